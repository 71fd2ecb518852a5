// scan_i8_diag.hip -- int8 MFMA, complete SNP tiles, screen mode
#include "scan_kernel.h"

extern "C" hipError_t kx_scan_i8_diag(const kx::ScanArgs* a, int ks, int grid, hipStream_t st) {
    using namespace kx;
    switch (ks) {
        case 1: return launch_one<I8, 1, DIAG, SCREEN>(*a, grid, st);
        case 2: return launch_one<I8, 2, DIAG, SCREEN>(*a, grid, st);
        case 3: return launch_one<I8, 3, DIAG, SCREEN>(*a, grid, st);
        case 4: return launch_one<I8, 4, DIAG, SCREEN>(*a, grid, st);
        default: return hipErrorInvalidValue;
    }
}
