// scan_i8_diag.hip -- int8 MFMA, complete SNP tiles, screen mode
#include "scan_kernel.h"

extern "C" hipError_t kx_scan_i8_diag(const kx::ScanArgs* a, int ks, int grid, hipStream_t st) {
    using namespace kx;
    switch (ks) {
        case 1: return launch_diag_screen<I8, 1>(*a, grid, st);
        case 2: return launch_diag_screen<I8, 2>(*a, grid, st);
        case 3: return launch_diag_screen<I8, 3>(*a, grid, st);
        case 4: return launch_diag_screen<I8, 4>(*a, grid, st);
        case 5: return launch_diag_screen<I8, 5>(*a, grid, st);
        case 6: return launch_diag_screen<I8, 6>(*a, grid, st);
        case 7: return launch_diag_screen<I8, 7>(*a, grid, st);
        case 8: return launch_diag_screen<I8, 8>(*a, grid, st);
        default: return hipErrorInvalidValue;
    }
}
