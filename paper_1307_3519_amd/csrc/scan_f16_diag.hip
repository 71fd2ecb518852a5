// scan_f16_diag.hip -- fp16 MFMA, complete SNP tiles, screen mode (the hot path)
#include "scan_kernel.h"

extern "C" hipError_t kx_scan_f16_diag(const kx::ScanArgs* a, int ks, int grid, hipStream_t st) {
    using namespace kx;
    switch (ks) {
        case 1: return launch_diag_screen<F16, 1>(*a, grid, st);
        case 2: return launch_diag_screen<F16, 2>(*a, grid, st);
        case 3: return launch_diag_screen<F16, 3>(*a, grid, st);
        case 4: return launch_diag_screen<F16, 4>(*a, grid, st);
        case 5: return launch_diag_screen<F16, 5>(*a, grid, st);
        case 6: return launch_diag_screen<F16, 6>(*a, grid, st);
        case 7: return launch_diag_screen<F16, 7>(*a, grid, st);
        case 8: return launch_diag_screen<F16, 8>(*a, grid, st);
        default: return hipErrorInvalidValue;
    }
}
