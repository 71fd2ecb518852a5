// scan_f16_diag.hip -- fp16 MFMA, complete SNP tiles, screen mode (the hot path)
#include "scan_kernel.h"

extern "C" hipError_t kx_scan_f16_diag(const kx::ScanArgs* a, int ks, int grid, hipStream_t st) {
    using namespace kx;
    switch (ks) {
        case 1: return a->ring == 2 ? launch_one<F16, 1, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 1, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 1, DIAG, SCREEN, 2>(*a, grid, st);
        case 2: return a->ring == 2 ? launch_one<F16, 2, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 2, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 2, DIAG, SCREEN, 2>(*a, grid, st);
        case 3: return a->ring == 2 ? launch_one<F16, 3, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 3, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 3, DIAG, SCREEN, 2>(*a, grid, st);
        case 4: return a->ring == 2 ? launch_one<F16, 4, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 4, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 4, DIAG, SCREEN, 2>(*a, grid, st);
        case 5: return a->ring == 2 ? launch_one<F16, 5, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 5, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 5, DIAG, SCREEN, 2>(*a, grid, st);
        case 6: return a->ring == 2 ? launch_one<F16, 6, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 6, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 6, DIAG, SCREEN, 2>(*a, grid, st);
        case 7: return a->ring == 2 ? launch_one<F16, 7, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 7, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 7, DIAG, SCREEN, 2>(*a, grid, st);
        case 8: return a->ring == 2 ? launch_one<F16, 8, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<F16, 8, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<F16, 8, DIAG, SCREEN, 2>(*a, grid, st);
        default: return hipErrorInvalidValue;
    }
}
