// scan_i8_diag.hip -- int8 MFMA, complete SNP tiles, screen mode
#include "scan_kernel.h"

extern "C" hipError_t kx_scan_i8_diag(const kx::ScanArgs* a, int ks, int grid, hipStream_t st) {
    using namespace kx;
    switch (ks) {
        case 1: return a->ring == 2 ? launch_one<I8, 1, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<I8, 1, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<I8, 1, DIAG, SCREEN, 2>(*a, grid, st);
        case 2: return a->ring == 2 ? launch_one<I8, 2, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<I8, 2, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<I8, 2, DIAG, SCREEN, 2>(*a, grid, st);
        case 3: return a->ring == 2 ? launch_one<I8, 3, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<I8, 3, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<I8, 3, DIAG, SCREEN, 2>(*a, grid, st);
        case 4: return a->ring == 2 ? launch_one<I8, 4, DIAG, SCREEN, 4, 3>(*a, grid, st)
                         : a->ring ? launch_one<I8, 4, DIAG, SCREEN, 3>(*a, grid, st)
                                   : launch_one<I8, 4, DIAG, SCREEN, 2>(*a, grid, st);
        default: return hipErrorInvalidValue;
    }
}
