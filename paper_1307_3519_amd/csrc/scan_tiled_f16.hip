// scan_tiled_f16.hip -- fp16 instances of the tiled scan (K > 128) and of
// the column expansion.
#include "scan_tiled.h"

extern "C" hipError_t kx_launch_tiled_f16(const kx::ScanArgs* a, const kx::TiledArgs* ta, int form,
                                          int mode, int grid, hipStream_t st) {
    using namespace kx;
    if (mode == SCREEN) {
        if (form == DIAG) return launch_tiled<F16, DIAG, SCREEN, false>(*a, *ta, grid, st);
        if (form == PLAIN) return launch_tiled<F16, PLAIN, SCREEN, false>(*a, *ta, grid, st);
        if (form == MISS3) return launch_tiled<F16, MISS3, SCREEN, false>(*a, *ta, grid, st);
    } else if (form == MISS3) {
        if (mode == FULL) return launch_tiled<F16, MISS3, FULL, false>(*a, *ta, grid, st);
        if (mode == SUMS) return launch_tiled<F16, MISS3, SUMS, false>(*a, *ta, grid, st);
    }
    return hipErrorInvalidValue;
}

extern "C" hipError_t kx_launch_expand_f16(const int8_t* G, int gstride, const kx::SnpInfo* info,
                                           int64_t n_tiles_pad, int ks, int form, void* Bf,
                                           int grid, hipStream_t st) {
    using namespace kx;
    if (form == DIAG)
        hipLaunchKernelGGL((expand_columns<F16, DIAG>), dim3(grid), dim3(256), 0, st, G, gstride, info, n_tiles_pad, ks, Bf);
    else if (form == PLAIN)
        hipLaunchKernelGGL((expand_columns<F16, PLAIN>), dim3(grid), dim3(256), 0, st, G, gstride, info, n_tiles_pad, ks, Bf);
    else if (form == MISS3)
        hipLaunchKernelGGL((expand_columns<F16, MISS3>), dim3(grid), dim3(256), 0, st, G, gstride, info, n_tiles_pad, ks, Bf);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
