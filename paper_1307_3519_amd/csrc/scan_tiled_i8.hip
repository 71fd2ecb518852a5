// scan_tiled_i8.hip -- int8 instances of the tiled scan: the centred rank
// split into bytes (two accumulator sets), indicator columns.
#include "scan_tiled.h"

extern "C" hipError_t kx_launch_tiled_i8(const kx::ScanArgs* a, const kx::TiledArgs* ta, int form,
                                         int mode, int grid, hipStream_t st) {
    using namespace kx;
    if (mode == SCREEN) {
        if (form == PLAIN) return launch_tiled<I8, PLAIN, SCREEN, true>(*a, *ta, grid, st);
        if (form == MISS3) return launch_tiled<I8, MISS3, SCREEN, true>(*a, *ta, grid, st);
    } else if (form == MISS3) {
        if (mode == FULL) return launch_tiled<I8, MISS3, FULL, true>(*a, *ta, grid, st);
        if (mode == SUMS) return launch_tiled<I8, MISS3, SUMS, true>(*a, *ta, grid, st);
    }
    return hipErrorInvalidValue;
}

extern "C" hipError_t kx_launch_expand_i8(const int8_t* G, int gstride, const kx::SnpInfo* info,
                                          int64_t n_tiles_pad, int ks, int form, void* Bf,
                                          int grid, hipStream_t st) {
    using namespace kx;
    if (form == PLAIN)
        hipLaunchKernelGGL((expand_columns<I8, PLAIN>), dim3(grid), dim3(256), 0, st, G, gstride, info, n_tiles_pad, ks, Bf);
    else if (form == MISS3)
        hipLaunchKernelGGL((expand_columns<I8, MISS3>), dim3(grid), dim3(256), 0, st, G, gstride, info, n_tiles_pad, ks, Bf);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
