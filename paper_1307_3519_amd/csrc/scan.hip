// scan.hip -- dispatch of the fused scan kernel over (element type, form,
// mode); the template instances live in scan_{f16,i8}_*.hip so that they
// compile in parallel.  The kernel itself is in scan_kernel.h.
#include "kx_args.h"

extern "C" {
hipError_t kx_scan_f16_diag(const kx::ScanArgs*, int, int, hipStream_t);
hipError_t kx_scan_f16_miss(const kx::ScanArgs*, int, int, hipStream_t);
hipError_t kx_scan_f16_full(const kx::ScanArgs*, int, int, hipStream_t);
hipError_t kx_scan_f16_sums(const kx::ScanArgs*, int, int, hipStream_t);
hipError_t kx_scan_i8_diag(const kx::ScanArgs*, int, int, hipStream_t);
hipError_t kx_scan_i8_miss(const kx::ScanArgs*, int, int, hipStream_t);
hipError_t kx_scan_i8_full(const kx::ScanArgs*, int, int, hipStream_t);
hipError_t kx_scan_i8_sums(const kx::ScanArgs*, int, int, hipStream_t);

hipError_t kx_launch_scan(const kx::ScanArgs* a, int elem, int ks, int form, int mode, int grid,
                          hipStream_t st) {
    using namespace kx;
    const bool f16 = elem == F16;
    if (elem != F16 && elem != I8) return hipErrorInvalidValue;
    if (mode == SCREEN && form == DIAG)
        return f16 ? kx_scan_f16_diag(a, ks, grid, st) : kx_scan_i8_diag(a, ks, grid, st);
    if (form != MISS3) return hipErrorInvalidValue;
    if (mode == SCREEN) return f16 ? kx_scan_f16_miss(a, ks, grid, st) : kx_scan_i8_miss(a, ks, grid, st);
    if (mode == FULL) return f16 ? kx_scan_f16_full(a, ks, grid, st) : kx_scan_i8_full(a, ks, grid, st);
    if (mode == SUMS) return f16 ? kx_scan_f16_sums(a, ks, grid, st) : kx_scan_i8_sums(a, ks, grid, st);
    return hipErrorInvalidValue;
}
}
