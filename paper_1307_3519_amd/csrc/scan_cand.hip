// scan_cand.hip -- launcher of the exact evaluation of screened pairs.
#include "scan_kernel.h"

namespace kx {

// Exact evaluation of the screened pairs collected by scan_kernel.
__global__ __launch_bounds__(256) void scan_candidates(ScanArgs a) {
    int64_t n = (int64_t)*a.n_cand;
    if (n > a.cand_cap) n = a.cand_cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 e = a.cand[i];
        eval_candidate(a, (int64_t)e.x, (int64_t)(e.y & kCandSnp), __uint_as_float(e.z),
                       __uint_as_float(e.w), e.y & ~kCandSnp);
    }
}

}  // namespace kx

extern "C" hipError_t kx_launch_candidates(const kx::ScanArgs* a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kx::scan_candidates, dim3(grid), dim3(256), 0, st, *a);
    return hipGetLastError();
}
