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

// Exact evaluation of the screened pairs of SNPs with missing genotypes
// (re-ranking over the kept samples), one pair per wave at a time.
__global__ __launch_bounds__(256) void scan_missing(ScanArgs a) {
    extern __shared__ int16_t s_buf[];   // per wave 2K entries
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int16_t* sb = s_buf + wave * 2 * a.K;
    int64_t n = (int64_t)*a.n_mcand;
    if (n > a.mcand_cap) n = a.mcand_cap;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; e < n; e += waves) {
        const int2 q = a.mcand[e];
        const int64_t v = a.row_v[q.x];
        if (v < 0) continue;             // padding row (uniform per wave)
        int df;
        int64_t s[3];
        const double H = coop_exact(a, v, q.y, sb, lane, &df, s);
        if (lane == 0) record(a, v, q.y, H, df);
    }
}

}  // namespace kx

extern "C" hipError_t kx_launch_missing(const kx::ScanArgs* a, int grid, hipStream_t st) {
    const size_t lds = (size_t)4 * 2 * a->K * sizeof(int16_t);
    hipLaunchKernelGGL(kx::scan_missing, dim3(grid), dim3(256), lds, st, *a);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_candidates(const kx::ScanArgs* a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kx::scan_candidates, dim3(grid), dim3(256), 0, st, *a);
    return hipGetLastError();
}
