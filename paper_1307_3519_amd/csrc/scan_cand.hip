// scan_cand.hip -- exact evaluation of the pairs that passed the screen.
#include "scan_kernel.h"

namespace kx {

// One launch evaluates both buffers filled by the scan kernels:
//  * candidates of complete SNPs, one lane each: exact H from the pair's
//    exact MFMA column values (eq. (2) with the tie factor), p, hit / min p;
//  * pairs of SNPs with missing genotypes, one wave each: the ranks are
//    re-derived over the kept samples (coop_exact), then the same.
__global__ __launch_bounds__(256) void scan_exact(ScanArgs a) {
    int64_t n = (int64_t)*a.n_cand;
    if (n > a.cand_cap) n = a.cand_cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 e = a.cand[i];
        eval_candidate(a, (int64_t)e.x, (int64_t)(e.y & kCandSnp), __uint_as_float(e.z),
                       __uint_as_float(e.w), e.y & ~kCandSnp);
    }
    if (!a.mcand) return;
    extern __shared__ __attribute__((aligned(16))) int16_t s_buf[];   // per wave coop_lds_entries(K)
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int16_t* sb = s_buf + wave * coop_lds_entries(a.K);
    int64_t nm = (int64_t)*a.n_mcand;
    if (nm > a.mcand_cap) nm = a.mcand_cap;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; e < nm; e += waves) {
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

extern "C" hipError_t kx_launch_exact(const kx::ScanArgs* a, int grid, hipStream_t st) {
    const size_t lds = (size_t)4 * kx::coop_lds_entries(a->K) * sizeof(int16_t);
    hipLaunchKernelGGL(kx::scan_exact, dim3(grid), dim3(256), lds, st, *a);
    return hipGetLastError();
}
