// sort.hip -- deterministic (trait, snp) order of the compacted hit list.
// Hits are appended by atomics in arbitrary order; the hits present are
// sorted by the key trait * 2^32 + snp with the radix sort of radix.h, then
// gathered into the caller's buffer.
#include <algorithm>
#include <cstring>
#include "kx_common.h"
#include "radix.h"

namespace kx {

__global__ void make_hit_keys(const HitRec* __restrict__ stage, const unsigned long long* n_hits,
                              int64_t cap, unsigned long long* __restrict__ keys,
                              uint32_t* __restrict__ idx) {
    int64_t n = (int64_t)*n_hits;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        idx[i] = (uint32_t)i;
        keys[i] = ((unsigned long long)(uint32_t)stage[i].trait << 32) | (uint32_t)stage[i].snp;
    }
}

__global__ void gather_hits(const HitRec* __restrict__ stage, const unsigned long long* n_hits,
                            int64_t cap, const uint32_t* __restrict__ idx,
                            HitRec* __restrict__ out, int64_t* __restrict__ n_out) {
    int64_t n = (int64_t)*n_hits;
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = n;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = stage[idx[i]];
}

// Empirical FDR curve (P-value calculation and empirical FDR correction):
// the p-values of a hit list as sortable keys (the bits of a positive double
// order as the double does)
__global__ void p_keys(const HitRec* __restrict__ hits, const int64_t* n_hits, int64_t cap,
                       unsigned long long* __restrict__ keys) {
    int64_t n = *n_hits;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        keys[i] = dbl_bits(hits[i].p);
}

// number of the first n sorted keys that are <= key
__device__ inline int64_t count_le(const unsigned long long* __restrict__ sorted, int64_t n,
                                   unsigned long long key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (sorted[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// fdr[i] = (#{permuted hits with p <= p_i} / P) / #{real hits with p <= p_i}
// for each real hit i, from both lists' sorted p-value keys.
__global__ void fdr_eval(const HitRec* __restrict__ real, const int64_t* n_real, int64_t real_cap,
                         const unsigned long long* __restrict__ real_sorted,
                         const int64_t* n_perm, int64_t perm_cap,
                         const unsigned long long* __restrict__ perm_sorted, int P,
                         double* __restrict__ fdr) {
    int64_t nr = *n_real, np = *n_perm;
    if (nr > real_cap) nr = real_cap;
    if (np > perm_cap) np = perm_cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long key = dbl_bits(real[i].p);
        const int64_t cr = count_le(real_sorted, nr, key);
        const int64_t cp = count_le(perm_sorted, np, key);
        fdr[i] = (double)cp / ((double)P * (double)cr);
    }
}

}  // namespace kx

extern "C" size_t kx_sort_tmp_bytes(int64_t cap) { return kx::radix_tmp_bytes(cap); }

// keys/idx: 2 x cap each (ping-pong halves); tmp of kx_sort_tmp_bytes(cap).
// The key of a hit is trait * 2^32 + snp; only the digits that can be
// non-zero are sorted: bits [0, snp_bits) and [32, 32 + trait_bits).
extern "C" hipError_t kx_sort_hits(const kx::HitRec* stage, const unsigned long long* n_hits,
                                   int64_t cap, unsigned long long* keys, uint32_t* idx,
                                   void* tmp, size_t tmp_bytes, kx::HitRec* out, int64_t* n_out,
                                   int trait_bits, int snp_bits, hipStream_t st) {
    (void)tmp_bytes;
    if (cap <= 0) {
        hipLaunchKernelGGL(kx::gather_hits, dim3(1), dim3(64), 0, st, stage, n_hits, (int64_t)0,
                           idx, out, n_out);
        return hipGetLastError();
    }
    const int grid = (int)std::min<int64_t>(kx::radix_blocks(cap) * 8, 2048);
    hipLaunchKernelGGL(kx::make_hit_keys, dim3(grid), dim3(256), 0, st, stage, n_hits, cap, keys,
                       idx);
    int shifts[8], n_pass = 0;
    for (int b = 0; b < std::max(snp_bits, 1); b += 8) shifts[n_pass++] = b;
    for (int b = 0; b < std::max(trait_bits, 1); b += 8) shifts[n_pass++] = 32 + b;
    int half = 0;
    hipError_t e = kx::radix_sort((uint64_t*)keys, idx, n_hits, cap, shifts, n_pass, tmp, st,
                                  &half);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kx::gather_hits, dim3(grid), dim3(256), 0, st, stage, n_hits, cap,
                       idx + (half ? cap : 0), out, n_out);
    return hipGetLastError();
}

extern "C" size_t kx_sort_keys_tmp_bytes(int64_t cap) { return kx::radix_tmp_bytes(cap); }

// keys_r: 2 x real_cap, keys_p: 2 x perm_cap (ping-pong halves); tmp of
// kx_sort_keys_tmp_bytes(max(real_cap, perm_cap)).  The p-value keys are the
// bits of positive doubles: all eight digits are sorted (an even number of
// passes, so the sorted keys end in the first half).
extern "C" hipError_t kx_fdr_curve(const kx::HitRec* real, const int64_t* n_real, int64_t real_cap,
                                   const kx::HitRec* perm, const int64_t* n_perm, int64_t perm_cap,
                                   int P, unsigned long long* keys_r, unsigned long long* keys_p,
                                   void* tmp, size_t tmp_bytes, double* fdr, hipStream_t st) {
    (void)tmp_bytes;
    if (real_cap <= 0) return hipSuccess;
    static const int kAll[8] = {0, 8, 16, 24, 32, 40, 48, 56};
    int half = 0;
    const int gr = (int)std::min<int64_t>(kx::radix_blocks(real_cap) * 8, 2048);
    hipLaunchKernelGGL(kx::p_keys, dim3(gr), dim3(256), 0, st, real, n_real, real_cap, keys_r);
    hipError_t e = kx::radix_sort((uint64_t*)keys_r, nullptr, (const unsigned long long*)n_real,
                                  real_cap, kAll, 8, tmp, st, &half);
    if (e != hipSuccess) return e;
    if (perm_cap > 0) {
        const int gp = (int)std::min<int64_t>(kx::radix_blocks(perm_cap) * 8, 2048);
        hipLaunchKernelGGL(kx::p_keys, dim3(gp), dim3(256), 0, st, perm, n_perm, perm_cap,
                           keys_p);
        e = kx::radix_sort((uint64_t*)keys_p, nullptr, (const unsigned long long*)n_perm,
                           perm_cap, kAll, 8, tmp, st, &half);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kx::fdr_eval, dim3(256), dim3(256), 0, st, real, n_real, real_cap,
                       keys_r, n_perm, perm_cap, keys_p, P, fdr);
    return hipGetLastError();
}
