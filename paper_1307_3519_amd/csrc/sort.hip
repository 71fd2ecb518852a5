// sort.hip -- deterministic (trait, snp) order of the compacted hit list.
// Hits are appended by atomics in arbitrary order; they are sorted by the
// key trait * 2^32 + snp with rocPRIM's device radix sort over the whole
// staging capacity (unused slots carry the largest key), then gathered into
// the caller's buffer.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include "kx_common.h"

namespace kx {

__global__ void make_hit_keys(const HitRec* __restrict__ stage, const unsigned long long* n_hits,
                              int64_t cap, unsigned long long* __restrict__ keys,
                              uint32_t* __restrict__ idx) {
    int64_t n = (int64_t)*n_hits;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
         i += (int64_t)gridDim.x * blockDim.x) {
        idx[i] = (uint32_t)i;
        keys[i] = i < n ? ((unsigned long long)(uint32_t)stage[i].trait << 32) |
                              (uint32_t)stage[i].snp
                        : ~0ull;
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
// order as the double does), unused slots +inf.
__global__ void p_keys(const HitRec* __restrict__ hits, const int64_t* n_hits, int64_t cap,
                       unsigned long long* __restrict__ keys) {
    int64_t n = *n_hits;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
         i += (int64_t)gridDim.x * blockDim.x)
        keys[i] = i < n ? dbl_bits(hits[i].p) : 0x7FF0000000000000ull;
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

extern "C" size_t kx_sort_tmp_bytes(int64_t cap) {
    size_t bytes = 0;
    (void)rocprim::radix_sort_pairs((void*)nullptr, bytes, (unsigned long long*)nullptr,
                                    (unsigned long long*)nullptr, (uint32_t*)nullptr,
                                    (uint32_t*)nullptr, (size_t)cap, 0, 64);
    return bytes;
}

// keys/idx: 2 x cap each (in, out); tmp of kx_sort_tmp_bytes(cap).
extern "C" hipError_t kx_sort_hits(const kx::HitRec* stage, const unsigned long long* n_hits,
                                   int64_t cap, unsigned long long* keys, uint32_t* idx,
                                   void* tmp, size_t tmp_bytes, kx::HitRec* out, int64_t* n_out,
                                   int key_bits, hipStream_t st) {
    if (cap <= 0) {
        hipLaunchKernelGGL(kx::gather_hits, dim3(1), dim3(64), 0, st, stage, n_hits, (int64_t)0,
                           idx, out, n_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(kx::make_hit_keys, dim3(256), dim3(256), 0, st, stage, n_hits, cap, keys,
                       idx);
    hipError_t e = rocprim::radix_sort_pairs(tmp, tmp_bytes, keys, keys + cap, idx, idx + cap,
                                             (size_t)cap, 0, key_bits, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kx::gather_hits, dim3(256), dim3(256), 0, st, stage, n_hits, cap,
                       idx + cap, out, n_out);
    return hipGetLastError();
}

extern "C" size_t kx_sort_keys_tmp_bytes(int64_t cap) {
    size_t bytes = 0;
    (void)rocprim::radix_sort_keys((void*)nullptr, bytes, (unsigned long long*)nullptr,
                                   (unsigned long long*)nullptr, (size_t)cap, 0, 64);
    return bytes;
}

// keys_r: 2 x real_cap, keys_p: 2 x perm_cap (in, out); tmp of
// kx_sort_keys_tmp_bytes(max(real_cap, perm_cap)).
extern "C" hipError_t kx_fdr_curve(const kx::HitRec* real, const int64_t* n_real, int64_t real_cap,
                                   const kx::HitRec* perm, const int64_t* n_perm, int64_t perm_cap,
                                   int P, unsigned long long* keys_r, unsigned long long* keys_p,
                                   void* tmp, size_t tmp_bytes, double* fdr, hipStream_t st) {
    if (real_cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(kx::p_keys, dim3(256), dim3(256), 0, st, real, n_real, real_cap, keys_r);
    hipError_t e = rocprim::radix_sort_keys(tmp, tmp_bytes, keys_r, keys_r + real_cap,
                                            (size_t)real_cap, 0, 64, st);
    if (e != hipSuccess) return e;
    if (perm_cap > 0) {
        hipLaunchKernelGGL(kx::p_keys, dim3(256), dim3(256), 0, st, perm, n_perm, perm_cap,
                           keys_p);
        e = rocprim::radix_sort_keys(tmp, tmp_bytes, keys_p, keys_p + perm_cap, (size_t)perm_cap,
                                     0, 64, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kx::fdr_eval, dim3(256), dim3(256), 0, st, real, n_real, real_cap,
                       keys_r + real_cap, n_perm, perm_cap, keys_p + perm_cap, P, fdr);
    return hipGetLastError();
}
