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
