// group.hip -- SNPs grouped by their pattern of missing genotypes (Handling
// missing values: one sub-problem per pattern, its samples removed from both
// matrices).  The kernels key each SNP by its pattern, check a group's
// members against the pattern, gather the sub-problem's columns and rows,
// and merge the sub-problems' hit lists and per-trait minima.
#include <algorithm>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_run_length_encode.hpp>
#include "kx_common.h"

namespace kx {

// splitmix64 finaliser (Steele, Lea and Flood, 2014): a 64-bit mixing of k
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline bool is_missing(int8_t g) { return g < 0 || g > 2; }

// key[m] = sum over the SNP's missing samples k of mix64(k) (mod 2^64); 0
// for a complete SNP.  One wave per SNP.
__global__ __launch_bounds__(256) void miss_keys(const int8_t* __restrict__ geno, int64_t M,
                                                 int64_t ld, int K, uint64_t* __restrict__ key) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t m = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); m < M;
         m += waves) {
        uint64_t h = 0;
        for (int k = lane; k < K; k += kWave)
            if (is_missing(geno[m * ld + k])) h += mix64((uint64_t)k);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
        if (lane == 0) key[m] = h;
    }
}

// Part of every SNP: the index of its key among the G sorted group keys, G
// (the ungrouped rest) when absent.  A stable sort of (part, SNP) then lists
// each part's SNPs in ascending order, the parts one after the other.
__global__ void part_ids(const uint64_t* __restrict__ key, int64_t M,
                         const uint64_t* __restrict__ big, int G, int32_t* __restrict__ pid,
                         int32_t* __restrict__ idx) {
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M;
         m += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[m];
        int lo = 0, hi = G;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (big[mid] < k) lo = mid + 1;
            else hi = mid;
        }
        pid[m] = (k != 0 && lo < G && big[lo] == k) ? lo : G;
        idx[m] = (int32_t)m;
    }
}

// qmask[g][k] = 1 when sample k is missing at the first SNP of group g's
// slice of list (any member: all are checked against it afterwards).
__global__ void pattern_mask(const int8_t* __restrict__ geno, int64_t ld, int K,
                             const int32_t* __restrict__ list, const int64_t* __restrict__ off,
                             int G, uint8_t* __restrict__ qmask) {
    const int64_t n = (int64_t)G * K;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = i / K;
        const int k = (int)(i - g * K);
        qmask[i] = is_missing(geno[(int64_t)list[off[g]] * ld + k]) ? 1 : 0;
    }
}

// Counts the SNPs of a list whose missing samples differ from qmask (1 =
// missing).  One wave per SNP.
__global__ __launch_bounds__(256) void check_pattern(const int8_t* __restrict__ geno, int64_t ld,
                                                     int K, const int32_t* __restrict__ snps,
                                                     int64_t n, const uint8_t* __restrict__ qmask,
                                                     unsigned long long* bad) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n;
         i += waves) {
        const int64_t m = snps[i];
        bool diff = false;
        for (int k = lane; k < K; k += kWave)
            diff = diff || (is_missing(geno[m * ld + k]) != (qmask[k] != 0));
        if (__any(diff) && lane == 0) atomicAdd(bad, 1ull);
    }
}

// out[t][j] = the rank of sample S[j] as a float (NaN for a missing
// expression value): ranking these reproduces the ranks over the kept samples
// (ranks order the samples as their values do, ties included).
__global__ void gather_rank_cols(const int16_t* __restrict__ ranks2, int64_t T, int K,
                                 const int32_t* __restrict__ S, int Kp, float* __restrict__ out) {
    const int64_t n = T * Kp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / Kp;
        const int j = (int)(i - t * Kp);
        const int a = ranks2[t * K + S[j]];
        out[i] = a == 0 ? __builtin_nanf("") : (float)a;
    }
}

// out[i][j] = geno[rows[i]][S[j]] (S null: j itself), row stride Kp.
__global__ void gather_geno(const int8_t* __restrict__ geno, int64_t ld,
                            const int32_t* __restrict__ rows, int64_t n,
                            const int32_t* __restrict__ S, int Kp, int8_t* __restrict__ out) {
    const int64_t total = n * Kp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / Kp;
        const int j = (int)(i - r * Kp);
        out[i] = geno[(int64_t)rows[r] * ld + (S ? S[j] : j)];
    }
}

// Appends a sub-problem's hits (SNP indices local to its list) to the merged
// staging list with the SNP mapped back; total receives the true count.
__global__ void append_hits(const HitRec* __restrict__ part, const int64_t* part_n, int64_t cap,
                            const int32_t* __restrict__ snp_map, int64_t snp_base,
                            HitRec* __restrict__ stage, unsigned long long* stored,
                            unsigned long long* total) {
    int64_t n = *part_n;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(total, (unsigned long long)n);
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        HitRec h = part[i];
        const unsigned long long idx = atomicAdd(stored, 1ull);
        if ((int64_t)idx >= cap) continue;
        h.snp = (int32_t)(snp_map[h.snp] + snp_base);
        stage[idx] = h;
    }
}

__global__ void min_merge(const double* __restrict__ part, double* __restrict__ acc, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc[i] = fmin(acc[i], part[i]);
}

// *n_out = the true count; the stored count is capped at cap.
__global__ void set_counts(int64_t* n_out, const unsigned long long* total,
                           unsigned long long* stored, int64_t cap) {
    *n_out = (int64_t)*total;
    if ((int64_t)*stored > cap) *stored = (unsigned long long)cap;
}

}  // namespace kx

extern "C" hipError_t kx_launch_miss_keys(const int8_t* geno, int64_t M, int64_t ld, int K,
                                          uint64_t* key, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kx::miss_keys, dim3(grid), dim3(256), 0, st, geno, M, ld, K, key);
    return hipGetLastError();
}

// Sorted copy of the keys and its runs: uniq[r], counts[r] for r < *n_runs.
extern "C" size_t kx_group_tmp_bytes(int64_t M) {
    size_t a = 0, b = 0;
    (void)rocprim::radix_sort_keys((void*)nullptr, a, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                   (size_t)M, 0, 64);
    (void)rocprim::run_length_encode((void*)nullptr, b, (uint64_t*)nullptr, (unsigned int)M,
                                     (uint64_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr);
    size_t c = 0;
    (void)rocprim::radix_sort_pairs((void*)nullptr, c, (const uint32_t*)nullptr,
                                    (uint32_t*)nullptr, (const int32_t*)nullptr,
                                    (int32_t*)nullptr, (size_t)M, 0, 31);
    return std::max(a, std::max(b, c));
}

extern "C" hipError_t kx_group_runs(const uint64_t* key, int64_t M, uint64_t* sorted,
                                    uint64_t* uniq, uint32_t* counts, uint32_t* n_runs, void* tmp,
                                    size_t tmp_bytes, hipStream_t st) {
    size_t bytes = tmp_bytes;
    hipError_t e = rocprim::radix_sort_keys(tmp, bytes, key, sorted, (size_t)M, 0, 64, st);
    if (e != hipSuccess) return e;
    bytes = tmp_bytes;
    return rocprim::run_length_encode(tmp, bytes, sorted, (unsigned int)M, uniq, counts, n_runs,
                                      st);
}

// pid, pid_sorted, idx: M int32 each; list receives the SNPs by part.
extern "C" hipError_t kx_group_parts(const uint64_t* key, int64_t M, const uint64_t* big, int G,
                                     int32_t* pid, int32_t* pid_sorted, int32_t* idx,
                                     int32_t* list, void* tmp, size_t tmp_bytes, int grid,
                                     hipStream_t st) {
    hipLaunchKernelGGL(kx::part_ids, dim3(grid), dim3(256), 0, st, key, M, big, G, pid, idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int bits = 1;
    while (bits < 31 && (1 << bits) <= G) ++bits;
    size_t bytes = tmp_bytes;
    return rocprim::radix_sort_pairs(tmp, bytes, (const uint32_t*)pid, (uint32_t*)pid_sorted,
                                     idx, list, (size_t)M, 0, bits, st);
}

extern "C" hipError_t kx_launch_pattern_mask(const int8_t* geno, int64_t ld, int K,
                                             const int32_t* list, const int64_t* off, int G,
                                             uint8_t* qmask, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kx::pattern_mask, dim3(grid), dim3(256), 0, st, geno, ld, K, list, off, G,
                       qmask);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_check_pattern(const int8_t* geno, int64_t ld, int K,
                                              const int32_t* snps, int64_t n,
                                              const uint8_t* qmask, unsigned long long* bad,
                                              int grid, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(kx::check_pattern, dim3(grid), dim3(256), 0, st, geno, ld, K, snps, n,
                       qmask, bad);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_gather_rank_cols(const int16_t* ranks2, int64_t T, int K,
                                                 const int32_t* S, int Kp, float* out, int grid,
                                                 hipStream_t st) {
    if (T * Kp <= 0) return hipSuccess;
    hipLaunchKernelGGL(kx::gather_rank_cols, dim3(grid), dim3(256), 0, st, ranks2, T, K, S, Kp,
                       out);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_gather_geno(const int8_t* geno, int64_t ld, const int32_t* rows,
                                            int64_t n, const int32_t* S, int Kp, int8_t* out,
                                            int grid, hipStream_t st) {
    if (n * Kp <= 0) return hipSuccess;
    hipLaunchKernelGGL(kx::gather_geno, dim3(grid), dim3(256), 0, st, geno, ld, rows, n, S, Kp,
                       out);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_append_hits(const kx::HitRec* part, const int64_t* part_n,
                                            int64_t cap, const int32_t* snp_map, int64_t snp_base,
                                            kx::HitRec* stage, unsigned long long* stored,
                                            unsigned long long* total, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kx::append_hits, dim3(grid), dim3(256), 0, st, part, part_n, cap, snp_map,
                       snp_base, stage, stored, total);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_min_merge(const double* part, double* acc, int64_t n, int grid,
                                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(kx::min_merge, dim3(grid), dim3(256), 0, st, part, acc, n);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_set_counts(int64_t* n_out, const unsigned long long* total,
                                           unsigned long long* stored, int64_t cap,
                                           hipStream_t st) {
    hipLaunchKernelGGL(kx::set_counts, dim3(1), dim3(1), 0, st, n_out, total, stored, cap);
    return hipGetLastError();
}
