// radix.h -- stable least-significant-digit radix sort of 64-bit keys, with
// optional 32-bit values, over an element count that lives on the device.
//
// Used for the hit lists and the p-value keys of the FDR curve, on streams
// that a caller may capture into a graph: every buffer is written by a kernel
// before it is read (no memset, no library temporaries), and only the
// n = min(*count, cap) elements present are moved.
//
// One pass per 8-bit digit of the requested bit positions, three kernels a
// pass:
//   radix_count    block b histograms the digits of its tile of 2048 keys
//                  into hist[digit][b] (blocks past n write zeros)
//   radix_scan     block d turns row hist[d][.] into exclusive offsets and
//                  writes the digit's total
//   radix_scatter  block b moves its keys (and values) to
//                  base(digit) + hist[digit][b] + rank; the rank of a key
//                  among equal digits of the tile follows the key order:
//                  within a wave from the digit's 8 ballots, across waves
//                  and rounds from per-digit counters in LDS
#pragma once
#include "kx_common.h"

namespace kx {

constexpr int kRadixBins = 256;
constexpr int kRadixThreads = 256;
constexpr int kRadixIpt = 8;                             // keys per thread
constexpr int kRadixTile = kRadixThreads * kRadixIpt;   // keys per block

__host__ __device__ inline int64_t radix_blocks(int64_t cap) {
    const int64_t b = (cap + kRadixTile - 1) / kRadixTile;
    return b > 0 ? b : 1;
}

// Bytes of the count table: hist[256][blocks] and the 256 digit totals.
inline size_t radix_tmp_bytes(int64_t cap) {
    return (size_t)(kRadixBins * radix_blocks(cap) + kRadixBins) * sizeof(uint32_t);
}

__device__ inline int64_t radix_n(const unsigned long long* count, int64_t cap) {
    const unsigned long long n = *count;
    return n < (unsigned long long)cap ? (int64_t)n : cap;
}

__global__ __launch_bounds__(kRadixThreads) void radix_count(
    const uint64_t* __restrict__ keys, const unsigned long long* count, int64_t cap, int shift,
    uint32_t* __restrict__ hist, int64_t nb) {
    __shared__ uint32_t h[kRadixBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = radix_n(count, cap);
    const int64_t b0 = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
    for (int j = 0; j < kRadixIpt; ++j) {
        const int64_t i = b0 + j * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kRadixBins - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the values of a block's threads (blockDim.x = 64 * W
// with W <= 16); *total receives the sum.
template <int THREADS>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* lds16, uint32_t* total) {
    constexpr int W = THREADS / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
    }
    if (lane == 63) lds16[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const uint32_t t = lds16[k];
        before += k < w ? t : 0u;
        all += t;
    }
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(1024) void radix_scan(uint32_t* __restrict__ hist, int64_t nb,
                                                   uint32_t* __restrict__ totals) {
    __shared__ uint32_t part[16];
    uint32_t* row = hist + (int64_t)blockIdx.x * nb;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += row[i];
    uint32_t total = 0;
    uint32_t run = block_excl_scan<1024>(s, part, &total);
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

template <bool VALS>
__global__ __launch_bounds__(kRadixThreads) void radix_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const unsigned long long* count, int64_t cap, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, int64_t nb) {
    __shared__ uint32_t base[kRadixBins];                          // next slot per digit
    __shared__ uint32_t wcnt[kRadixThreads / 64][kRadixBins];     // per wave, this round
    __shared__ uint32_t part[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t n = radix_n(count, cap);
    const int64_t b0 = (int64_t)blockIdx.x * kRadixTile;
    if (b0 >= n) return;                                           // uniform per block
    uint32_t all = 0;
    const uint32_t dbase = block_excl_scan<kRadixThreads>(totals[t], part, &all);
    base[t] = dbase + hist[(int64_t)t * nb + blockIdx.x];
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int j = 0; j < kRadixIpt; ++j) {
#pragma unroll
        for (int k = 0; k < kRadixThreads / 64; ++k) wcnt[k][t] = 0;
        __syncthreads();
        const int64_t i = b0 + j * kRadixThreads + t;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & (kRadixBins - 1);
        // lanes of this wave holding a key with the same digit
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long b = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? b : ~b;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        if (valid && rank + 1 == cnt) wcnt[w][d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + rank;
            for (int k = 0; k < w; ++k) off += wcnt[k][d];
            kout[off] = key;
            if constexpr (VALS) vout[off] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < kRadixThreads / 64; ++k) add += wcnt[k][t];
        base[t] += add;
        __syncthreads();
    }
}

// Sorts keys[0, n) (and vals[0, n) along) on the digits at `shifts`
// (n_pass entries, ascending), ping-ponging with keys[cap, 2 cap) and
// vals[cap, 2 cap).  Returns the half (0 or 1) that holds the result.
// tmp: radix_tmp_bytes(cap) bytes.
inline hipError_t radix_sort(uint64_t* keys, uint32_t* vals, const unsigned long long* count,
                             int64_t cap, const int* shifts, int n_pass, void* tmp,
                             hipStream_t st, int* half) {
    const int64_t nb = radix_blocks(cap);
    uint32_t* hist = (uint32_t*)tmp;
    uint32_t* totals = hist + (int64_t)kRadixBins * nb;
    int h = 0;
    for (int ps = 0; ps < n_pass; ++ps) {
        uint64_t* kin = keys + (h ? cap : 0);
        uint64_t* kout = keys + (h ? 0 : cap);
        uint32_t* vin = vals ? vals + (h ? cap : 0) : nullptr;
        uint32_t* vout = vals ? vals + (h ? 0 : cap) : nullptr;
        hipLaunchKernelGGL(radix_count, dim3((unsigned)nb), dim3(kRadixThreads), 0, st, kin,
                           count, cap, shifts[ps], hist, nb);
        hipLaunchKernelGGL(radix_scan, dim3(kRadixBins), dim3(1024), 0, st, hist, nb, totals);
        if (vals)
            hipLaunchKernelGGL(radix_scatter<true>, dim3((unsigned)nb), dim3(kRadixThreads), 0, st,
                               kin, vin, kout, vout, count, cap, shifts[ps], hist, totals, nb);
        else
            hipLaunchKernelGGL(radix_scatter<false>, dim3((unsigned)nb), dim3(kRadixThreads), 0,
                               st, kin, vin, kout, vout, count, cap, shifts[ps], hist, totals, nb);
        h ^= 1;
    }
    *half = h;
    return hipGetLastError();
}

}  // namespace kx
