// rank.hip -- per-trait doubled midranks and tie term (the ranking step of
// the paper's input-data section and the tie term of its tied-data section).
//
// K > 256: one workgroup per trait row.  The row is sorted in LDS as 64-bit words
// (order-preserving 32-bit key of the value << 32 | sample index) by a
// bitonic network; a value's tie run [lo, hi) in the sorted row then gives
//   less = lo, eq = hi - lo,  a = 2 less + eq + 1 = lo + hi + 1,
// and the run contributes eq^2 - 1 per member, i.e. t^3 - t per tie group.
// NaN sorts last (key 0xFFFFFFFF, above +inf) and is not ranked.
#include "kx_common.h"

namespace kx {

__device__ inline uint32_t order_key(float v) {
    if (isnan(v)) return 0xFFFFFFFFu;
    if (v == 0.0f) v = 0.0f;                 // -0 and +0 are one value
    uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// first index in [0, n) whose word is >= w (words sorted ascending)
__device__ inline int lower_bound64(const uint64_t* s, int n, uint64_t w) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (s[mid] < w) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int NT>
__global__ __launch_bounds__(NT) void rank_rows(const float* __restrict__ expr, int64_t T,
                                                int K, int64_t ld, int kp2,
                                                int16_t* __restrict__ ranks2,
                                                int64_t* __restrict__ tiesum,
                                                int32_t* __restrict__ nvalid) {
    extern __shared__ uint64_t sk[];
    __shared__ unsigned long long ts_acc;
    __shared__ int n_obs;
    const int tid = threadIdx.x;
    for (int64_t row = blockIdx.x; row < T; row += gridDim.x) {
        const float* x = expr + row * ld;
        for (int i = tid; i < kp2; i += NT) {
            uint32_t key = 0xFFFFFFFFu;
            if (i < K) key = order_key(x[i]);
            sk[i] = ((uint64_t)key << 32) | (uint32_t)i;
        }
        if (tid == 0) ts_acc = 0ull;
        __syncthreads();
        for (int size = 2; size <= kp2; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = tid; t < (kp2 >> 1); t += NT) {
                    int i = (t / stride) * 2 * stride + (t % stride);
                    int j = i + stride;
                    bool up = (i & size) == 0;
                    uint64_t a = sk[i], b = sk[j];
                    if ((a > b) == up) { sk[i] = b; sk[j] = a; }
                }
                __syncthreads();
            }
        }
        if (tid == 0) n_obs = lower_bound64(sk, kp2, 0xFFFFFFFF00000000ull);
        __syncthreads();
        const int n = n_obs;
        unsigned long long local = 0;
        int16_t* r = ranks2 + row * (int64_t)K;
        for (int j = tid; j < kp2; j += NT) {
            uint64_t w = sk[j];
            int idx = (int)(w & 0xFFFFFFFFu);
            if (j < n) {
                uint64_t kw = w & 0xFFFFFFFF00000000ull;
                int lo = lower_bound64(sk, n, kw);
                // sample indices are < 2^32 - 1, so this is the end of the run
                int hi = lower_bound64(sk, n, kw | 0xFFFFFFFFull);
                r[idx] = (int16_t)(lo + hi + 1);
                long long eq = hi - lo;
                local += (unsigned long long)(eq * eq - 1);
            } else if (idx < K) {
                r[idx] = 0;
            }
        }
        if (local) atomicAdd(&ts_acc, local);
        __syncthreads();
        if (tid == 0) {
            tiesum[row] = (int64_t)ts_acc;
            if (nvalid) nvalid[row] = n;
        }
        __syncthreads();
    }
}

// K <= 256: one wave per row, ranks by counting.  The row's keys sit in
// LDS; every lane takes up to four samples and counts, over all samples,
// the keys below and equal to each (a broadcast LDS read per sample), so
//   a = 2 less + eq + 1,  sumT += eq^2 - 1,
// the same numbers as the sort above.  NaN (the largest key) is neither
// below nor equal to an observed value.
constexpr int kCountMaxK = 256;

template <int NJ>   // samples per lane: ceil(K / 64)
__global__ __launch_bounds__(256) void rank_rows_count(const float* __restrict__ expr,
                                                       int64_t T, int K, int64_t ld,
                                                       int16_t* __restrict__ ranks2,
                                                       int64_t* __restrict__ tiesum,
                                                       int32_t* __restrict__ nvalid) {
    __shared__ uint4 s_keys[4][kCountMaxK / 4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* keys = (uint32_t*)s_keys[wave];
    const int K4 = (K + 3) & ~3;          // padded with the NaN key (never below or equal)
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wave; row < T; row += n_waves) {
        const float* x = expr + row * ld;
        uint32_t mine[NJ];
        int n_valid = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int k = lane + 64 * j;
            const uint32_t key = k < K ? order_key(x[k]) : 0xFFFFFFFFu;
            if (k < K4) keys[k] = key;
            mine[j] = key;
            n_valid += __popcll(__ballot(k < K && key != 0xFFFFFFFFu));
        }
        __builtin_amdgcn_wave_barrier();
        int less[NJ], eq[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) { less[j] = 0; eq[j] = 0; }
        const uint4* k4 = s_keys[wave];
        for (int i = 0; i < K4 / 4; ++i) {
            const uint4 q = k4[i];        // broadcast read of four keys
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                less[j] += (q.x < mine[j]) + (q.y < mine[j]) + (q.z < mine[j]) + (q.w < mine[j]);
                eq[j] += (q.x == mine[j]) + (q.y == mine[j]) + (q.z == mine[j]) + (q.w == mine[j]);
            }
        }
        unsigned long long ts = 0;
        int16_t* r = ranks2 + row * (int64_t)K;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int k = lane + 64 * j;
            if (k < K) {
                if (mine[j] == 0xFFFFFFFFu) {
                    r[k] = 0;
                } else {
                    r[k] = (int16_t)(2 * less[j] + eq[j] + 1);
                    ts += (unsigned long long)((long long)eq[j] * eq[j] - 1);
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ts += __shfl_xor(ts, o, 64);
        if (lane == 0) {
            tiesum[row] = (int64_t)ts;
            if (nvalid) nvalid[row] = n_valid;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace kx

// Host launcher (called from the C ABI layer).
extern "C" hipError_t kx_launch_rank(const float* expr, int64_t T, int K, int64_t ld,
                                     int16_t* ranks2, int64_t* tiesum, int32_t* nvalid,
                                     int max_blocks, hipStream_t stream) {
    if (T <= 0) return hipSuccess;
    if (K <= kx::kCountMaxK) {
        int64_t grid = (T + 3) / 4;
        grid = grid < max_blocks ? grid : max_blocks;
        const int nj = (K + 63) / 64;
        auto kern = nj == 1 ? kx::rank_rows_count<1>
                  : nj == 2 ? kx::rank_rows_count<2>
                  : nj == 3 ? kx::rank_rows_count<3> : kx::rank_rows_count<4>;
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, expr, T, K, ld, ranks2,
                           tiesum, nvalid);
        return hipGetLastError();
    }
    int kp2 = 2;
    while (kp2 < K) kp2 <<= 1;
    size_t lds = (size_t)kp2 * sizeof(uint64_t);
    int64_t grid = T < max_blocks ? T : max_blocks;
    if (grid <= 0) return hipSuccess;
    if (kp2 <= 256) {
        hipLaunchKernelGGL(kx::rank_rows<64>, dim3((unsigned)grid), dim3(64), lds, stream,
                           expr, T, K, ld, kp2, ranks2, tiesum, nvalid);
    } else {
        hipLaunchKernelGGL(kx::rank_rows<256>, dim3((unsigned)grid), dim3(256), lds, stream,
                           expr, T, K, ld, kp2, ranks2, tiesum, nvalid);
    }
    return hipGetLastError();
}
