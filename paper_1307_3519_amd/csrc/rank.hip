// rank.hip -- per-trait doubled midranks and tie term (the ranking step of
// the paper's input-data section and the tie term of its tied-data section).
//
// One workgroup per trait row.  The row is sorted in LDS as 64-bit words
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

}  // namespace kx

// Host launcher (called from the C ABI layer).
extern "C" hipError_t kx_launch_rank(const float* expr, int64_t T, int K, int64_t ld,
                                     int16_t* ranks2, int64_t* tiesum, int32_t* nvalid,
                                     int max_blocks, hipStream_t stream) {
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
