// multi_mfma.hip -- multi-allelic markers (classes 0..l, l + 1 = G <= 5) on
// the MFMA rank-sum GEMM, K <= 128 (eq. (1) with one product per class,
// Calculation of the Kruskal-Wallis test statistic; P-value calculation).
//
// For a trait n and a SNP m whose samples all have a class and an
// expression value, the twice-centred class sums D_c = C I_c^T (C the
// centred doubled ranks, I_c the 0/1 indicators of class c) give
//   f = sum_{N_c>0} D_c^2 / N_c,  H = 3 (K-1) f / (K^3 - K - sumT_n),
// and, because the centred ranks of a trait sum to zero, D_0 = -sum_{c>0} D_c:
// G - 1 MFMA columns per SNP.  SNP-stationary like the two-allele kernel: a
// wave builds its 32-SNP tile's indicator fragments once per work item and
// streams 32-trait tiles of centred ranks through v_mfma_f32_32x32x16_f16
// (two waves per SIMD: one wave's loads and epilogue overlap the other's
// MFMAs).  The epilogue screens every
// pair in fp32 against the chi-square threshold of its df at the screen
// level (slack 1e-5, the smallest K^3 - K - sumT of the tile); the pairs
// that pass are staged per wave in LDS and written to a candidate buffer
// {operand row, SNP, D_1..D_{G-1}} (the class sums are exact integers in
// fp32), from which multi_exact evaluates H exactly.  When the buffer is full
// the pair is evaluated here.  Lanes of SNPs with a removed code and
// rows of traits with a NaN value never pass: scan_multi takes those pairs.
#include "multi_common.h"

namespace kx {

typedef _Float16 mhalf8 __attribute__((ext_vector_type(8)));
typedef float mf32x16 __attribute__((ext_vector_type(16)));

constexpr int kMultiStage = 64;

// A value no kernel writes while this one runs, read through the scalar cache
// (uniform address): its wait does not cover the vector loads in flight.
__device__ inline float const_load(const float* p) {
    return *(const __attribute__((address_space(4))) float*)p;
}

// Out of line: keeps the exact evaluation's registers out of the scan loop.
template <int G>
__device__ __attribute__((noinline)) void multi_eval_fallback(const MultiArgs& a,
                                                              const MultiCand& e) {
    const int64_t trait = a.row_v[e.row];
    if (trait >= 0) multi_eval_sums<G>(a, trait, e);
}

template <int G>
__device__ inline void multi_flush(const MultiArgs& a, const MultiArgs* a_lds, MultiCand* stage,
                                   int& sn, int lane) {
    if (sn == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.n_cand, (unsigned long long)sn);
    base = __shfl(base, 0, 64);
    for (int i = lane; i < sn; i += kWave) {
        const MultiCand e = stage[i];
        const unsigned long long idx = base + (unsigned long long)i;
        if ((int64_t)idx < a.cand_cap) a.cand[idx] = e;
        else multi_eval_fallback<G>(*a_lds, e);
    }
    sn = 0;
    __builtin_amdgcn_wave_barrier();
}

// 0/1 fp16 indicators of class c at eight codes.
__device__ inline mhalf8 class_frag(uint2 w, int c) {
    uint8_t codes[8];
    __builtin_memcpy(codes, &w, 8);
    mhalf8 f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = codes[e] == c ? (_Float16)1.0f : (_Float16)0.0f;
    return f;
}

template <int KS, int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void scan_multi_mfma(MultiArgs a) {
    constexpr int NC = G - 1;
    __shared__ MultiCand s_stage[kWavesPerBlock][kMultiStage];
    __shared__ MultiArgs s_args;
    if (threadIdx.x == 0) s_args = a;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    MultiCand* stage = s_stage[wave];
    int sn = 0;
    const int64_t n_tiles = (a.n_rows + kTile - 1) / kTile;
    const int64_t tpr = a.tiles_per_range;
    const int64_t n_ranges = (n_tiles + tpr - 1) / tpr;
    const int64_t n_blocks = (a.n_snp_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t items = n_ranges * n_blocks;
    const uint4* A = (const uint4*)a.A;
    const float kslack = 1.0f + kScreenSlack;
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;

    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int64_t rg = item / n_blocks;
        const int64_t st = (item % n_blocks) * kWavesPerBlock + wave;
        if (st >= a.n_snp_tiles) continue;            // per wave: no block barrier below
        const int64_t m = st * kTile + (lane & 31);
        const bool in_range = m < a.M;
        MultiInfo inf{};
        if (in_range) inf = a.info[m];
        // screen weights: 3 (K-1) (1 + slack) / (H_c(df) N_c); zero for a SNP
        // with a removed code or at most one class (never a candidate)
        const bool live = in_range && inf.nmiss == 0 && inf.df > 0;
        const float fac = live ? 3.0f * (float)(a.K - 1) * kslack * a.inv_hc[inf.df] : 0.0f;
        float w[G];
#pragma unroll
        for (int c = 0; c < G; ++c) w[c] = inf.w[c] * fac;
        // indicator fragments of classes 1..G-1 for this lane's SNP
        mhalf8 B[KS][NC];
        const uint8_t* grow = a.packed + m * (int64_t)a.pstride + 8 * (lane >> 5);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const uint2 cw = in_range ? *(const uint2*)(grow + 16 * s) : make_uint2(~0u, ~0u);
#pragma unroll
            for (int c = 0; c < NC; ++c) B[s][c] = class_frag(cw, c + 1);
        }
        const int64_t t0 = rg * tpr;
        const int64_t t1 = t0 + tpr < n_tiles ? t0 + tpr : n_tiles;
        // (as 16-byte words: a loop-carried vector of halves is split by the
        // compiler into 16-bit pieces and reassembled before every MFMA)
        auto load_tile = [&](int64_t t, uint4 (&Ad)[KS]) {
#pragma unroll
            for (int s = 0; s < KS; ++s) Ad[s] = A[(t * KS + s) * kWave + lane];
        };
        // The A fragments of the next tile are loaded into the same registers
        // once the current tile's MFMAs have been issued, so that the loads
        // land while the current tile is screened.
        uint4 Ac[KS];
        if (t0 < t1) load_tile(t0, Ac);
        for (int64_t t = t0; t < t1; ++t) {
            mf32x16 acc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = mf32x16{};
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(mhalf8, Ac[s]),
                                                                     B[s][c], acc[c], 0, 0, 0);
            const float th = const_load(a.theta + t);
            if (t + 1 < t1) load_tile(t + 1, Ac);
            // screen value of a pair: sum_c w_c D_c^2 - theta, D_0 = -sum_{c>0} D_c
            auto screen = [&](int r) {
                float d0 = 0.0f, v = -th;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float d = acc[c][r];
                    d0 -= d;
                    v = fmaf(w[c + 1] * d, d, v);
                }
                return fmaf(w[0] * d0, d0, v);
            };
            float vmax = -__builtin_inff();
#pragma unroll
            for (int r = 0; r < 16; ++r) vmax = fmaxf(vmax, screen(r));
            if (!__any(vmax > 0.0f)) continue;
            const int64_t rb = t * kTile + 4 * (lane >> 5);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const bool cand = screen(r) > 0.0f;
                const unsigned long long msk = __ballot(cand);
                if (!msk) continue;
                const int n = __popcll(msk);
                if (sn + n > kMultiStage) multi_flush<G>(a, &s_args, stage, sn, lane);
                if (cand) {
                    MultiCand e;
                    e.row = (uint32_t)(rb + 8 * (r >> 2) + (r & 3));
                    e.snp = (uint32_t)m;
#pragma unroll
                    for (int c = 0; c < 6; ++c) e.d[c] = c < NC ? (int32_t)acc[c < NC ? c : 0][r] : 0;
                    stage[sn + __popcll(msk & lt)] = e;
                }
                sn += n;
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    multi_flush<G>(a, &s_args, stage, sn, lane);
}

// `grid` is the number of work items; the persistent launch uses at most the
// blocks that fit on the device at once.
template <int KS, int G>
hipError_t launch_multi_mfma_ks(const MultiArgs& a, int grid, hipStream_t st) {
    auto kern = scan_multi_mfma<KS, G>;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, 0) != hipSuccess || occ < 1)
        occ = 1;
    int dev = 0, n_cu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t resident = (int64_t)n_cu * occ;
    const int g = (int)(grid < resident ? grid : resident);
    if (g < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int G>
hipError_t launch_multi_mfma_g(const MultiArgs& a, int ks, int grid, hipStream_t st) {
    switch (ks) {
#define KX_KS(k) case k: return launch_multi_mfma_ks<k, G>(a, grid, st);
        KX_KS(1) KX_KS(2) KX_KS(3) KX_KS(4) KX_KS(5) KX_KS(6) KX_KS(7) KX_KS(8)
#undef KX_KS
        default: return hipErrorInvalidValue;
    }
}

}  // namespace kx

// ks = ceil(K / 16) <= 8; n_classes 2..5.
extern "C" hipError_t kx_launch_multi_mfma(const kx::MultiArgs* a, int n_classes, int ks, int grid,
                                           hipStream_t st) {
    switch (n_classes) {
        case 2: return kx::launch_multi_mfma_g<2>(*a, ks, grid, st);
        case 3: return kx::launch_multi_mfma_g<3>(*a, ks, grid, st);
        case 4: return kx::launch_multi_mfma_g<4>(*a, ks, grid, st);
        case 5: return kx::launch_multi_mfma_g<5>(*a, ks, grid, st);
        default: return hipErrorInvalidValue;
    }
}
