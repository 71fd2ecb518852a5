// multi.hip -- multi-allelic markers: genotype classes 0..l (l + 1 <= 8
// groups), eq. (2) over the classes present among a pair's kept samples and
// the chi-square tail for df = (non-empty classes - 1) (P-value calculation).
//
//   multi_pack     genotype rows copied to an aligned stride, codes 0..l
//                  kept and every other code 0xFF
//   multi_info     per-SNP class sizes, removed samples, df and 1/N_c
//   scan_multi     one wave per (trait, 64 SNPs), one lane per pair: the
//                  trait's ranks are staged in LDS, the lane sums them per
//                  class and re-ranks its pair when samples are removed (a
//                  code outside 0..l where the trait has a value: Handling
//                  missing values); evaluates every pair, or only the pairs
//                  the MFMA screen cannot take (a trait with a NaN value or a
//                  SNP with a removed code), or a list of traits (minimum p)
//   multi_exact    exact H and p of the pairs that passed the MFMA screen
//                  (multi_mfma.hip) from their class sums, one lane per pair
// H is the exact rational of eq. (2) divided by the tie factor, rounded once.
#include "multi_common.h"

namespace kx {

// Genotype rows copied to an aligned stride, classes 0..G-1 kept and every
// other code (and the padding past K) set to 0xFF.
__global__ void multi_pack(const int8_t* __restrict__ geno, int64_t ld, int64_t M, int K, int G,
                           int stride, uint8_t* __restrict__ out) {
    const int64_t n = M * stride;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / stride;
        const int k = (int)(i - m * stride);
        const int code = k < K ? geno[m * ld + k] : -1;
        out[i] = (code >= 0 && code < G) ? (uint8_t)code : (uint8_t)0xFF;
    }
}

// Per-SNP constants: class sizes over the samples with a class code, the
// number of removed samples, df and 1/N_c.  One wave per SNP.  A SNP with a
// removed sample sets *any_missing.
__global__ __launch_bounds__(256) void multi_info(const uint8_t* __restrict__ packed, int pstride,
                                                  int64_t M, int K, int G,
                                                  MultiInfo* __restrict__ info,
                                                  int32_t* __restrict__ any_missing) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t m = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); m < M;
         m += waves) {
        const uint8_t* row = packed + m * (int64_t)pstride;
        int n[kMaxClasses];
#pragma unroll
        for (int c = 0; c < kMaxClasses; ++c) n[c] = 0;
        int nq = 0;
        for (int k = lane; k < K; k += kWave) {
            const int code = row[k];
#pragma unroll
            for (int c = 0; c < kMaxClasses; ++c) n[c] += code == c;
            nq += code == 0xFF;
        }
        MultiInfo out{};
        int ne = 0;
#pragma unroll
        for (int c = 0; c < kMaxClasses; ++c) {
            int v = n[c];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            out.n[c] = (int16_t)(c < G ? v : 0);
            out.w[c] = (c < G && v > 0) ? 1.0f / (float)v : 0.0f;
            ne += c < G && v > 0;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) nq += __shfl_xor(nq, o, 64);
        out.nmiss = (int16_t)nq;
        out.df = (int16_t)(ne > 0 ? ne - 1 : 0);
        if (lane == 0) {
            info[m] = out;
            if (nq > 0) *any_missing = 1;
        }
    }
}

// Exact H and p of the pairs that passed the MFMA screen, one lane each.
template <int G>
__global__ __launch_bounds__(256) void multi_exact(MultiArgs a) {
    int64_t n = (int64_t)*a.n_cand;
    if (n > a.cand_cap) n = a.cand_cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const MultiCand e = a.cand[i];
        const int64_t trait = a.row_v[e.row];
        if (trait >= 0) multi_eval_sums<G>(a, trait, e);
    }
}

template <int G, int MODE>
__global__ __launch_bounds__(256) void scan_multi(MultiArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t s_words[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int K = a.K;
    const int KW = ((K + 15) & ~15) >> 2;          // words of four samples, a multiple of 4
    // per wave: low rank bytes, high rank bytes, observed flags (KW words
    // each), then the ranks as int16 (4 KW)
    uint32_t* slo = s_words + (size_t)wave * 5 * KW;
    uint32_t* shi = slo + KW;
    uint32_t* sob = shi + KW;
    int16_t* srk = (int16_t*)(sob + KW);
    const bool wide = 2 * K > 255;
    // nothing for this pass when no trait has a NaN value and no SNP a removed code
    if (a.only_incomplete && *a.n_nan == 0 && *a.any_missing == 0) return;
    int64_t n_tr = a.T;
    if (a.trait_list) {
        const int64_t d = *a.n_list;
        n_tr = d < n_tr ? d : n_tr;
    }
    const int64_t nb = (a.M + kWave - 1) / kWave;
    const int64_t items = n_tr * nb;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    double pmin = 2.0;                               // the lane's smallest p of the item
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < items; it += waves) {
        const int64_t ti = it / nb;
        const int64_t blk = it - ti * nb;
        const int64_t trait = a.trait_list ? (int64_t)a.trait_list[ti] : ti;
        const int64_t m = blk * kWave + lane;
        bool work = m < a.M;
        if (a.only_incomplete) {
            const bool nan_trait = a.nan_flag && a.nan_flag[trait];
            work = work && (nan_trait || a.info[m].nmiss > 0);
            if (!__any(work)) continue;              // uniform: nothing for this wave
        }
        int kobs = 0;
        for (int i = lane; i < KW; i += kWave) {
            uint32_t lo = 0, hi = 0, ob = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int k = 4 * i + b;
                const int ak = k < K ? (int)a.ranks2[trait * K + k] : 0;
                lo |= (uint32_t)(ak & 0xFF) << (8 * b);
                hi |= (uint32_t)(ak >> 8) << (8 * b);
                ob |= (uint32_t)(ak != 0) << (8 * b);
                kobs += ak != 0;
                srk[k] = (int16_t)ak;
            }
            slo[i] = lo;
            shi[i] = hi;
            sob[i] = ob;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) kobs += __shfl_xor(kobs, o, 64);
        __builtin_amdgcn_wave_barrier();
        if (work) {
            const uint8_t* row = a.packed + m * (int64_t)a.pstride;
            // classes 1..G-1 by indicator; class 0 from the totals below
            uint32_t sl[G], sh[G], n[G];
#pragma unroll
            for (int c = 0; c < G; ++c) { sl[c] = 0; sh[c] = 0; n[c] = 0; }
            uint32_t nq = 0, ql = 0, qh = 0;     // removed samples: count, rank bytes
            for (int i0 = 0; i0 < KW; i0 += 4) {
                const uint4 g4 = *(const uint4*)(row + 4 * i0);
                const uint4 l4 = *(const uint4*)(slo + i0);
                const uint4 o4 = *(const uint4*)(sob + i0);
                const uint4 h4 = wide ? *(const uint4*)(shi + i0) : make_uint4(0, 0, 0, 0);
                const uint32_t gw[4] = {g4.x, g4.y, g4.z, g4.w};
                const uint32_t lw[4] = {l4.x, l4.y, l4.z, l4.w};
                const uint32_t ow[4] = {o4.x, o4.y, o4.z, o4.w};
                const uint32_t hw[4] = {h4.x, h4.y, h4.z, h4.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // codes are 0..7 or 0xFF: a class's indicator bytes are
                    // the AND of its three low bits, each taken as is or
                    // inverted (0xFF matches only code 7, which also needs
                    // the top bit clear)
                    const uint32_t w = gw[j];
                    const uint32_t b0 = w & 0x01010101u, b1 = (w >> 1) & 0x01010101u;
                    const uint32_t b2 = (w >> 2) & 0x01010101u, top = (w >> 7) & 0x01010101u;
#pragma unroll
                    for (int c = 1; c < G; ++c) {
                        uint32_t ind = (c & 1) ? b0 : (b0 ^ 0x01010101u);
                        ind &= (c & 2) ? b1 : (b1 ^ 0x01010101u);
                        ind &= (c & 4) ? b2 : (b2 ^ 0x01010101u);
                        if (c == 7) ind &= ~top;
                        sl[c] = __builtin_amdgcn_udot4(ind, lw[j], sl[c], false);
                        n[c] = __builtin_amdgcn_udot4(ind, ow[j], n[c], false);
                        if (wide) sh[c] = __builtin_amdgcn_udot4(ind, hw[j], sh[c], false);
                    }
                    const uint32_t indq = top;                 // the missing code
                    nq = __builtin_amdgcn_udot4(indq, ow[j], nq, false);
                    ql = __builtin_amdgcn_udot4(indq, lw[j], ql, false);
                    if (wide) qh = __builtin_amdgcn_udot4(indq, hw[j], qh, false);
                }
            }
            // observed samples: doubled ranks summing to kobs (kobs + 1);
            // class 0 holds the observed ones neither removed nor in 1..G-1
            int64_t s[G];
            s[0] = (int64_t)kobs * (kobs + 1) - ((int64_t)ql + ((int64_t)qh << 8));
            n[0] = (uint32_t)kobs - nq;
#pragma unroll
            for (int c = 1; c < G; ++c) {
                s[c] = (int64_t)sl[c] + ((int64_t)sh[c] << 8);
                s[0] -= s[c];
                n[0] -= n[c];
            }
            // removed samples (K' counts only the kept ones), in sample
            // order: each lowers every kept doubled rank above its own by 2
            // and every tied one by 1, and its tie group (current size t)
            // loses 3 t (t - 1) of the tie term.  Samples past K read rank 0.
            int64_t ts = a.tiesum[trait];
            if (nq > 0) {
                for (int j = 0; j < K; ++j) {
                    const int aj = srk[j];
                    if (!(row[j] == 0xFF && aj != 0)) continue;
                    int e = 0, before = 0;
                    for (int k = 0; k < K; ++k) {
                        const int code = row[k];
                        const int ak = srk[k];
                        const int f = (ak > aj) + (ak >= aj);
#pragma unroll
                        for (int c = 0; c < G; ++c)
                            if (code == c) s[c] -= f;
                        e += ak == aj;
                        before += k < j && ak == aj && code == 0xFF;
                    }
                    const int64_t t = e - before;
                    ts -= 3 * t * (t - 1);
                }
            }
            const int64_t kp = kobs - (int64_t)nq;
            int ne = 0;
            int nn[G];
            int64_t D[G];
#pragma unroll
            for (int c = 0; c < G; ++c) {
                nn[c] = (int)n[c];
                ne += n[c] > 0;
                D[c] = s[c] - (int64_t)n[c] * (kp + 1);
            }
            const int df = ne > 0 ? ne - 1 : 0;
            const double H = exact_H_classes<G>(D, nn, kp, ts, df);
            if (MODE == FULL) {
                a.H_out[trait * a.M + m] = H;
                a.p_out[trait * a.M + m] = chi2_upper(H, df);
            } else {
                if (a.minp_bits && df > 0) pmin = fmin(pmin, chi2_upper(H, df));
                if (a.record_hits && df > 0 && H > a.hc[df]) {
                    const unsigned long long idx = atomicAdd(a.n_hits, 1ull);
                    if ((int64_t)idx < a.hit_cap) {
                        HitRec h;
                        h.trait = (int32_t)trait;
                        h.snp = (int32_t)(a.snp_base + m);
                        h.H = H;
                        h.p = chi2_upper(H, df);
                        a.hits[idx] = h;
                    }
                }
            }
        }
        if (MODE != FULL && a.minp_bits) {
            // every lane of the wave holds the same trait: one update per wave
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) pmin = fmin(pmin, __shfl_xor(pmin, o, 64));
            if (lane == 0 && pmin <= 1.0)
                atomicMin(&a.minp_bits[trait], (unsigned long long)__double_as_longlong(pmin));
            pmin = 2.0;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void fill_flag(int32_t* f) {
    if (threadIdx.x == 0) *f = 0;
}

template <int G>
hipError_t launch_multi_g(const MultiArgs& a, int mode, int grid, hipStream_t st) {
    const size_t lds = (size_t)4 * 5 * (((a.K + 15) & ~15) >> 2) * sizeof(uint32_t);
    if (mode == FULL)
        hipLaunchKernelGGL((scan_multi<G, FULL>), dim3(grid), dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL((scan_multi<G, SCREEN>), dim3(grid), dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace kx

extern "C" hipError_t kx_launch_multi_pack(const int8_t* geno, int64_t ld, int64_t M, int K,
                                           int G, int stride, uint8_t* out, int grid,
                                           hipStream_t st) {
    if (M * stride <= 0) return hipSuccess;
    hipLaunchKernelGGL(kx::multi_pack, dim3(grid), dim3(256), 0, st, geno, ld, M, K, G, stride,
                       out);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_multi_info(const uint8_t* packed, int pstride, int64_t M, int K,
                                           int G, kx::MultiInfo* info, int32_t* any_missing,
                                           int grid, hipStream_t st) {
    hipLaunchKernelGGL(kx::fill_flag, dim3(1), dim3(64), 0, st, any_missing);
    if (M > 0)
        hipLaunchKernelGGL(kx::multi_info, dim3(grid), dim3(256), 0, st, packed, pstride, M, K, G,
                           info, any_missing);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_multi_exact(const kx::MultiArgs* a, int n_classes, int grid,
                                            hipStream_t st) {
    switch (n_classes) {
#define KX_CASE(g) case g: hipLaunchKernelGGL(kx::multi_exact<g>, dim3(grid), dim3(256), 0, st, *a); break;
        KX_CASE(2) KX_CASE(3) KX_CASE(4) KX_CASE(5) KX_CASE(6) KX_CASE(7) KX_CASE(8)
#undef KX_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_multi(const kx::MultiArgs* a, int n_classes, int mode, int grid,
                                      hipStream_t st) {
    switch (n_classes) {
        case 2: return kx::launch_multi_g<2>(*a, mode, grid, st);
        case 3: return kx::launch_multi_g<3>(*a, mode, grid, st);
        case 4: return kx::launch_multi_g<4>(*a, mode, grid, st);
        case 5: return kx::launch_multi_g<5>(*a, mode, grid, st);
        case 6: return kx::launch_multi_g<6>(*a, mode, grid, st);
        case 7: return kx::launch_multi_g<7>(*a, mode, grid, st);
        case 8: return kx::launch_multi_g<8>(*a, mode, grid, st);
        default: return hipErrorInvalidValue;
    }
}
