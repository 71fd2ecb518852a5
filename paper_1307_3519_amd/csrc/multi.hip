// multi.hip -- multi-allelic markers: genotype classes 0..l (l + 1 <= 8
// groups), eq. (2) over the classes present among a pair's kept samples and
// the chi-square tail for df = (non-empty classes - 1) (P-value calculation).
// One wave per (trait, 64 SNPs), one lane per pair: the trait's ranks are
// staged in LDS, the lane sums them per class and re-ranks its pair when
// samples are removed (a genotype code outside 0..l where the trait has a
// value: Handling missing values).  No GEMM: the two-allele path keeps the
// MFMA scan.
#include "kx_args.h"

namespace kx {

// Upper tail of chi-square with df degrees of freedom at H: Q(df/2, H/2) from
// its closed forms, exp(-x) sum_{k < df/2} x^k / k! for even df and
// erfc(sqrt x) + exp(-x) sum_{k=1}^{(df-1)/2} x^(k-1/2) / Gamma(k + 1/2) for
// odd df (x = H/2).
__device__ inline double chi2_upper(double H, int df) {
    if (df <= 0) return 1.0;
    const double x = 0.5 * H;
    if ((df & 1) == 0) {
        double term = 1.0, total = 1.0;
        for (int k = 1; k < df / 2; ++k) {
            term *= x / k;
            total += term;
        }
        return exp(-x) * total;
    }
    double total = erfc(sqrt(x));
    if (df > 1) {
        double term = sqrt(x) / 0.88622692545275801365;   // Gamma(3/2) = sqrt(pi)/2
        double s = term;
        for (int k = 2; k <= (df - 1) / 2; ++k) {
            term *= x / (k - 0.5);
            s += term;
        }
        total += exp(-x) * s;
    }
    return total;
}

__device__ inline bool multi_missing(int code, int G) { return code < 0 || code >= G; }

template <int G, int MODE>
__global__ __launch_bounds__(256) void scan_multi(MultiArgs a) {
    extern __shared__ __attribute__((aligned(16))) int16_t s_rk[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int K = a.K;
    const int K16 = (K + 15) & ~15;
    int16_t* srk = s_rk + wave * K16;
    const int64_t nb = (a.M + kWave - 1) / kWave;
    const int64_t items = a.T * nb;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < items; it += waves) {
        const int64_t trait = it / nb;
        const int64_t blk = it - trait * nb;
        int kobs = 0;
        for (int k = lane; k < K16; k += kWave) {
            const int16_t ak = k < K ? a.ranks2[trait * K + k] : (int16_t)0;
            srk[k] = ak;
            kobs += ak != 0;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) kobs += __shfl_xor(kobs, o, 64);
        __builtin_amdgcn_wave_barrier();
        const int64_t m = blk * kWave + lane;
        if (m < a.M) {
            const int8_t* row = a.geno + m * a.ld;
            int64_t s[G];
            int n[G];
#pragma unroll
            for (int c = 0; c < G; ++c) { s[c] = 0; n[c] = 0; }
            int nq = 0;
            for (int k = 0; k < K; ++k) {
                const int code = row[k];
                const int ak = srk[k];
#pragma unroll
                for (int c = 0; c < G; ++c)
                    if (code == c) { s[c] += ak; n[c] += ak != 0; }
                nq += multi_missing(code, G) && ak != 0;
            }
            // removed samples, in sample order: each lowers every kept
            // doubled rank above its own by 2 and every tied one by 1, and
            // its tie group (current size t) loses 3 t (t - 1) of the tie term
            int64_t ts = a.tiesum[trait];
            if (nq > 0) {
                for (int j = 0; j < K; ++j) {
                    const int aj = srk[j];
                    if (!(multi_missing(row[j], G) && aj != 0)) continue;
                    int e = 0, before = 0;
                    for (int k = 0; k < K; ++k) {
                        const int code = row[k];
                        const int ak = srk[k];
                        const int f = (ak > aj) + (ak >= aj);
#pragma unroll
                        for (int c = 0; c < G; ++c)
                            if (code == c) s[c] -= f;
                        e += ak == aj;
                        before += k < j && ak == aj && multi_missing(code, G);
                    }
                    const int64_t t = e - before;
                    ts -= 3 * t * (t - 1);
                }
            }
            const int64_t kp = kobs - nq;
            int ne = 0;
#pragma unroll
            for (int c = 0; c < G; ++c) ne += n[c] > 0;
            const int df = ne > 0 ? ne - 1 : 0;
            const int64_t E = kp * kp * kp - kp - ts;
            double H = 0.0;
            if (df > 0 && kp >= 2 && E > 0) {
                // D_c^2 < 2^53 and N_c are exact doubles; all terms are
                // non-negative (relative error a few ulp)
                double f = 0.0;
#pragma unroll
                for (int c = 0; c < G; ++c)
                    if (n[c]) {
                        const double d = (double)(s[c] - (int64_t)n[c] * (kp + 1));
                        f += d * d / (double)n[c];
                    }
                H = 3.0 * (double)(kp - 1) * f / (double)E;
            }
            if (MODE == FULL) {
                a.H_out[trait * a.M + m] = H;
                a.p_out[trait * a.M + m] = chi2_upper(H, df);
            } else if (df > 0 && H > a.hc[df]) {
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
        __builtin_amdgcn_wave_barrier();
    }
}

template <int G>
hipError_t launch_multi_g(const MultiArgs& a, int mode, int grid, hipStream_t st) {
    const size_t lds = (size_t)4 * ((a.K + 15) & ~15) * sizeof(int16_t);
    if (mode == FULL)
        hipLaunchKernelGGL((scan_multi<G, FULL>), dim3(grid), dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL((scan_multi<G, SCREEN>), dim3(grid), dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace kx

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
