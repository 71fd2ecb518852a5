// fp64.hip -- comparator path: the paper's matrix formulation on the GPU.
//
// For a slice of SNPs, the rank-sum matrices S_i = R * I_i^T of eq. (1) are
// formed for all l + 1 = 3 genotype classes with one rocBLAS fp64 GEMM (the
// stacked indicator matrices), written to HBM, and an element-wise pass then
// turns them into H, the tie correction, p and hits (eq. (2), tied-data and
// P-value sections), slice after slice (the paper's data slicing).  It
// computes the same exact statistic as the fused MFMA path, so its results
// are identical; it exists to be timed beside it.
#include <rocblas/rocblas.h>

#include <algorithm>

#include "kx_host.h"

namespace kx {

__global__ void ranks_to_f64(const int16_t* __restrict__ r, int64_t n, double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)r[i];
}

// Stacked indicators of a slice: row (i * S + j) is I_i(m0 + j, :); counts per SNP.
__global__ void indicators_f64(const int8_t* __restrict__ geno, int64_t ld, int K, int64_t m0,
                               int S, int S_act, double* __restrict__ I,
                               int4* __restrict__ cnt) {
    int64_t total = (int64_t)S * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int j = (int)(e / K), k = (int)(e % K);
        int g = -1;
        if (j < S_act) {
            int8_t v = geno[(m0 + j) * ld + k];
            g = (v >= 0 && v <= 2) ? v : -1;
        }
        for (int i = 0; i < 3; ++i) I[((int64_t)i * S + j) * K + k] = (g == i) ? 1.0 : 0.0;
    }
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < S; j += gridDim.x * blockDim.x) {
        int4 c = make_int4(0, 0, 0, 0);
        if (j < S_act) {
            const int8_t* row = geno + (m0 + j) * ld;
            for (int k = 0; k < K; ++k) {
                int8_t v = row[k];
                if (v == 0) c.x++; else if (v == 1) c.y++; else if (v == 2) c.z++; else c.w++;
            }
        }
        cnt[j] = c;
    }
}

struct F64Args {
    const double* C;            // [T][3S] doubled rank sums (sum over kept samples)
    const int4* cnt;            // [S] n0, n1, n2, nmiss
    int64_t T;
    int S, S_act, K;
    int64_t m0, M, snp_base;
    const int64_t* tiesum;
    const int16_t* ranks2;
    const int8_t* geno;
    int64_t ld;
    double hc1, hc2;
    HitRec* hits; int64_t hit_cap; unsigned long long* n_hits;
    unsigned long long* maxH;   // [T][2] bits of the max H per df (min p)
    double* H_out; double* p_out; int32_t* sums_out;
};

// Exact H of a pair with missing genotypes or missing expression values, one
// thread: the samples without a genotype are removed and the ranks re-derived
// over the rest; samples without an expression value (rank 0) are not part of
// the trait's ranking and drop out of the pair.  Group sizes, K' and df are
// the pair's own.
__device__ double rerank_pair(const F64Args& a, int64_t t, int64_t m, int64_t* s_out, int* df_out) {
    const int K = a.K;
    const int16_t* rk = a.ranks2 + t * K;
    const int8_t* gr = a.geno + m * a.ld;
    long long ts = a.tiesum[t];
    int nq = 0, kobs = 0;
    long long s[3] = {0, 0, 0};
    int n[3] = {0, 0, 0};
    // tie term: remove the missing samples one at a time
    for (int j = 0; j < K; ++j) {
        const int aj = rk[j];
        if (aj == 0) continue;
        ++kobs;
        int8_t gj = gr[j];
        if (gj >= 0 && gj <= 2) continue;
        int tcnt = 0;
        for (int k = 0; k < K; ++k) {
            if (rk[k] != aj) continue;
            int8_t gk = gr[k];
            bool removed_before = !(gk >= 0 && gk <= 2) && k < j;
            if (!removed_before) ++tcnt;
        }
        ts -= 3ll * tcnt * (tcnt - 1);
        ++nq;
    }
    for (int k = 0; k < K; ++k) {
        int8_t gk = gr[k];
        const int ak = rk[k];
        if (!(gk >= 0 && gk <= 2) || ak == 0) continue;
        int w = 0;
        for (int j = 0; j < K; ++j) {
            int8_t gj = gr[j];
            const int aj = rk[j];
            if ((gj >= 0 && gj <= 2) || aj == 0) continue;
            w += aj < ak ? 2 : (aj == ak ? 1 : 0);
        }
        s[gk] += ak - w;
        ++n[gk];
    }
    int64_t kp = kobs - nq;
    s_out[0] = s[0]; s_out[1] = s[1]; s_out[2] = s[2];
    int ne = (n[0] > 0) + (n[1] > 0) + (n[2] > 0);
    int df = ne > 0 ? ne - 1 : 0;
    *df_out = df;
    return exact_H(s[0] - (int64_t)n[0] * (kp + 1), s[1] - (int64_t)n[1] * (kp + 1),
                   s[2] - (int64_t)n[2] * (kp + 1), n[0], n[1], n[2], kp, ts, df);
}

__global__ __launch_bounds__(256) void f64_epilogue(F64Args a) {
  for (int64_t t = blockIdx.y; t < a.T; t += gridDim.y) {
    double best[2] = {0.0, 0.0};
    // a trait with missing expression values takes the re-rank path for
    // every pair (its group sizes and K' depend on the pair)
    bool zero = false;
    for (int k = threadIdx.x; k < a.K; k += blockDim.x) zero = zero || a.ranks2[t * a.K + k] == 0;
    const bool nan_t = __syncthreads_or(zero);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < a.S_act; j += gridDim.x * blockDim.x) {
        const int4 c = a.cnt[j];
        const int64_t m = a.m0 + j;
        const double* row = a.C + t * 3 * (int64_t)a.S;
        int64_t s[3] = {(int64_t)row[j], (int64_t)row[a.S + j], (int64_t)row[2 * a.S + j]};
        int ne = (c.x > 0) + (c.y > 0) + (c.z > 0);
        int df = ne > 0 ? ne - 1 : 0;
        double H;
        if (c.w == 0 && !nan_t) {
            const int64_t k1 = a.K + 1;
            H = exact_H(s[0] - c.x * k1, s[1] - c.y * k1, s[2] - c.z * k1, c.x, c.y, c.z, a.K,
                        a.tiesum[t], df);
        } else {
            H = rerank_pair(a, t, m, s, &df);
        }
        if (a.H_out) {
            a.H_out[t * a.M + m] = H;
            a.p_out[t * a.M + m] = pvalue(H, df);
        }
        if (a.sums_out) {
            int64_t TM = a.T * a.M;
            a.sums_out[t * a.M + m] = (int32_t)s[0];
            a.sums_out[TM + t * a.M + m] = (int32_t)s[1];
            a.sums_out[2 * TM + t * a.M + m] = (int32_t)s[2];
        }
        if (df >= 1) {
            if (H > best[df - 1]) best[df - 1] = H;
            if (a.hits && H > (df == 1 ? a.hc1 : a.hc2)) {
                unsigned long long idx = atomicAdd(a.n_hits, 1ull);
                if ((int64_t)idx < a.hit_cap) {
                    HitRec h;
                    h.trait = (int32_t)t;
                    h.snp = (int32_t)(a.snp_base + m);
                    h.H = H;
                    h.p = pvalue(H, df);
                    a.hits[idx] = h;
                }
            }
        }
    }
    if (a.maxH) {
        for (int d = 0; d < 2; ++d) {
            double v = best[d];
            for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
            if ((threadIdx.x & 63) == 0 && v > 0.0) atomicMax(&a.maxH[t * 2 + d], dbl_bits(v));
        }
    }
  }
}

__global__ void f64_min_p(const unsigned long long* maxH, int64_t T, double* out) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T;
         t += (int64_t)gridDim.x * blockDim.x) {
        double h1 = __longlong_as_double((long long)maxH[2 * t]);
        double h2 = __longlong_as_double((long long)maxH[2 * t + 1]);
        double p1 = h1 > 0.0 ? pvalue(h1, 1) : 1.0;
        double p2 = h2 > 0.0 ? pvalue(h2, 2) : 1.0;
        out[t] = p1 < p2 ? p1 : p2;
    }
}

}  // namespace kx

namespace {
krux_status hip_fail(krux_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return KRUX_OK;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return kx_fail(c, KRUX_ERR_HIP, buf);
}
}  // namespace

void kx_fp64_release(krux_ctx* c) {
    void** h = kx_blas_handle(c);
    if (*h) {
        rocblas_destroy_handle((rocblas_handle)*h);
        *h = nullptr;
    }
}

krux_status kx_fp64_test(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                         int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno,
                         int64_t snp_base, double p_c, int32_t mode, krux_hit* hits,
                         int64_t hit_capacity, int64_t* n_hits, double* min_p, double* H,
                         double* p, int32_t* sums, hipStream_t st) {
    krux_status s = KRUX_OK;
    hipError_t e = hipSetDevice(kx_ctx_device(c));
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    void** hp = kx_blas_handle(c);
    if (!*hp) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success)
            return kx_fail(c, KRUX_ERR_HIP, "rocblas_create_handle failed");
        *hp = h;
    }
    rocblas_handle blas = (rocblas_handle)*hp;
    rocblas_set_stream(blas, st);

    // slice size: the three T x S fp64 rank-sum matrices stay below ~4 GB
    int64_t S = (int64_t)(4.0e9 / (24.0 * std::max<int64_t>(T, 1)));
    S = std::max<int64_t>(256, std::min<int64_t>(S, 65536));
    S = std::min<int64_t>(S, std::max<int64_t>(M, 1));
    double* R = (double*)kx_ws(c, kx_slot_f64_r(), (size_t)std::max<int64_t>(T, 1) * K * 8, &s);
    double* I = (double*)kx_ws(c, kx_slot_f64_i(), (size_t)3 * S * K * 8 + (size_t)S * 16, &s);
    double* C = (double*)kx_ws(c, kx_slot_f64_s(), (size_t)3 * S * std::max<int64_t>(T, 1) * 8, &s);
    if (s != KRUX_OK) return s;
    int4* cnt = (int4*)(I + 3 * S * K);
    kx::HitRec* stage = nullptr;
    unsigned long long* nh = nullptr;
    unsigned long long* maxH = nullptr;
    int64_t cap = hit_capacity;
    if (mode == KRUX_MODE_HITS) {
        stage = (kx::HitRec*)kx_ws(c, kx_slot_stage(), (size_t)std::max<int64_t>(cap, 1) * 24, &s);
        nh = (unsigned long long*)kx_ws(c, kx_slot_nhits(), 256, &s);
        if (min_p)
            maxH = (unsigned long long*)kx_ws(c, kx_slot_minp(), (size_t)std::max<int64_t>(T, 1) * 16, &s);
        if (s != KRUX_OK) return s;
        if ((e = kx_launch_fill_u64(nh, 1, 0ull, st)) != hipSuccess) return hip_fail(c, e, "fill");
        if (maxH && (e = kx_launch_fill_u64(maxH, 2 * T, 0ull, st)) != hipSuccess)
            return hip_fail(c, e, "fill");
    }
    if (T > 0) {
        hipLaunchKernelGGL(kx::ranks_to_f64, dim3(1024), dim3(256), 0, st, ranks2, T * K, R);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "ranks_to_f64");
    }
    const double one = 1.0, zero = 0.0;
    for (int64_t m0 = 0; m0 < M && T > 0; m0 += S) {
        int S_act = (int)std::min<int64_t>(S, M - m0);
        hipLaunchKernelGGL(kx::indicators_f64, dim3(1024), dim3(256), 0, st, geno, ld_geno, K, m0,
                           (int)S, S_act, I, cnt);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "indicators_f64");
        // column-major view: C'(3S x T) = I'(K x 3S)^T * R'(K x T)
        rocblas_status bs = rocblas_dgemm(blas, rocblas_operation_transpose,
                                          rocblas_operation_none, (rocblas_int)(3 * S),
                                          (rocblas_int)T, K, &one, I, K, R, K, &zero, C,
                                          (rocblas_int)(3 * S));
        if (bs != rocblas_status_success) return kx_fail(c, KRUX_ERR_HIP, "rocblas_dgemm failed");
        kx::F64Args a{};
        a.C = C; a.cnt = cnt; a.T = T; a.S = (int)S; a.S_act = S_act; a.K = K;
        a.m0 = m0; a.M = M; a.snp_base = snp_base; a.tiesum = tiesum; a.ranks2 = ranks2;
        a.geno = geno; a.ld = ld_geno;
        a.hc1 = kx_threshold_of(mode == KRUX_MODE_HITS ? p_c : 1.0, 1);
        a.hc2 = kx_threshold_of(mode == KRUX_MODE_HITS ? p_c : 1.0, 2);
        a.hits = stage; a.hit_cap = cap; a.n_hits = nh; a.maxH = maxH;
        if (mode == KRUX_MODE_FULL) { a.H_out = H; a.p_out = p; }
        if (mode == KRUX_MODE_SUMS) a.sums_out = sums;
        dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((S_act + 255) / 256, 64)),
                  (unsigned)std::min<int64_t>(T, 65535));
        hipLaunchKernelGGL(kx::f64_epilogue, grid, dim3(256), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "f64_epilogue");
    }
    if (mode != KRUX_MODE_HITS) return KRUX_OK;
    if (min_p && T > 0) {
        hipLaunchKernelGGL(kx::f64_min_p, dim3(256), dim3(256), 0, st, maxH, T, min_p);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "f64_min_p");
    } else if (min_p) {
        // nothing to do for T == 0
    }
    size_t tmp_bytes = kx_sort_tmp_bytes(std::max<int64_t>(cap, 1));
    unsigned long long* keys =
        (unsigned long long*)kx_ws(c, kx_slot_keys(), (size_t)std::max<int64_t>(cap, 1) * 16, &s);
    uint32_t* idx = (uint32_t*)kx_ws(c, kx_slot_idx(), (size_t)std::max<int64_t>(cap, 1) * 8, &s);
    void* tmp = kx_ws(c, kx_slot_sort_tmp(), tmp_bytes, &s);
    if (s != KRUX_OK) return s;
    // digits that can be non-zero: traits below T, SNP numbers below snp_base + M
    auto bits = [](int64_t v) {
        int b = 0;
        while (b < 32 && ((int64_t)1 << b) <= v) ++b;
        return b;
    };
    e = kx_sort_hits(stage, nh, cap, keys, idx, tmp, tmp_bytes, (kx::HitRec*)hits, n_hits,
                     bits(T - 1), bits(snp_base + M - 1), st);
    return hip_fail(c, e, "sort hits");
}
