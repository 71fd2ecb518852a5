// scan_cand.hip -- exact evaluation of the pairs that passed the screen.
#include "scan_kernel.h"

namespace kx {

// Rank-aware bound for a pair (row v, SNP m) whose SNP has missing genotypes
// (sample exclusion with re-ranking over the rest, section 2).  With D~_i the
// sums of full-sample centred ranks over the observed members of group i (the
// scan's columns; D~_0 = -D~_1 - D~_2 - sum of the missing samples' centred
// ranks), the re-ranked sums are D'_i = D~_i - sum_q s_i(q), where for each
// missing sample q, s_i(q) = #{kept k in group i above q} - #{kept k in group i
// below q}.  At most L_q = (a_q - 2) / 2 samples lie below q and at most
// G_q = K - a_q / 2 above it (a_q: doubled midrank, its tie group holds q), so
// s_i(q) lies in [-min(N_i, L_q), min(N_i, G_q)].  The largest f over these
// intervals, with E' >= K'^3 - K' - sumT, bounds H'.  Returns false when the
// bound stays below the pass's screen level (never for a level of 0), or when
// the pair can only matter for its row's minimum p and cannot lower it.  All
// lanes of the wave take part; the result is uniform.
__device__ inline bool missing_pair_may_pass(const ScanArgs& a, int64_t v, int64_t m, int d1,
                                             int d2, int lane) {
    const int K = a.K;
    const int64_t trait = v % a.T, perm = v / a.T;
    const int16_t* rk = a.ranks2 + trait * K;
    const int32_t* pm = a.perms ? a.perms + perm * K : nullptr;
    const int8_t* gr = a.G + m * (int64_t)a.gstride;
    const SnpInfo inf = a.info[m];
    const int n[3] = {inf.n0, inf.n1, inf.n2};
    int nq = 0, sq = 0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    auto add_missing = [&](int aq) {
        const int below = (aq - 2) >> 1, above = K - ((aq + 1) >> 1);
        ++nq;
        sq += aq - (K + 1);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo[i] -= min(n[i], below);
            hi[i] += min(n[i], above);
        }
    };
    // each lane scans 16 consecutive codes per 16-byte load (the packed row
    // stride is a multiple of 32 bytes, so the load stays inside the row);
    // bytes equal to the missing code are found four at a time.  The first
    // four missing samples of a lane have their ranks loaded together, any
    // further ones one by one.
    for (int k0 = 0; k0 < K; k0 += 16 * kWave) {
        const int kb = k0 + 16 * lane;
        const uint4 w = kb < K ? *(const uint4*)(gr + kb) : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
        int np = 0, p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        bool more = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = words[j] ^ (0x01010101u * (uint32_t)kMissingCode);
            // high bit of each byte of z set iff that byte of x is zero
            uint32_t z = ~((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x)) & 0x80808080u;
            while (z) {
                const int k = kb + 4 * j + (__builtin_ctz(z) >> 3);
                z &= z - 1u;
                if (k >= K) continue;
                if (np == 4) { more = true; break; }
                p0 = np == 0 ? k : p0; p1 = np == 1 ? k : p1;
                p2 = np == 2 ? k : p2; p3 = np == 3 ? k : p3;
                ++np;
            }
        }
        // unused slots load sample 0 (no branches around the loads)
        int i0 = p0, i1 = p1, i2 = p2, i3 = p3;
        if (pm) {
            i0 = pm[p0]; i1 = pm[p1]; i2 = pm[p2]; i3 = pm[p3];
        }
        const int a0 = rk[i0], a1 = rk[i1], a2 = rk[i2], a3 = rk[i3];
        if (np > 0) add_missing(a0);
        if (np > 1) add_missing(a1);
        if (np > 2) add_missing(a2);
        if (np > 3) add_missing(a3);
        if (more) {
            // the lane's missing samples after its fourth
            int seen = 0;
            for (int e = 0; e < 16; ++e) {
                const int k = kb + e;
                if (k >= K) break;
                if (gr[k] != kMissingCode) continue;
                if (++seen <= 4) continue;
                add_missing(rk[pm ? pm[k] : k]);
            }
        }
    }
    nq = wave_sum(nq);
    sq = wave_sum(sq);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lo[i] = wave_sum(lo[i]);
        hi[i] = wave_sum(hi[i]);
    }
    const int df = snp_df(inf);
    if (df <= 0) return false;                  // never recorded
    const int64_t kp = K - nq;
    const int64_t E = cube_minus(kp) - a.tiesum[trait];
    if (kp < 2 || E <= 0) return true;          // no bound: evaluate
    const int64_t D[3] = {-(int64_t)d1 - d2 - sq, d1, d2};
    double f = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (n[i] == 0) continue;
        const int64_t x0 = D[i] - hi[i], x1 = D[i] - lo[i];
        const int64_t x = max(x0 < 0 ? -x0 : x0, x1 < 0 ? -x1 : x1);
        f += (double)(x * x) / (double)n[i];
    }
    const double Hup = 3.0 * (double)(kp - 1) * f / (double)E * (1.0 + 1e-9);
    if (Hup < a.hc_screen[df]) return false;
    // Below every count level and the hit level the pair matters only for
    // its row's minimum p: skip it when even its bound cannot lower the
    // minimum found so far (read without synchronisation: a stale, larger
    // value only skips less)
    bool counted = false;
    for (int l = 0; l < a.n_lev; ++l) counted = counted || !(Hup < a.hc[l][df - 1]);
    if (counted || !a.minp_bits) return true;
    const double cur = __longlong_as_double((long long)a.minp_bits[v]);
    return pvalue(Hup, df) < cur;
}

// Exact evaluation of the candidates of complete SNPs, one lane each: exact
// H from the pair's exact MFMA column values (eq. (2) with the tie factor),
// p, hit / min p.
__global__ __launch_bounds__(256) void scan_exact(ScanArgs a) {
    int64_t n = (int64_t)*a.n_cand;
    if (n > a.cand_cap) n = a.cand_cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 e = a.cand[i];
        eval_candidate(a, (int64_t)e.x, (int64_t)(e.y & kCandSnp), __uint_as_float(e.z),
                       __uint_as_float(e.w), e.y & ~kCandSnp);
    }
}

// Pairs of SNPs with missing genotypes, one wave each: a rank-aware bound
// (missing_pair_may_pass) drops most of them; for the rest the ranks are
// re-derived over the kept samples (coop_exact), then as above.  The next
// entry of the wave's stride is loaded one iteration ahead.  The pass is
// bound by the latency of each pair's dependent gathers, so it runs at six
// waves per SIMD (80 registers; the spills stay outside the sample loops;
// measured on the cohort workload: 3 waves 19.5 ms, 4 16.3, 5 15.3, 6 14.9),
// as a kernel of its own so that the complete-SNP path does not set its
// register budget.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6)))
void scan_exact_missing(ScanArgs a) {
    extern __shared__ __attribute__((aligned(16))) int16_t s_buf[];   // per wave coop_lds_entries(K)
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int16_t* sb = s_buf + wave * coop_lds_entries(a.K);
    int64_t nm = (int64_t)*a.n_mcand;
    if (nm > a.mcand_cap) nm = a.mcand_cap;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    int4 q = e < nm ? a.mcand[e] : make_int4(0, 0, 0, 0);
    for (; e < nm; e += waves) {
        const int4 qn = e + waves < nm ? a.mcand[e + waves] : make_int4(0, 0, 0, 0);
        const int64_t v = a.row_v[q.x];
        if (v >= 0 &&                    // padding row (uniform per wave)
            missing_pair_may_pass(a, v, q.y, q.z, q.w, lane)) {
            int df;
            int64_t s[3];
            const double H = coop_exact<4>(a, v, q.y, sb, lane, &df, s);
            if (lane == 0) record(a, v, q.y, H, df);
        }
        q = qn;
    }
}

// Traits with missing expression values (a doubled midrank of 0, see
// krux_rank): one wave per trait sets flag[t] and appends t to list.  Their
// operand rows are padding in the scans (prep), and scan_nan_traits evaluates
// their pairs.
__global__ __launch_bounds__(256) void flag_nan_traits(const int16_t* __restrict__ ranks2,
                                                       int64_t T, int K, uint8_t* flag,
                                                       int32_t* list, int32_t* n_list) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < T;
         t += waves) {
        bool zero = false;
        for (int k = lane; k < K; k += kWave) zero = zero || ranks2[t * K + k] == 0;
        const bool any = __any(zero);
        if (lane == 0) {
            flag[t] = any ? 1 : 0;
            if (any) list[atomicAdd(n_list, 1)] = (int32_t)t;
        }
    }
}

// Every pair of the flagged traits, exactly (missing expression values,
// Handling missing values: each pair keeps the samples with both an
// expression value and a genotype, with K' of them): one wave per (trait,
// permutation, 64 SNPs), one lane per SNP.  A SNP without missing genotypes
// needs no re-ranking (the trait's ranks are already over its observed
// samples): the lane sums ranks and counts per group over the observed
// samples.  SNPs with missing genotypes are re-ranked by the wave
// (coop_exact), one after the other.
template <int MODE>
__global__ __launch_bounds__(256) void scan_nan_traits(ScanArgs a, const int32_t* list,
                                                       const int32_t* n_list, int P) {
    extern __shared__ __attribute__((aligned(16))) int16_t s_buf[];   // per wave coop_lds_entries(K)
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int16_t* sb = s_buf + wave * coop_lds_entries(a.K);
    const int K = a.K;
    const int64_t nb = (a.M + kWave - 1) / kWave;
    const int64_t items = (int64_t)*n_list * P * nb;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < items; it += waves) {
        const int64_t blk = it % nb;
        const int64_t rest = it / nb;
        const int perm = (int)(rest % P);
        const int64_t trait = list[rest / P];
        const int64_t v = (int64_t)perm * a.T + trait;
        const int16_t* rk = a.ranks2 + trait * K;
        const int32_t* pm = a.perms ? a.perms + (int64_t)perm * K : nullptr;
        const int64_t m = blk * kWave + lane;
        const bool active = m < a.M;
        const SnpInfo inf = a.info[active ? m : 0];
        const bool rerank = active && inf.nmiss > 0;
        if (active && !rerank) {
            const int8_t* gr = a.G + m * (int64_t)a.gstride;
            int64_t s[3] = {0, 0, 0};
            int n[3] = {0, 0, 0};
            int kobs = 0;
            for (int k = 0; k < K; ++k) {
                const int ak = rk[pm ? pm[k] : k];       // the same for every lane
                const int code = gr[k];
                if (ak == 0) continue;
                ++kobs;
                if (code == 0) { s[0] += ak; ++n[0]; }
                else if (code == 1) { s[1] += ak; ++n[1]; }
                else if (code == 2) { s[2] += ak; ++n[2]; }
            }
            const int64_t k1 = kobs + 1;
            const int ne = (n[0] > 0) + (n[1] > 0) + (n[2] > 0);
            const int df = ne > 0 ? ne - 1 : 0;
            const double H = exact_H(s[0] - n[0] * k1, s[1] - n[1] * k1, s[2] - n[2] * k1, n[0],
                                     n[1], n[2], kobs, a.tiesum[trait], df);
            if (MODE == SCREEN) record(a, v, m, H, df);
            else emit_full<MODE>(a, v, m, H, df, s[0], s[1], s[2]);
        }
        unsigned long long todo = __ballot(rerank);
        while (todo) {
            const int j = __builtin_ctzll(todo);
            todo &= todo - 1ull;
            const int64_t mj = blk * kWave + j;
            int df;
            int64_t s[3];
            const double H = coop_exact<4>(a, v, mj, sb, lane, &df, s);
            if (lane == 0) {
                if (MODE == SCREEN) record(a, v, mj, H, df);
                else emit_full<MODE>(a, v, mj, H, df, s[0], s[1], s[2]);
            }
        }
    }
}

}  // namespace kx

extern "C" hipError_t kx_launch_flag_nan(const int16_t* ranks2, int64_t T, int K, uint8_t* flag,
                                         int32_t* list, int32_t* n_list, int grid,
                                         hipStream_t st) {
    hipLaunchKernelGGL(kx::flag_nan_traits, dim3(grid), dim3(256), 0, st, ranks2, T, K, flag,
                       list, n_list);
    return hipGetLastError();
}

extern "C" hipError_t kx_launch_nan_traits(const kx::ScanArgs* a, const int32_t* list,
                                           const int32_t* n_list, int P, int mode, int grid,
                                           hipStream_t st) {
    const size_t lds = (size_t)4 * kx::coop_lds_entries(a->K) * sizeof(int16_t);
    if (mode == kx::SCREEN)
        hipLaunchKernelGGL(kx::scan_nan_traits<kx::SCREEN>, dim3(grid), dim3(256), lds, st, *a,
                           list, n_list, P);
    else if (mode == kx::FULL)
        hipLaunchKernelGGL(kx::scan_nan_traits<kx::FULL>, dim3(grid), dim3(256), lds, st, *a,
                           list, n_list, P);
    else
        hipLaunchKernelGGL(kx::scan_nan_traits<kx::SUMS>, dim3(grid), dim3(256), lds, st, *a,
                           list, n_list, P);
    return hipGetLastError();
}

// Both exact-evaluation launches of one scan (the second only when the
// missing-genotype buffer is in use).
extern "C" hipError_t kx_launch_exact(const kx::ScanArgs* a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(kx::scan_exact, dim3(grid), dim3(256), 0, st, *a);
    if (!a->mcand) return hipGetLastError();
    const size_t lds = (size_t)4 * kx::coop_lds_entries(a->K) * sizeof(int16_t);
    hipLaunchKernelGGL(kx::scan_exact_missing, dim3(grid), dim3(256), lds, st, *a);
    return hipGetLastError();
}
