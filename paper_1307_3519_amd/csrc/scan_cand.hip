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
// s_i(q) lies in [-min(N_i, L_q), min(N_i, G_q)].  Counting q's tie partners
// (t_q - 1 of them) too, 2 #below + (t_q - 1) = a_q - 2 and
// 2 #above + (t_q - 1) = 2K - a_q exactly; with #above_i + #below_i <= N_i and
// the tied members of group i at most t_q - 1, s_i(q) <= 2K - a_q - N_i and
// s_i(q) >= N_i - (a_q - 2), which is tighter for a q near either end of
// the ranks (a q at the top has nearly all of group i below it).  The kept samples'
// re-centred ranks sum to zero, so the shifts also satisfy
// sum_i sum_q s_i(q) = -(sum of the missing samples' centred ranks).  The
// largest f over these intervals and that plane (at a vertex of the polygon
// they cut, f being convex), with E' >= K'^3 - K' - sumT, bounds H'.
// missing_bound returns false when the bound stays below the pass's screen
// level (never for a level of 0), or when the pair can only matter for its
// row's minimum p and cannot lower it.  nq, sq, lo and hi are the pair's
// count of missing samples, the sum of their centred ranks and the summed
// per-sample shift intervals of the three groups.
__device__ inline bool missing_bound(const ScanArgs& a, int64_t v, int64_t trait,
                                     const SnpInfo& inf, int nq, int sq, const int (&lo)[3],
                                     const int (&hi)[3], int d1, int d2) {
    const int K = a.K;
    const int n[3] = {inf.n0, inf.n1, inf.n2};
    const int df = snp_df(inf);
    if (df <= 0) return false;                  // never recorded
    const int64_t kp = K - nq;
    const int64_t E = cube_minus(kp) - a.tiesum[trait];
    if (kp < 2 || E <= 0) return true;          // no bound: evaluate
    const int64_t D[3] = {-(int64_t)d1 - d2 - sq, d1, d2};
    // D'_i = D_i - s_i with s_i in [lo_i, hi_i], and the kept samples'
    // re-centred ranks sum to zero: sum_i s_i = sum_i D_i = -sq.  f is convex,
    // so its largest value over the box cut by that plane is at a vertex (two
    // shifts at an end of their interval, the third from the sum and within
    // its own); the box alone (each |D'_i| at its largest) is the fallback
    double f = -1.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int o1 = j == 0 ? 1 : 0, o2 = j == 2 ? 1 : 2;
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
            const int64_t s1 = (sg & 1) ? hi[o1] : lo[o1];
            const int64_t s2 = (sg & 2) ? hi[o2] : lo[o2];
            const int64_t sj = -(int64_t)sq - s1 - s2;
            if (sj < lo[j] || sj > hi[j]) continue;
            const int64_t x[3] = {j == 0 ? D[0] - sj : o1 == 0 ? D[0] - s1 : D[0] - s2,
                                  j == 1 ? D[1] - sj : o1 == 1 ? D[1] - s1 : D[1] - s2,
                                  j == 2 ? D[2] - sj : o1 == 2 ? D[2] - s1 : D[2] - s2};
            double fv = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (n[i]) fv += (double)(x[i] * x[i]) / (double)n[i];
            f = fv > f ? fv : f;
        }
    }
    if (f < 0.0) {
        f = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (n[i] == 0) continue;
            const int64_t x0 = D[i] - hi[i], x1 = D[i] - lo[i];
            const int64_t x = max(x0 < 0 ? -x0 : x0, x1 < 0 ? -x1 : x1);
            f += (double)(x * x) / (double)n[i];
        }
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

// One missing sample of doubled midrank aq: its centred rank joins sq and
// its shift intervals join lo and hi.
__device__ inline void add_missing_sample(int K, const int (&n)[3], int aq, int& sq,
                                          int (&lo)[3], int (&hi)[3]) {
    const int below = (aq - 2) >> 1, above = K - ((aq + 1) >> 1);
    sq += aq - (K + 1);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lo[i] -= min(min(n[i], below), aq - 2 - n[i]);
        hi[i] += min(min(n[i], above), 2 * K - aq - n[i]);
    }
}

// The bound of pair (v, m) by the whole wave, for a SNP with any number of
// missing samples (found in its packed row).  All lanes take part; the
// result is uniform.
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
        ++nq;
        add_missing_sample(K, n, aq, sq, lo, hi);
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
    return missing_bound(a, v, trait, inf, nq, sq, lo, hi, d1, d2);
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

// The same bound for one lane's pair, from the SNP's listed missing samples
// (at most kLaneMiss of them): their ranks are gathered eight at a time.
__device__ inline bool lane_pair_may_pass(const ScanArgs& a, int64_t v, int64_t m,
                                          const SnpInfo& inf, int d1, int d2) {
    const int K = a.K;
    const int64_t trait = v % a.T, perm = v / a.T;
    const int16_t* rk = a.ranks2 + trait * K;
    const int32_t* pm = a.perms ? a.perms + perm * K : nullptr;
    const int16_t* mp = a.mpos + m * kLaneMiss;
    const int n[3] = {inf.n0, inf.n1, inf.n2};
    const int nq = inf.nmiss;
    int sq = 0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int j0 = 0; j0 < nq; j0 += 8) {
        // 8 positions per 16-byte load (a SNP's list is 64 bytes, 16-byte
        // aligned); slots past nq load sample 0 and are not counted
        const uint4 w = *(const uint4*)(mp + j0);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        int aq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            int k = j0 + u < nq ? (int)((ws[u >> 1] >> (16 * (u & 1))) & 0xFFFFu) : 0;
            if (pm) k = pm[k];
            aq[u] = rk[k];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < nq) add_missing_sample(K, n, aq[u], sq, lo, hi);
    }
    return missing_bound(a, v, trait, inf, nq, sq, lo, hi, d1, d2);
}

// Sum over the wave by DPP moves (no LDS round trips): pairs and quads
// within each row of 16 lanes, then the row halves and the rows, then row
// sums broadcast into rows 1 and 3 and rows 0-1 into rows 2-3; lane 63 ends
// with the total.
__device__ inline int wave_sum_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);   // row_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Exact evaluation of pair (v, m) by the whole wave when the SNP's missing
// samples are listed (1..kLaneMiss of them, K from 32 to 2047) and the trait
// has every expression value: the re-ranked sums of coop_exact without its
// staging pass.  The missing samples' ranks (one lane each) go into a bitmap
// over the doubled ranks 0..2K with per-word prefix counts; every sample's
// rank and code are read from global memory, U per lane in flight together
// (the first U issued with the missing positions, so that their latency
// overlaps the bitmap's), and for sample k the bitmap gives the number of
// missing ranks below a_k (lt) and whether one equals it (eq): its re-ranked
// doubled rank is a_k - 2 lt - eq.  Only groups 1 and 2 are summed: the kept
// samples' re-ranked doubled ranks sum to K'(K' + 1).  All sums fit 32 bits
// (K (2K + 1) < 2^31).  A tie group of size t that loses its one missing
// member takes 3 t (t - 1) off the tie term (t counted per missing rank, the
// missing sample included).  Returns false, having evaluated nothing, when
// two missing samples share a rank (coop_exact handles that case).
template <int U>
__device__ inline bool coop_exact_listed(const ScanArgs& a, int64_t v, int64_t m,
                                         int16_t* sbuf, int lane, double* H_out, int* df_out) {
    const int K = a.K;
    const int64_t trait = v % a.T, perm = v / a.T;
    const int16_t* rk = a.ranks2 + trait * K;
    const int32_t* pm = a.perms ? a.perms + perm * K : nullptr;
    const int8_t* gr = a.G + m * (int64_t)a.gstride;
    const SnpInfo inf = a.info[m];
    const int nq = inf.nmiss;
    int pos = lane < nq ? (int)a.mpos[m * kLaneMiss + lane] : 0;
    // the first U samples of this lane (loads at clamped indices, all in
    // flight together; samples past K are masked afterwards)
    int code[U], ak[U];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = min(k0 + u * kWave + lane, K - 1);
            code[u] = (int)gr[k];
            ak[u] = (int)rk[pm ? pm[k] : k];
        }
    };
    load(0);
    if (pm) pos = pm[pos];
    const int qa = lane < nq ? (int)rk[pos] : 0;
    uint4* bm = (uint4*)(sbuf + coop_bitmap_offset(K));
    int32_t* tc = (int32_t*)(sbuf + 2 * K + 64);
    const int W = ((2 * K) >> 6) + 1;            // 64-bit words covering 0..2K
    __builtin_amdgcn_wave_barrier();
    if (lane < W) bm[lane] = make_uint4(0u, 0u, 0u, 0u);
    tc[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    bool dup = false;
    if (lane < nq) {
        const uint32_t bit = 1u << (qa & 31);
        const uint32_t old = atomicOr((uint32_t*)&bm[qa >> 6] + ((qa >> 5) & 1), bit);
        dup = (old & bit) != 0u;
    }
    if (__any(dup)) return false;
    __builtin_amdgcn_wave_barrier();
    {
        const uint4 e = lane < W ? bm[lane] : make_uint4(0u, 0u, 0u, 0u);
        const int c = __popc(e.x) + __popc(e.y);
        const int incl = wave_incl_scan(c, lane);
        if (lane < W) bm[lane].z = (uint32_t)(incl - c);
    }
    __builtin_amdgcn_wave_barrier();
    const long long ts0 = a.tiesum[trait];
    int s1 = 0, s2 = 0;
    for (int k0 = 0;;) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool valid = k0 + u * kWave + lane < K;
            const uint4 e = bm[ak[u] >> 6];
            const int b = ak[u] & 63;
            const unsigned long long bits = (unsigned long long)e.x |
                                            ((unsigned long long)e.y << 32);
            const int lt = (int)e.z + __popcll(bits & ((1ull << b) - 1ull));
            const int eq = (int)((bits >> b) & 1ull);
            const int ap = ak[u] - 2 * lt - eq;
            s1 += (valid && code[u] == 1) ? ap : 0;
            s2 += (valid && code[u] == 2) ? ap : 0;
            if (ts0 != 0 && valid && eq) atomicAdd(&tc[lt], 1);
        }
        k0 += U * kWave;
        if (k0 >= K) break;
        load(k0);
    }
    s1 = wave_sum_dpp(s1);
    s2 = wave_sum_dpp(s2);
    long long ts = ts0;
    if (ts0 != 0) {
        __builtin_amdgcn_wave_barrier();
        int corr = 0;
        if (lane < nq) {
            const int t = tc[lane];
            corr = 3 * t * (t - 1);
        }
        ts -= wave_sum_dpp(corr);
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t kp = K - nq;
    const int64_t s0 = kp * (kp + 1) - s1 - s2;
    const int df = snp_df(inf);
    *df_out = df;
    *H_out = exact_H(s0 - (int64_t)inf.n0 * (kp + 1), s1 - (int64_t)inf.n1 * (kp + 1),
                     s2 - (int64_t)inf.n2 * (kp + 1), inf.n0, inf.n1, inf.n2, kp, ts, df);
    return true;
}

// Pairs of SNPs with missing genotypes that passed the scan's bound.  A wave
// takes up to 64 queued pairs at a time, one lane each: the lane bounds its
// pair from the listed missing samples (missing_bound, a few gathers); then
// the whole wave re-derives the ranks over the kept samples
// (coop_exact_listed, else coop_exact) of each pair that the bound keeps,
// one after the other, and of a SNP with
// more missing samples than the list holds it first takes the bound as a
// wave (missing_pair_may_pass).  When there are fewer queued pairs than
// lanes in the grid, each wave takes fewer of them so that every wave gets
// some.  The pass is bound by the latency of the re-ranks' dependent loads,
// so it runs at six waves per SIMD, as a kernel of its own so that the
// complete-SNP path does not set its register budget.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6)))
void scan_exact_missing(ScanArgs a) {
    extern __shared__ __attribute__((aligned(16))) int16_t s_buf[];   // per wave coop_lds_entries(K)
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int16_t* sb = s_buf + wave * coop_lds_entries(a.K);
    int64_t nm = (int64_t)*a.n_mcand;
    if (nm > a.mcand_cap) nm = a.mcand_cap;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w_id = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    // pairs per wave and round: 1..64
    const int per = (int)min((int64_t)kWave, max((int64_t)1, (nm + waves - 1) / waves));
    for (int64_t base = w_id * per; base < nm; base += waves * per) {
        const int64_t e = base + lane;
        bool have = lane < per && e < nm;
        const int4 q = have ? a.mcand[e] : make_int4(0, 0, 0, 0);
        const int64_t v = have ? (int64_t)a.row_v[q.x] : -1;
        have = have && v >= 0;            // padding rows can pass the scan's bound
        bool listed = false, pass = false;
        if (have) {
            const SnpInfo inf = a.info[q.y];
            listed = inf.nmiss <= kLaneMiss;
            if (listed) pass = lane_pair_may_pass(a, v, q.y, inf, q.z, q.w);
        }
        unsigned long long todo = __ballot(have && (pass || !listed));
        while (todo) {
            const int j = __builtin_ctzll(todo);
            todo &= todo - 1ull;
            // j is uniform: the pair's fields are read from its lane
            const int64_t vj = __builtin_amdgcn_readlane((int)v, j);
            const int mj = __builtin_amdgcn_readlane(q.y, j);
            const bool lj = __builtin_amdgcn_readlane((int)listed, j) != 0;
            if (!lj && !missing_pair_may_pass(a, vj, mj, __builtin_amdgcn_readlane(q.z, j),
                                              __builtin_amdgcn_readlane(q.w, j), lane))
                continue;
            int df;
            double H;
            bool done = false;
            if (lj && a.K >= 32 && a.K <= 2047)
                // eight samples per lane in flight (sixteen spilled registers
                // at this kernel's six waves per SIMD: cohort step 53.6 ms
                // against 51.3)
                done = a.K > 256 ? coop_exact_listed<8>(a, vj, mj, sb, lane, &H, &df)
                                 : coop_exact_listed<4>(a, vj, mj, sb, lane, &H, &df);
            if (!done) {
                int64_t sums[3];
                H = coop_exact<4>(a, vj, mj, sb, lane, &df, sums);
            }
            if (lane == 0) record(a, vj, mj, H, df);
        }
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

// Screen-mode tallies of one lane over pairs of one virtual row v: counts
// per level and the largest H at df 1 and at df 2 (p falls as H grows at
// fixed df, so the minimum p over the pairs is that of one of the two);
// hits are written at once.  The wave's tallies reach memory in one flush.
struct RowTally {
    unsigned cnt[kMaxLevels];
    double h1, h2;
};

__device__ inline void tally_pair(const ScanArgs& a, RowTally& r, int64_t v, int64_t m,
                                  double H, int df) {
    if (df <= 0) return;
#pragma unroll
    for (int l = 0; l < kMaxLevels; ++l)
        if (l < a.n_lev && H > a.hc[l][df - 1]) ++r.cnt[l];
    if (df == 1) r.h1 = fmax(r.h1, H);
    else r.h2 = fmax(r.h2, H);
    if (a.hits && H > a.hc[0][df - 1]) {
        const unsigned long long idx = atomicAdd(a.n_hits, 1ull);
        if ((int64_t)idx < a.hit_cap) {
            HitRec h;
            h.trait = (int32_t)v;     // perm * T + trait (the trait without permutations)
            h.snp = (int32_t)(a.snp_base + m);
            h.H = H;
            h.p = pvalue(H, df);
            a.hits[idx] = h;
        }
    }
}

// All lanes of the wave call this together.
__device__ inline void tally_flush(const ScanArgs& a, const RowTally& r, int64_t v, int lane) {
    if (a.counts) {
        const int64_t perm = v / a.T;
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l) {
            if (l >= a.n_lev) break;
            const int c = wave_sum((int)r.cnt[l]);
            if (lane == 0 && c) atomicAdd(&a.counts[perm * a.n_lev + l], (unsigned long long)c);
        }
    }
    if (a.minp_bits) {
        double h1 = r.h1, h2 = r.h2;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            h1 = fmax(h1, __shfl_xor(h1, o, 64));
            h2 = fmax(h2, __shfl_xor(h2, o, 64));
        }
        double p = 2.0;
        if (h1 >= 0.0) p = pvalue(h1, 1);
        if (h2 >= 0.0) p = fmin(p, pvalue(h2, 2));
        if (lane == 0 && p <= 1.0) atomicMin(&a.minp_bits[v], dbl_bits(p));
    }
}

// LDS of one wave of scan_nan_traits: the staged rank words (three arrays of
// nan_words(K) words), the ranks as int16 (4 nan_words(K) of them), then the
// coop_exact buffer.
__host__ __device__ inline int nan_words(int K) { return ((K + 15) & ~15) >> 2; }
__host__ __device__ inline int nan_wave_lds_bytes(int K) {
    return 20 * nan_words(K) + 2 * coop_lds_entries(K);
}
constexpr int kNoRank = 0x7FFF;   // above every doubled rank (2K <= 16384)

// Every pair of the flagged traits, exactly (missing expression values,
// Handling missing values: each pair keeps the samples with both an
// expression value and a genotype, K' of them).  One wave per (virtual row,
// chunk of SNP blocks of 64), one lane per SNP; the rows vary fastest over
// the items, so the waves that run together read the same genotype rows.
// The row's ranks are staged once per item in LDS as bytes, four samples a
// word: low bytes, high bytes, and 1 for an observed sample (a zero rank
// counts nowhere).  A SNP without missing genotypes needs no re-ranking (the
// trait's ranks are already over its observed samples): the lane turns 16
// genotype codes at a time into byte indicators of groups 1 and 2 and takes
// their dot products with the rank and observation bytes (v_dot4_u32_u8);
// group 0 follows from the row's totals, K' observed samples whose doubled
// ranks sum to K' (K' + 1).  A SNP with up to four removed samples (a
// missing genotype where the trait has a value) is re-ranked by its lane: a
// second pass subtracts each removal's effect on the group sums and counts
// the removed ranks' tie groups for the tie term (Handling tied data).  SNPs
// with more are re-ranked by the wave (coop_exact), one after the other.
// Four waves per SIMD (128
// registers, a few spilled) against two at the compiler's choice: 8.3 ->
// 7.2 ms per step with 402 such traits of 20 000 against 500 000 SNPs.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void scan_nan_traits(ScanArgs a, const int32_t* list,
                                                       const int32_t* n_list, int P) {
    extern __shared__ __attribute__((aligned(16))) int16_t s_buf[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int K = a.K;
    const int KW = nan_words(K);                  // a multiple of 4
    uint32_t* slo = (uint32_t*)((char*)s_buf + (size_t)wave * nan_wave_lds_bytes(K));
    uint32_t* shi = slo + KW;
    uint32_t* sob = shi + KW;
    int16_t* srk = (int16_t*)(sob + KW);          // the ranks, 4 KW of them (zero past K)
    int16_t* sb = srk + 4 * KW;                   // coop_exact buffer
    const bool wide = 2 * K > 255;                // ranks above one byte
    const int64_t nb = (a.M + kWave - 1) / kWave;
    const int64_t rows = (int64_t)*n_list * P;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    if (rows <= 0 || nb <= 0) return;
    // about two items per wave of the grid
    const int64_t chunk = max((int64_t)1, (nb * rows + 2 * waves - 1) / (2 * waves));
    const int64_t n_chunks = (nb + chunk - 1) / chunk;
    const int64_t items = rows * n_chunks;
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; it < items; it += waves) {
        const int64_t row = it % rows;
        const int64_t c = it / rows;
        const int perm = (int)(row % P);
        const int64_t trait = list[row / P];
        const int64_t v = (int64_t)perm * a.T + trait;
        const int16_t* rk = a.ranks2 + trait * K;
        const int32_t* pm = a.perms ? a.perms + (int64_t)perm * K : nullptr;
        int kobs = 0;
        for (int i = lane; i < KW; i += kWave) {
            uint32_t lo = 0, hi = 0, ob = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int k = 4 * i + b;
                const int ak = k < K ? (int)rk[pm ? pm[k] : k] : 0;
                lo |= (uint32_t)(ak & 0xFF) << (8 * b);
                hi |= (uint32_t)(ak >> 8) << (8 * b);
                ob |= (uint32_t)(ak != 0) << (8 * b);
                kobs += ak != 0;
            }
            slo[i] = lo;
            shi[i] = hi;
            sob[i] = ob;
        }
        for (int k = lane; k < 4 * KW; k += kWave) srk[k] = k < K ? rk[pm ? pm[k] : k] : 0;
        kobs = wave_sum(kobs);
        __builtin_amdgcn_wave_barrier();
        const int64_t k1 = kobs + 1;
        const int64_t tsum = a.tiesum[trait];
        RowTally tl;
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l) tl.cnt[l] = 0;
        tl.h1 = -1.0;
        tl.h2 = -1.0;
        const int64_t b_end = min(nb, (c + 1) * chunk);
        for (int64_t blk = c * chunk; blk < b_end; ++blk) {
            const int64_t m = blk * kWave + lane;
            const bool active = m < a.M;
            const int nmiss = active ? (int)a.info[m].nmiss : 0;
            const int8_t* gr = a.G + (active ? m : 0) * (int64_t)a.gstride;
            uint32_t s1 = 0, s2 = 0, n1 = 0, n2 = 0, h1 = 0, h2 = 0;
            // removed samples: a missing genotype where the trait has a
            // value.  The lane keeps the ranks of up to four (kNoRank: none);
            // a SNP with more is re-ranked by the wave.
            int nq = 0;
            int q0 = kNoRank, q1 = kNoRank, q2 = kNoRank, q3 = kNoRank;
            // pass 1: group sums and counts over the observed samples, and
            // (only in waves that have a SNP with a missing genotype) the
            // ranks of the removed samples
            auto pass1 = [&](auto with_miss) {
                // the packed row stride is a multiple of 32 bytes: 16-byte
                // loads stay inside the row (codes past K meet zero ranks)
                for (int i0 = 0; i0 < KW; i0 += 4) {
                    const uint4 g4 = *(const uint4*)(gr + 4 * i0);
                    const uint4 l4 = *(const uint4*)(slo + i0);
                    const uint4 o4 = *(const uint4*)(sob + i0);
                    const uint32_t gw[4] = {g4.x, g4.y, g4.z, g4.w};
                    const uint32_t lw[4] = {l4.x, l4.y, l4.z, l4.w};
                    const uint32_t ow[4] = {o4.x, o4.y, o4.z, o4.w};
                    uint32_t i1[4], i2[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        // codes are 0..3: bit 0 alone marks group 1, bit 1
                        // alone group 2, both the missing code
                        const uint32_t w = gw[j], t = w >> 1;
                        i1[j] = (w & 0x01010101u) & ~t;
                        i2[j] = (t & 0x01010101u) & ~w;
                        s1 = __builtin_amdgcn_udot4(i1[j], lw[j], s1, false);
                        s2 = __builtin_amdgcn_udot4(i2[j], lw[j], s2, false);
                        n1 = __builtin_amdgcn_udot4(i1[j], ow[j], n1, false);
                        n2 = __builtin_amdgcn_udot4(i2[j], ow[j], n2, false);
                        if (decltype(with_miss)::value && nmiss) {
                            uint32_t m3 = (w & t) & 0x01010101u;
                            while (m3) {
                                const int k = 4 * (i0 + j) + (__builtin_ctz(m3) >> 3);
                                m3 &= m3 - 1u;
                                const int aq = srk[k];
                                if (aq != 0) {
                                    q0 = nq == 0 ? aq : q0;
                                    q1 = nq == 1 ? aq : q1;
                                    q2 = nq == 2 ? aq : q2;
                                    q3 = nq == 3 ? aq : q3;
                                    ++nq;
                                }
                            }
                        }
                    }
                    if (wide) {
                        const uint4 h4 = *(const uint4*)(shi + i0);
                        const uint32_t hw[4] = {h4.x, h4.y, h4.z, h4.w};
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            h1 = __builtin_amdgcn_udot4(i1[j], hw[j], h1, false);
                            h2 = __builtin_amdgcn_udot4(i2[j], hw[j], h2, false);
                        }
                    }
                }
            };
            if (__ballot(nmiss > 0)) {
                if (active) pass1(std::true_type{});
            } else if (active) {
                pass1(std::false_type{});
            }
            const bool lane_ok = active && nq <= 4;
            // Removing sample j lowers every kept doubled rank above a_j by 2
            // and every tied one by 1, so group i loses
            // sum_{k in group i} ([a_k > a_j] + [a_k >= a_j]); e_j is the
            // size of a_j's tie group before any removal.
            int nqw = lane_ok ? nq : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) nqw = max(nqw, __shfl_xor(nqw, o, 64));
            int64_t c1 = 0, c2 = 0;
            int e0 = 0, e1 = 0, e2 = 0, e3 = 0;
            if (nqw > 0 && lane_ok && nq > 0) {
                for (int i0 = 0; i0 < KW; i0 += 4) {
                    const uint4 g4 = *(const uint4*)(gr + 4 * i0);
                    const uint32_t gw[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int ak = srk[4 * (i0 + j) + b];
                            const uint32_t code = (gw[j] >> (8 * b)) & 3u;
                            auto one = [&](int q, int& e) {
                                const int f = (ak > q) + (ak >= q);
                                c1 += code == 1u ? f : 0;
                                c2 += code == 2u ? f : 0;
                                e += ak == q;
                            };
                            one(q0, e0);
                            if (nqw > 1) one(q1, e1);
                            if (nqw > 2) one(q2, e2);
                            if (nqw > 3) one(q3, e3);
                        }
                    }
                }
            }
            if (lane_ok) {
                const int kp = kobs - nq;
                const int64_t kp1 = kp + 1;
                const int64_t S1 = (int64_t)s1 + ((int64_t)h1 << 8) - c1;
                const int64_t S2 = (int64_t)s2 + ((int64_t)h2 << 8) - c2;
                const int N1 = (int)n1, N2 = (int)n2, N0 = kp - N1 - N2;
                const int64_t S0 = (int64_t)kp * kp1 - S1 - S2;
                // tie term: a removal from a tie group of current size t
                // takes 3 t (t - 1) off (t^3 - t)
                int64_t ts = tsum;
                auto drop = [&](int64_t t) { ts -= 3 * t * (t - 1); };
                if (nq > 0) drop(e0);
                if (nq > 1) drop(e1 - (q1 == q0));
                if (nq > 2) drop(e2 - (q2 == q0) - (q2 == q1));
                if (nq > 3) drop(e3 - (q3 == q0) - (q3 == q1) - (q3 == q2));
                const int ne = (N0 > 0) + (N1 > 0) + (N2 > 0);
                const int df = ne > 0 ? ne - 1 : 0;
                const double H = exact_H(S0 - N0 * kp1, S1 - N1 * kp1, S2 - N2 * kp1, N0, N1, N2,
                                         kp, ts, df);
                if (MODE == SCREEN) tally_pair(a, tl, v, m, H, df);
                else emit_full<MODE>(a, v, m, H, df, S0, S1, S2);
            }
            unsigned long long todo = __ballot(active && !lane_ok);
            while (todo) {
                const int j = __builtin_ctzll(todo);
                todo &= todo - 1ull;
                const int64_t mj = blk * kWave + j;
                int dfj;
                int64_t sj[3];
                const double Hj = coop_exact<4>(a, v, mj, sb, lane, &dfj, sj);
                if (lane == 0) {
                    if (MODE == SCREEN) tally_pair(a, tl, v, mj, Hj, dfj);
                    else emit_full<MODE>(a, v, mj, Hj, dfj, sj[0], sj[1], sj[2]);
                }
            }
        }
        if (MODE == SCREEN) tally_flush(a, tl, v, lane);
        __builtin_amdgcn_wave_barrier();
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
    const size_t lds = (size_t)4 * kx::nan_wave_lds_bytes(a->K);
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
