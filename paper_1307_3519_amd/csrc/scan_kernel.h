// scan_kernel.h -- rank-sum GEMM on MFMA with the Kruskal-Wallis statistic, tie
// correction, chi-square p-value and hit compaction fused into its epilogue.
//
// What is computed (eq. (1), eq. (2), tied-data and P-value sections): for a
// trait n with centred doubled ranks c_nk = a_nk - (K+1) and a SNP m with
// genotype groups g_i, the twice-centred group sums
//     D_i(n,m) = sum_{k in g_i} c_nk          (a product R * I_i^T, eq. (1))
// give  f = sum_{N_i>0} D_i^2 / N_i  and  H = 3 (K-1) f / (K^3 - K - sumT_n),
// which is eq. (2) divided by the tie factor, written without the
// cancelling "- 3(K+1)" term.  sum_i D_i = 0 when no genotype is missing, so
// two MFMA columns per SNP suffice (the paper uses l + 1 products).
//
// Kernel organisation (SNP-stationary): a block has 4 waves; each wave owns
// one tile of 32 SNPs whose genotype columns it expands once into MFMA
// B fragments held in registers, then streams 32-trait A tiles (centred
// ranks, fragment order, L2 resident) through v_mfma 32x32 instructions.
// The 32x32 accumulator tile never leaves registers: a 4-operation fp32
// screen per pair compares f against the per-trait threshold; the rare
// survivors are re-evaluated exactly (integer D_i -> exact rational H ->
// fp64 p) and appended to the hit list with one atomic each.
//
// Forms of the two/three MFMA columns per SNP:
//   DIAG   Y = cy1 D1 + cy2 D2 and Z = D2 (integer coefficients chosen so that
//          f = wy Y^2 + wz Z^2); exact while |Y| stays below 2^24
//   PLAIN  Y = D1, Z = D2 and f = a0 (D1+D2)^2 + a1 D1^2 + a2 D2^2
//   MISS3  D0, D1, D2 with indicators that are 0 at missing genotypes; pairs
//          whose SNP has missing genotypes use a rigorous upper bound of H
//          and survivors are recomputed by the wave cooperatively with the
//          ranks re-derived over the remaining samples.
#pragma once
#include "kx_args.h"
#include <type_traits>

namespace kx {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int int4v __attribute__((ext_vector_type(4)));


template <int E> struct ET;
template <> struct ET<F16> {
    using frag = half8;
    using acc = f32x16;
    static constexpr int kps = 16;     // samples per k-step
    static constexpr int per_lane = 8; // samples per lane per k-step
    __device__ static acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    __device__ static float val(const acc& c, int r) { return c[r]; }
    __device__ static frag make(const int8_t* codes, float v0, float v1, float v2) {
        frag f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int c = codes[e];
            float v = c == 0 ? v0 : c == 1 ? v1 : c == 2 ? v2 : 0.0f;
            f[e] = (_Float16)v;
        }
        return f;
    }
};
template <> struct ET<I8> {
    using frag = int4v;
    using acc = i32x16;
    static constexpr int kps = 32;
    static constexpr int per_lane = 16;
    __device__ static acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
    }
    __device__ static float val(const acc& c, int r) { return (float)c[r]; }
    __device__ static frag make(const int8_t* codes, float v0, float v1, float v2) {
        frag f;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint32_t u = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                int c = codes[4 * w + b];
                int v = c == 0 ? (int)v0 : c == 1 ? (int)v1 : c == 2 ? (int)v2 : 0;
                u |= (uint32_t)(uint8_t)(int8_t)v << (8 * b);
            }
            f[w] = (int)u;
        }
        return f;
    }
};

// Load through a global-address-space pointer: keeps the hot loads out of
// the flat path (flat loads also count against the LDS counter, so a wait for
// them would also wait for every outstanding prefetch).
template <class V>
__device__ inline V gload(const V* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    V v;
    __builtin_memcpy(&v, (const __attribute__((address_space(1))) V*)p, sizeof(V));
    return v;
#else
    return *p;
#endif
}

// Wave-uniform load through the constant address space (scalar load).
__device__ inline float cload(const float* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) float*)p;
#else
    return *p;
#endif
}

__device__ inline int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline long long wave_sum64(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Record one exactly evaluated pair (screen mode).
__device__ inline void record(const ScanArgs& a, int64_t v, int64_t m, double H, int df) {
    if (df <= 0) return;
    const int64_t perm = v / a.T;
    if (a.counts) {
        for (int l = 0; l < a.n_lev; ++l)
            if (H > a.hc[l][df - 1]) atomicAdd(&a.counts[perm * a.n_lev + l], 1ull);
    }
    const bool hit = H > a.hc[0][df - 1];
    if (!(a.minp_bits || (a.hits && hit))) return;
    double p = pvalue(H, df);
    if (a.minp_bits) atomicMin(&a.minp_bits[v], dbl_bits(p));
    if (a.hits && hit) {
        unsigned long long idx = atomicAdd(a.n_hits, 1ull);
        if ((int64_t)idx < a.hit_cap) {
            HitRec h;
            h.trait = (int32_t)v;     // perm * T + trait (the trait without permutations)
            h.snp = (int32_t)(a.snp_base + m);
            h.H = H;
            h.p = p;
            a.hits[idx] = h;
        }
    }
}

// Write the FULL / SUMS outputs of one pair.
template <int MODE>
__device__ inline void emit_full(const ScanArgs& a, int64_t v, int64_t m, double H, int df,
                                 int64_t s0, int64_t s1, int64_t s2) {
    if (m >= a.M || v < 0) return;
    if (MODE == FULL) {
        a.H_out[v * a.M + m] = H;
        a.p_out[v * a.M + m] = pvalue(H, df);
    } else if (MODE == SUMS) {
        int64_t TM = a.T * a.M;
        a.sums_out[v * a.M + m] = (int32_t)s0;
        a.sums_out[TM + v * a.M + m] = (int32_t)s1;
        a.sums_out[2 * TM + v * a.M + m] = (int32_t)s2;
    }
}

// Exact evaluation of one screened pair of a SNP without missing genotypes
// from its two exact MFMA column values: (Y, Z) of the DIAG form or
// (D1, D2) of the PLAIN form; D0 = -D1 - D2.
__device__ inline void eval_candidate(const ScanArgs& a, int64_t row, int64_t m, float y,
                                      float z, uint32_t flags) {
    const SnpInfo inf = a.info[m];
    const int64_t v = a.row_v[row];
    if (v < 0) return;                // padding row of a partial tile
    int64_t D1, D2;
    if (flags & kCandPlain) {
        D1 = (int64_t)y;
        D2 = (int64_t)z;
    } else {
        const int64_t Y = (int64_t)y;
        if (flags & kCandZs) {
            // z = q D2 exactly; the quotient is an integer
            const float q = diag_zscale(inf);
            D2 = q > 0.0f ? (int64_t)rint((double)z / (double)q) : 0;
        } else {
            D2 = (int64_t)z;
        }
        D1 = inf.cy1 ? (Y - (int64_t)inf.cy2 * D2) / inf.cy1 : 0;
    }
    const int64_t D0 = -D1 - D2;
    const int df = snp_df(inf);
    const double H = exact_H(D0, D1, D2, inf.n0, inf.n1, inf.n2, a.K, a.tiesum[v % a.T], df);
    record(a, v, m, H, df);
}

// Used only when the candidate buffer is full: keeps its registers out of
// the scan loop.
__device__ __attribute__((noinline)) void eval_candidate_fallback(const ScanArgs& a, int64_t row,
                                                                   int64_t m, float y, float z,
                                                                   uint32_t flags) {
    eval_candidate(a, row, m, y, z, flags);
}

// Block barrier without a memory fence (the LDS-DMA waits are explicit);
// the empty asm statements keep the compiler from moving memory accesses
// across it.
__device__ inline void block_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Screened pairs are staged per wave in LDS and copied to the global
// candidate buffer in bursts (one atomic per burst); a pair that does not fit
// in the global buffer is evaluated on the spot.
constexpr int kStageCap = 64;

__device__ inline void flush_stage(const ScanArgs& a, const ScanArgs* a_lds, uint4* stage, int& sn,
                                   int lane) {
    if (sn == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.n_cand, (unsigned long long)sn);
    base = __shfl(base, 0, 64);
    for (int i = lane; i < sn; i += kWave) {
        const uint4 e = stage[i];
        const unsigned long long idx = base + (unsigned long long)i;
        if ((int64_t)idx < a.cand_cap) {
            a.cand[idx] = e;
        } else {
            eval_candidate_fallback(*a_lds, (int64_t)e.x, (int64_t)(e.y & kCandSnp),
                                    __uint_as_float(e.z), __uint_as_float(e.w),
                                    e.y & ~kCandSnp);
        }
    }
    sn = 0;
    __builtin_amdgcn_wave_barrier();
}

// Called by all lanes of a wave (uniform control flow); `cand` per lane.
__device__ inline void stage_candidates(const ScanArgs& a, const ScanArgs* a_lds, uint4* stage,
                                        int& sn, int lane, bool cand, int64_t row, int64_t m,
                                        float y, float z, uint32_t flags) {
    const unsigned long long msk = __ballot(cand);
    if (!msk) return;
    const int n = __popcll(msk);
    if (sn + n > kStageCap) flush_stage(a, a_lds, stage, sn, lane);
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (cand)
        stage[sn + __popcll(msk & lt)] =
            make_uint4((uint32_t)row, (uint32_t)m | flags,
                       __float_as_uint(y), __float_as_uint(z));
    sn += n;
    __builtin_amdgcn_wave_barrier();
}

// Exact evaluation of pair (v, m) whose SNP has missing genotypes: the
// missing samples are removed and the ranks re-derived over the rest,
//   a'_k = a_k - sum_{j missing} (2 [a_j < a_k] + [a_j == a_k]),
// the tie term loses 3 t (t - 1) for each removal from a tie group of
// current size t.  All 64 lanes of the wave take part; the result is uniform.
// sbuf (coop_lds_entries(K) int16 entries of this wave's LDS, 16-byte
// aligned): [0, K) the pair's samples (rank | code << 13, ranks are below 2^13
// for K <= 4095), [K, 2K + 64) the ranks of its missing samples (the rank
// bitmap of the fast path sits past the first 64), then 64 int32 counters.
constexpr int kCodeShift = 13;
constexpr int kRankMask = (1 << kCodeShift) - 1;
constexpr int kAbsentCode = 4;   // sample without an expression value (rank 0)
__host__ __device__ inline int coop_lds_entries(int K) { return (2 * K + 64 + 128 + 7) & ~7; }
// int16 offset of the fast path's rank bitmap (16-byte aligned)
__device__ inline int coop_bitmap_offset(int K) { return (K + 64 + 7) & ~7; }

// Ascending sort of one value per lane across the wave (bitonic network).
__device__ inline int wave_sort(int v, int lane) {
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int o = __shfl_xor(v, j, 64);
            const bool up = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            v = (lower == up) ? min(v, o) : max(v, o);
        }
    }
    return v;
}

__device__ inline int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// U: samples per lane whose loads are in flight together in the first pass;
// BITMAP: rank-bitmap lookups instead of binary searches when the missing
// ranks are distinct (the out-of-line copy called from the scan kernels takes
// U = 1 and no bitmap, to stay small).
template <int U = 8, bool BITMAP = true>
__device__ inline double coop_exact(const ScanArgs& a, int64_t v, int64_t m, int16_t* sbuf,
                                    int lane, int* df_out, int64_t* s_out) {
    const int K = a.K;
    const int64_t trait = v % a.T, perm = v / a.T;
    const int16_t* rk = a.ranks2 + trait * K;
    const int32_t* pm = a.perms ? a.perms + perm * K : nullptr;
    const int8_t* gr = a.G + m * (int64_t)a.gstride;
    uint16_t* sr = (uint16_t*)sbuf;
    int16_t* qb = sbuf + K;
    int32_t* tc = (int32_t*)(sbuf + 2 * K + 64);   // 4-byte aligned: 2K + 64 is even
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // one pass over global memory, eight loads of each kind in flight per lane:
    // rank and genotype code of every sample into LDS, the ranks of the
    // missing samples compacted into qb
    int nq = 0;
    int kobs = 0;            // samples with an expression value
    auto pass = [&](auto with_perm) {
        for (int k0 = 0; k0 < K; k0 += U * kWave) {
            // loads at clamped indices (no branches, so all are in flight
            // together); lanes past K are masked afterwards
            int code[U], ak[U], idx[U];
#pragma unroll
            for (int u = 0; u < U; ++u) idx[u] = min(k0 + u * kWave + lane, K - 1);
#pragma unroll
            for (int u = 0; u < U; ++u) code[u] = (int)gr[idx[u]];
            if constexpr (decltype(with_perm)::value) {
#pragma unroll
                for (int u = 0; u < U; ++u) idx[u] = pm[idx[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) ak[u] = (int)rk[idx[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + u * kWave + lane;
                // a missing expression value (rank 0) takes the sample out of
                // the pair whatever its genotype
                const int cu = ak[u] == 0 ? kAbsentCode : code[u];
                if (k < K) sr[k] = (uint16_t)(ak[u] | (cu << kCodeShift));
                const bool miss = k < K && cu == kMissingCode;
                const unsigned long long msk = __ballot(miss);
                if (miss) qb[nq + __popcll(msk & lt)] = (int16_t)ak[u];
                nq += __popcll(msk);
                kobs += __popcll(__ballot(k < K && cu != kAbsentCode));
            }
        }
    };
    if (pm) pass(std::true_type{});
    else pass(std::false_type{});
    __builtin_amdgcn_wave_barrier();
    long long ts = a.tiesum[trait];
    long long s0 = 0, s1 = 0, s2 = 0;
    int n0 = 0, n1 = 0, n2 = 0;              // kept samples per group
    auto add = [&](int code, int ap) {
        if (code == 0) { s0 += ap; ++n0; } else if (code == 1) { s1 += ap; ++n1; } else { s2 += ap; ++n2; }
    };
    const int W = ((2 * K) >> 6) + 1;      // 64-bit words covering doubled ranks 0..2K
    int qv = 0x7FFF;
    bool dup = false;
    if (nq <= kWave) {
        qv = wave_sort(lane < nq ? (int)qb[lane] : 0x7FFF, lane);
        const int prev = __shfl_up(qv, 1, 64);
        dup = __any(lane > 0 && lane < nq && prev == qv);
        __builtin_amdgcn_wave_barrier();
        qb[lane] = (int16_t)qv;
        tc[lane] = 0;
        __builtin_amdgcn_wave_barrier();
    }
    if (BITMAP && nq <= kWave && !dup && W <= kWave && K >= 32) {
        // Up to 64 missing samples with distinct ranks: a bitmap of their ranks
        // with per-word prefix counts gives, for sample k, the number of
        // missing ranks below a_k (lt) and whether one equals it, in one LDS
        // read.  The shift of a_k is 2 lt + eq; a sample equal to a missing
        // rank adds one to that rank's tie-group counter (index lt in sorted
        // order).  A tie group of size t that loses its one missing member
        // takes 3 t (t - 1) off the tie term.
        uint4* bm = (uint4*)(sbuf + coop_bitmap_offset(K));
        if (lane < W) bm[lane] = make_uint4(0u, 0u, 0u, 0u);
        __builtin_amdgcn_wave_barrier();
        if (lane < nq) atomicOr((uint32_t*)&bm[qv >> 6] + ((qv >> 5) & 1), 1u << (qv & 31));
        __builtin_amdgcn_wave_barrier();
        {
            const uint4 e = lane < W ? bm[lane] : make_uint4(0u, 0u, 0u, 0u);
            const int c = __popc(e.x) + __popc(e.y);
            const int incl = wave_incl_scan(c, lane);
            __builtin_amdgcn_wave_barrier();
            if (lane < W) bm[lane].z = (uint32_t)(incl - c);
        }
        __builtin_amdgcn_wave_barrier();
        constexpr int V4 = 4;
        for (int k0 = 0; k0 < K; k0 += V4 * kWave) {
            int x[V4];
            uint4 e[V4];
#pragma unroll
            for (int u = 0; u < V4; ++u) {
                const int k = k0 + u * kWave + lane;
                x[u] = k < K ? (int)sr[k] : (kMissingCode << kCodeShift);
            }
#pragma unroll
            for (int u = 0; u < V4; ++u) e[u] = bm[(x[u] & kRankMask) >> 6];
            int eqi[V4];
#pragma unroll
            for (int u = 0; u < V4; ++u) {
                const int k = k0 + u * kWave + lane;
                const int ak = x[u] & kRankMask;
                const int b = ak & 63;
                const unsigned long long bits = (unsigned long long)e[u].x |
                                                ((unsigned long long)e[u].y << 32);
                const int below = (int)e[u].z + __popcll(bits & ((1ull << b) - 1ull));
                const int eq = (int)((bits >> b) & 1ull);
                const int code = x[u] >> kCodeShift;
                if (k < K && code <= 2) add(code, ak - 2 * below - eq);
                eqi[u] = (k < K && eq) ? below : -1;
            }
            if (ts != 0) {
#pragma unroll
                for (int u = 0; u < V4; ++u)
                    if (eqi[u] >= 0) atomicAdd(&tc[eqi[u]], 1);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (ts != 0) {
            long long corr = 0;
            if (lane < nq) {
                const long long t = tc[lane];
                corr = 3 * t * (t - 1);
            }
            ts -= wave_sum64(corr);
        }
    } else if (nq <= kWave) {
        // Up to 64 missing samples, some tied: binary search in the sorted
        // missing ranks for lt / le = number below / at most a_k; the shift is
        // 2 lt + (le - lt).  A tie group of size t that loses r members takes
        // (t^3 - t) - ((t-r)^3 - (t-r)) off the tie term.
        for (int k0 = 0; k0 < K; k0 += kWave) {
            const int k = k0 + lane;
            if (k < K) {
                const int x = sr[k];
                const int code = x >> kCodeShift;
                const int ak = x & kRankMask;
                int lo = 0, hi = nq;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (qb[mid] < ak) lo = mid + 1; else hi = mid;
                }
                const int below = lo;
                hi = nq;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (qb[mid] <= ak) lo = mid + 1; else hi = mid;
                }
                const int equal = lo - below;
                if (code <= 2) add(code, ak - 2 * below - equal);
                if (equal && ts != 0) atomicAdd(&tc[below], 1);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (ts != 0) {
            long long corr = 0;
            if (lane < nq && (lane == 0 || qb[lane - 1] != qv)) {
                int r = 1;
                while (lane + r < nq && qb[lane + r] == qv) ++r;
                const long long t = tc[lane];
                corr = (t * t * t - t) - ((t - r) * (t - r) * (t - r) - (t - r));
            }
            ts -= wave_sum64(corr);
        }
    } else {
    if (ts != 0) {
        for (int qi = 0; qi < nq; ++qi) {
            const int aj = qb[qi];
            int cnt = 0;
            for (int k0 = 0; k0 < K; k0 += kWave) {
                const int k = k0 + lane;
                if (k < K) cnt += ((sr[k] & kRankMask) == aj);
            }
            for (int q0 = 0; q0 < qi; q0 += kWave) {
                const int qq = q0 + lane;
                if (qq < qi) cnt -= (qb[qq] == aj);
            }
            const int t = wave_sum(cnt);
            ts -= 3ll * t * (t - 1);
        }
    }
    for (int k0 = 0; k0 < K; k0 += kWave) {
        const int k = k0 + lane;
        const int x = k < K ? sr[k] : (kMissingCode << kCodeShift);
        const int code = x >> kCodeShift;
        if (code <= 2) {
            const int ak = x & kRankMask;
            int w = 0;
            for (int qi = 0; qi < nq; ++qi) {
                const int aj = qb[qi];
                w += (aj < ak) ? 2 : (aj == ak ? 1 : 0);
            }
            add(code, ak - w);
        }
    }
    }
    s0 = wave_sum64(s0); s1 = wave_sum64(s1); s2 = wave_sum64(s2);
    n0 = wave_sum(n0); n1 = wave_sum(n1); n2 = wave_sum(n2);
    // group sizes, K' and df over the pair's kept samples (the SNP's own
    // counts when the trait has every expression value)
    const int64_t kp = kobs - nq;
    const int64_t D0 = s0 - (int64_t)n0 * (kp + 1);
    const int64_t D1 = s1 - (int64_t)n1 * (kp + 1);
    const int64_t D2 = s2 - (int64_t)n2 * (kp + 1);
    const int ne = (n0 > 0) + (n1 > 0) + (n2 > 0);
    const int df = ne > 0 ? ne - 1 : 0;
    *df_out = df;
    s_out[0] = s0; s_out[1] = s1; s_out[2] = s2;
    __builtin_amdgcn_wave_barrier();
    return exact_H(D0, D1, D2, n0, n1, n2, kp, ts, df);
}

// Out-of-line entry for the scan kernels' own (rare, or FULL / SUMS) use, so
// that the re-rank's registers do not weigh on the scan loop.
__device__ __attribute__((noinline)) double coop_exact_call(const ScanArgs& a, int64_t v,
                                                            int64_t m, int16_t* sbuf, int lane,
                                                            int* df_out, int64_t* s_out) {
    return coop_exact<1, false>(a, v, m, sbuf, lane, df_out, s_out);
}

// Empties a wave's queue of screened pairs of SNPs with missing genotypes.
// In screen mode the pairs go to the global buffer (one atomic per burst) for
// scan_exact, which runs them at full occupancy instead of stalling the
// scan; pairs beyond its capacity, and the FULL / SUMS outputs, are
// evaluated here.
template <int MODE>
__device__ inline void drain(const ScanArgs& a, int4* queue, int& qn, int16_t* qbuf, int lane) {
    int e0 = 0;
    if constexpr (MODE == SCREEN) {
        if (a.mcand) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(a.n_mcand, (unsigned long long)qn);
            base = __shfl(base, 0, 64);
            const int64_t room = a.mcand_cap - (int64_t)base;
            const int fit = room <= 0 ? 0 : (room < qn ? (int)room : qn);
            for (int i = lane; i < fit; i += kWave) a.mcand[base + i] = queue[i];
            e0 = fit;
        }
    }
    for (int e = e0; e < qn; ++e) {
        int4 q = queue[e];
        int64_t v = a.row_v[q.x];
        // padding rows (zero operand) can pass the missing-genotype bound; the
        // entry is the same for the whole wave, so the skip is uniform
        if (v < 0) continue;
        int64_t m = q.y;
        int df;
        int64_t s[3];
        double H = coop_exact_call(a, v, m, qbuf, lane, &df, s);
        if (lane == 0) {
            if (MODE == SCREEN) record(a, v, m, H, df);
            else emit_full<MODE>(a, v, m, H, df, s[0], s[1], s[2]);
        }
    }
    qn = 0;
    __builtin_amdgcn_wave_barrier();
}

// WPE: waves per SIMD the register budget is sized for.
// PF: 0 = load-then-compute per tile; 1 = next tile prefetched into a second
// register buffer; 2 = software pipeline (MFMAs of the next tile interleaved
// with the screen of the current one; screen mode, complete SNPs only);
// 3 = the same pipeline fed from an LDS ring shared by the block; 4 = the
// LDS ring, one tile at a time; 5 = the LDS ring, two tiles per step.
template <int E, int KS, int FORM, int MODE,
          int PF = (MODE == SCREEN && FORM != MISS3) ? 2 : 0, int WPE = 2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void scan_kernel(ScanArgs a) {
    using T_ = ET<E>;
    using frag = typename T_::frag;
    using acc_t = typename T_::acc;
    constexpr int NC = FORM == MISS3 ? 3 : 2;
    constexpr bool QUEUE = FORM == MISS3;
    constexpr bool RING = (PF == 3 || PF == 4 || PF == 5) && MODE == SCREEN && FORM != MISS3;
    // ring slots (a power of two): two tiles per step with PF == 5
    constexpr int NSLOT = PF == 5 ? 8 : 4;
    // fp16 DIAG: second column scaled by q (diag_zscale), screen Y^2 + Z^2
    constexpr bool ZS = E == F16 && FORM == DIAG;
    // int8 DIAG: the same two-square screen with Z scaled in fp32 after the
    // conversion (the int8 B operand cannot carry q)
    constexpr bool ZF = E == I8 && FORM == DIAG;
    constexpr uint32_t kDiagFlags = ZS ? kCandZs : 0u;

    __shared__ int4 s_queue[QUEUE ? kWavesPerBlock : 1][QUEUE ? kQueueCap : 1];
    __shared__ uint4 s_stage[MODE == SCREEN ? kWavesPerBlock : 1][kStageCap];
    // copy of the arguments for the out-of-line fallback (taking the address
    // of the kernel argument itself would move it to the stack)
    __shared__ ScanArgs s_args;
    // LDS ring of A tiles shared by the block's waves (PF == 3, 4, 5)
    __shared__ frag s_ring[RING ? NSLOT * KS * kWave : 1];
    if (threadIdx.x == 0) s_args = a;
    __syncthreads();
    extern __shared__ __attribute__((aligned(16))) int16_t s_qbuf[];   // MISS3: per wave coop_lds_entries(K)

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
    int4* queue = s_queue[QUEUE ? wave : 0];
    uint4* stage = s_stage[MODE == SCREEN ? wave : 0];
    int sn = 0;
    int16_t* qbuf = s_qbuf + (QUEUE ? wave * coop_lds_entries(a.K) : 0);
    int qn = 0;

    // tile_flags[n_snp_tiles] is set when any SNP has a missing genotype,
    // tile_flags[n_snp_tiles + 1] when any tile has none
    if (a.want_flag == 1 && a.tile_flags[a.n_snp_tiles] == 0) return;
    if (a.want_flag == 0 && a.tile_flags[a.n_snp_tiles + 1] == 0) return;
    int64_t n_rows = a.n_rows;
    if (a.d_nrows) {
        int64_t d = *a.d_nrows;
        n_rows = d < n_rows ? d : n_rows;
    }
    const int64_t n_tiles = (n_rows + kTile - 1) / kTile;
    const int64_t n_ranges = (n_tiles + a.tiles_per_range - 1) / a.tiles_per_range;
    const int64_t n_blocks = (a.n_snp_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t items = n_ranges * n_blocks;
    const frag* A = (const frag*)a.A;
    const float kslack = 1.0f + kScreenSlack;

    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int64_t rg = item / n_blocks;
        const int64_t st = (item % n_blocks) * kWavesPerBlock + wave;
        const bool active = st < a.n_snp_tiles &&
                            (a.want_flag < 0 || a.tile_flags[st] == a.want_flag);
        if constexpr (RING) {
            // the waves of a block meet at barriers: skip items as a block only;
            // an inactive wave runs with all-zero columns (never a candidate)
            if (!__syncthreads_or(active)) continue;
        } else {
            if (!active) continue;
        }
        const int64_t m = active ? st * kTile + (lane & 31) : 0;
        SnpInfo inf{};
        if (active) inf = gload(a.info + m);

        // B fragments of this lane's SNP column, built once per item
        float cv[NC][3];
        if constexpr (FORM == DIAG) {
            cv[0][0] = 0.f; cv[0][1] = inf.cy1; cv[0][2] = inf.cy2;
            cv[1][0] = 0.f; cv[1][1] = 0.f; cv[1][2] = ZS ? diag_zscale(inf) : 1.f;
        } else if (FORM == PLAIN) {
            cv[0][0] = 0.f; cv[0][1] = 1.f; cv[0][2] = 0.f;
            cv[1][0] = 0.f; cv[1][1] = 0.f; cv[1][2] = 1.f;
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) cv[c][i] = (c == i) ? 1.f : 0.f;
        }
        frag B[KS][NC];
        const int8_t* grow = a.G + m * (int64_t)a.gstride + T_::per_lane * (lane >> 5);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            int8_t codes[T_::per_lane];
            if constexpr (T_::per_lane == 8) {
                uint2 w = active ? gload((const uint2*)(grow + s * T_::kps)) : make_uint2(~0u, ~0u);
                __builtin_memcpy(codes, &w, 8);
            } else {
                uint4 w = active ? gload((const uint4*)(grow + s * T_::kps))
                                 : make_uint4(~0u, ~0u, ~0u, ~0u);
                __builtin_memcpy(codes, &w, 16);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) B[s][c] = T_::make(codes, cv[c][0], cv[c][1], cv[c][2]);
        }

        // per-lane screen constants
        const int kp = a.K - inf.nmiss;
        const float fac = 3.0f * (float)(kp - 1) * kslack * a.inv_hc[snp_df(inf)];
        const float wy = inf.wy * fac, wz = inf.wz * fac;
        const float w0 = inf.a0 * fac, w1 = inf.a1 * fac, w2 = inf.a2 * fac;
        const bool lane_miss = inf.nmiss > 0;
        const float qn0 = (float)inf.nmiss * inf.n0, qn1 = (float)inf.nmiss * inf.n1,
                    qn2 = (float)inf.nmiss * inf.n2;
        const float delta = (float)(cube_minus(a.K) - cube_minus(kp));
        // MISS3: w_i (|D_i| + nmiss N_i)^2 as (|D_i| r_i + q_i)^2, r_i = sqrt(w_i)
        const float r0 = sqrtf(w0), r1 = sqrtf(w1), r2 = sqrtf(w2);
        const float q0 = qn0 * r0, q1 = qn1 * r1, q2 = qn2 * r2;
        // ZS: candidate iff Y^2 + Z^2 > theta * invc (inf when wy * fac = 0);
        // ZF: Y^2 + (zq Z)^2 with zq = sqrt(wz / wy) rounded up
        const float invc = (ZS || ZF) ? 1.0f / (inf.wy * fac) : 0.0f;
        float zq = 0.0f;
        if constexpr (ZF) {
            if (inf.wy > 0.0f) {
                zq = sqrtf(inf.wz / inf.wy);
                zq = __uint_as_float(__float_as_uint(zq) + 1u);   // next float up
            }
        }

        const int64_t t0 = rg * a.tiles_per_range;
        const int64_t t1 = (t0 + a.tiles_per_range < n_tiles) ? t0 + a.tiles_per_range : n_tiles;

        // g = (screen value of f) - theta, > 0 for every pair beyond the
        // screen level (the weights carry 3(K-1)(1+slack)/H_c(df));
        // theta is the smallest threshold of the tile's 32 traits, which
        // can only admit more candidates than the per-trait one
        auto screen = [&](const acc_t (&acc)[NC], const float th, int r) -> float {
            if constexpr (ZS) {
                float y = T_::val(acc[0], r), z = T_::val(acc[1], r);
                return fmaf(y, y, z * z) - th * invc;
            } else if constexpr (ZF) {
                float y = T_::val(acc[0], r), z = zq * T_::val(acc[1], r);
                return fmaf(y, y, z * z) - th * invc;
            } else if constexpr (FORM == DIAG) {
                float y = T_::val(acc[0], r), z = T_::val(acc[1], r);
                return fmaf(wy * y, y, fmaf(wz * z, z, -th));
            } else if constexpr (FORM == PLAIN) {
                float d1 = T_::val(acc[0], r), d2 = T_::val(acc[1], r);
                float d0 = -(d1 + d2);
                return fmaf(w0 * d0, d0, fmaf(w1 * d1, d1, fmaf(w2 * d2, d2, -th)));
            } else {
                // |D'_i - D_i| <= nmiss * N_i and E' >= K'^3 - K' - sumT
                // (complete SNPs: q_i = 0, delta = 0 and a threshold lowered
                // by 1e-6, which only admits more candidates; the weights'
                // 1e-5 slack covers the rounding of r_i and q_i)
                const float e0 = fmaf(fabsf(T_::val(acc[0], r)), r0, q0);
                const float e1 = fmaf(fabsf(T_::val(acc[1], r)), r1, q1);
                const float e2 = fmaf(fabsf(T_::val(acc[2], r)), r2, q2);
                const float tl = delta - th * 0.99999905f;
                return fmaf(e0, e0, fmaf(e1, e1, fmaf(e2, e2, tl)));
            }
        };
        // the rare path: stage the pairs that pass the screen
        auto screen_cands = [&](const int64_t t, const acc_t (&acc)[NC], const float th) {
            const int64_t rb = t * kTile + 4 * (lane >> 5);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = rb + 8 * (r >> 2) + (r & 3);
                bool cand = screen(acc, th, r) > 0.0f;
                if constexpr (QUEUE) {
                    bool qpush = cand && lane_miss;
                    unsigned long long msk = __ballot(qpush);
                    if (msk) {
                        if (qn + 64 > kQueueCap) drain<MODE>(a, queue, qn, qbuf, lane);
                        const unsigned long long lt =
                            (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                        if (qpush)
                            queue[qn + __popcll(msk & lt)] =
                                make_int4((int)row, (int)m, (int)T_::val(acc[1], r),
                                          (int)T_::val(acc[2], r));
                        qn += __popcll(msk);
                    }
                    cand = cand && !lane_miss;
                }
                if constexpr (FORM == DIAG)
                    stage_candidates(a, &s_args, stage, sn, lane, cand, row, m, T_::val(acc[0], r),
                                     T_::val(acc[1], r), kDiagFlags);
                else if constexpr (FORM == PLAIN)
                    stage_candidates(a, &s_args, stage, sn, lane, cand, row, m, T_::val(acc[0], r),
                                     T_::val(acc[1], r), kCandPlain);
                else   // complete SNP in a MISS3 tile: D0 = -D1 - D2
                    stage_candidates(a, &s_args, stage, sn, lane, cand, row, m, T_::val(acc[1], r),
                                     T_::val(acc[2], r), kCandPlain);
            }
            // screen mode: the queue carries over to the next tile and is
            // drained when nearly full and at the end of the kernel (one
            // atomic per burst of up to 128 pairs, not one per tile)
        };
        // largest screen value of a tile (VALU only, no branches)
        auto screen_max = [&](const acc_t (&acc)[NC], const float th) -> float {
            if constexpr (ZS || ZF) {
                float smax = 0.0f;
#pragma unroll
                for (int r = 0; r < 16; r += 2) {
                    float z0 = T_::val(acc[1], r), z1 = T_::val(acc[1], r + 1);
                    if constexpr (ZF) {
                        z0 *= zq;
                        z1 *= zq;
                    }
                    const float y0 = T_::val(acc[0], r), y1 = T_::val(acc[0], r + 1);
                    smax = fmaxf(smax, fmaxf(fmaf(y0, y0, z0 * z0), fmaf(y1, y1, z1 * z1)));
                }
                return smax - th * invc;
            }
            float gmax = -__builtin_inff();
#pragma unroll
            for (int r = 0; r < 16; r += 2)
                gmax = fmaxf(gmax, fmaxf(screen(acc, th, r), screen(acc, th, r + 1)));
            return gmax;
        };
        // MFMA chain of one 32-trait tile into registers
        auto mma_tile = [&](const frag (&Af)[KS], acc_t (&acc)[NC]) {
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = acc_t{};
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] = T_::mma(Af[s], B[s][c], acc[c]);
        };
        // epilogue of one tile (all modes)
        auto tile_epilogue = [&](const int64_t t, const acc_t (&acc)[NC], const float th) {
            const int64_t rb = t * kTile + 4 * (lane >> 5);
            if constexpr (MODE == SCREEN) {
                (void)rb;
                if (__any(screen_max(acc, th) > 0.0f)) screen_cands(t, acc, th);
            } else if constexpr (FORM == MISS3) {
                // FULL / SUMS: every pair exactly (MISS3 columns)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t row = rb + 8 * (r >> 2) + (r & 3);
                    const int64_t v = a.row_v[row];
                    bool want = v >= 0 && m < a.M;
                    if constexpr (QUEUE) {
                        bool qpush = want && lane_miss;
                        unsigned long long msk = __ballot(qpush);
                        if (msk) {
                            if (qn + 64 > kQueueCap) drain<MODE>(a, queue, qn, qbuf, lane);
                            const unsigned long long lt =
                                (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                            if (qpush) queue[qn + __popcll(msk & lt)] = make_int4((int)row, (int)m, 0, 0);
                            qn += __popcll(msk);
                        }
                        want = want && !lane_miss;
                    }
                    if (want) {
                        int64_t D0 = (int64_t)T_::val(acc[0], r);
                        int64_t D1 = (int64_t)T_::val(acc[1], r);
                        int64_t D2 = (int64_t)T_::val(acc[2], r);
                        const double H = exact_H(D0, D1, D2, inf.n0, inf.n1, inf.n2, a.K,
                                                 a.tiesum[v % a.T], snp_df(inf));
                        const int64_t k1 = a.K + 1;
                        emit_full<MODE>(a, v, m, H, snp_df(inf), D0 + inf.n0 * k1, D1 + inf.n1 * k1,
                                        D2 + inf.n2 * k1);
                    }
                }
                if (QUEUE && qn) drain<MODE>(a, queue, qn, qbuf, lane);
            }
        };
        auto tile_body = [&](const int64_t t, const frag (&Af)[KS], const float th) {
            acc_t acc[NC];
            mma_tile(Af, acc);
            tile_epilogue(t, acc, th);
        };
        // A fragments and the (wave-uniform) threshold of tile t
        auto load_tile = [&](const int64_t t, frag (&Af)[KS], float& th) {
#pragma unroll
            for (int s = 0; s < KS; ++s) Af[s] = gload(A + (t * KS + s) * kWave + lane);
            th = cload(a.theta + t);
        };
        if constexpr (RING) {
            // As PF == 2, but the A tiles come through a ring of 4 LDS slots
            // shared by the block's 4 waves (they walk the same trait range):
            // each wave copies its share of the k-steps of tile t + 2 straight
            // from global memory into the ring (LDS-DMA loads, no registers),
            // waits for its own copies of tile t, and after one block barrier
            // every wave reads tile t from LDS.  This reads each A tile once
            // per block instead of once per wave, and keeps two tiles in
            // flight without registers.  A slot is rewritten two barriers
            // after its last read.
            constexpr int LPW = (KS + kWavesPerBlock - 1) / kWavesPerBlock;  // copies per wave
            // The copies are issued from inline assembly: they have no
            // register result, and keeping them out of the compiler's view
            // stops it from waiting for every copy in flight before each
            // read of the ring; arrive() does the exact wait instead.
            auto issue = [&](const int64_t tt) {
                const int64_t tc = tt < t1 ? tt : t1 - 1;
#pragma unroll
                for (int j = 0; j < LPW; ++j) {
                    int ks = wave + j * kWavesPerBlock;
                    ks = ks < KS ? ks : KS - 1;     // the spare copy repeats the last k-step
                    const frag* src = A + (tc * KS + ks) * kWave + lane;
                    const uint32_t dst = (uint32_t)(uintptr_t)(
                        (__attribute__((address_space(3))) frag*)&s_ring[((tt & (NSLOT - 1)) * KS + ks) * kWave]);
                    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                                 :
                                 : "s"(__builtin_amdgcn_readfirstlane(dst)), "v"(src)
                                 : "memory");
                }
            };
            // this wave's copies of the oldest tile in flight have landed
            // (vmcnt counts in issue order; the two younger tiles may still
            // be in flight), then the block barrier publishes them
            auto arrive = [&]() {
                __builtin_amdgcn_s_waitcnt((2 * LPW) | (0x7 << 4) | (0xF << 8));
                block_barrier();
            };
            auto lread = [&](const int64_t tt, frag (&Af)[KS]) {
#pragma unroll
                for (int s = 0; s < KS; ++s) Af[s] = s_ring[((tt & (NSLOT - 1)) * KS + s) * kWave + lane];
            };
            auto thr = [&](const int64_t tt) { return cload(a.theta + (tt < t1 ? tt : t1 - 1)); };
            frag Af[KS];
            // every wave is done with the ring of the previous item (its last
            // reads fed MFMAs that have issued)
            __builtin_amdgcn_s_waitcnt(0);
            block_barrier();
            issue(t0);
            issue(t0 + 1);
            if constexpr (PF == 5) {
                // two tiles per step (two accumulator sets, one barrier per
                // step), four tiles in flight: the copies issued in a step go
                // into the slots read two steps before, which every wave has
                // finished reading once it has passed the previous barrier
                issue(t0 + 2);
                issue(t0 + 3);
                frag Ag[KS];
                for (int64_t t = t0; t < t1; t += 2) {
                    issue(t + 4);
                    issue(t + 5);
                    // tiles t and t+1 landed; t+2 .. t+5 may be in flight
                    __builtin_amdgcn_s_waitcnt((4 * LPW) | (0x7 << 4) | (0xF << 8));
                    block_barrier();
                    lread(t, Af);
                    lread(t + 1, Ag);
                    const float th0 = thr(t), th1 = thr(t + 1);
                    acc_t c0[NC], c1[NC];
                    mma_tile(Af, c0);
                    mma_tile(Ag, c1);
                    if (__any(screen_max(c0, th0) > 0.0f)) screen_cands(t, c0, th0);
                    if (t + 1 < t1 && __any(screen_max(c1, th1) > 0.0f))
                        screen_cands(t + 1, c1, th1);
                }
                __builtin_amdgcn_s_waitcnt(0);
            } else if constexpr (PF == 4) {
                // one accumulator set, tile after tile: the MFMA / screen overlap
                // comes from the other waves of the SIMD (three per SIMD)
                for (int64_t t = t0; t < t1; ++t) {
                    issue(t + 2);
                    arrive();
                    lread(t, Af);
                    // all k-steps of the tile are read before the first MFMA
                    // (one LDS latency per tile; left to itself the scheduler
                    // interleaves pairs of reads with the MFMAs)
                    __builtin_amdgcn_sched_barrier(0);
                    const float th = thr(t);
                    acc_t c[NC];
                    mma_tile(Af, c);
                    if (__any(screen_max(c, th) > 0.0f)) screen_cands(t, c, th);
                }
                __builtin_amdgcn_s_waitcnt(0);
            } else {
            acc_t c0[NC], c1[NC];
            issue(t0 + 2);
            arrive();
            lread(t0, Af);
            float th0 = thr(t0), th1 = 0.0f;
            mma_tile(Af, c0);
            for (int64_t t = t0; t < t1; t += 2) {
                // half 1: MFMAs of t+1 || screen of t
                issue(t + 3);
                arrive();
                lread(t + 1, Af);
                th1 = thr(t + 1);
                mma_tile(Af, c1);
                const float g0 = screen_max(c0, th0);
#pragma unroll
                for (int i = 0; i < NC * KS; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
                }
                if (__any(g0 > 0.0f)) screen_cands(t, c0, th0);
                // half 2: MFMAs of t+2 || screen of t+1
                issue(t + 4);
                arrive();
                lread(t + 2, Af);
                th0 = thr(t + 2);
                mma_tile(Af, c0);
                const float g1 = screen_max(c1, th1);
#pragma unroll
                for (int i = 0; i < NC * KS; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 1);
                }
                if (t + 1 < t1 && __any(g1 > 0.0f)) screen_cands(t + 1, c1, th1);
            }
            // the copies past the range end are still landing in the ring
            __builtin_amdgcn_s_waitcnt(0);
            }
        } else if constexpr (PF == 2 && MODE == SCREEN && FORM != MISS3) {
            // Software pipeline over pairs of tiles: the MFMA chain of the next
            // tile is issued in the same basic block as the fp32 screen of the
            // current one (two accumulator sets), and the scheduler is asked to
            // interleave one MFMA with a group of VALU operations, so that the
            // matrix core and the vector ALU work at the same time within the
            // wave.  The tile count of a range is even (the operand is padded
            // with a zero tile whose threshold is +inf); loads of the tile after
            // next are clamped into the range instead of branching.
            frag A0[KS], A1[KS];
            acc_t c0[NC], c1[NC];
            float h0, h1;
            const int64_t tl = t1 - 1;
            load_tile(t0, A0, h0);
            load_tile(t0 + 1 < t1 ? t0 + 1 : tl, A1, h1);
            mma_tile(A0, c0);
            for (int64_t t = t0; t < t1; t += 2) {
                // half 1: MFMAs of tile t+1 || screen of tile t
                const float th0 = h0;
                load_tile(t + 2 < t1 ? t + 2 : tl, A0, h0);
                mma_tile(A1, c1);
                const float g0 = screen_max(c0, th0);
#pragma unroll
                for (int i = 0; i < NC * KS; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
                }
                if (__any(g0 > 0.0f)) screen_cands(t, c0, th0);
                // half 2: MFMAs of tile t+2 || screen of tile t+1
                const float th1 = h1;
                load_tile(t + 3 < t1 ? t + 3 : tl, A1, h1);
                mma_tile(A0, c0);
                const float g1 = screen_max(c1, th1);
#pragma unroll
                for (int i = 0; i < NC * KS; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 1);
                }
                if (t + 1 < t1 && __any(g1 > 0.0f)) screen_cands(t + 1, c1, th1);
            }
        } else if constexpr (PF == 0) {
            for (int64_t t = t0; t < t1; ++t) {
                frag Ac[KS];
                float hc;
                load_tile(t, Ac, hc);
                tile_body(t, Ac, hc);
            }
        } else {
            // two register buffers, alternating: tile t+1 loads while t computes
            frag A0[KS], A1[KS];
            float h0 = 0.f, h1 = 0.f;
            if (t0 < t1) load_tile(t0, A0, h0);
            for (int64_t t = t0; t < t1; t += 2) {
                if (t + 1 < t1) load_tile(t + 1, A1, h1);
                tile_body(t, A0, h0);
                if (t + 1 < t1) {
                    if (t + 2 < t1) load_tile(t + 2, A0, h0);
                    tile_body(t + 1, A1, h1);
                }
            }
        }
    }
    if constexpr (QUEUE && MODE == SCREEN) {
        if (qn) drain<MODE>(a, queue, qn, qbuf, lane);
    }
    if constexpr (MODE == SCREEN) flush_stage(a, &s_args, stage, sn, lane);
}

// Complete-SNP screen (DIAG form) with two SNP tiles per wave: every A tile
// the block copies into its LDS ring feeds 2 SNP tiles x 2 columns x KS
// MFMAs per wave, so the ring's LDS reads, barrier and copies per MFMA are
// half those of the one-tile pipeline (PF 4), at two waves per SIMD (the B
// fragments of both tiles stay in registers).  The screen is the two-square
// form of the one-tile kernel (fp16: Z pre-scaled by q in B; int8: scaled in
// fp32 after the conversion).
template <int E, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void scan_kernel_ns2(ScanArgs a) {
    using T_ = ET<E>;
    using frag = typename T_::frag;
    using acc_t = typename T_::acc;
    constexpr int NC = 2, NS = 2, NSLOT = 4;
    constexpr int TPB = kWavesPerBlock * NS;          // SNP tiles per block
    constexpr bool ZS = E == F16;
    constexpr uint32_t kFlags = ZS ? kCandZs : 0u;
    __shared__ uint4 s_stage[kWavesPerBlock][kStageCap];
    __shared__ ScanArgs s_args;
    __shared__ frag s_ring[NSLOT * KS * kWave];
    if (threadIdx.x == 0) s_args = a;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint4* stage = s_stage[wave];
    int sn = 0;
    if (a.want_flag == 1 && a.tile_flags[a.n_snp_tiles] == 0) return;
    if (a.want_flag == 0 && a.tile_flags[a.n_snp_tiles + 1] == 0) return;
    int64_t n_rows = a.n_rows;
    if (a.d_nrows) {
        const int64_t d = *a.d_nrows;
        n_rows = d < n_rows ? d : n_rows;
    }
    const int64_t n_tiles = (n_rows + kTile - 1) / kTile;
    const int64_t n_ranges = (n_tiles + a.tiles_per_range - 1) / a.tiles_per_range;
    const int64_t n_blocks = (a.n_snp_tiles + TPB - 1) / TPB;
    const int64_t items = n_ranges * n_blocks;
    const frag* A = (const frag*)a.A;
    const float kslack = 1.0f + kScreenSlack;
    constexpr int LPW = (KS + kWavesPerBlock - 1) / kWavesPerBlock;   // copies per wave

    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int64_t rg = item / n_blocks;
        const int64_t sb = item % n_blocks;
        // the wave's SNP tiles (uniform); a lane's SNP is st * 32 + lane % 32
        const int64_t st0 = sb * TPB + wave * NS;
        bool act[NS];
        bool any = false;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int64_t st = st0 + j;
            act[j] = st < a.n_snp_tiles && (a.want_flag < 0 || a.tile_flags[st] == a.want_flag);
            any = any || act[j];
        }
        // block-uniform skip: the waves meet at the ring's barriers
        if (!__syncthreads_or(any)) continue;
        frag B[NS][KS][NC];
        float invc[NS], zq[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int64_t mj = (st0 + j) * kTile + (lane & 31);
            SnpInfo inf{};
            if (act[j]) inf = gload(a.info + mj);
            const float cz = ZS ? diag_zscale(inf) : 1.f;
            const int8_t* grow = a.G + mj * (int64_t)a.gstride + T_::per_lane * (lane >> 5);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                int8_t codes[T_::per_lane];
                if constexpr (T_::per_lane == 8) {
                    const uint2 w = act[j] ? gload((const uint2*)(grow + s * T_::kps))
                                           : make_uint2(~0u, ~0u);
                    __builtin_memcpy(codes, &w, 8);
                } else {
                    const uint4 w = act[j] ? gload((const uint4*)(grow + s * T_::kps))
                                           : make_uint4(~0u, ~0u, ~0u, ~0u);
                    __builtin_memcpy(codes, &w, 16);
                }
                B[j][s][0] = T_::make(codes, 0.f, inf.cy1, inf.cy2);
                B[j][s][1] = T_::make(codes, 0.f, 0.f, cz);
            }
            const float fac = 3.0f * (float)(a.K - 1) * kslack * a.inv_hc[snp_df(inf)];
            invc[j] = 1.0f / (inf.wy * fac);          // inf when the SNP is never screened in
            zq[j] = 0.0f;
            if (!ZS && inf.wy > 0.0f)
                zq[j] = __uint_as_float(__float_as_uint(sqrtf(inf.wz / inf.wy)) + 1u);
        }
        const int64_t t0 = rg * a.tiles_per_range;
        const int64_t t1 = (t0 + a.tiles_per_range < n_tiles) ? t0 + a.tiles_per_range : n_tiles;
        auto issue = [&](const int64_t tt) {
            const int64_t tc = tt < t1 ? tt : t1 - 1;
#pragma unroll
            for (int jj = 0; jj < LPW; ++jj) {
                int ks = wave + jj * kWavesPerBlock;
                ks = ks < KS ? ks : KS - 1;
                const frag* src = A + (tc * KS + ks) * kWave + lane;
                const uint32_t dst = (uint32_t)(uintptr_t)(
                    (__attribute__((address_space(3))) frag*)&s_ring[((tt & (NSLOT - 1)) * KS + ks) * kWave]);
                asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                             :
                             : "s"(__builtin_amdgcn_readfirstlane(dst)), "v"(src)
                             : "memory");
            }
        };
        // every wave is done with the ring of the previous item
        __builtin_amdgcn_s_waitcnt(0);
        block_barrier();
        issue(t0);
        issue(t0 + 1);
        for (int64_t t = t0; t < t1; ++t) {
            issue(t + 2);
            // this wave's copies of tile t have landed, then the barrier
            __builtin_amdgcn_s_waitcnt((2 * LPW) | (0x7 << 4) | (0xF << 8));
            block_barrier();
            frag Af[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) Af[s] = s_ring[((t & (NSLOT - 1)) * KS + s) * kWave + lane];
            const float th = cload(a.theta + t);
            acc_t acc[NS][NC];
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[j][c] = acc_t{};
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int j = 0; j < NS; ++j)
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[j][c] = T_::mma(Af[s], B[j][s][c], acc[j][c]);
            // largest Y^2 + Z^2 of each SNP tile (Z scaled), against theta * invc
            float g = -__builtin_inff();
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                float smax = 0.0f;
#pragma unroll
                for (int r = 0; r < 16; r += 2) {
                    float z0 = T_::val(acc[j][1], r), z1 = T_::val(acc[j][1], r + 1);
                    if constexpr (!ZS) {
                        z0 *= zq[j];
                        z1 *= zq[j];
                    }
                    const float y0 = T_::val(acc[j][0], r), y1 = T_::val(acc[j][0], r + 1);
                    smax = fmaxf(smax, fmaxf(fmaf(y0, y0, z0 * z0), fmaf(y1, y1, z1 * z1)));
                }
                g = fmaxf(g, smax - th * invc[j]);
            }
            if (__any(g > 0.0f)) {
                const int64_t rb = t * kTile + 4 * (lane >> 5);
#pragma unroll
                for (int j = 0; j < NS; ++j) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float y = T_::val(acc[j][0], r), zr = T_::val(acc[j][1], r);
                        const float z = ZS ? zr : zq[j] * zr;
                        const bool cand = act[j] && fmaf(y, y, z * z) - th * invc[j] > 0.0f;
                        stage_candidates(a, &s_args, stage, sn, lane, cand,
                                         rb + 8 * (r >> 2) + (r & 3),
                                         (st0 + j) * kTile + (lane & 31), y, zr, kFlags);
                    }
                }
            }
        }
        // the copies past the range end are still landing in the ring
        __builtin_amdgcn_s_waitcnt(0);
    }
    flush_stage(a, &s_args, stage, sn, lane);
}

}  // namespace kx

// ---------------------------------------------------------------------------
// Launch of one (element type, k-steps, form, mode) instance.
// ---------------------------------------------------------------------------

// `grid` is the number of work items (an upper bound); the persistent launch
// uses min(items, resident blocks) = min(grid, n_cu * occupancy).
namespace kx {
template <int E, int KS, int FORM, int MODE,
          int PF = (MODE == kx::SCREEN && FORM != kx::MISS3) ? 2 : 0, int WPE = 2>
inline hipError_t launch_one(const kx::ScanArgs& a, int grid, hipStream_t st) {
    size_t lds = FORM == kx::MISS3 ? (size_t)kx::kWavesPerBlock * kx::coop_lds_entries(a.K) * sizeof(int16_t) : 0;
    auto kern = kx::scan_kernel<E, KS, FORM, MODE, PF, WPE>;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, lds) != hipSuccess || occ < 1)
        occ = 1;
    int dev = 0, n_cu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t resident = (int64_t)n_cu * occ;
    int g = (int)(grid < resident ? grid : resident);
    hipLaunchKernelGGL(kern, dim3(g), dim3(256), lds, st, a);
    return hipGetLastError();
}

// Complete-SNP screen pass with the A-operand pipeline selected by a.ring:
// 0 register double buffer (2 waves per SIMD), 1 LDS ring with the two-tile
// software pipeline, 2 LDS ring one tile at a time (3 waves per SIMD),
// 3 LDS ring two tiles per step (2 waves per SIMD), 4 LDS ring one tile at a
// time with two SNP tiles per wave (2 waves per SIMD).
template <int E, int KS>
inline hipError_t launch_ns2(const kx::ScanArgs& a, int grid, hipStream_t st) {
    auto kern = kx::scan_kernel_ns2<E, KS>;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, 0) != hipSuccess || occ < 1)
        occ = 1;
    int dev = 0, n_cu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t resident = (int64_t)n_cu * occ;
    const int g = (int)(grid < resident ? grid : resident);
    hipLaunchKernelGGL(kern, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int E, int KS>
inline hipError_t launch_diag_screen(const kx::ScanArgs& a, int grid, hipStream_t st) {
    switch (a.ring) {
        case 4: return launch_ns2<E, KS>(a, grid, st);
        case 3: return launch_one<E, KS, kx::DIAG, kx::SCREEN, 5, 2>(a, grid, st);
        case 2: return launch_one<E, KS, kx::DIAG, kx::SCREEN, 4, 3>(a, grid, st);
        case 1: return launch_one<E, KS, kx::DIAG, kx::SCREEN, 3>(a, grid, st);
        default: return launch_one<E, KS, kx::DIAG, kx::SCREEN, 2>(a, grid, st);
    }
}
}  // namespace kx
