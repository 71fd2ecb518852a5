// multi_common.h -- device helpers of the multi-allelic scan (genotype
// classes 0..l, l + 1 <= 8): the chi-square tail for any df, the statistic as
// an exact rational rounded once, and the exact evaluation of a screened pair
// from its class sums.
#pragma once
#include "kx_args.h"

namespace kx {

typedef unsigned __int128 u128;

__device__ inline int bitlen128(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64);
    return hi ? 64 + bitlen64(hi) : bitlen64((uint64_t)v);
}

// Nearest double (ties to even) to num / den for den < 2^127 and a quotient
// below 2^64 (here H <= K - 1).  Operands below 2^53 are exact doubles and
// one IEEE division rounds once; otherwise long division, bit by bit.
__device__ inline double rat128_to_double(u128 num, u128 den) {
    if (num == 0 || den == 0) return 0.0;
    if ((num >> 53) == 0 && (den >> 53) == 0)
        return (double)(uint64_t)num / (double)(uint64_t)den;
    const int nb = bitlen128(num);
    uint64_t q = 0;
    u128 r = 0;
    for (int i = nb - 1; i >= 0; --i) {
        r = (r << 1) | ((num >> i) & 1u);
        q <<= 1;
        if (r >= den) {
            r -= den;
            q |= 1ull;
        }
    }
    int e = 0, sticky;
    const int qb = bitlen64(q);
    if (qb >= 54) {
        const int sh = qb - 54;
        sticky = ((q & ((1ull << sh) - 1ull)) != 0) || (r != 0);
        q >>= sh;
        e = sh;
    } else {
        while (bitlen64(q) < 54) {
            r <<= 1;
            q <<= 1;
            if (r >= den) {
                r -= den;
                q |= 1ull;
            }
            --e;
        }
        sticky = (r != 0);
    }
    uint64_t mant = q >> 1;
    const int rb = (int)(q & 1ull);
    if (rb && (sticky || (mant & 1ull))) ++mant;
    if (mant == (1ull << 53)) {
        mant >>= 1;
        ++e;
    }
    return ldexp((double)mant, e + 1);
}

// H over G classes from twice-centred class sums D_c (centred at K'+1),
// class sizes n_c, K' and the tie term: eq. (2) divided by the tie factor,
//   H = 3 (K'-1) sum_{n_c>0} D_c^2 / n_c / (K'^3 - K' - sumT),
// as the rational 3 (K'-1) A / (L E) with L = prod_{n_c>0} n_c and
// A = sum_c D_c^2 L / n_c, rounded once.  With K' <= 2048 and at most eight
// classes, L <= 2^64, A < 2^96, the numerator < 2^108 and L E < 2^97.
template <int G>
__device__ inline double exact_H_classes(const int64_t (&D)[G], const int (&n)[G], int64_t kp,
                                         int64_t tiesum, int df) {
    const int64_t E = cube_minus(kp) - tiesum;
    if (df <= 0 || kp < 2 || E <= 0) return 0.0;
    u128 L = 1;
#pragma unroll
    for (int c = 0; c < G; ++c)
        if (n[c]) L *= (u128)(uint32_t)n[c];
    u128 A = 0;
#pragma unroll
    for (int c = 0; c < G; ++c) {
        if (!n[c]) continue;
        u128 cof = 1;                                // L / n_c: the other sizes
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (j != c && n[j]) cof *= (u128)(uint32_t)n[j];
        A += (u128)(uint64_t)(D[c] * D[c]) * cof;
    }
    return rat128_to_double((u128)(uint64_t)(3 * (kp - 1)) * A, L * (u128)(uint64_t)E);
}

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

// Records one exactly evaluated pair: the hit list (H > hc[df]) and the
// trait's minimum p.
__device__ inline void multi_record(const MultiArgs& a, int64_t trait, int64_t m, double H, int df) {
    if (df <= 0) return;
    const bool hit = a.record_hits && a.hits && H > a.hc[df];
    if (!hit && !a.minp_bits) return;
    const double p = chi2_upper(H, df);
    if (a.minp_bits) atomicMin(&a.minp_bits[trait], (unsigned long long)__double_as_longlong(p));
    if (hit) {
        const unsigned long long idx = atomicAdd(a.n_hits, 1ull);
        if ((int64_t)idx < a.hit_cap) {
            HitRec h;
            h.trait = (int32_t)trait;
            h.snp = (int32_t)(a.snp_base + m);
            h.H = H;
            h.p = p;
            a.hits[idx] = h;
        }
    }
}

// Exact evaluation of one screened complete pair from its class sums (the
// MFMA screen's integers) and the SNP's class sizes: no pass over the samples.
template <int G>
__device__ inline void multi_eval_sums(const MultiArgs& a, int64_t trait, const MultiCand& e) {
    const int64_t m = (int64_t)e.snp;
    const MultiInfo inf = a.info[m];
    int64_t D[G];
    int n[G];
    int64_t d0 = 0;
#pragma unroll
    for (int c = 1; c < G; ++c) {
        D[c] = (int64_t)e.d[c - 1];
        d0 -= D[c];
        n[c] = inf.n[c];
    }
    D[0] = d0;
    n[0] = inf.n[0];
    const double H = exact_H_classes<G>(D, n, a.K, a.tiesum[trait], inf.df);
    multi_record(a, trait, m, H, inf.df);
}

}  // namespace kx
