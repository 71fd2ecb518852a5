/*
 * krux_oracle.c -- plain, slow CPU oracle for the Kruskal-Wallis SNP x trait
 * scan of kruX (Qi, Foroughi Asl, Bjorkegren, Michoel, arXiv:1307.3519).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - per trait, ranks over the observed samples (Implementation, "Input
 *     data"); ties get the average rank, the tie term is the sum over tie
 *     groups of t^3 - t ("Handling tied data");
 *   - per SNP x trait pair, the Kruskal-Wallis statistic of eq. (2) divided
 *     by the tie factor 1 - sum(T)/(K^3 - K), with empty genotype groups
 *     dropped so the degrees of freedom fall ("Calculation of the
 *     Kruskal-Wallis test statistic by matrix multiplication");
 *   - the chi-square tail p-value of that statistic, and the statistic
 *     threshold that corresponds to a p-value threshold P_c ("P-value
 *     calculation and empirical FDR correction");
 *   - a sample whose genotype is missing is removed from that pair and the
 *     ranks are recomputed over the remaining samples ("Handling missing
 *     values", missing genotypes);
 *   - permuted data: the columns of the rank matrix are permuted, the same
 *     permutation for every trait ("P-value calculation and empirical FDR
 *     correction").
 *
 * It follows the plain definition of the test, pair by pair, not the
 * paper's matrix formulation: ranks by counting, group sums by looping over
 * samples, and H as an exact rational rounded once to the nearest double.
 *
 * Ranks are stored doubled (2 x midrank, always an integer):
 *   a_k = 2 #{j : x_j < x_k} + #{j : x_j == x_k} + 1.
 * With D_i = sum_{k in group i} a_k - N_i (K+1) (twice the centred rank sum
 * of group i) and E = K^3 - K - sum(T), eq. (2) divided by the tie factor is
 *   H = 3 (K-1) * sum_{N_i>0} D_i^2 / N_i / E,
 * evaluated here as the exact rational 3(K-1) P / (L E) with
 * L = prod_{N_i>0} N_i and P = sum_{N_i>0} D_i^2 (L / N_i).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Number of OpenMP threads a scan will use, and a way to change it (the
 * benchmark times the oracle on all cores and on one). */
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* ------------------------------------------------------------------------ */
/* Exact rational -> nearest double (round half to even).                    */
/* ------------------------------------------------------------------------ */
static int bitlen128(u128 v) {
    int n = 0;
    while (v) { v >>= 1; n++; }
    return n;
}

double oracle_rational_to_double(u128 num, u128 den) {
    if (num == 0 || den == 0) return 0.0;
    u128 q = num / den;
    u128 r = num % den;
    int exp2 = 0;           /* value = q * 2^exp2 (+ remainder) */
    int sticky = 0;
    int b = bitlen128(q);
    if (b >= 54) {
        int sh = b - 54;
        u128 mask = (((u128)1) << sh) - 1;
        sticky = ((q & mask) != 0) || (r != 0);
        q >>= sh;
        exp2 = sh;
    } else {
        /* produce further quotient bits from the remainder */
        while (bitlen128(q) < 54) {
            r <<= 1;
            q <<= 1;
            if (r >= den) { r -= den; q |= 1; }
            exp2--;
        }
        sticky = (r != 0);
    }
    /* q holds 54 significant bits: 53 kept + one rounding bit */
    uint64_t mant = (uint64_t)(q >> 1);
    int round_bit = (int)(q & 1);
    if (round_bit && (sticky || (mant & 1))) mant++;
    if (mant == (((uint64_t)1) << 53)) { mant >>= 1; exp2++; }
    return ldexp((double)mant, exp2 + 1);
}

/* test hook: numerator/denominator given as (hi, lo) 64-bit halves */
double oracle_rational_to_double_parts(uint64_t num_hi, uint64_t num_lo,
                                       uint64_t den_hi, uint64_t den_lo) {
    u128 num = (((u128)num_hi) << 64) | num_lo;
    u128 den = (((u128)den_hi) << 64) | den_lo;
    return oracle_rational_to_double(num, den);
}

/* ------------------------------------------------------------------------ */
/* chi-square upper tail for df = 1, 2 and the statistic threshold.          */
/* ------------------------------------------------------------------------ */
double oracle_pvalue(double H, int df) {
    if (df <= 0) return 1.0;
    if (df == 1) return erfc(sqrt(H / 2.0));
    if (df == 2) return exp(-H / 2.0);
    return NAN; /* more than three genotype classes is not covered */
}

static uint64_t dbits(double v) { uint64_t u; memcpy(&u, &v, 8); return u; }
static double bitsd(uint64_t u) { double v; memcpy(&v, &u, 8); return v; }

/* The threshold of the paper's P-value section: the largest double h >= 0
 * whose tail probability (as evaluated by this host's libm) is still >= P_c,
 * so that "H > h" selects exactly the statistics with p < P_c.  Found by
 * bisection over the ordered bit patterns of non-negative doubles. */
double oracle_threshold(double p_c, int df) {
    if (!(p_c > 0.0 && p_c <= 1.0) || df < 1 || df > 2) return NAN;
    uint64_t lo = dbits(0.0), hi = dbits(4096.0);
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (oracle_pvalue(bitsd(mid), df) >= p_c) lo = mid; else hi = mid;
    }
    return bitsd(lo);
}

/* ------------------------------------------------------------------------ */
/* Ranks of one trait row over the samples with keep[k] != 0.               */
/* NaN expression values are not observed and get rank 0.                   */
/* ------------------------------------------------------------------------ */
static void rank_row(const float* x, const uint8_t* keep, int K,
                     int32_t* a2, int64_t* tiesum, int32_t* kobs) {
    int64_t ts = 0;
    int32_t n = 0;
    for (int k = 0; k < K; k++) {
        if (!keep[k] || isnan(x[k])) { a2[k] = 0; continue; }
        int64_t less = 0, eq = 0;
        for (int j = 0; j < K; j++) {
            if (!keep[j] || isnan(x[j])) continue;
            if (x[j] < x[k]) less++;
            else if (x[j] == x[k]) eq++;
        }
        a2[k] = (int32_t)(2 * less + eq + 1);
        ts += eq * eq - 1;
        n++;
    }
    *tiesum = ts;
    *kobs = n;
}

/* Public: ranks of a T x K matrix (row stride ld).  Every sample kept. */
void oracle_rank(const float* expr, int64_t T, int32_t K, int64_t ld,
                 int32_t* ranks2, int64_t* tiesum, int32_t* nvalid) {
    #pragma omp parallel
    {
        uint8_t* keep = (uint8_t*)malloc((size_t)K);
        memset(keep, 1, (size_t)K);
        #pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < T; t++) {
            int32_t kobs;
            rank_row(expr + t * ld, keep, K, ranks2 + t * (int64_t)K,
                     tiesum + t, &kobs);
            if (nvalid) nvalid[t] = kobs;
        }
        free(keep);
    }
}

/* ------------------------------------------------------------------------ */
/* One SNP x trait pair.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double H, p;
    int32_t df, kobs;
    int32_t n[3];       /* group sizes N_0, N_1, N_2 over the kept samples */
    int64_t s2[3];      /* doubled rank sums of the three groups */
    int64_t tiesum;     /* tie term over the kept samples */
} oracle_pair;

/* H, df and p from group sizes, doubled rank sums and the tie term. */
static void pair_from_sums(oracle_pair* o) {
    int64_t Kp = o->kobs;
    int nonempty = 0;
    for (int i = 0; i < 3; i++) nonempty += (o->n[i] > 0);
    o->df = nonempty > 0 ? nonempty - 1 : 0;
    int64_t E = Kp * Kp * Kp - Kp - o->tiesum;
    if (o->df == 0 || Kp < 2 || E <= 0) { o->H = 0.0; o->p = 1.0; return; }
    u128 L = 1;
    for (int i = 0; i < 3; i++) if (o->n[i] > 0) L *= (u128)o->n[i];
    u128 P = 0;
    for (int i = 0; i < 3; i++) {
        if (o->n[i] == 0) continue;
        int64_t D = o->s2[i] - (int64_t)o->n[i] * (Kp + 1);
        u128 D2 = (u128)((__int128)D * (__int128)D);
        P += D2 * (L / (u128)o->n[i]);
    }
    u128 num = (u128)(3 * (Kp - 1)) * P;
    u128 den = L * (u128)E;
    o->H = oracle_rational_to_double(num, den);
    o->p = oracle_pvalue(o->H, o->df);
}

/* Pair statistic from a trait row x (K values) and a genotype row g (codes
 * 0,1,2 or -1 = missing).  a2_full / ts_full: ranks and tie term of x over all
 * samples (valid whenever g has no missing code); scratch: 2K bytes + K ints */
static void pair_stat(const float* x, const int8_t* g, int32_t K,
                      const int32_t* a2_full, int64_t ts_full, int32_t kobs_full,
                      uint8_t* keep, int32_t* a2_tmp, oracle_pair* o) {
    /* a genotype is a code 0..2; anything else (-1 by convention) is missing */
    int missing = 0;
    for (int k = 0; k < K; k++) missing |= (g[k] < 0 || g[k] > 2);
    const int32_t* a2 = a2_full;
    o->tiesum = ts_full;
    o->kobs = kobs_full;
    if (missing) {
        for (int k = 0; k < K; k++) keep[k] = (uint8_t)(g[k] >= 0 && g[k] <= 2);
        rank_row(x, keep, K, a2_tmp, &o->tiesum, &o->kobs);
        a2 = a2_tmp;
    }
    for (int i = 0; i < 3; i++) { o->n[i] = 0; o->s2[i] = 0; }
    for (int k = 0; k < K; k++) {
        int gi = g[k];
        if (gi < 0 || gi > 2 || a2[k] == 0) continue;
        o->n[gi] += 1;
        o->s2[gi] += a2[k];
    }
    pair_from_sums(o);
}

/* Public: one pair, for tests. out: H, p; df_out, n_out[3], s2_out[3]. */
void oracle_one_pair(const float* x, const int8_t* g, int32_t K,
                     double* H, double* p, int32_t* df, int32_t* n_out,
                     int64_t* s2_out, int64_t* tiesum_out, int32_t* kobs_out) {
    uint8_t* keep = (uint8_t*)malloc((size_t)K);
    int32_t* a2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
    int32_t* a2t = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
    int64_t ts; int32_t kobs;
    memset(keep, 1, (size_t)K);
    rank_row(x, keep, K, a2, &ts, &kobs);
    oracle_pair o;
    pair_stat(x, g, K, a2, ts, kobs, keep, a2t, &o);
    *H = o.H; *p = o.p; *df = o.df;
    for (int i = 0; i < 3; i++) { n_out[i] = o.n[i]; s2_out[i] = o.s2[i]; }
    *tiesum_out = o.tiesum; *kobs_out = o.kobs;
    free(keep); free(a2); free(a2t);
}

/* ------------------------------------------------------------------------ */
/* Scans over all pairs.                                                     */
/*   expr: T x K (row stride ld_e), geno: M x K (row stride ld_g).           */
/*   perm: optional K-vector; the rank matrix columns are permuted, i.e.     */
/*   trait row n is read as x'(k) = x(perm[k]) (same permutation for every   */
/*   trait).  Permuting the expression columns and re-ranking gives the same */
/*   ranks as permuting the rank columns.                                    */
/* Per trait callback-free outputs:                                          */
/*   H, p     : optional T x M full matrices                                 */
/*   sums     : optional 3 x T x M doubled group rank sums (int64)           */
/*   counts   : optional n_thr hit counts (H > H_c(df, level))               */
/*   min_p    : optional T per-trait minimum p over all SNPs                 */
/*   hits     : optional per-trait hit lists at thr index 0, returned via    */
/*              hit_trait/hit_snp/hit_H/hit_p arrays of capacity hit_cap;    */
/*              *n_hits gets the true count; order is (trait, snp).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t snp;
    double H, p;
} hit_rec;

int oracle_scan(const float* expr, int64_t T, int32_t K, int64_t ld_e,
                const int8_t* geno, int64_t M, int64_t ld_g,
                const int32_t* perm,
                const double* Hc /* n_thr x 2: threshold for df=1, df=2 */,
                int32_t n_thr,
                double* H_out, double* p_out, int64_t* sums_out,
                int64_t* counts, double* min_p,
                int32_t* hit_trait, int32_t* hit_snp, double* hit_H,
                double* hit_p, int64_t hit_cap, int64_t* n_hits) {
    hit_rec** lists = NULL;
    int64_t* nlist = NULL;
    if (n_hits) {
        lists = (hit_rec**)calloc((size_t)T, sizeof(hit_rec*));
        nlist = (int64_t*)calloc((size_t)T, sizeof(int64_t));
    }
    if (counts) {
        for (int i = 0; i < n_thr; i++) counts[i] = 0;
    }
    #pragma omp parallel
    {
        uint8_t* keep = (uint8_t*)malloc((size_t)K);
        int32_t* a2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
        int32_t* a2t = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
        float* xp = (float*)malloc(sizeof(float) * (size_t)K);
        int64_t* cnt = (int64_t*)calloc((size_t)(n_thr > 0 ? n_thr : 1), sizeof(int64_t));
        #pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < T; t++) {
            const float* x = expr + t * ld_e;
            if (perm) {
                for (int k = 0; k < K; k++) xp[k] = x[perm[k]];
                x = xp;
            }
            int64_t ts; int32_t kobs;
            memset(keep, 1, (size_t)K);
            rank_row(x, keep, K, a2, &ts, &kobs);
            double best = 1.0;
            int64_t cap = 0, nh = 0;
            hit_rec* lst = NULL;
            for (int64_t m = 0; m < M; m++) {
                oracle_pair o;
                pair_stat(x, geno + m * ld_g, K, a2, ts, kobs, keep, a2t, &o);
                if (H_out) H_out[t * M + m] = o.H;
                if (p_out) p_out[t * M + m] = o.p;
                if (sums_out)
                    for (int i = 0; i < 3; i++)
                        sums_out[((int64_t)i * T + t) * M + m] = o.s2[i];
                if (o.p < best) best = o.p;
                if (o.df >= 1 && o.df <= 2) {
                    for (int l = 0; l < n_thr; l++) {
                        if (o.H > Hc[2 * l + (o.df - 1)]) {
                            cnt[l]++;
                            if (l == 0 && n_hits) {
                                if (nh == cap) {
                                    cap = cap ? 2 * cap : 16;
                                    lst = (hit_rec*)realloc(lst, (size_t)cap * sizeof(hit_rec));
                                }
                                lst[nh].snp = (int32_t)m;
                                lst[nh].H = o.H;
                                lst[nh].p = o.p;
                                nh++;
                            }
                        }
                    }
                }
            }
            if (min_p) min_p[t] = best;
            if (n_hits) { lists[t] = lst; nlist[t] = nh; } else free(lst);
        }
        if (counts) {
            #pragma omp critical
            for (int l = 0; l < n_thr; l++) counts[l] += cnt[l];
        }
        free(keep); free(a2); free(a2t); free(xp); free(cnt);
    }
    if (n_hits) {
        int64_t pos = 0;
        for (int64_t t = 0; t < T; t++) {
            for (int64_t j = 0; j < nlist[t]; j++) {
                if (pos < hit_cap) {
                    hit_trait[pos] = (int32_t)t;
                    hit_snp[pos] = lists[t][j].snp;
                    hit_H[pos] = lists[t][j].H;
                    hit_p[pos] = lists[t][j].p;
                }
                pos++;
            }
            free(lists[t]);
        }
        *n_hits = pos;
        free(lists); free(nlist);
    }
    return 0;
}
