/*
 * krux.h -- C ABI of the MI355X (gfx950) Kruskal-Wallis SNP x trait scan.
 *
 * The method is kruX (Qi, Foroughi Asl, Bjorkegren, Michoel,
 * arXiv:1307.3519): per-trait ranks with a tie term, per-genotype-group rank
 * sums as products of the rank matrix with genotype indicator matrices
 * (eq. (1)), the Kruskal-Wallis statistic of eq. (2) divided by the tie
 * factor 1 - sum(T)/(K^3-K), and a chi-square p-value per SNP x trait pair.
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers unless marked (host).  Matrices are
 *     row-major with the sample index contiguous.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it and the call returns after enqueue, except where
 *     a function says it synchronises.
 *   - Argument errors are found before anything is launched; then nothing is
 *     launched, the call returns a status other than KRUX_OK and
 *     krux_last_error() describes the problem.
 *   - The caller owns every buffer it passes; the library never frees caller
 *     memory.  The context owns its scratch memory (allocated at first use,
 *     grown as needed, freed by krux_destroy).  Calls on one context must not
 *     overlap in time (one context per host thread).
 *   - Graph capture: krux_rank, krux_test (fp16 and int8), krux_permute,
 *     krux_permute_hits, krux_fdr_curve, krux_test_multi and
 *     krux_test_batched enqueue kernels only (no host synchronisation, no
 *     memset nodes), so the caller may capture a call into a HIP graph and
 *     replay it.  A call made while its stream is being captured must not
 *     need more scratch than an earlier call on the same context already
 *     allocated: otherwise it returns KRUX_ERR_UNSUPPORTED (run the same call
 *     once without capture first).  Once a call has been captured, a later
 *     call that needs a larger scratch buffer gets a new one and the old one
 *     is kept until krux_destroy, so captured graphs stay valid.  Replays of
 *     a graph and other calls on the same context must not overlap in time.
 *     krux_test_grouped, krux_autotune and the fp64 comparator synchronise
 *     and are refused under capture.
 *   - Doubled midranks: a = 2 x (average rank), i.e.
 *     a_k = 2 #{j: x_j < x_k} + #{j: x_j == x_k} + 1, an integer in [2, 2K];
 *     0 marks a missing (NaN) expression value.
 *   - Genotype codes: 0, 1, 2 (copies of the minor allele).  Any other code
 *     (-1 by convention) is missing: that sample is removed from that pair
 *     and the ranks are recomputed over the remaining samples (the paper's
 *     missing-genotype rule).
 *   - The statistic H of a pair is the exact rational value of eq. (2)
 *     divided by the tie factor, rounded once to the nearest double; groups
 *     with no sample are dropped (df = #non-empty groups - 1, the paper's
 *     NaN-to-zero rule).  p = exp(-H/2) for df = 2, erfc(sqrt(H/2)) for
 *     df = 1, and H = 0, p = 1 for df = 0 or an all-tied trait.
 *   - A pair is a hit at threshold P_c iff df >= 1 and H > H_c(df), with
 *     H_c from krux_threshold (the paper's statistic-threshold rule).
 */
#ifndef KRUX_H
#define KRUX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KRUX_OK = 0,
    KRUX_ERR_ARG = 1,         /* null pointer, negative size, bad enum, ... */
    KRUX_ERR_SHAPE = 2,       /* inconsistent sizes or strides */
    KRUX_ERR_UNSUPPORTED = 3, /* valid but outside what this build handles */
    KRUX_ERR_NOMEM = 4,       /* scratch allocation failed */
    KRUX_ERR_HIP = 5          /* a HIP runtime call failed */
} krux_status;

typedef struct krux_ctx krux_ctx;

/* One significant pair.  `snp` is global: snp_base + local SNP index. */
typedef struct {
    int32_t trait;
    int32_t snp;
    double H;
    double p;
} krux_hit;

enum {
    KRUX_MODE_HITS = 0, /* compacted hit list (+ optional per-trait min p) */
    KRUX_MODE_FULL = 1, /* H and p for every pair (T x M doubles each) */
    KRUX_MODE_SUMS = 2  /* doubled group rank sums for every pair */
};

enum {
    KRUX_PREC_FP16 = 0, /* fp16 MFMA, fp32 accumulation: exact rank sums, K <= 2049 */
    KRUX_PREC_INT8 = 1, /* int8 MFMA, i32 accumulation (byte split above K = 127) */
    KRUX_PREC_FP64 = 2  /* comparator: the paper's matrix formulation with fp64
                           GEMMs of the rank and indicator matrices (one per
                           genotype class) and an element-wise pass */
};

/* Largest supported sample count of each path. */
#define KRUX_MAX_K_RANK 8192
#define KRUX_MAX_K_FP16 2049

/* Create a context on HIP device `device`.  Returns KRUX_OK and *out, or an
 * error (then *out is NULL).  Tuned launch configurations are loaded into a
 * context afterwards with krux_load_tuning (or found by krux_autotune). */
krux_status krux_create(krux_ctx** out, int device);

/* Free a context and all its scratch memory.  Synchronises its device. */
void krux_destroy(krux_ctx* ctx);

/* Message for the last failing call on `ctx` (or on a NULL ctx). Never NULL. */
const char* krux_last_error(const krux_ctx* ctx);

/* Statistic threshold for a p-value threshold (P-value calculation section):
 * *H_c (host) = the largest double h >= 0 whose chi-square tail at df,
 * evaluated on the host, is still >= p_c.  So H > H_c exactly when the
 * host-evaluated p-value of H is below p_c.  p_c in (0, 1]; df in {1, 2}. */
krux_status krux_threshold(double p_c, int32_t df, double* H_c);

/* Per-row ranking (Implementation, input data; handling tied data).
 *   expr    T x K float32, row stride ld_expr >= K (elements).
 *   ranks2  T x K int16 doubled midranks (row stride K); 0 for NaN entries,
 *           which are excluded from the ranking.
 *   tiesum  T int64: sum over tie groups of t^3 - t (over non-NaN values).
 *   nvalid  T int32 or NULL: number of non-NaN values per row.
 * -0.0 and +0.0 are one value.  1 <= K <= KRUX_MAX_K_RANK. */
krux_status krux_rank(krux_ctx* ctx, const float* expr, int64_t T, int32_t K,
                      int64_t ld_expr, int16_t* ranks2, int64_t* tiesum,
                      int32_t* nvalid, void* stream);

/* Kruskal-Wallis test of every trait against every SNP of a slice
 * (eq. (1), eq. (2), tie factor, P-value calculation; data slicing).
 *   ranks2, tiesum  from krux_rank.  A 0 rank marks a missing (NaN)
 *                   expression value: such a sample is left out of every pair
 *                   of its trait, as a missing genotype is, and the ranks,
 *                   tie term, group sizes and df of the pair are taken over
 *                   the samples observed on both sides (traits with a 0 rank
 *                   are evaluated exactly per pair, outside the MFMA scan).
 *   geno            M x K int8, row stride ld_geno >= K (bytes).
 *   snp_base        added to the SNP index of every hit (slice start).
 *   p_c             p-value threshold, (0, 1] (HITS mode).
 *   mode            KRUX_MODE_*; precision KRUX_PREC_*.
 * HITS: hits[hit_capacity] receives the pairs with H > H_c(df) sorted by
 *       (trait, snp); *n_hits (device int64) the true count, which may exceed
 *       hit_capacity (then the kept subset is unspecified: call again with a
 *       larger buffer).  min_p (device, T doubles, may be NULL) receives the
 *       minimum p over the slice's SNPs per trait.
 * FULL: H and p (device, T x M doubles each, row stride M) for every pair.
 * SUMS: sums (device, 3 x T x M int32): doubled rank sums of genotype groups
 *       0, 1, 2 (sum of ranks2 over the group's non-missing samples, with the
 *       ranks recomputed when the SNP has missing genotypes).
 * Unused outputs may be NULL. */
krux_status krux_test(krux_ctx* ctx, const int16_t* ranks2, const int64_t* tiesum,
                      int64_t T, int32_t K, const int8_t* geno, int64_t M,
                      int64_t ld_geno, int64_t snp_base, double p_c,
                      int32_t mode, int32_t precision,
                      krux_hit* hits, int64_t hit_capacity, int64_t* n_hits,
                      double* min_p, double* H, double* p, int32_t* sums,
                      void* stream);

/* Bytes of the static device scratch of krux_test_noalloc (one array per
 * GPU the library runs on, held until the process ends). */
#define KRUX_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* krux_test without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture (no earlier eager call is needed),
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * modes, results and output ownership as krux_test for the fp16 and int8
 * precisions (KRUX_PREC_FP64 is refused: its GEMM library allocates).  Every
 * working buffer is carved from a static device array of
 * KRUX_NOALLOC_SCRATCH_BYTES per GPU instead of the context's scratch; no
 * hipMalloc, hipFree or allocating library routine is called.  A call whose
 * working set (about 224 B per SNP at K <= 128, more for the tiled K > 128
 * path; the A operand, twice with per-trait minimum p; 48 B per hit of
 * hit_capacity) exceeds the array returns KRUX_ERR_UNSUPPORTED before
 * anything is launched.  The screened-pair buffers are capped at a few MB
 * (pairs beyond them are evaluated inside the scan kernels: slower, same
 * results).  All calls on one GPU share its array, which keeps the last
 * call's contents: calls that overlap in time on one GPU, from any contexts
 * or streams, race and give wrong results. */
krux_status krux_test_noalloc(krux_ctx* ctx, const int16_t* ranks2, const int64_t* tiesum,
                              int64_t T, int32_t K, const int8_t* geno, int64_t M,
                              int64_t ld_geno, int64_t snp_base, double p_c,
                              int32_t mode, int32_t precision,
                              krux_hit* hits, int64_t hit_capacity, int64_t* n_hits,
                              double* min_p, double* H, double* p, int32_t* sums,
                              void* stream);

/* HITS-mode scan with the SNPs grouped by their pattern of missing genotypes
 * (Handling missing values: one sub-problem per unique pattern, with the
 * pattern's samples removed from the genotype and expression matrices).
 * Every pattern shared by at least min_group SNPs (>= 1) becomes a complete
 * sub-problem over its remaining samples; the other SNPs are scanned as by
 * krux_test.  Same arguments, outputs and results as krux_test in HITS mode
 * (hits sorted by (trait, snp), true count in *n_hits, min_p per trait);
 * faster when many SNPs share their missing samples (a failed sample).
 * Synchronises `stream` a few times (the host reads the patterns' counts
 * and masks), so it cannot be captured into a graph. */
krux_status krux_test_grouped(krux_ctx* ctx, const int16_t* ranks2, const int64_t* tiesum,
                              int64_t T, int32_t K, const int8_t* geno, int64_t M,
                              int64_t ld_geno, int64_t snp_base, double p_c, int32_t precision,
                              int64_t min_group, krux_hit* hits, int64_t hit_capacity,
                              int64_t* n_hits, double* min_p, void* stream);

/* Multi-allelic markers (Input data: genotype values 0..l; Calculation of
 * the Kruskal-Wallis test statistic, eq. (2), over l + 1 groups; P-value
 * calculation for df up to l).  Genotype codes 0..n_classes-1 are classes,
 * any other code is missing (the sample is removed from the pair and the
 * ranks recomputed, as in krux_test); a 0 rank is a missing expression value.
 * df = non-empty classes - 1, p = the chi-square tail at df.  H is the exact
 * rational value rounded once to the nearest double, as in krux_test.  In
 * HITS mode with K <= 128 and n_classes <= 5, the pairs whose samples all
 * have a class and an expression value go through the MFMA rank-sum GEMM
 * (n_classes - 1 indicator columns per SNP) with an fp32 screen, and the
 * pairs that pass are evaluated exactly from the GEMM's class sums (exact
 * integers); every other pair (and FULL mode) is evaluated exactly by one GPU
 * lane over its samples.
 *   n_classes  2..8 (l + 1); K <= 2048.
 *   mode       KRUX_MODE_HITS: hits (sorted by (trait, snp)) with
 *              H > H_c(df), the largest double whose chi-square tail at df is
 *              >= p_c; *n_hits the true count; min_p (device, T doubles, may
 *              be NULL) the minimum p over the SNPs per trait.
 *              KRUX_MODE_FULL: H and p (device, T x M doubles).
 * Other arguments as krux_test (snp_base + M must fit int32); unused outputs
 * may be NULL. */
krux_status krux_test_multi(krux_ctx* ctx, const int16_t* ranks2, const int64_t* tiesum,
                            int64_t T, int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno,
                            int32_t n_classes, int64_t snp_base, double p_c, int32_t mode,
                            krux_hit* hits, int64_t hit_capacity, int64_t* n_hits,
                            double* min_p, double* H, double* p, void* stream);

/* Permuted-data repeats for the empirical FDR (P-value calculation and
 * empirical FDR correction): for each permutation pi (perms, P x K int32,
 * each a permutation of 0..K-1) the rank matrix columns are permuted, the
 * same pi for every trait: trait row n is read as a'(k) = a(n, pi(k)).
 *   p_cs    (host) n_thr p-value thresholds, each in (0, 1].
 *   counts  P x n_thr int64: number of hits at each threshold.
 *   min_p   P x T doubles or NULL: per permutation and trait, min p over SNPs.
 * Every permutation of the batch is scanned by the same kernel launches (rows
 * perm * T + trait of one operand).  The call enqueues kernels only, so the
 * caller may capture it into a graph and replay it (see the conventions). */
krux_status krux_permute(krux_ctx* ctx, const int16_t* ranks2, const int64_t* tiesum,
                         int64_t T, int32_t K, const int8_t* geno, int64_t M,
                         int64_t ld_geno, const int32_t* perms, int32_t P,
                         const double* p_cs, int32_t n_thr, int64_t* counts,
                         double* min_p, void* stream);

/* The permuted-data hits themselves (P-value calculation and empirical FDR
 * correction: the P-value calculation repeated with the same P_c on data
 * with permuted rank columns), for the full FDR curve.  Same inputs as
 * krux_permute; p_c in (0, 1].
 *   hits[hit_capacity]  receives every permuted pair with H > H_c(df) at p_c,
 *                       sorted by (row, snp), where the trait field holds the
 *                       row perm * T + trait (perm indexes perms).
 *   n_hits              device int64: the true count (may exceed
 *                       hit_capacity; then the kept subset is unspecified). */
krux_status krux_permute_hits(krux_ctx* ctx, const int16_t* ranks2, const int64_t* tiesum,
                              int64_t T, int32_t K, const int8_t* geno, int64_t M,
                              int64_t ld_geno, const int32_t* perms, int32_t P, double p_c,
                              krux_hit* hits, int64_t hit_capacity, int64_t* n_hits,
                              void* stream);

/* Empirical FDR at the p-value of every real hit (P-value calculation and
 * empirical FDR correction: the mean over the P permutations of the number of
 * permuted associations with p' <= P, over the number of real associations
 * with p' <= P):
 *   fdr[i] = #{permuted hits j: p_j <= p_i} / (P * #{real hits j: p_j <= p_i})
 * computed in double from the two integer counts (one rounding).
 *   real, n_real   hit list of krux_test (HITS mode) with its device count;
 *                  min(*n_real, real_capacity) entries are used.
 *   perm, n_perm   hit list of krux_permute_hits over P permutations at the
 *                  same p_c, likewise.
 *   fdr            device, real_capacity doubles; entry i is written for
 *                  every used real hit i (same order as real).
 * All pointers are device pointers; n_real and n_perm are never NULL. */
krux_status krux_fdr_curve(krux_ctx* ctx, const krux_hit* real, const int64_t* n_real,
                           int64_t real_capacity, const krux_hit* perm, const int64_t* n_perm,
                           int64_t perm_capacity, int32_t P, double* fdr, void* stream);

/* One cohort of a batched scan: its own samples (K), traits and genotype
 * matrix over a shared SNP panel of M SNPs.  Pointers are device pointers. */
typedef struct {
    const int16_t* ranks2;  /* T x K */
    const int64_t* tiesum;  /* T */
    int64_t T;
    int32_t K;
    const int8_t* geno;     /* M x K, row stride ld_geno */
    int64_t ld_geno;
    krux_hit* hits;         /* hit_capacity entries, sorted (trait, snp) */
    int64_t hit_capacity;
    int64_t* n_hits;        /* device int64: true hit count */
    double* min_p;          /* T or NULL */
} krux_cohort;

/* HITS-mode scan of several cohorts of uneven sample counts against one SNP
 * panel (cohorts: host array of n_cohorts descriptors). */
krux_status krux_test_batched(krux_ctx* ctx, const krux_cohort* cohorts,
                              int32_t n_cohorts, int64_t M, double p_c,
                              int32_t precision, void* stream);

/* Limits on the two screened-pair buffers of the context (entries; 0 = the
 * built-in sizes, which grow with the expected number of screened pairs):
 * `candidates` bounds the buffer of pairs of complete SNPs that pass the fp32
 * screen (16 B each, 32 B in krux_test_multi; built in: at least 2^22),
 * `missing_pairs` the buffer of
 * pairs of SNPs with missing genotypes that pass the missing-genotype bound
 * (16 B each; built in: at least 2^16).  Pairs beyond a full buffer are
 * evaluated inside the scan kernels instead (slower, identical results), so
 * a limit bounds scratch memory, and a tiny limit exercises those paths.
 * Applies to later krux_test / krux_permute / krux_permute_hits /
 * krux_test_grouped / krux_test_batched / krux_test_multi calls on this
 * context. */
krux_status krux_set_pair_buffer_limits(krux_ctx* ctx, int64_t candidates,
                                        int64_t missing_pairs);

/* Instrumentation of the fused scan kernels (the rank-sum GEMM with its
 * epilogue): after krux_timer_start, each main pass of krux_test /
 * krux_permute (one per cohort for krux_test_batched) brackets its two scan
 * launches with HIP events on the launch stream: the complete-SNP kernel and
 * the missing-genotype kernel (which returns at once when no SNP has a
 * missing genotype); a krux_test_multi call on the MFMA path brackets its
 * screen kernel.  krux_timer_read synchronises those events, returns the
 * summed kernel time (host, ms) and the number of timed launches (two per
 * main pass), and stops the timer.  Meant for benchmarks. */
krux_status krux_timer_start(krux_ctx* ctx);
krux_status krux_timer_read(krux_ctx* ctx, double* total_ms, int64_t* launches);

/* Autotuner of the launch configuration (Data slicing: the work is tiled
 * over traits and SNP blocks; how large a trait range each work item covers,
 * the pipeline of the K <= 128 kernel, and the tile shape and item order of
 * the K > 128 kernel are machine- and shape-dependent).  Times krux_test (hit mode, P_c = 1e-5, no minimum p) on
 * the caller's inputs -- device arrays as for krux_test; a representative
 * slice of a few 1e9 pairs is enough -- for every candidate configuration of
 * the kernel that serves (K, precision), and keeps the fastest in the context:
 * later krux_test / krux_permute / krux_test_batched calls with that K and
 * precision use it.  precision: KRUX_PREC_FP16 or KRUX_PREC_INT8 (the fp64
 * comparator has nothing to tune: KRUX_ERR_UNSUPPORTED).  cache_path (host,
 * nullable): the choice is appended to this text file as one JSON object per
 * line keyed by architecture, K, precision and mode.  best_ms (host,
 * nullable): time of the chosen configuration per call.  Synchronises the
 * stream.  Results of the scan do not depend on the configuration. */
krux_status krux_autotune(krux_ctx* ctx, const int16_t* ranks2, const int64_t* tiesum,
                          int64_t T, int32_t K, const int8_t* geno, int64_t M,
                          int64_t ld_geno, int32_t precision, const char* cache_path,
                          double* best_ms, void* stream);

/* Loads the entries of a cache file written by krux_autotune that match this
 * device's architecture (later lines win; other lines are ignored). */
krux_status krux_load_tuning(krux_ctx* ctx, const char* cache_path);

/* The configuration in use for (K, precision).  K <= 128 kernel: ring
 * (0 register double buffer, 1 LDS ring with the two-tile pipeline, 2 LDS
 * ring one tile at a time, 3 LDS ring two tiles per step, 4 LDS ring with two
 * SNP tiles per wave) and range_kb
 * (trait-range operand budget).
 * K > 128 kernel: grouped (XCD-grouped item order) and shape (0 wide tiles,
 * one wave per SIMD; 1 two waves per SIMD; 2 as 1 with the complete-SNP
 * screen reading the packed genotype codes, PLAIN form; 3 as 2 with
 * eight-wave blocks, also for the missing-genotype screen, which runs as
 * under 1 in shape 2).  -1 / 0 mean the built-in rule.
 * Host outputs, each nullable. */
krux_status krux_tuning_of(krux_ctx* ctx, int32_t K, int32_t precision, int32_t* ring,
                           int32_t* range_kb, int32_t* grouped, int32_t* shape);

#ifdef __cplusplus
}
#endif
#endif /* KRUX_H */
