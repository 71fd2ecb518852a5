// kx_args.h -- argument blocks of the operand-preparation and scan kernels,
// shared by the kernels and by the host code that fills them.
#pragma once
#include "kx_common.h"

namespace kx {

struct PrepArgs {
    const int16_t* ranks2;   // T x K
    const int64_t* tiesum;   // T
    const int32_t* perms;    // P x K or null
    const int32_t* rows;     // list of virtual rows or null (identity)
    const int32_t* d_nrows;  // device count of rows (with list) or null
    int64_t n_rows;          // host bound on the number of operand rows
    int64_t n_alloc_rows;    // rows written (>= n_rows; the rest are zero padding)
    int64_t T;
    int K;
    int ks;                  // k-steps of the operand
    void* A;                 // fp16: half8 [tiles][ks][64]; int8: 16 B [tiles][ks][64]
    void* A_hi;              // int8 byte split: high plane, else null
    float* theta;            // [tiles] min over the tile's rows of K^3 - K - sumT
    int32_t* row_v;          // [tiles * 32]
    unsigned long long* zero;  // counters cleared by the kernel (the next scan's), or null
    int n_zero;
    const uint8_t* nan_flag;  // [T] 1: the trait has missing expression values (its rows
                              // become padding here; scan_nan_traits evaluates them), or null
};

enum { DIAG = 0, PLAIN = 1, MISS3 = 2 };
enum { SCREEN = 0, FULL = 1, SUMS = 2 };
enum { F16 = 0, I8 = 1 };

constexpr int kQueueCap = 128;     // per-wave queue of pairs needing a re-rank
constexpr int kLaneMiss = 32;      // missing-sample positions listed per SNP (int16 each)

struct ScanArgs {
    const void* A;            // operand tiles in fragment order
    const float* theta;       // [tiles] min over the tile's rows of K^3 - K - sumT (float)
    const int32_t* row_v;     // [tiles*32] virtual row (perm*T + trait), -1 padding
    const int32_t* d_nrows;   // device row count (fix-up passes) or null
    int64_t n_rows;           // host bound on operand rows
    int64_t T;                // traits
    const int64_t* tiesum;    // [T]
    const int16_t* ranks2;    // [T][K] doubled midranks (re-rank path)
    const int32_t* perms;     // [P][K] column permutations or null
    const int8_t* G;          // packed genotypes [m_pad][gstride]
    int gstride;
    const SnpInfo* info;      // [m_pad]
    const int32_t* tile_flags;// [n_snp_tiles] 1 = has a missing genotype, then "some tile has
                              // one" and "some tile has none"
    int64_t M;
    int64_t n_snp_tiles;
    int K;
    int tiles_per_range;
    int ring;                 // complete-SNP screen: 0 register double buffer, 1 block LDS
                              // ring (pipelined), 2 LDS ring, one tile at a time, 3 waves/SIMD,
                              // 3 LDS ring, two tiles per step
    int group_items;          // tiled kernel: XCD-grouped item order
    int tile_shape;           // tiled kernel: TiledShape variant
    int want_flag;            // process SNP tiles with this flag; -1 = all
    float inv_hc[3];          // screen level: 1/H_c(df), [0] = 0
    double hc_screen[3];      // screen level: H_c(df) in double, [0] unused
    double hc[kMaxLevels][2]; // exact thresholds per level, df = 1, 2
    int n_lev;
    HitRec* hits;
    int64_t hit_cap;
    unsigned long long* n_hits;
    int64_t snp_base;
    unsigned long long* minp_bits;  // [virtual rows] bits of the min p
    unsigned long long* counts;     // [P][n_lev]
    double* H_out;            // FULL: [T][M]
    double* p_out;
    int32_t* sums_out;        // SUMS: [3][T][M]
    // pairs that passed the fp32 screen, evaluated exactly by scan_exact:
    // {operand row, SNP | form << 31, column-1 value, column-2 value}
    uint4* cand;
    int64_t cand_cap;
    unsigned long long* n_cand;
    // screen mode: pairs of SNPs with missing genotypes that passed the
    // bound, {operand row, SNP, D~1, D~2} (the group-1 and group-2 sums of
    // centred full-sample ranks over the observed samples), evaluated by
    // scan_exact (null: in the scan)
    int4* mcand;
    int64_t mcand_cap;
    unsigned long long* n_mcand;
    // [m_pad][kLaneMiss] positions of the missing samples of each SNP with 1
    // to kLaneMiss of them, ascending (written by pack_snps); other entries
    // are unused
    const int16_t* mpos;
};

// Multi-allelic scan (classes 0..n_classes-1, at most kMaxClasses).
constexpr int kMaxClasses = 8;

// Per-SNP constants of a multi-allelic scan (over the samples whose code is a
// class; a SNP with a removed code is evaluated per pair, not screened).
struct alignas(16) MultiInfo {
    float w[kMaxClasses];     // 1/N_c, 0 for an empty class
    int16_t n[kMaxClasses];   // class sizes
    int16_t nmiss;            // samples whose code is not a class
    int16_t df;               // non-empty classes - 1 (0 for at most one)
    int16_t pad[2];
};
static_assert(sizeof(MultiInfo) == 64, "MultiInfo is 64 bytes");

// A multi-allelic pair that passed the MFMA screen: its operand row, SNP and
// the centred doubled-rank sums D_1..D_{G-1} of classes 1..G-1 (exact
// integers from the screen's GEMM; D_0 = -(D_1 + ... + D_{G-1}), the centred
// ranks of a trait without missing values summing to zero).
struct alignas(16) MultiCand {
    uint32_t row;
    uint32_t snp;
    int32_t d[6];
};
static_assert(sizeof(MultiCand) == 32, "MultiCand is 32 bytes");

struct MultiArgs {
    const int16_t* ranks2;   // T x K doubled midranks, 0 = missing value
    const int64_t* tiesum;   // T
    int64_t T;
    int K;
    int G;                   // classes
    const uint8_t* packed;   // M rows of pstride bytes: class 0..G-1, else 0xFF
    int pstride;             // a multiple of 32, >= K
    int64_t M;
    double hc[kMaxClasses];  // hc[df]: threshold on H at df (hits)
    HitRec* hits;
    int64_t hit_cap;
    unsigned long long* n_hits;
    int64_t snp_base;
    double* H_out;           // full mode: T x M
    double* p_out;
    unsigned long long* minp_bits;  // hits mode: [T] bits of the per-trait min p, or null
    // which pairs the lane-per-pair kernel evaluates
    const MultiInfo* info;        // [M] per-SNP constants, or null
    const uint8_t* nan_flag;      // [T] 1: the trait has a missing expression value, or null
    const int32_t* trait_list;    // traits to scan, or null for 0..T-1
    const int32_t* n_list;        // device count of trait_list
    int only_incomplete;          // 1: only pairs of a NaN trait or of a SNP with nmiss > 0
    int record_hits;              // 0: minimum p only
    const int32_t* n_nan;         // device: number of NaN traits
    const int32_t* any_missing;   // device: 1 if some SNP has nmiss > 0
    // MFMA screen of the complete pairs (SNP-stationary, fp16)
    const void* A;                // centred ranks in fragment order (prep_ranks_f16)
    const float* theta;           // [tiles] min over the tile's rows of K^3 - K - sumT
    const int32_t* row_v;         // [tiles * 32] trait of each operand row, -1 padding
    int64_t n_rows;
    int64_t n_snp_tiles;
    int tiles_per_range;
    float inv_hc[kMaxClasses];    // screen level: 1/H_c(df) (capped), [0] = 0
    MultiCand* cand;              // screened pairs with their class sums
    int64_t cand_cap;
    unsigned long long* n_cand;
};

// Extra operands of the tiled large-K kernels.
struct TiledArgs {
    const void* Bf;      // [snp tiles][ks][NC][64] fragments
    const void* A_hi;    // int8 byte split: high plane of A, else null
    int ks;              // k-steps of both operands (even)
    int shape;           // tile shape: 0 wide (one wave per SIMD), 1 two waves per SIMD
};

// candidate entry flags (high bits of the SNP word): column values are
// (D1, D2) of the PLAIN form, else (Y, Z) of DIAG; kCandZs: the DIAG Z column
// carries the per-SNP scale q (Z = q D2, see diag_zscale)
constexpr uint32_t kCandPlain = 0x80000000u;
constexpr uint32_t kCandZs = 0x40000000u;
constexpr uint32_t kCandSnp = 0x3FFFFFFFu;

}  // namespace kx
