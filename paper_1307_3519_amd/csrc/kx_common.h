// kx_common.h -- types and device helpers shared by the gfx950 kernels of the
// Kruskal-Wallis scan and by the host side that launches them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace kx {

constexpr int kWave = 64;            // CDNA wavefront
constexpr int kTile = 32;            // 32x32 MFMA output tile: 32 traits x 32 SNPs
constexpr int kWavesPerBlock = 4;    // one SNP tile per wave, 128 SNPs per block
constexpr int kMaxLevels = 4;        // p-value thresholds counted in one pass
constexpr float kScreenSlack = 1.0e-5f;  // relative margin of the fp32 screen

// Packed genotype code for "not a genotype" (missing or padding).
constexpr int8_t kMissingCode = 3;

// Per-SNP constants written by the pack kernel.  Counts are over the
// non-missing samples.  The two MFMA columns of an SNP are
//   Y = cy1 * D1 + cy2 * D2,  Z = D2          (no missing genotype)
// where D_i is twice the centred rank sum of genotype group i; with
// D0 = -D1 - D2 the statistic numerator f = sum_i D_i^2 / N_i equals
// wy * Y^2 + wz * Z^2 (the quadratic form written as a sum of two squares).
struct alignas(16) SnpInfo {
    float wy, wz;        // diagonal weights of f in (Y, Z)
    float a0, a1, a2;    // 1/N_i (0 for an empty group)
    int16_t cy1, cy2;    // integer coefficients of column Y
    int16_t n0, n1, n2;  // group sizes over observed samples
    int16_t nmiss;       // samples with a missing genotype
};
static_assert(sizeof(SnpInfo) == 32, "SnpInfo is 32 bytes");

// degrees of freedom: number of non-empty genotype groups - 1 (0..2)
__host__ __device__ inline int snp_df(const SnpInfo& s) {
    int ne = (s.n0 > 0) + (s.n1 > 0) + (s.n2 > 0);
    return ne > 0 ? ne - 1 : 0;
}

// Scale of the fp16 DIAG screen's second column: q = sqrt(wz / wy) rounded
// up to an fp16 value, so that with Z = q D2 the screen reads
// f / wy <= Y^2 + Z^2 (two VALU operations per pair).  Z stays exact: the
// partial sums of q * D2 have at most 11 + 13 significant bits while
// sum_k |c_k| < 2^13 (K <= 128).  0 when wy = 0 (a SNP without groups 0
// and 1, which is monomorphic and never screened in).
__device__ inline float diag_zscale(const SnpInfo& s) {
    if (!(s.wy > 0.0f) || !(s.wz > 0.0f)) return 0.0f;
    const double x = sqrt((double)s.wz / (double)s.wy);
    _Float16 h = (_Float16)x;
    if ((double)h < x) {
        uint16_t b;
        __builtin_memcpy(&b, &h, 2);
        ++b;                                   // next fp16 up (x > 0, finite)
        __builtin_memcpy(&h, &b, 2);
    }
    return (float)h;
}

// Hit record, identical layout to krux_hit of the C ABI.
struct HitRec {
    int32_t trait;
    int32_t snp;
    double H;
    double p;
};
static_assert(sizeof(HitRec) == 24, "hit record is 24 bytes");

__host__ __device__ inline int64_t cube_minus(int64_t k) { return k * k * k - k; }

// f(std::integral_constant<int, i>) for i = 0 .. N-1, expanded at compile
// time: loop indices that select registers (accumulator tiles, vector
// elements) stay constants even where the compiler would not unroll a large
// loop body, which would otherwise put the whole array in scratch memory.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ inline int bitlen64(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

// Nearest double (ties to even) to num / den, for den < 2^63 and an integer
// quotient below 2^64 (always true here: 0 <= H <= K - 1).
__device__ inline double rat_to_double(unsigned __int128 num, uint64_t den) {
    if (num == 0 || den == 0) return 0.0;
    if ((num >> 53) == 0 && den < (1ull << 53))
        return (double)(uint64_t)num / (double)den;   // one IEEE division: exact operands
    uint64_t nh = (uint64_t)(num >> 64), nl = (uint64_t)num;
    int nb = nh ? 64 + bitlen64(nh) : bitlen64(nl);
    uint64_t q = 0, r = 0;
    for (int i = nb - 1; i >= 0; --i) {
        uint64_t bit = i >= 64 ? (nh >> (i - 64)) & 1ull : (nl >> i) & 1ull;
        r = (r << 1) | bit;
        q <<= 1;
        if (r >= den) { r -= den; q |= 1ull; }
    }
    int e = 0;
    int sticky;
    int qb = bitlen64(q);
    if (qb >= 54) {
        int sh = qb - 54;
        sticky = ((q & ((1ull << sh) - 1ull)) != 0) || (r != 0);
        q >>= sh;
        e = sh;
    } else {
        while (bitlen64(q) < 54) {
            r <<= 1;
            q <<= 1;
            if (r >= den) { r -= den; q |= 1ull; }
            --e;
        }
        sticky = (r != 0);
    }
    uint64_t mant = q >> 1;
    int rb = (int)(q & 1ull);
    if (rb && (sticky || (mant & 1ull))) ++mant;
    if (mant == (1ull << 53)) { mant >>= 1; ++e; }
    return ldexp((double)mant, e + 1);
}

// Exact H of one pair from twice-centred group sums D_i (centred at K'+1),
// group sizes, observed sample count K' and tie term:
//   H = 3 (K'-1) sum_{N_i>0} D_i^2 / N_i / (K'^3 - K' - sumT),
// evaluated as the rational 3(K'-1) P / (L E), L = prod N_i, rounded once.
__device__ inline double exact_H(int64_t D0, int64_t D1, int64_t D2, int n0, int n1,
                                 int n2, int64_t kp, int64_t tiesum, int df) {
    int64_t E = cube_minus(kp) - tiesum;
    if (df <= 0 || kp < 2 || E <= 0) return 0.0;
    uint64_t L = 1;
    if (n0) L *= (uint64_t)n0;
    if (n1) L *= (uint64_t)n1;
    if (n2) L *= (uint64_t)n2;
    uint64_t P = 0;
    if (n0) P += (uint64_t)(D0 * D0) * (L / (uint64_t)n0);
    if (n1) P += (uint64_t)(D1 * D1) * (L / (uint64_t)n1);
    if (n2) P += (uint64_t)(D2 * D2) * (L / (uint64_t)n2);
    unsigned __int128 num = (unsigned __int128)(uint64_t)(3 * (kp - 1)) * P;
    uint64_t den = L * (uint64_t)E;
    return rat_to_double(num, den);
}

__device__ inline double pvalue(double H, int df) {
    if (df == 2) return exp(-H * 0.5);
    if (df == 1) return erfc(sqrt(H * 0.5));
    return 1.0;
}

__device__ inline uint64_t dbl_bits(double v) { return (uint64_t)__double_as_longlong(v); }

}  // namespace kx
