// prep.hip -- operand preparation for the rank-sum GEMM.
//
// pack_snps: genotype rows -> (a) a packed copy with a fixed, 32-byte aligned
//   row stride in which every code outside {0,1,2} (missing) and the padding
//   become kMissingCode, (b) per-SNP constants (group sizes N_i, df, the
//   integer coefficients of the MFMA columns and the weights of the
//   statistic numerator), (c) a per-32-SNP-tile flag "has a missing
//   genotype" (and whether any tile has one, and any none), (d) the positions of the missing samples of each SNP that has
//   at most kLaneMiss of them.  Counting N_i is the paper's
//   N_i = sum_k I_i(m,k) (eq. (1)).
//
// prep_ranks: doubled midranks -> the MFMA A operand in fragment order,
//   centred c = a - (K+1) (an integer in [-(K-1), K-1], exact in fp16 for
//   K <= 2049 and in int8 for K <= 128), optionally through a row list
//   (fix-up passes) and a column permutation (permuted data for the FDR).
//   Also the screen threshold of each 32-row tile, the smallest of
//   K^3 - K - sumT (the tie factor's numerator, eq. (2) with the tied-data
//   correction) over its rows (+inf for rows without a finite threshold), and
//   the map operand row -> virtual row (perm * T + trait), -1 for padding.
#include "kx_args.h"

namespace kx {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef int int4v __attribute__((ext_vector_type(4)));

// Per-SNP constants from the group counts (one thread per SNP).
__device__ inline SnpInfo snp_constants(int c0, int c1, int c2, int cm, int diag_ok) {
    SnpInfo s;
    s.n0 = (int16_t)c0; s.n1 = (int16_t)c1; s.n2 = (int16_t)c2;
    s.nmiss = (int16_t)cm;
    double a0 = c0 ? 1.0 / c0 : 0.0, a1 = c1 ? 1.0 / c1 : 0.0, a2 = c2 ? 1.0 / c2 : 0.0;
    s.a0 = (float)a0; s.a1 = (float)a1; s.a2 = (float)a2;
    // f = a0 D0^2 + a1 D1^2 + a2 D2^2 with D0 = -D1 - D2, completed to a
    // square in D1:  f = wy * Y^2 + wz * D2^2,  Y = cy1 D1 + cy2 D2.
    double wy = 0.0, wz = a2;
    int cy1 = 0, cy2 = 0;
    if (c0 > 0 && c1 > 0) {
        cy1 = c0 + c1; cy2 = c1;
        wy = 1.0 / ((double)c0 * c1 * (c0 + c1));
        wz = 1.0 / (double)(c0 + c1) + a2;
    } else if (c1 > 0) {        // group 0 empty: f = a1 D1^2 + a2 D2^2
        cy1 = 1; cy2 = 0; wy = a1;
    } else if (c0 > 0) {        // group 1 empty: D0 = -D2, f = (a0 + a2) D2^2
        cy1 = 1; cy2 = 1; wy = a0;
    }
    if (!diag_ok) { cy1 = 1; cy2 = 0; }
    s.cy1 = (int16_t)cy1; s.cy2 = (int16_t)cy2;
    s.wy = (float)wy; s.wz = (float)wz;
    return s;
}

// Counts of the codes 0, 1, 2, 3 among the four bytes of w (codes 0..3).
__device__ inline void count_codes(uint32_t w, int& c0, int& c1, int& c2, int& c3) {
    const uint32_t b0 = w & 0x01010101u, b1 = (w >> 1) & 0x01010101u;
    c3 += __popc(b0 & b1);
    c1 += __popc(b0 & ~b1);
    c2 += __popc(~b0 & b1);
    c0 += __popc(~(b0 | b1) & 0x01010101u);
}

// A block packs kPackRows SNP rows through LDS, one column chunk of
// kPackCols bytes at a time: the block loads the chunk's input bytes
// (consecutive threads take consecutive bytes of a row), rewrites them as
// codes and stores them to the packed rows, then each thread counts the codes
// of its own row in LDS.  gstride: packed row bytes (>= K, multiple of 32).
constexpr int kPackRows = 256;
constexpr int kPackCols = 128;
constexpr int kPackLds = kPackCols + 4;     // padded LDS row: conflict-free dword reads
constexpr int kPackUnroll = 16;
static_assert((kPackRows * kPackCols) % (256 * kPackUnroll) == 0, "whole batches");

__global__ __launch_bounds__(256) void pack_snps(const int8_t* __restrict__ geno, int64_t M,
                                                 int64_t ld, int K, int64_t m_pad, int gstride,
                                                 int diag_ok, int8_t* __restrict__ gp,
                                                 SnpInfo* __restrict__ info,
                                                 int32_t* __restrict__ tile_flags,
                                                 int16_t* __restrict__ mpos) {
    __shared__ uint32_t s_rows[kPackRows * kPackLds / 4];
    uint8_t* s_bytes = (uint8_t*)s_rows;
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * kPackRows;
    const int64_t m_me = m0 + tid;
    int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    for (int col0 = 0; col0 < gstride; col0 += kPackCols) {
        const int w = gstride - col0 < kPackCols ? gstride - col0 : kPackCols;
        // batches of kPackUnroll independent byte loads per thread, so that a
        // thread waits once per batch rather than once per byte
        for (int base = 0; M > 0 && base < kPackRows * kPackCols; base += 256 * kPackUnroll) {
            int8_t g[kPackUnroll];
#pragma unroll
            for (int u = 0; u < kPackUnroll; ++u) {
                // branch-free: the address is clamped into the matrix (M >= 1
                // here) and out-of-range elements are replaced afterwards
                const int idx = base + u * 256 + tid;
                const int r = idx / kPackCols, cc = idx % kPackCols;
                const int64_t m = m0 + r;
                const int col = col0 + cc;
                const int64_t mc = m < M ? m : M - 1;
                const int colc = col < K ? col : K - 1;
                const int8_t raw = geno[mc * ld + colc];
                g[u] = (cc < w && m < M && col < K) ? raw : (int8_t)kMissingCode;
            }
#pragma unroll
            for (int u = 0; u < kPackUnroll; ++u) {
                const int idx = base + u * 256 + tid;
                const int r = idx / kPackCols, cc = idx % kPackCols;
                if (cc >= w) continue;
                const int64_t m = m0 + r;
                const int8_t code = (g[u] >= 0 && g[u] <= 2) ? g[u] : (int8_t)kMissingCode;
                s_bytes[r * kPackLds + cc] = (uint8_t)code;
                if (m < m_pad) gp[m * (int64_t)gstride + col0 + cc] = code;
            }
        }
        __syncthreads();
        // this thread's row: only the K real columns count
        const int valid = K - col0 < w ? (K - col0 > 0 ? K - col0 : 0) : w;
        const uint32_t* row = s_rows + tid * (kPackLds / 4);
        const int full = valid >> 2;
        // counts of the word's codes, and the positions of its missing ones
        // while the row has at most kLaneMiss of them
        auto word = [&](uint32_t w, int col) {
            uint32_t mb = w & (w >> 1) & 0x01010101u;
            if (mpos && m_me < M) {
                int j = c3;
                while (mb) {
                    if (j < kLaneMiss)
                        mpos[m_me * kLaneMiss + j] = (int16_t)(col + (__builtin_ctz(mb) >> 3));
                    mb &= mb - 1u;
                    ++j;
                }
            }
            count_codes(w, c0, c1, c2, c3);
        };
        for (int q = 0; q < full; ++q) word(row[q], col0 + 4 * q);
        if (valid & 3) {
            const uint32_t keep = (1u << (8 * (valid & 3))) - 1u;
            // masked-off bytes read as code 0: subtract them afterwards
            word(row[full] & keep, col0 + 4 * full);
            c0 -= 4 - (valid & 3);
        }
        __syncthreads();
    }
    const bool real = m_me < M;
    if (!real) { c0 = c1 = c2 = c3 = 0; }
    if (m_me < m_pad) info[m_me] = snp_constants(c0, c1, c2, c3, diag_ok);
    // per 32-SNP tile: has a missing genotype (tiles past the last SNP are
    // never read as tile flags; the first two of them hold "some tile has a
    // missing genotype" and "some tile has none", so that a launch for the
    // other kind of tile returns at once)
    // (one read and at most one atomic per block and flag: every tile taking
    // an atomic on the same word serialised them, 70 -> 200 us at 500 000 SNPs)
    const unsigned long long miss = __ballot(real && c3 > 0);
    const int lane = tid & 63;
    const int64_t n_real = (M + 31) >> 5;
    const int64_t tile = m_me >> 5;
    const uint32_t bits = (uint32_t)(miss >> (lane & 32));
    const bool lead = (lane & 31) == 0 && tile < n_real;
    if (lead) tile_flags[tile] = bits ? 1 : 0;
    const int any_miss = __syncthreads_or(lead && bits != 0u);
    const int any_full = __syncthreads_or(lead && bits == 0u);
    if (tid == 0) {
        if (any_miss && tile_flags[n_real] == 0) atomicOr(&tile_flags[n_real], 1);
        if (any_full && tile_flags[n_real + 1] == 0) atomicOr(&tile_flags[n_real + 1], 1);
    }
}

// Fill an int32 array (used instead of a memset so captured graphs stay safe).
__global__ void fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}


__device__ inline int rank_at(const PrepArgs& a, int64_t v, int k) {
    int64_t trait = v % a.T, perm = v / a.T;
    int kk = a.perms ? a.perms[perm * a.K + k] : k;
    return a.ranks2[trait * a.K + kk];
}

// Operand row r belongs to a trait with missing expression values: it is
// written as padding (zero operand, virtual row -1) and its pairs are left to
// scan_nan_traits.
__device__ inline bool nan_row(const PrepArgs& a, int64_t r) {
    if (!a.nan_flag) return false;
    const int64_t v = a.rows ? a.rows[r] : r;
    return a.nan_flag[v % a.T] != 0;
}

__device__ inline int64_t count_rows(const PrepArgs& a) {
    if (a.d_nrows) {
        int64_t n = *a.d_nrows;
        return n < a.n_rows ? n : a.n_rows;
    }
    return a.n_rows;
}

__device__ inline float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline void clear_counters(const PrepArgs& a) {
    if (a.zero && blockIdx.x == 0 && (int)threadIdx.x < a.n_zero) a.zero[threadIdx.x] = 0ull;
}

// fp16 operand: one thread per (tile, k-step, lane) writes 8 halves.  The
// grid-stride loop keeps the 64 threads of one (tile, k-step) in one wave
// (the stride is a multiple of 64).
__global__ __launch_bounds__(256) void prep_ranks_f16(PrepArgs a) {
    clear_counters(a);
    const int64_t n_tiles = (a.n_alloc_rows + kTile - 1) / kTile;
    const int64_t total = n_tiles * a.ks * kWave;
    const int64_t nr = count_rows(a);
    half8* A = (half8*)a.A;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int lane = (int)(i % kWave);
        int64_t ts = i / kWave;
        int s = (int)(ts % a.ks);
        int64_t tile = ts / a.ks;
        int64_t r = tile * kTile + (lane & 31);
        half8 h;
        for (int e = 0; e < 8; ++e) h[e] = (_Float16)0.0f;
        const bool live = r < nr && !nan_row(a, r);
        if (live) {
            int64_t v = a.rows ? a.rows[r] : r;
            int k0 = s * 16 + 8 * (lane >> 5);
            for (int e = 0; e < 8; ++e) {
                int k = k0 + e;
                if (k < a.K) h[e] = (_Float16)(float)(rank_at(a, v, k) - (a.K + 1));
            }
        }
        A[i] = h;
        if (s == 0) {
            // the 64 threads of (tile, k-step 0) are one wave: lanes 0..31 hold
            // the tile's rows; the wave's minimum is the tile's threshold
            float th = __builtin_inff();
            if (lane < 32 && live) {
                int64_t v = a.rows ? a.rows[r] : r;
                int64_t E = cube_minus(a.K) - a.tiesum[v % a.T];
                if (E > 0) th = (float)E;
                a.row_v[r] = (int32_t)v;
            } else if (lane < 32) {
                a.row_v[r] = -1;
            }
            th = wave_min(th);
            if (lane == 0) a.theta[tile] = th;
        }
    }
}

// int8 operand: 16 samples per lane per k-step of 32.  With A_hi set, the
// centred rank is split c = 128 h + l, l in [0, 127].
__global__ __launch_bounds__(256) void prep_ranks_i8(PrepArgs a) {
    clear_counters(a);
    const int64_t n_tiles = (a.n_alloc_rows + kTile - 1) / kTile;
    const int64_t total = n_tiles * a.ks * kWave;
    const int64_t nr = count_rows(a);
    int4v* A = (int4v*)a.A;
    int4v* Ah = (int4v*)a.A_hi;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int lane = (int)(i % kWave);
        int64_t ts = i / kWave;
        int s = (int)(ts % a.ks);
        int64_t tile = ts / a.ks;
        int64_t r = tile * kTile + (lane & 31);
        int8_t lo[16], hi[16];
        for (int e = 0; e < 16; ++e) { lo[e] = 0; hi[e] = 0; }
        const bool live = r < nr && !nan_row(a, r);
        if (live) {
            int64_t v = a.rows ? a.rows[r] : r;
            int k0 = s * 32 + 16 * (lane >> 5);
            for (int e = 0; e < 16; ++e) {
                int k = k0 + e;
                if (k < a.K) {
                    int c = rank_at(a, v, k) - (a.K + 1);
                    if (Ah) {
                        int h = c >> 7;               // floor(c / 128)
                        lo[e] = (int8_t)(c - h * 128);
                        hi[e] = (int8_t)h;
                    } else {
                        lo[e] = (int8_t)c;
                    }
                }
            }
        }
        int4v wl, wh;
        for (int w = 0; w < 4; ++w) {
            uint32_t ul = 0, uh = 0;
            for (int b = 0; b < 4; ++b) {
                ul |= (uint32_t)(uint8_t)lo[4 * w + b] << (8 * b);
                uh |= (uint32_t)(uint8_t)hi[4 * w + b] << (8 * b);
            }
            wl[w] = (int)ul; wh[w] = (int)uh;
        }
        A[i] = wl;
        if (Ah) Ah[i] = wh;
        if (s == 0) {
            // the 64 threads of (tile, k-step 0) are one wave: lanes 0..31 hold
            // the tile's rows; the wave's minimum is the tile's threshold
            float th = __builtin_inff();
            if (lane < 32 && live) {
                int64_t v = a.rows ? a.rows[r] : r;
                int64_t E = cube_minus(a.K) - a.tiesum[v % a.T];
                if (E > 0) th = (float)E;
                a.row_v[r] = (int32_t)v;
            } else if (lane < 32) {
                a.row_v[r] = -1;
            }
            th = wave_min(th);
            if (lane == 0) a.theta[tile] = th;
        }
    }
}

// A pass whose screen level is p_L evaluates exactly every pair with p < p_L,
// so a row whose minimum over the evaluated pairs is below p_L (less a margin
// for host/device rounding of p) is final.  The other rows (limit_bits =
// bits of that bound) are listed for the next, looser pass.
__global__ void list_unresolved(const unsigned long long* __restrict__ minp_bits,
                                unsigned long long limit_bits,
                                const int32_t* __restrict__ rows_in,
                                const int32_t* __restrict__ d_n_in, int64_t n_in_max,
                                int32_t* __restrict__ rows_out, int32_t* __restrict__ d_n_out) {
    int64_t n_in = d_n_in ? (*d_n_in < n_in_max ? *d_n_in : n_in_max) : n_in_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_in;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = rows_in ? rows_in[i] : (int32_t)i;
        if (minp_bits[v] >= limit_bits) {
            int pos = atomicAdd(d_n_out, 1);
            rows_out[pos] = v;
        }
    }
}

__global__ void bits_to_double(const unsigned long long* __restrict__ bits, int64_t n,
                               double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = __longlong_as_double((long long)bits[i]);
}

}  // namespace kx

extern "C" {

hipError_t kx_launch_pack(const int8_t* geno, int64_t M, int64_t ld, int K, int64_t m_pad,
                          int gstride, int diag_ok, int8_t* gp, kx::SnpInfo* info,
                          int32_t* tile_flags, int16_t* mpos, int grid, hipStream_t st) {
    int64_t n_tiles = m_pad / 32;
    hipLaunchKernelGGL(kx::fill_i32, dim3(64), dim3(256), 0, st, tile_flags, n_tiles + 2, 0);
    (void)grid;
    const int64_t blocks = (m_pad + kx::kPackRows - 1) / kx::kPackRows;
    if (blocks > 0)
        hipLaunchKernelGGL(kx::pack_snps, dim3((unsigned)blocks), dim3(256), 0, st, geno, M, ld,
                           K, m_pad, gstride, diag_ok, gp, info, tile_flags, mpos);
    return hipGetLastError();
}

hipError_t kx_launch_prep(const kx::PrepArgs* a, int is_i8, int grid, hipStream_t st) {
    if (is_i8)
        hipLaunchKernelGGL(kx::prep_ranks_i8, dim3(grid), dim3(256), 0, st, *a);
    else
        hipLaunchKernelGGL(kx::prep_ranks_f16, dim3(grid), dim3(256), 0, st, *a);
    return hipGetLastError();
}

hipError_t kx_launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    hipLaunchKernelGGL(kx::fill_i32, dim3(256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t kx_launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v,
                              hipStream_t st) {
    hipLaunchKernelGGL(kx::fill_u64, dim3(512), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t kx_launch_list_unresolved(const unsigned long long* minp_bits,
                                     unsigned long long limit_bits, const int32_t* rows_in,
                                     const int32_t* d_n_in, int64_t n_in_max, int32_t* rows_out,
                                     int32_t* d_n_out, hipStream_t st) {
    hipLaunchKernelGGL(kx::fill_i32, dim3(1), dim3(64), 0, st, d_n_out, 1, 0);
    hipLaunchKernelGGL(kx::list_unresolved, dim3(256), dim3(256), 0, st, minp_bits, limit_bits,
                       rows_in, d_n_in, n_in_max, rows_out, d_n_out);
    return hipGetLastError();
}

hipError_t kx_launch_bits_to_double(const unsigned long long* bits, int64_t n, double* out,
                                    hipStream_t st) {
    hipLaunchKernelGGL(kx::bits_to_double, dim3(256), dim3(256), 0, st, bits, n, out);
    return hipGetLastError();
}

}  // extern "C"
