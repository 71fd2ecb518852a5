// scan_tiled.h -- the rank-sum GEMM with its fused epilogue for sample counts
// too large to keep a SNP tile's genotype columns in registers (K > 128).
//
// Same computation as scan_kernel (eq. (1), eq. (2) with the tie factor, the
// chi-square screen and exact evaluation of candidates), organised as a
// classic two-operand tiled GEMM: each wave computes 2 or 4 trait tiles x 1
// or 2 SNP tiles, in blocks of four waves (one or two blocks per CU) or of
// eight (one per CU); see TiledShape for the four shapes.  The K loop runs
// over chunks of two 16-sample (fp16) or 32-sample (int8) k-steps (four in
// the fp16 eight-wave blocks when the k-step count allows) whose A
// (centred ranks) fragments and B side (genotype columns expanded once into
// MFMA fragment order, or the packed genotype codes themselves, from which
// the fragments are built in registers) are copied into an LDS ring by
// LDS-DMA loads, with one block barrier per chunk.  With int8 and K > 127
// the centred rank is split into bytes, c = 128 h + l, and two accumulator
// sets give D = 128 D_h + D_l exactly.
#pragma once
#include "scan_kernel.h"

namespace kx {


// Per-lane screen constants of one SNP column.  The missing-genotype form
// takes the square roots r_i of its weights and q_i = nmiss N_i r_i, so that
// w_i (|D_i| + nmiss N_i)^2 = (|D_i| r_i + q_i)^2: one fma and one square per
// column, the same for complete SNPs (q_i = 0, delta = 0).
struct LaneK {
    float wy, wz, w0, w1, w2, qn0, qn1, qn2, delta;
    float r0, r1, r2, q0, q1, q2;
    bool miss;
};

__device__ inline LaneK lane_constants(const SnpInfo& inf, int K, const float* inv_hc) {
    LaneK c;
    const int kp = K - inf.nmiss;
    const float fac = 3.0f * (float)(kp - 1) * (1.0f + kScreenSlack) * inv_hc[snp_df(inf)];
    c.wy = inf.wy * fac; c.wz = inf.wz * fac;
    c.w0 = inf.a0 * fac; c.w1 = inf.a1 * fac; c.w2 = inf.a2 * fac;
    c.miss = inf.nmiss > 0;
    c.qn0 = (float)inf.nmiss * inf.n0; c.qn1 = (float)inf.nmiss * inf.n1;
    c.qn2 = (float)inf.nmiss * inf.n2;
    c.delta = (float)(cube_minus(K) - cube_minus(kp));
    c.r0 = sqrtf(c.w0); c.r1 = sqrtf(c.w1); c.r2 = sqrtf(c.w2);
    c.q0 = c.qn0 * c.r0; c.q1 = c.qn1 * c.r1; c.q2 = c.qn2 * c.r2;
    return c;
}

// Screen value (> 0: candidate) of one pair from its column values.
template <int FORM>
__device__ inline float screen_value(const LaneK& c, float th, float v0, float v1, float v2) {
    if constexpr (FORM == DIAG) {
        return fmaf(c.wy * v0, v0, fmaf(c.wz * v1, v1, -th));
    } else if constexpr (FORM == PLAIN) {
        const float d0 = -(v0 + v1);
        return fmaf(c.w0 * d0, d0, fmaf(c.w1 * v0, v0, fmaf(c.w2 * v1, v1, -th)));
    } else {
        // |D'_i - D_i| <= nmiss N_i and E' >= K'^3 - K' - sumT (complete SNPs:
        // the plain screen, with a threshold lowered by 1e-6, which only
        // admits more candidates); the weights' 1e-5 slack covers the
        // rounding of r_i and q_i
        const float e0 = fmaf(fabsf(v0), c.r0, c.q0);
        const float e1 = fmaf(fabsf(v1), c.r1, c.q1);
        const float e2 = fmaf(fabsf(v2), c.r2, c.q2);
        const float tl = c.delta - th * 0.99999905f;
        return fmaf(e0, e0, fmaf(e1, e1, fmaf(e2, e2, tl)));
    }
}

// Tile shape of the tiled kernel.
//  V = 0 ("wide"): up to 4 trait tiles x 2 SNP tiles per wave (accumulators up
//        to 256 registers, fewest LDS reads per MFMA), one wave per SIMD;
//  V = 1 ("two waves"): 4 (or 2) trait tiles x 1 SNP tile per wave, so that
//        two waves share each SIMD and one wave's epilogue overlaps the
//        other's MFMAs; its LDS ring is kept small enough for two blocks;
//  V = 2 ("codes", PLAIN form): the tiles of V = 1, with the B side copied
//        as the packed genotype codes (1 byte per sample instead of 2 bytes
//        per sample and column) and turned into fragments in registers (byte
//        permutes), so that a chunk is 18 KB instead of 24 KB, the LDS ring
//        holds four chunks instead of three, and no expanded columns are
//        built;
//  V = 3 ("one block per CU"): eight waves per block (two per SIMD), the
//        B side from the codes in the PLAIN form and in the fp16
//        missing-genotype form (three indicator columns, classes 0..2, built
//        in registers; a chunk of 8 KB of A and 4 KB of codes feeds 96 MFMAs
//        where the expanded columns took 16 KB and 12 KB, and the ring holds
//        eight chunks instead of four), expanded in the int8 missing-genotype
//        form.
template <int FORM, bool SPLIT, int V, int KCX = 2>
struct TiledShape {
    static constexpr int NC = FORM == MISS3 ? 3 : 2;
    static constexpr int NP = SPLIT ? 2 : 1;
    // fp16 missing-genotype form in eight-wave blocks: codes as well (three
    // indicator columns, classes 0..2)
    static constexpr bool CODES = (V >= 2 && FORM == PLAIN) || (V == 3 && FORM == MISS3 && !SPLIT);
    static constexpr int NW = V == 3 ? 8 : 4;            // waves per block
    // SNP groups (waves per trait group): eight-wave blocks take one trait
    // group of eight SNP tiles in the fp16 codes form (codes are the small
    // side; K = 500 3.68 -> 3.62 ms, K = 1000 6.72 -> 6.51 ms against 2 x 4),
    // two of four in the int8 one (its A side has two planes; 1 x 8 4.17 ->
    // 4.38 ms), two of four in the fp16 missing-genotype form (two trait
    // tiles per wave; cohort step 53.5 ms against 52.8 with 1 x 8) and four
    // trait groups of two SNP tiles in the int8 one (its three expanded
    // columns are the large side; K = 1000 17.9 -> 17.5 ms)
    static constexpr int GSW = V == 3 ? (FORM == MISS3 ? (CODES ? 4 : 2) : SPLIT ? 4 : 8) : 2;
    static constexpr int GTW = NW / GSW;                 // trait groups
    static constexpr int WS = V == 0 ? ((NC == 2 && !SPLIT) ? 2 : 1) : 1;
    static constexpr int WT = V == 0 ? ((FORM != MISS3 && NP * 4 * WS * NC * 16 <= 256) ? 4 : 2)
                                     : (NP * NC <= 2 ? 4 : 2);
    static constexpr int BT = GTW * WT;                  // trait tiles per block
    static constexpr int BS = GSW * WS;                  // SNP tiles per block
    static constexpr int ACC = NP * WT * WS * NC * 16;   // accumulator registers
    static constexpr int WPE_MIN = (V != 0 && ACC <= 128) ? 2 : 1;
    static constexpr int RING_BYTES =
        V == 0 ? 128 * 1024 : V == 3 ? (FORM == MISS3 ? 128 * 1024 : 140 * 1024) : 72 * 1024;
    static constexpr int KC = KCX;                       // k-steps per chunk (2 or 4)
    // codes shapes: 1 KB copies of codes (64 lanes x 16 codes: 32 samples of
    // 32 SNPs), KC / 2 per SNP tile and chunk in fp16 (16-sample k-steps),
    // KC in int8 (32-sample k-steps)
    static constexpr int CPT = SPLIT ? KC : KC / 2;
    static constexpr int NFA = BT * KC * NP;             // A fragments per chunk
    static constexpr int NFB = CODES ? BS * CPT : BS * KC * NC;
    static constexpr int NF = NFA + NFB;                 // 1 KB copies per chunk
    // ring of R chunk slots of NF copies (64 lanes x 16 bytes each)
    static constexpr int R = (CODES || V == 3) ? (RING_BYTES / (NF * kWave * 16) < 8
                                                      ? RING_BYTES / (NF * kWave * 16) : 8)
                                               : (NF * kWave * 16 * 4 <= RING_BYTES ? 4 : 3);
    static constexpr int RING_USED = R * NF * kWave * 16;
};

// Fragments of the B side built from packed genotype codes (V = 2): code
// bytes 0..2 are genotype classes, 3 a missing genotype or padding.
// v_perm_b32 picks bytes of {S0 (bytes 4-7), S1 (bytes 0-3)} by selector.
//
// fp16, one dword (two samples b, b + 1 of a lane's eight) of the indicator
// of class k: the selector [4, code_b, 4, code_b+1] picks 0 for the low
// bytes and byte code of 0x3C << 8k (fp16 1.0 = 0x3C00) for the high bytes.
__device__ inline uint32_t f16_ind_sel(uint32_t w, int b) {
    return __builtin_amdgcn_perm(0x04040404u, w,
                                 0x04u | ((uint32_t)b << 8) | (0x04u << 16) | ((uint32_t)(b + 1) << 24));
}
__device__ inline uint32_t f16_ind(uint32_t sel, int k) {
    return __builtin_amdgcn_perm(0u, k < 3 ? 0x3Cu << (8 * k) : 0u, sel);
}
// fp16 DIAG: the selector [2 code_b, 2 code_b + 1, 2 code_b+1, 2 code_b+1 + 1]
// picks the two bytes of the code's fp16 entry of an 8-byte table.
__device__ inline uint32_t f16_tab_sel(uint32_t w, int b) {
    const uint32_t t = __builtin_amdgcn_perm(0u, w,
                                             (uint32_t)b | ((uint32_t)b << 8) |
                                                 ((uint32_t)(b + 1) << 16) | ((uint32_t)(b + 1) << 24));
    return (t << 1) + 0x01000100u;
}
// int8, one dword (four samples) of the indicator of class k: the codes
// themselves select byte code of 1 << 8k.
__device__ inline uint32_t i8_ind(uint32_t w, int k) {
    return __builtin_amdgcn_perm(0u, k < 3 ? 1u << (8 * k) : 0u, w);
}

// The missing-genotype form re-ranks pairs in its epilogue with per-wave LDS
// scratch (coop_lds_entries); the ring is idle then and holds it when large
// enough, else the launch adds dynamic LDS.
template <int FORM, bool SPLIT, int V, int KCX = 2>
__host__ __device__ inline bool tiled_scratch_in_ring(int K) {
    return (int64_t)TiledShape<FORM, SPLIT, V, KCX>::NW * coop_lds_entries(K) * (int64_t)sizeof(int16_t) <=
           TiledShape<FORM, SPLIT, V, KCX>::RING_USED;
}

template <int E, int FORM, int MODE, bool SPLIT, int V, int KCX = 2>
__global__ __launch_bounds__((TiledShape<FORM, SPLIT, V, KCX>::NW * 64))
__attribute__((amdgpu_waves_per_eu(TiledShape<FORM, SPLIT, V, KCX>::WPE_MIN, 2)))
void scan_tiled(ScanArgs a, TiledArgs ta) {
    using T_ = ET<E>;
    using frag = typename T_::frag;
    using acc_t = typename T_::acc;
    using SH = TiledShape<FORM, SPLIT, V, KCX>;
    constexpr int NC = SH::NC;
    constexpr int WS = SH::WS;                         // SNP tiles per wave
    constexpr int NP = SH::NP;                         // A planes
    constexpr int KC = SH::KC;                         // k-steps per chunk
    constexpr int WT = SH::WT;                         // trait tiles per wave
    constexpr int NW = SH::NW;                         // waves per block
    constexpr int GSW = SH::GSW;                       // waves per trait group
    constexpr int BT = SH::BT;                         // trait tiles per block
    constexpr int BS = SH::BS;                         // SNP tiles per block
    constexpr int NFA = BT * KC * NP;                  // A fragments per chunk
    constexpr int NFB = SH::NFB;                       // B fragments (or code copies) per chunk
    constexpr int NF = NFA + NFB;
    static_assert(NFA == SH::NFA && NF == SH::NF, "fragment count");
    constexpr bool CODES = SH::CODES;
    static_assert(!CODES || (WS == 1 && FORM != DIAG && SPLIT == (E == I8)),
                  "the codes shapes build the indicator columns of one SNP tile per wave");
    // copies per wave per chunk: a contiguous run of NF / NW copies, or
    // (codes shapes and eight-wave blocks) copies wave, wave + NW, ..., which
    // leaves some waves one fewer
    constexpr bool SPREAD = CODES || V == 3;
    constexpr int FPW = (NF + NW - 1) / NW;
    constexpr int FPW_MIN = NF / NW;
    static_assert(SPREAD || NF % NW == 0, "every wave copies the same number of fragments");
    constexpr bool QUEUE = FORM == MISS3;
    // ring of R chunk slots filled D = R - 1 chunks ahead by LDS-DMA copies
    constexpr int R = SH::R;
    static_assert(NF * kWave * 16 * R <= 140 * 1024, "ring fits the LDS budget");
    constexpr int D = R - 1;
    // a wave with FPW copies per chunk waits for D - 1 more of its copies
    // than it needs to (still exact for the chunk it is about to read)
    constexpr int kWaitVm = (D - 1) * FPW_MIN;
    static_assert(kWaitVm <= 63, "wait count fits the vmcnt field");

    __shared__ frag s_buf[R][NF][kWave];
    __shared__ int4 s_queue[QUEUE ? NW : 1][QUEUE ? kQueueCap : 1];
    __shared__ uint4 s_stage[MODE == SCREEN ? NW : 1][kStageCap];
    __shared__ ScanArgs s_args;
    extern __shared__ __attribute__((aligned(16))) int16_t s_qbuf[];
    if (threadIdx.x == 0) s_args = a;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
    int4* queue = s_queue[QUEUE ? wave : 0];
    uint4* stage = s_stage[MODE == SCREEN ? wave : 0];
    int sn = 0, qn = 0;
    int16_t* qbuf = (QUEUE && tiled_scratch_in_ring<FORM, SPLIT, V, KCX>(a.K) ? (int16_t*)&s_buf[0][0][0]
                                                                          : s_qbuf) +
                    (QUEUE ? wave * coop_lds_entries(a.K) : 0);

    // LDS address of the ring (the LDS-DMA destination operand)
    const uint32_t ring_lds =
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) frag*)&s_buf[0][0][0];

    if (a.want_flag == 1 && a.tile_flags[a.n_snp_tiles] == 0) return;
    if (a.want_flag == 0 && a.tile_flags[a.n_snp_tiles + 1] == 0) return;
    int64_t n_rows = a.n_rows;
    if (a.d_nrows) {
        int64_t d = *a.d_nrows;
        n_rows = d < n_rows ? d : n_rows;
    }
    const int KS = ta.ks;
    const int64_t n_tiles = (n_rows + kTile - 1) / kTile;
    const int64_t n_tb = (n_tiles + BT - 1) / BT;
    const int64_t n_sb = (a.n_snp_tiles + BS - 1) / BS;
    const int64_t items = n_tb * n_sb;
    const frag* A = (const frag*)a.A;
    const frag* Ah = (const frag*)ta.A_hi;
    const frag* Bf = (const frag*)ta.Bf;
    const int nchunks = KS / KC;

    // Item order: blocks go round-robin to the 8 XCDs, so the blocks of one
    // XCD (b, b + 8, ...) take, round after round, one 8 x (G/64) group of
    // (trait block, SNP block) items: the group's A and B slices stay in that
    // XCD's L2 while its blocks share them.  Without a multiple of 8 blocks,
    // plain row-major order.
    const bool grouped = a.group_items && (gridDim.x % 8) == 0 && gridDim.x >= 64;
    const int64_t per_xcd = gridDim.x / 8;
    const int64_t GT = 8, GS = grouped ? per_xcd / 8 : 1;
    const int64_t n_gt = (n_tb + GT - 1) / GT, n_gs = (n_sb + GS - 1) / GS;
    const int64_t n_rounds = grouped ? (n_gt * n_gs + 7) / 8 : (items + gridDim.x - 1) / gridDim.x;
    for (int64_t round = 0; round < n_rounds; ++round) {
        int64_t tb, sb;
        if (grouped) {
            const int64_t grp = round * 8 + blockIdx.x % 8;
            const int64_t j = blockIdx.x / 8;
            if (grp >= n_gt * n_gs || j >= GT * GS) continue;
            tb = (grp % n_gt) * GT + j % GT;
            sb = (grp / n_gt) * GS + j / GT;
        } else {
            const int64_t item = round * gridDim.x + blockIdx.x;
            if (item >= items) continue;
            sb = item / n_tb;
            tb = item % n_tb;
        }
        if (tb >= n_tb || sb >= n_sb) continue;
        // SNP tiles of this wave and whether each is handled by this kernel
        int64_t stl[WS];
        bool act[WS];
        bool any = false;
#pragma unroll
        for (int j = 0; j < WS; ++j) {
            stl[j] = sb * BS + (wave % GSW) * WS + j;
            act[j] = stl[j] < a.n_snp_tiles &&
                     (a.want_flag < 0 || a.tile_flags[stl[j]] == a.want_flag);
            any = any || act[j];
        }
        if (!__syncthreads_or(any)) continue;   // block-uniform skip

        // LDS-DMA copies: the k-th round of an item fetches chunk
        // min(k, nchunks - 1) into slot k % R, this wave's FPW fragments,
        // each 64 lanes x 16 bytes, contiguous in global memory and in the
        // slot.  Issued from inline assembly so
        // that the compiler does not wait for every copy in flight before
        // reading the ring; the waits below are exact.
        // The wave's FPW copies per chunk: per-lane source pointers at the
        // item's first chunk, advanced by a fixed stride per chunk (up to the
        // last chunk, which the copies past the end repeat), so that a chunk
        // costs one 64-bit add per copy instead of the address arithmetic.
        // (the codes shape copies the B side straight from the packed
        // genotype rows: lane l takes 16 codes of SNP l % 32 of the tile, the
        // first or second half of the chunk's samples per k-step part)
        auto copy_of = [&](int i) { return SPREAD ? wave + NW * i : wave * FPW + i; };
        const uint8_t* cp[FPW];
        int cstride[FPW];                              // bytes per chunk
#pragma unroll
        for (int i = 0; i < FPW; ++i) {
            const int f = copy_of(i);
            if (f < NFA) {
                const int p = f / (BT * KC), r = f % (BT * KC);
                const int tt = r / KC, kk = r % KC;
                const int64_t tile = tb * BT + tt;
                cp[i] = (const uint8_t*)((p ? Ah : A) + (tile * KS + kk) * kWave + lane);
                cstride[i] = KC * kWave * 16;
            } else if constexpr (CODES) {
                const int g = f < NF ? f - NFA : 0;
                const int s2 = g / SH::CPT, part = g % SH::CPT;
                const int64_t m = (sb * BS + s2) * kTile + (lane & 31);
                cp[i] = (const uint8_t*)a.G + m * (int64_t)a.gstride + part * 32 +
                        16 * (lane >> 5);
                cstride[i] = KC * T_::kps;
            } else {
                const int g = f < NF ? f - NFA : 0;
                const int s2 = g / (KC * NC), r = g % (KC * NC);
                const int kk = r / NC, c = r % NC;
                const int64_t st = sb * BS + s2;
                cp[i] = (const uint8_t*)(Bf + ((st * KS + kk) * NC + c) * kWave + lane);
                cstride[i] = KC * NC * kWave * 16;
            }
        }
        int n_issued = 0;                              // chunks issued for this item
        auto issue_next = [&]() {
            const uint32_t sbase = ring_lds + (uint32_t)((n_issued % R) * NF * kWave * 16);
#pragma unroll
            for (int i = 0; i < FPW; ++i) {
                const int f = copy_of(i);
                if (SPREAD && f >= NF) continue;       // uniform per wave
                const uint32_t dst = sbase + (uint32_t)(f * kWave * 16);
                asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                             :
                             : "s"(__builtin_amdgcn_readfirstlane(dst)), "v"(cp[i])
                             : "memory");
            }
            if (n_issued < nchunks - 1) {
#pragma unroll
                for (int i = 0; i < FPW; ++i) cp[i] += cstride[i];
            }
            ++n_issued;
        };
        // the item's first k-step starts its accumulators from zero (an
        // MFMA with a zero C operand: no clearing of 64 to 192 registers per
        // item), hence the first chunk's body separately
        acc_t acc[NP][WT][WS][NC];

        // every wave is done reading the ring of the previous item
        __builtin_amdgcn_s_waitcnt(0);
        block_barrier();
#pragma unroll
        for (int d = 0; d < D; ++d) issue_next();
        auto chunk = [&](int ch, auto first_c) {
            constexpr bool FIRST = decltype(first_c)::value;
            // this wave's copies of chunk ch have landed (the D - 1 younger
            // chunks may still be in flight); the barrier publishes every
            // wave's copies and certifies that chunk ch - 1, whose slot the
            // next copy reuses, has been read by all waves
            // vmcnt: low four bits in [3:0], high two in [15:14]; no wait on
            // the export and LDS/scalar counters
            __builtin_amdgcn_s_waitcnt((kWaitVm & 0xF) | ((kWaitVm >> 4) << 14) | (0x7 << 4) |
                                       (0xF << 8));
            block_barrier();
            issue_next();
            const int buf = ch % R;
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                frag fa[NP][WT], fb[WS][NC];
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int ti = 0; ti < WT; ++ti)
                        fa[p][ti] = s_buf[buf][p * BT * KC + ((wave / GSW) * WT + ti) * KC + kk][lane];
                if constexpr (CODES) {
                    // indicator columns of classes 1 and 2 from this lane's codes
                    // of the k-step
                    const uint8_t* cb = (const uint8_t*)&s_buf[buf][NFA + (wave % GSW) * SH::CPT][0];
                    if constexpr (E == F16) {
                        // samples 8 (lane / 32) .. + 7 of k-step kk: copy lane
                        // l % 32 + 32 kk, bytes 8 (lane / 32) .. + 7
                        const uint2 w = *(const uint2*)(cb + ((lane & 31) + 32 * kk) * 16 +
                                                        8 * (lane >> 5));
                        uint32_t sel[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) sel[q] = f16_ind_sel(q < 2 ? w.x : w.y, 2 * (q & 1));
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            const int k = FORM == MISS3 ? c : c + 1;
                            const uint4 o = make_uint4(f16_ind(sel[0], k), f16_ind(sel[1], k),
                                                       f16_ind(sel[2], k), f16_ind(sel[3], k));
                            fb[0][c] = __builtin_bit_cast(frag, o);
                        }
                    } else {
                        // samples 16 (lane / 32) .. + 15 of k-step kk: part kk,
                        // this lane's 16 bytes
                        const uint4 w = *(const uint4*)(cb + kk * kWave * 16 + lane * 16);
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            const int k = FORM == MISS3 ? c : c + 1;
                            const uint4 o = make_uint4(i8_ind(w.x, k), i8_ind(w.y, k),
                                                       i8_ind(w.z, k), i8_ind(w.w, k));
                            fb[0][c] = __builtin_bit_cast(frag, o);
                        }
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < WS; ++j)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            fb[j][c] = s_buf[buf][NFA + ((wave % GSW) * WS + j) * KC * NC + kk * NC + c][lane];
                }
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                        for (int j = 0; j < WS; ++j)
#pragma unroll
                            for (int c = 0; c < NC; ++c)
                                acc[p][ti][j][c] = T_::mma(fa[p][ti], fb[j][c],
                                                           FIRST && kk == 0 ? acc_t{} : acc[p][ti][j][c]);
            }
        };
        chunk(0, std::true_type{});
        for (int ch = 1; ch < nchunks; ++ch) chunk(ch, std::false_type{});
        // the clamped copies past the last chunk are still landing; with the
        // re-rank scratch in the ring, every wave's copies must have landed
        __builtin_amdgcn_s_waitcnt(0);
        if constexpr (QUEUE) block_barrier();

        // epilogue over the wave's 2 x WS output tiles (compile-time indices
        // throughout: see static_for)
        static_for<WS>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if (!act[j]) return;
            const int64_t m = stl[j] * kTile + (lane & 31);
            const SnpInfo inf = gload(a.info + m);
            const LaneK lk = lane_constants(inf, a.K, a.inv_hc);
            static_for<WT>([&](auto tic) {
                constexpr int ti = decltype(tic)::value;
                const int64_t tt = tb * BT + (wave / GSW) * WT + ti;
                if (tt >= n_tiles) return;
                const int64_t rb = tt * kTile + 4 * (lane >> 5);
                auto colv = [&](auto cc, auto rc) -> float {
                    constexpr int c = decltype(cc)::value, r = decltype(rc)::value;
                    if constexpr (SPLIT)
                        return (float)(128 * acc[1][ti][j][c][r] + acc[0][ti][j][c][r]);
                    else
                        return T_::val(acc[0][ti][j][c], r);
                };
                using C0 = std::integral_constant<int, 0>;
                using C1 = std::integral_constant<int, 1>;
                using CL = std::integral_constant<int, NC - 1>;
                if constexpr (MODE == SCREEN) {
                    const float th = cload(a.theta + tt);
                    // the missing-genotype form in eight-wave blocks: the rows
                    // with a passing pair as a mask in the same pass (most of
                    // its tiles have one); the others: the largest value
                    uint32_t pm = 0;
                    float gmax = -__builtin_inff();
                    static_for<16>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        const float sv = screen_value<FORM>(lk, th, colv(C0{}, rc), colv(C1{}, rc),
                                                            NC == 3 ? colv(CL{}, rc) : 0.0f);
                        if constexpr (QUEUE && V == 3) pm |= sv > 0.0f ? (1u << r) : 0u;
                        else gmax = fmaxf(gmax, sv);
                    });
                    if constexpr (QUEUE && V == 3) {
                        if (!__any(pm != 0u)) return;
                    } else {
                        if (!__any(gmax > 0.0f)) return;
                    }
                    if constexpr (QUEUE && V == 3) {
                        // The rows with a passing pair (per lane, then over the
                        // wave), then one loop over those rows: the queue and
                        // staging code (and the drains and fallbacks inlined in
                        // it) appear once instead of once per row, a quarter of
                        // the instructions (K = 1000: 17.6 -> 16.3 ms).  In the
                        // four-wave tiles the extra mask work outweighs it
                        // (K = 233: 9.1 -> 10.3 ms), so they keep the unrolled
                        // rows.
                        const uint32_t qm = lk.miss ? pm : 0u, cm = lk.miss ? 0u : pm;
                        uint32_t rows = pm;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) rows |= (uint32_t)__shfl_xor((int)rows, o, 64);
                        rows = __builtin_amdgcn_readfirstlane(rows);
                        while (rows) {
                            const int r = __builtin_ctz(rows);      // uniform
                            rows &= rows - 1u;
                            const int64_t row = rb + 8 * (r >> 2) + (r & 3);
                            // the row's column values, selected with compile-time
                            // register indices
                            float v1 = 0.0f, v2 = 0.0f;
                            static_for<16>([&](auto rc) {
                                constexpr int rr = decltype(rc)::value;
                                if (r == rr) {
                                    v1 = colv(C1{}, rc);
                                    v2 = colv(CL{}, rc);
                                }
                            });
                            const bool qpush = (qm >> r) & 1u;
                            const unsigned long long msk = __ballot(qpush);
                            if (msk) {
                                if (qn + 64 > kQueueCap) drain<MODE>(a, queue, qn, qbuf, lane);
                                const unsigned long long lt =
                                    (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                                if (qpush)
                                    queue[qn + __popcll(msk & lt)] =
                                        make_int4((int)row, (int)m, (int)v1, (int)v2);
                                qn += __popcll(msk);
                            }
                            const bool cand = (cm >> r) & 1u;
                            stage_candidates(a, &s_args, stage, sn, lane, cand, row, m, v1, v2, kCandPlain);
                        }
                    } else {
                    static_for<16>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        const int64_t row = rb + 8 * (r >> 2) + (r & 3);
                        const float v0 = colv(C0{}, rc), v1 = colv(C1{}, rc);
                        const float v2 = NC == 3 ? colv(CL{}, rc) : 0.0f;
                        bool cand = screen_value<FORM>(lk, th, v0, v1, v2) > 0.0f;
                        if constexpr (QUEUE) {
                            const bool qpush = cand && lk.miss;
                            const unsigned long long msk = __ballot(qpush);
                            if (msk) {
                                if (qn + 64 > kQueueCap) drain<MODE>(a, queue, qn, qbuf, lane);
                                const unsigned long long lt =
                                    (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                                if (qpush)
                                    queue[qn + __popcll(msk & lt)] =
                                        make_int4((int)row, (int)m, (int)v1, (int)v2);
                                qn += __popcll(msk);
                            }
                            cand = cand && !lk.miss;
                        }
                        if constexpr (FORM == DIAG)
                            stage_candidates(a, &s_args, stage, sn, lane, cand, row, m, v0, v1, 0u);
                        else if constexpr (FORM == PLAIN)
                            stage_candidates(a, &s_args, stage, sn, lane, cand, row, m, v0, v1, kCandPlain);
                        else
                            stage_candidates(a, &s_args, stage, sn, lane, cand, row, m, v1, v2, kCandPlain);
                    });
                    }
                    // the queue carries over to the next tile (drained when
                    // nearly full and at the end of the kernel)
                } else if constexpr (FORM == MISS3) {
                    static_for<16>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        const int64_t row = rb + 8 * (r >> 2) + (r & 3);
                        const int64_t v = a.row_v[row];
                        bool want = v >= 0 && m < a.M;
                        const bool qpush = want && lk.miss;
                        const unsigned long long msk = __ballot(qpush);
                        if (msk) {
                            if (qn + 64 > kQueueCap) drain<MODE>(a, queue, qn, qbuf, lane);
                            const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                            if (qpush) queue[qn + __popcll(msk & lt)] = make_int4((int)row, (int)m, 0, 0);
                            qn += __popcll(msk);
                        }
                        want = want && !lk.miss;
                        if (want) {
                            const int64_t D0 = (int64_t)colv(C0{}, rc), D1 = (int64_t)colv(C1{}, rc),
                                          D2 = (int64_t)colv(CL{}, rc);
                            const double H = exact_H(D0, D1, D2, inf.n0, inf.n1, inf.n2, a.K,
                                                     a.tiesum[v % a.T], snp_df(inf));
                            const int64_t k1 = a.K + 1;
                            emit_full<MODE>(a, v, m, H, snp_df(inf), D0 + inf.n0 * k1,
                                            D1 + inf.n1 * k1, D2 + inf.n2 * k1);
                        }
                    });
                    if (qn) drain<MODE>(a, queue, qn, qbuf, lane);
                }
            });
        });
    }
    if constexpr (QUEUE && MODE == SCREEN) {
        if (qn) drain<MODE>(a, queue, qn, qbuf, lane);
    }
    if constexpr (MODE == SCREEN) flush_stage(a, &s_args, stage, sn, lane);
}

// B fragments of every SNP tile: column c of SNP m at sample k is
// coef(c, code(m, k)) for the form's coefficients, 0 at missing samples.
template <int E, int FORM>
__global__ __launch_bounds__(256) void expand_columns(const int8_t* __restrict__ G, int gstride,
                                                      const SnpInfo* __restrict__ info,
                                                      int64_t n_tiles_pad, int KS, void* Bf) {
    using T_ = ET<E>;
    using frag = typename T_::frag;
    constexpr int NC = FORM == MISS3 ? 3 : 2;
    frag* out = (frag*)Bf;
    const int64_t total = n_tiles_pad * KS * NC * kWave;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(i % kWave);
        int64_t q = i / kWave;
        const int c = (int)(q % NC);
        q /= NC;
        const int s = (int)(q % KS);
        const int64_t st = q / KS;
        const int64_t m = st * kTile + (lane & 31);
        const SnpInfo inf = info[m];
        float cv[3];
        if constexpr (FORM == DIAG) {
            if (c == 0) { cv[0] = 0.f; cv[1] = inf.cy1; cv[2] = inf.cy2; }
            else { cv[0] = 0.f; cv[1] = 0.f; cv[2] = 1.f; }
        } else if constexpr (FORM == PLAIN) {
            cv[0] = 0.f; cv[1] = c == 0 ? 1.f : 0.f; cv[2] = c == 1 ? 1.f : 0.f;
        } else {
            cv[0] = c == 0 ? 1.f : 0.f; cv[1] = c == 1 ? 1.f : 0.f; cv[2] = c == 2 ? 1.f : 0.f;
        }
        int8_t codes[T_::per_lane];
        const int8_t* src = G + m * (int64_t)gstride + s * T_::kps + T_::per_lane * (lane >> 5);
#pragma unroll
        for (int e = 0; e < T_::per_lane; ++e) codes[e] = src[e];
        out[i] = T_::make(codes, cv[0], cv[1], cv[2]);
    }
}

template <int E, int FORM, int MODE, bool SPLIT, int V, int KCX = 2>
inline hipError_t launch_tiled_v(const ScanArgs& a, const TiledArgs& ta, int grid, hipStream_t st) {
    using SH = TiledShape<FORM, SPLIT, V, KCX>;
    const size_t lds = FORM == MISS3 && !tiled_scratch_in_ring<FORM, SPLIT, V, KCX>(a.K)
                           ? (size_t)SH::NW * coop_lds_entries(a.K) * sizeof(int16_t) : 0;
    auto kern = scan_tiled<E, FORM, MODE, SPLIT, V, KCX>;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, SH::NW * 64, lds) != hipSuccess ||
        occ < 1)
        occ = 1;
    int dev = 0, n_cu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t resident = (int64_t)n_cu * occ;
    int g = (int)(grid < resident ? grid : resident);
    hipLaunchKernelGGL(kern, dim3(g), dim3(SH::NW * 64), lds, st, a, ta);
    return hipGetLastError();
}

// The codes shapes (2, 3) cover the complete-SNP screen (the host runs PLAIN
// in place of DIAG there); the missing-genotype form reads the codes in the
// fp16 eight-wave blocks of shape 3 and keeps expanded columns otherwise
// (the host runs it as shape 1 under shape 2).  The fp16 eight-wave blocks
// take four k-steps per ring chunk when the k-step count allows (half the
// block barriers and waits per MFMA).
template <int E, int FORM, int MODE, bool SPLIT>
inline hipError_t launch_tiled(const ScanArgs& a, const TiledArgs& ta, int grid, hipStream_t st) {
    if constexpr (FORM == PLAIN) {
        if constexpr (!SPLIT)
            if (ta.shape == 3 && ta.ks % 4 == 0)
                return launch_tiled_v<E, FORM, MODE, SPLIT, 3, 4>(a, ta, grid, st);
        if (ta.shape == 3) return launch_tiled_v<E, FORM, MODE, SPLIT, 3>(a, ta, grid, st);
        if (ta.shape == 2) return launch_tiled_v<E, FORM, MODE, SPLIT, 2>(a, ta, grid, st);
    } else if constexpr (FORM == MISS3) {
        if constexpr (!SPLIT)
            if (ta.shape == 3 && ta.ks % 4 == 0)
                return launch_tiled_v<E, FORM, MODE, SPLIT, 3, 4>(a, ta, grid, st);
        if (ta.shape == 3) return launch_tiled_v<E, FORM, MODE, SPLIT, 3>(a, ta, grid, st);
    }
    if (ta.shape == 0) return launch_tiled_v<E, FORM, MODE, SPLIT, 0>(a, ta, grid, st);
    return launch_tiled_v<E, FORM, MODE, SPLIT, 1>(a, ta, grid, st);
}

}  // namespace kx
