// api.cpp -- the C ABI of include/krux.h: argument checks, context scratch
// memory, and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/krux.h"
#include "kx_common.h"
#include "kx_host.h"
#include "kx_args.h"

namespace {

enum Slot {
    S_PACKED, S_INFO, S_FLAGS, S_MPOS, S_A, S_THETA, S_ROWV, S_A2, S_THETA2, S_ROWV2,
    S_LIST_A, S_LIST_B, S_COUNT_A, S_COUNT_B, S_MINP, S_STAGE, S_NHITS, S_KEYS, S_IDX,
    S_SORT_TMP, S_F64_R, S_F64_I, S_F64_S, S_COUNT_PREV, S_CAND, S_NCAND, S_MCAND, S_NMCAND,
    S_TUNE_HITS, S_TUNE_N,
    S_AH, S_AH2, S_BF, S_BF3, S_NAN_FLAG, S_NAN_LIST, S_NAN_N,
    S_G_KEYS, S_G_QMASK, S_G_SNPS, S_G_SAMPLES, S_G_EXPR, S_G_R, S_G_TS, S_G_GENO, S_G_STAGE,
    S_G_CNT, S_G_MINP, S_G_PHITS, S_G_PN, S_G_PMINP, S_MINFO, S_MFLAG,
    S_N_SLOTS
};

struct Buf {
    void* p = nullptr;
    size_t n = 0;
};

}  // namespace

// Launch configuration chosen by krux_autotune for one (K, precision).
// -1 / 0: the built-in rule.
struct Tuning {
    int ring = -1;       // SNP-stationary kernel: 0 register double buffer, 1 LDS ring,
                         // 2 LDS ring without the two-tile pipeline (3 waves per SIMD),
                         // 3 LDS ring, two tiles per step, 4 LDS ring with two SNP
                         // tiles per wave
    int range_kb = 0;    // SNP-stationary kernel: trait-range operand budget
    int grouped = -1;    // tiled kernel: XCD-grouped item order
    int shape = -1;      // tiled kernel: tile shape (0 wide, 1 two waves per SIMD, 2 the same
                         // with the B side from the packed genotype codes, 3 codes with
                         // eight-wave blocks)
    double ms = 0.0;     // time of the tuning run
};

struct krux_ctx {
    int device = 0;
    int n_cu = 256;
    char arch[32] = {0};
    std::map<std::pair<int, int>, Tuning> tuned;   // (K, precision) -> configuration
    std::string err;
    Buf bufs[S_N_SLOTS];
    void* blas = nullptr;   // rocBLAS handle of the fp64 comparator (created on first use)
    bool timing = false;    // krux_timer_start .. krux_timer_read
    std::vector<hipEvent_t> ev;   // start/stop pairs of timed launches
    size_t ev_used = 0;
    // limits on the two screened-pair buffers (krux_set_pair_buffer_limits; 0: none)
    int64_t cand_limit = 0, mcand_limit = 0;
    // graph capture: `capturing` holds while a call enqueues into a stream that
    // is being captured (no buffer may grow then); once anything has been
    // captured, a growing buffer keeps its old allocation in `retired` (freed by
    // krux_destroy) because a graph may still read it
    bool capturing = false;
    bool captured = false;
    std::vector<void*> retired;
    // krux_test_noalloc: the slots are carved from the device's static
    // scratch array instead of allocated.  arena 1 = sizing pass (offsets are
    // assigned, nothing is launched: every HIP call is skipped), 2 = carving
    // pass (the same offsets, kernels launched)
    int arena = 0;
    uint8_t* arena_base = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    size_t arena_off[S_N_SLOTS] = {}, arena_len[S_N_SLOTS] = {};
    void* noalloc_scratch = nullptr;   // this device's static scratch (hipGetSymbolAddress)
};

// Device scratch of krux_test_noalloc: one copy per GPU, held until the
// process ends.  Host code never uses this name as an address: krux_create
// looks up each device's copy with hipGetSymbolAddress and keeps the pointer.
static __device__ __align__(256) uint8_t scratch[KRUX_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};     // per device, from hipGetSymbolAddress
hipError_t g_scratch_err[kMaxDevices] = {};

// Address of `scratch` on `device` (current), looked up once per device.
void* scratch_address(int device, hipError_t* err) {
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) g_scratch_err[device] = e != hipSuccess ? e : hipErrorUnknown;
        else g_scratch_ptr[device] = ptr;
    }
    *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}

std::string g_err_null = "no error";
thread_local std::string g_err_noctx;

krux_status fail(krux_ctx* c, krux_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_err_noctx = buf;
    return s;
}

// A HIP call (a kernel launch, an event, a copy) with its error returned as
// KRUX_ERR_HIP.  Skipped in the sizing pass of krux_test_noalloc, which runs
// the host side of a call only to learn its scratch layout.
#define HIP_TRY(c, expr)                                                                   \
    do {                                                                                   \
        if ((c)->arena != 1) {                                                             \
            hipError_t e_ = (expr);                                                        \
            if (e_ != hipSuccess)                                                          \
                return fail(c, KRUX_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
        }                                                                                  \
    } while (0)

// Grow-only scratch buffer of the context.  Growing is refused while the
// call's stream is being captured (an allocation cannot be captured, and the
// graph would hold the old pointer); after a capture the old allocation is
// kept, not freed, so that captured graphs stay valid.
void* ws(krux_ctx* c, int slot, size_t bytes, krux_status* st) {
    Buf& b = c->bufs[slot];
    if (bytes == 0) bytes = 256;
    if (c->arena) {
        // static scratch: a slot keeps its offset for the rest of the call;
        // the same margin as an allocation below
        if (c->arena_len[slot] >= bytes) return c->arena_base + c->arena_off[slot];
        const size_t off = (c->arena_used + 255) & ~(size_t)255;
        const size_t len = bytes + bytes / 8 + 4096;
        if (c->arena == 2 && off + len > c->arena_cap) {
            *st = fail(c, KRUX_ERR_UNSUPPORTED, "the call needs more than the %zu bytes of static "
                       "scratch", c->arena_cap);
            return nullptr;
        }
        c->arena_off[slot] = off;
        c->arena_len[slot] = len;
        c->arena_used = off + len;
        return c->arena_base + off;
    }
    if (b.n >= bytes) return b.p;
    if (c->capturing) {
        *st = fail(c, KRUX_ERR_UNSUPPORTED,
                   "a scratch buffer must grow to %zu bytes while the stream is being captured: "
                   "run the same call once without capture first", bytes);
        return nullptr;
    }
    if (b.p) {
        if (c->captured) {
            c->retired.push_back(b.p);
        } else {
            (void)hipDeviceSynchronize();
            (void)hipFree(b.p);
        }
        b.p = nullptr;
        b.n = 0;
    }
    size_t want = bytes + bytes / 8 + 4096;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        *st = fail(c, KRUX_ERR_NOMEM, "device allocation of %zu bytes failed", want);
        return nullptr;
    }
    b.n = want;
    return b.p;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Start of an entry point that enqueues on `st`: notes whether the stream is
// being captured into a graph.  Calls that synchronise pass may_capture =
// false and are refused under capture.
krux_status begin_call(krux_ctx* c, hipStream_t st, bool may_capture = true) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamIsCapturing(st, &cs));
    c->capturing = cs == hipStreamCaptureStatusActive;
    if (c->capturing && !may_capture)
        return fail(c, KRUX_ERR_UNSUPPORTED, "this call synchronises its stream and cannot be captured");
    if (c->capturing) c->captured = true;
    return KRUX_OK;
}

// Entries of a screened-pair buffer after the context's limit.
int64_t pair_limit(int64_t want, int64_t limit) {
    return limit > 0 ? std::min(want, limit) : want;
}

// Capacity of the screened-pair buffer (16 B per entry).  When a scan finds
// more candidates than this, the extra ones are evaluated inside the scan.
// Candidate buffer entries: sized for about four times the expected number of
// screened pairs of a main pass (the screen level times the pair count), at
// least 2^22 and at most 2^28 (4 GiB); pairs beyond it are evaluated in the
// scan kernel itself.
int64_t candidate_capacity(int64_t rows, int64_t M, double p_screen) {
    const double want = 4.0 * (double)rows * (double)M * p_screen + (double)(1 << 20);
    return (int64_t)std::min(std::max(want, (double)(1 << 22)), (double)(1LL << 28));
}

double host_pvalue(double H, int df) {
    if (df == 1) return std::erfc(std::sqrt(H / 2.0));
    if (df == 2) return std::exp(-H / 2.0);
    return 1.0;
}

double threshold_of(double p_c, int df) {
    // largest double h >= 0 with host_pvalue(h, df) >= p_c (bisection on bits)
    uint64_t lo, hi;
    double d0 = 0.0, d1 = 4096.0;
    std::memcpy(&lo, &d0, 8);
    std::memcpy(&hi, &d1, 8);
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        double h;
        std::memcpy(&h, &mid, 8);
        if (host_pvalue(h, df) >= p_c) lo = mid; else hi = mid;
    }
    double r;
    std::memcpy(&r, &lo, 8);
    return r;
}

bool valid_p(double p) { return p > 0.0 && p <= 1.0; }

// Everything one scan needs about the genotype side.
struct SnpSide {
    int8_t* G = nullptr;
    kx::SnpInfo* info = nullptr;
    int32_t* flags = nullptr;
    int16_t* mpos = nullptr;
    int gstride = 0;
    int64_t n_snp_tiles = 0;
};

krux_status pack_snps(krux_ctx* c, const int8_t* geno, int64_t M, int64_t ld, int K, bool diag_ok,
                      int64_t row_bytes, hipStream_t st, SnpSide* out) {
    krux_status s = KRUX_OK;
    // packed rows cover every sample the kernels read (k-steps x samples per step)
    out->gstride = (int)ceil_div(std::max<int64_t>(K, row_bytes), 32) * 32;
    out->n_snp_tiles = ceil_div(M, kx::kTile);
    // rounded to whole blocks of 8 SNP tiles: the tiled kernel reads them
    int64_t m_pad = std::max<int64_t>(ceil_div(out->n_snp_tiles, 8) * 8, 8) * kx::kTile;
    out->G = (int8_t*)ws(c, S_PACKED, (size_t)m_pad * out->gstride, &s);
    out->info = (kx::SnpInfo*)ws(c, S_INFO, (size_t)m_pad * sizeof(kx::SnpInfo), &s);
    out->flags = (int32_t*)ws(c, S_FLAGS, (size_t)(m_pad / kx::kTile + 2) * 4, &s);
    out->mpos = (int16_t*)ws(c, S_MPOS, (size_t)m_pad * kx::kLaneMiss * sizeof(int16_t), &s);
    if (s != KRUX_OK) return s;
    // one wave per SNP row, enough blocks to cover every row at once (the
    // kernel is latency-bound when waves loop over many rows)
    int grid = (int)std::min<int64_t>(ceil_div(m_pad, 4), (int64_t)INT32_MAX / 4);
    HIP_TRY(c, kx_launch_pack(geno, M, ld, K, m_pad, out->gstride, diag_ok ? 1 : 0, out->G,
                              out->info, out->flags, out->mpos, std::max(grid, 1), st));
    return KRUX_OK;
}

// Operand of the rank side: fragment-ordered centred ranks.
struct RankSide {
    void* A = nullptr;
    void* A_hi = nullptr;
    float* theta = nullptr;
    int32_t* row_v = nullptr;
};

struct Variant {
    int elem;    // kx F16 / I8
    int ks;      // k-steps
    int form;    // kx DIAG / PLAIN / MISS3 of the complete-SNP kernel
    bool tiled;  // two-operand tiled GEMM (K > 128) instead of the SNP-stationary one
    bool split;  // int8 with the centred rank split into two bytes
};

// Samples one operand row spans: k-steps x samples per k-step.
int64_t row_bytes(const Variant& v) { return (int64_t)v.ks * (v.elem == kx::F16 ? 16 : 32); }

// Genotype columns in MFMA fragment order for the tiled kernel.
struct Columns {
    void* Bf = nullptr;     // complete-SNP form
    void* Bf3 = nullptr;    // three indicator columns (SNPs with missing genotypes)
};

krux_status prep_ranks(krux_ctx* c, const Variant& v, const int16_t* ranks2, const int64_t* tiesum,
                       int64_t T, int K, const int32_t* perms, const int32_t* rows,
                       const int32_t* d_nrows, int64_t n_rows, int slotA, int slotTh, int slotRv,
                       hipStream_t st, RankSide* out, int slotAh, const uint8_t* nan_flag) {
    krux_status s = KRUX_OK;
    // the tiled kernel reads whole blocks of up to 8 trait tiles
    const int64_t n_alloc = v.tiled ? ceil_div(std::max<int64_t>(n_rows, 1), 256) * 256
                                    : std::max<int64_t>(n_rows, 1);
    int64_t n_tiles = ceil_div(n_alloc, kx::kTile);
    out->A = ws(c, slotA, (size_t)n_tiles * v.ks * kx::kWave * 16, &s);
    out->A_hi = v.split ? ws(c, slotAh, (size_t)n_tiles * v.ks * kx::kWave * 16, &s) : nullptr;
    out->theta = (float*)ws(c, slotTh, (size_t)n_tiles * 4, &s);
    out->row_v = (int32_t*)ws(c, slotRv, (size_t)n_tiles * kx::kTile * 4, &s);
    if (s != KRUX_OK) return s;
    kx::PrepArgs a{};
    a.ranks2 = ranks2; a.tiesum = tiesum; a.perms = perms; a.rows = rows; a.d_nrows = d_nrows;
    a.n_rows = n_rows; a.n_alloc_rows = n_alloc; a.T = T; a.K = K; a.ks = v.ks;
    a.A = out->A; a.A_hi = out->A_hi; a.theta = out->theta; a.row_v = out->row_v;
    // the prep kernel also clears the candidate counters of the scan that follows it
    a.zero = (unsigned long long*)ws(c, S_NCAND, 256, &s);
    a.n_zero = 2;
    a.nan_flag = nan_flag;
    if (s != KRUX_OK) return s;
    int64_t total = n_tiles * v.ks * kx::kWave;
    int grid = (int)std::min<int64_t>(ceil_div(total, 256), (int64_t)c->n_cu * 16);
    HIP_TRY(c, kx_launch_prep(&a, v.elem == kx::I8 ? 1 : 0, std::max(grid, 1), st));
    return KRUX_OK;
}

// Traits with missing expression values (a rank of 0): a flag per trait for
// the operand preparation, which turns their rows into padding, and the list
// that scan_nan_traits walks after the scan.  Stream-ordered, no host sync.
struct NanSide {
    uint8_t* flag = nullptr;
    int32_t* list = nullptr;
    int32_t* n = nullptr;
};

krux_status flag_nan(krux_ctx* c, const int16_t* ranks2, int64_t T, int K, hipStream_t st,
                     NanSide* out) {
    krux_status s = KRUX_OK;
    out->flag = (uint8_t*)ws(c, S_NAN_FLAG, (size_t)std::max<int64_t>(T, 1), &s);
    out->list = (int32_t*)ws(c, S_NAN_LIST, (size_t)std::max<int64_t>(T, 1) * 4, &s);
    out->n = (int32_t*)ws(c, S_NAN_N, 256, &s);
    if (s != KRUX_OK) return s;
    HIP_TRY(c, kx_launch_fill_i32(out->n, 1, 0, st));
    if (T > 0) {
        const int grid = (int)std::min<int64_t>(ceil_div(T, 4), (int64_t)c->n_cu * 8);
        HIP_TRY(c, kx_launch_flag_nan(ranks2, T, K, out->flag, out->list, out->n, grid, st));
    }
    return KRUX_OK;
}

// Exact evaluation of every pair of the flagged traits (P permutations).
krux_status run_nan_traits(krux_ctx* c, const kx::ScanArgs& a, const NanSide& ns, int P,
                           int mode, hipStream_t st) {
    if (a.M <= 0) return KRUX_OK;
    HIP_TRY(c, kx_launch_nan_traits(&a, ns.list, ns.n, P, mode, c->n_cu * 8, st));
    return KRUX_OK;
}

// Kernel variant per (K, precision).  The SNP-stationary kernel keeps a SNP
// tile's columns in registers (K <= 128); larger K uses the tiled kernel.
// The DIAG form's integer column coefficients keep the fp32 accumulation
// exact while K^3/4 < 2^24 (K <= 406); beyond that the plain indicators.
krux_status choose_variant(krux_ctx* c, int K, int precision, Variant* v) {
    if (precision == KRUX_PREC_FP16) {
        if (K <= 128) {
            *v = {kx::F16, (int)ceil_div(K, 16), kx::DIAG, false, false};
        } else {
            *v = {kx::F16, (int)ceil_div(ceil_div(K, 16), 2) * 2, K <= 400 ? kx::DIAG : kx::PLAIN,
                  true, false};
        }
        return KRUX_OK;
    }
    if (precision == KRUX_PREC_INT8) {
        if (K <= 127) {
            *v = {kx::I8, (int)ceil_div(K, 32), kx::DIAG, false, false};
        } else {
            *v = {kx::I8, (int)ceil_div(ceil_div(K, 32), 2) * 2, kx::PLAIN, true, true};
        }
        return KRUX_OK;
    }
    return fail(c, KRUX_ERR_UNSUPPORTED, "precision %d not handled by the MFMA path", precision);
}

// Tile shape of the tiled kernel for (K, precision): the tuned one, else,
// where the complete-SNP screen is PLAIN (K > 400), the B side from the
// packed codes, with eight-wave blocks in fp16 (shape 3) and in int8 from
// K = 768 (shape 2, four-wave blocks, below), and shape 1 with the DIAG
// screen up to K = 400.  Complete-SNP kernel times of one A/B run, shapes
// 1 / 2 / 3: K = 500 fp16 3.87 / 3.77 / 3.53 ms, int8 4.14 / 4.04 / 4.19
// ms, K = 1000 fp16 8.66 / 7.27 / 6.27 ms, K = 200 fp16 1.90 / 1.97 / 2.09
// ms.  The missing-genotype screen (shape 1 against 3): K = 1000 fp16 20.9
// -> 17.9 ms and int8 12.3 -> 9.5 ms, K = 512 18.0 -> 16.9 ms, K = 380
// 5.2 -> 5.6 ms.
int tile_shape_for(krux_ctx* c, int K, int precision) {
    auto it = c->tuned.find({K, precision});
    const int t = it != c->tuned.end() ? it->second.shape : -1;
    if (t >= 0) return t;
    if (K <= 400) return 1;
    return precision == KRUX_PREC_INT8 && K < 768 ? 2 : 3;
}

// Expanded B columns of the tiled kernel; with the codes shapes (2, 3) the
// complete-SNP screen reads the packed genotype rows, and only the
// missing-genotype columns are built (none for fp16 in shape 3, whose
// missing-genotype form reads the codes too).
krux_status expand_columns(krux_ctx* c, const Variant& v, const SnpSide& sn, int shape,
                           hipStream_t st, Columns* out) {
    if (!v.tiled) return KRUX_OK;
    krux_status s = KRUX_OK;
    const int64_t n_pad = ceil_div(std::max<int64_t>(sn.n_snp_tiles, 1), 4) * 4;
    const size_t per_col = (size_t)n_pad * v.ks * kx::kWave * 16;
    // fp16 in eight-wave blocks: the missing-genotype form reads the codes too
    const bool miss_codes = shape == 3 && v.elem == kx::F16;
    if (shape < 2) out->Bf = ws(c, S_BF, per_col * 2, &s);
    if (!miss_codes) out->Bf3 = ws(c, S_BF3, per_col * 3, &s);
    if (s != KRUX_OK) return s;
    int grid = (int)std::min<int64_t>(ceil_div(n_pad * v.ks * 3 * kx::kWave, 256), (int64_t)c->n_cu * 16);
    if (v.elem == kx::F16) {
        if (shape < 2)
            HIP_TRY(c, kx_launch_expand_f16(sn.G, sn.gstride, sn.info, n_pad, v.ks, v.form, out->Bf, grid, st));
        if (!miss_codes)
            HIP_TRY(c, kx_launch_expand_f16(sn.G, sn.gstride, sn.info, n_pad, v.ks, kx::MISS3, out->Bf3, grid, st));
    } else {
        if (shape < 2)
            HIP_TRY(c, kx_launch_expand_i8(sn.G, sn.gstride, sn.info, n_pad, v.ks, v.form, out->Bf, grid, st));
        HIP_TRY(c, kx_launch_expand_i8(sn.G, sn.gstride, sn.info, n_pad, v.ks, kx::MISS3, out->Bf3, grid, st));
    }
    return KRUX_OK;
}

// One scan launch: the kernel family follows the variant.
krux_status launch_scan(krux_ctx* c, const kx::ScanArgs& a, const Variant& v, const Columns& col,
                        const void* A_hi, int form, int mode, int grid, hipStream_t st) {
    if (!v.tiled) {
        HIP_TRY(c, kx_launch_scan(&a, v.elem, v.ks, form, mode, grid, st));
        return KRUX_OK;
    }
    // the codes shapes build indicator columns only: PLAIN in place of DIAG
    if (a.tile_shape >= 2 && form == kx::DIAG) form = kx::PLAIN;
    kx::TiledArgs ta{};
    ta.Bf = form == kx::MISS3 ? col.Bf3 : col.Bf;
    ta.A_hi = A_hi;
    ta.ks = v.ks;
    ta.shape = a.tile_shape;
    // the missing-genotype form: shape 2 runs it in the four-wave tiles of
    // shape 1 (expanded columns), shape 3 in eight-wave blocks (from the codes
    // in fp16)
    if (form == kx::MISS3 && ta.shape == 2) ta.shape = 1;
    if (v.elem == kx::F16) HIP_TRY(c, kx_launch_tiled_f16(&a, &ta, form, mode, grid, st));
    else HIP_TRY(c, kx_launch_tiled_i8(&a, &ta, form, mode, grid, st));
    return KRUX_OK;
}

// Trait tiles per work item of the SNP-stationary kernel.  Concurrent blocks
// walk consecutive SNP blocks of one trait range, so the operand slices of
// the ranges in flight are what every XCD's L2 (4 MB) must hold: about
// 1 + resident blocks / SNP blocks ranges are in flight, and together they
// get ~2.5 MB.  At least two ranges, so that the persistent grid's last
// round is short.
int trait_range(const Variant& v, int64_t n_rows, int64_t n_snp_tiles, int n_cu,
                int budget_kb = 2560) {
    const int64_t n_tiles = std::max<int64_t>(ceil_div(n_rows, kx::kTile), 1);
    const int64_t tile_bytes = (int64_t)v.ks * kx::kWave * 16;
    const int64_t snp_blocks = std::max<int64_t>(ceil_div(n_snp_tiles, kx::kWavesPerBlock), 1);
    const double in_flight = 1.0 + 2.0 * n_cu / (double)snp_blocks;   // 2 blocks per CU
    const int64_t budget = std::max<int64_t>((int64_t)((double)budget_kb * 1024.0 / in_flight),
                                             64 << 10);
    int64_t ranges = ceil_div(n_tiles * tile_bytes, budget);
    if (n_tiles >= 128) ranges = std::max<int64_t>(ranges, 2);
    const int64_t tpr = ceil_div(ceil_div(n_tiles, ranges), 2) * 2;
    return (int)std::min<int64_t>(tpr, 1 << 20);
}

// Pipeline of the SNP-stationary screen kernel: the A tiles come through
// the block's LDS ring (one L2 read per block instead of one per wave), one
// tile at a time with three waves per SIMD (2), which on the paper-scale
// workload beats the register double buffer (0) by ~6 % and the two-tile
// pipelined ring at two waves per SIMD (1) by ~7 %.
int use_ring(const Variant& v, int64_t n_rows) {
    (void)n_rows;
    return v.tiled ? 0 : 2;
}

// Launch parameters of a scan: the autotuned configuration for (K,
// precision) if krux_autotune or krux_load_tuning provided one, else the rules
// above.
void apply_tuning(krux_ctx* c, int K, int precision, const Variant& v, int64_t n_rows,
                  int64_t n_snp_tiles, kx::ScanArgs* a) {
    Tuning t;
    auto it = c->tuned.find({K, precision});
    if (it != c->tuned.end()) t = it->second;
    a->tiles_per_range = trait_range(v, n_rows, n_snp_tiles, c->n_cu,
                                     t.range_kb > 0 ? t.range_kb : 2560);
    a->ring = t.ring >= 0 ? t.ring : use_ring(v, n_rows);
    // XCD-grouped item order: K = 500 4.27 ms against 5.11 ms row-major,
    // K = 200 2.28 against 2.37, within 1 % elsewhere
    a->group_items = t.grouped >= 0 ? t.grouped : 1;
    // two waves per SIMD (shape 1) measured 25-35 % faster than the wide
    // tiles at K = 200 and 500, fp16 and int8
    a->tile_shape = tile_shape_for(c, K, precision);
}

// Work items of one scan launch (an upper bound; the kernels stop early).
int64_t scan_items(const Variant& v, int64_t n_rows, int64_t n_snp_tiles, int tiles_per_range) {
    const int64_t n_tiles = ceil_div(n_rows, kx::kTile);
    if (v.tiled) return ceil_div(n_tiles, 4) * ceil_div(n_snp_tiles, 2);
    return ceil_div(n_tiles, tiles_per_range) * ceil_div(n_snp_tiles, kx::kWavesPerBlock);
}

void set_levels(kx::ScanArgs* a, const double* p_cs, int n) {
    a->n_lev = n;
    for (int l = 0; l < kx::kMaxLevels; ++l) {
        double pc = l < n ? p_cs[l] : 1.0;
        a->hc[l][0] = threshold_of(pc, 1);
        a->hc[l][1] = threshold_of(pc, 2);
    }
}

void set_screen(kx::ScanArgs* a, double p_screen) {
    a->inv_hc[0] = 0.0f;
    a->hc_screen[0] = 0.0;
    for (int df = 1; df <= 2; ++df) {
        double h = threshold_of(p_screen, df);
        a->inv_hc[df] = (float)(1.0 / h);
        a->hc_screen[df] = h;
    }
}

// Two launches cover every SNP tile: complete tiles on the fast form, tiles
// with a missing genotype on the MISS3 form (each kernel skips the others).
krux_status run_screen(krux_ctx* c, kx::ScanArgs a, const Variant& v, const Columns& col,
                       const void* A_hi, hipStream_t st, int64_t n_rows_max, bool timed = false) {
    int64_t items = scan_items(v, n_rows_max, a.n_snp_tiles, a.tiles_per_range);
    if (items <= 0) return KRUX_OK;
    int grid = (int)std::min<int64_t>(items, (int64_t)INT32_MAX);
    // screened pairs go to the candidate buffer and are evaluated exactly after the scan
    krux_status s = KRUX_OK;
    a.cand = (uint4*)ws(c, S_CAND, (size_t)a.cand_cap * sizeof(uint4), &s);
    a.n_cand = (unsigned long long*)ws(c, S_NCAND, 256, &s);
    // pairs of SNPs with missing genotypes that pass the bound: up to 1/16 of
    // the pairs, at most 2^27 entries (2 GB of the 288 GB); the rest are
    // evaluated in the scan kernel itself, which is several times slower (at
    // the 16/M-64/M screen level of a min-p run, a few percent of the pairs
    // pass)
    a.mcand_cap = pair_limit(
        std::min<int64_t>(std::max<int64_t>(n_rows_max * a.M / 16, 1 << 16), 1LL << 27),
        c->mcand_limit);
    a.mcand = (int4*)ws(c, S_MCAND, (size_t)a.mcand_cap * sizeof(int4), &s);
    a.n_mcand = a.n_cand + 1;      // both counters were cleared by the preceding prep kernel
    if (s != KRUX_OK) return s;
    a.want_flag = 0;
    // timed: one event pair around each of the two scan launches
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (timed && c->timing) {
        while (c->ev.size() < c->ev_used + 4) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
        for (int i = 0; i < 4; ++i) ev[i] = c->ev[c->ev_used + i];
        c->ev_used += 4;
    }
    if (ev[0]) HIP_TRY(c, hipEventRecord(ev[0], st));
    if ((s = launch_scan(c, a, v, col, A_hi, v.form, kx::SCREEN, grid, st)) != KRUX_OK) return s;
    if (ev[1]) HIP_TRY(c, hipEventRecord(ev[1], st));
    a.want_flag = 1;
    if (ev[2]) HIP_TRY(c, hipEventRecord(ev[2], st));
    if ((s = launch_scan(c, a, v, col, A_hi, kx::MISS3, kx::SCREEN, grid, st)) != KRUX_OK) return s;
    if (ev[3]) HIP_TRY(c, hipEventRecord(ev[3], st));
    HIP_TRY(c, kx_launch_exact(&a, c->n_cu * 8, st));
    return KRUX_OK;
}

// Main-pass screen level when per-row minima are wanted.  The chi-square
// p-values of the test are conservative in the far tail (a trait's smallest p
// over M null SNPs is typically several times 1/M), so the level is a
// multiple of 1/M: then nearly every row has an exactly evaluated pair below
// it and the fix-up passes see few rows, while the pairs staged and evaluated
// grow with the level.  At 8/M a quarter of the rows stayed open at K = 48
// and an eighth at K = 102; at K = 102, 16/M against 64/M took the
// 200-permutation step from 156 to 140 ms and the paper-scale hit step from
// 3.44 to 3.39 ms (8/M: 155 and 4.13 ms).  Below 96 samples, where the tail
// is coarser, the level stays 64/M.
double screen_level_for_min_p(double p_c, int64_t M, int K) {
    const double per_m = K >= 96 ? 16.0 : 64.0;
    return std::max(p_c, std::min(1.0, per_m / (double)std::max<int64_t>(M, 1)));
}

int bit_length(int64_t v) {
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) <= v) ++b;
    return b;
}

// The staged hits (appended in any order) sorted by (row, snp) into the
// caller's buffer; *n_hits receives the true count.  Rows are below `rows`,
// SNP numbers below `snp_end`.
krux_status sort_stage(krux_ctx* c, const kx::HitRec* stage, const unsigned long long* nh,
                       int64_t cap, krux_hit* hits, int64_t* n_hits, int64_t rows,
                       int64_t snp_end, hipStream_t st) {
    krux_status s = KRUX_OK;
    size_t tmp_bytes = kx_sort_tmp_bytes(std::max<int64_t>(cap, 1));
    unsigned long long* keys = (unsigned long long*)ws(c, S_KEYS, (size_t)std::max<int64_t>(cap, 1) * 16, &s);
    uint32_t* idx = (uint32_t*)ws(c, S_IDX, (size_t)std::max<int64_t>(cap, 1) * 8, &s);
    void* tmp = ws(c, S_SORT_TMP, tmp_bytes, &s);
    if (s != KRUX_OK) return s;
    HIP_TRY(c, kx_sort_hits(stage, nh, cap, keys, idx, tmp, tmp_bytes, (kx::HitRec*)hits, n_hits,
                            std::min(32, bit_length(rows - 1)), std::min(32, bit_length(snp_end - 1)),
                            st));
    return KRUX_OK;
}

// Per-row minimum p: rows still at p = 1 after the main pass are re-run with
// a looser screen (every pair whose p falls below the level is evaluated
// exactly), first at p_mid, then at p = 1 (every pair with H > 0).
krux_status resolve_min_p(krux_ctx* c, kx::ScanArgs base, const Variant& v, const Columns& col,
                          const int16_t* ranks2, const int64_t* tiesum, int64_t T, int K,
                          const int32_t* perms, int64_t V, double p_main, int64_t M,
                          const uint8_t* nan_flag, hipStream_t st) {
    std::vector<double> levels;
    double p_mid = std::min(1.0, std::max(p_main * 16.0, 1024.0 / std::max<int64_t>(M, 1)));
    if (p_mid > p_main && p_mid < 1.0) levels.push_back(p_mid);
    levels.push_back(1.0);
    krux_status s = KRUX_OK;
    int32_t* listA = (int32_t*)ws(c, S_LIST_A, (size_t)V * 4, &s);
    int32_t* listB = (int32_t*)ws(c, S_LIST_B, (size_t)V * 4, &s);
    int32_t* cntA = (int32_t*)ws(c, S_COUNT_A, 256, &s);
    int32_t* cntB = (int32_t*)ws(c, S_COUNT_B, 256, &s);
    if (s != KRUX_OK) return s;
    const int32_t* rows_in = nullptr;
    const int32_t* n_in = nullptr;
    double p_prev = p_main;   // screen level of the pass that just ran
    for (size_t li = 0; li < levels.size(); ++li) {
        int32_t* rows_out = (li % 2 == 0) ? listA : listB;
        int32_t* n_out = (li % 2 == 0) ? cntA : cntB;
        double bound = p_prev * (1.0 - 1e-12);
        unsigned long long limit;
        std::memcpy(&limit, &bound, 8);
        HIP_TRY(c, kx_launch_list_unresolved(base.minp_bits, limit, rows_in, n_in, V, rows_out,
                                             n_out, st));
        p_prev = levels[li];
        RankSide r2;
        s = prep_ranks(c, v, ranks2, tiesum, T, K, perms, rows_out, n_out, V, S_A2, S_THETA2,
                       S_ROWV2, st, &r2, S_AH2, nan_flag);
        if (s != KRUX_OK) return s;
        kx::ScanArgs a = base;
        a.A = r2.A; a.theta = r2.theta; a.row_v = r2.row_v;
        a.d_nrows = n_out; a.n_rows = V;
        a.hits = nullptr; a.counts = nullptr; a.n_lev = 0;
        set_screen(&a, levels[li]);
        s = run_screen(c, a, v, col, r2.A_hi, st, V);
        if (s != KRUX_OK) return s;
        rows_in = rows_out;
        n_in = n_out;
    }
    return KRUX_OK;
}

krux_status check_ranks(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                        int32_t K) {
    if (T < 0) return fail(c, KRUX_ERR_ARG, "T = %lld < 0", (long long)T);
    if (K < 1) return fail(c, KRUX_ERR_ARG, "K = %d < 1", K);
    if (K > KRUX_MAX_K_FP16)
        return fail(c, KRUX_ERR_UNSUPPORTED, "K = %d > %d", K, KRUX_MAX_K_FP16);
    if (T > 0 && (!ranks2 || !tiesum)) return fail(c, KRUX_ERR_ARG, "ranks2/tiesum is NULL");
    if (T > INT32_MAX / 2) return fail(c, KRUX_ERR_UNSUPPORTED, "T too large");
    return KRUX_OK;
}

krux_status check_geno(krux_ctx* c, const int8_t* geno, int64_t M, int64_t ld, int32_t K) {
    if (M < 0) return fail(c, KRUX_ERR_ARG, "M = %lld < 0", (long long)M);
    // SNP indices share a 32-bit word with two flag bits in the candidate buffer
    if (M > (1LL << 30) - 4096) return fail(c, KRUX_ERR_UNSUPPORTED, "M too large");
    if (M > 0 && !geno) return fail(c, KRUX_ERR_ARG, "geno is NULL");
    if (ld < K) return fail(c, KRUX_ERR_SHAPE, "ld_geno = %lld < K = %d", (long long)ld, K);
    return KRUX_OK;
}

krux_status test_impl(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                      int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno, int64_t snp_base,
                      double p_c, int32_t mode, int32_t precision, krux_hit* hits,
                      int64_t hit_capacity, int64_t* n_hits, double* min_p, double* H, double* p,
                      int32_t* sums, hipStream_t st) {
    krux_status s = check_ranks(c, ranks2, tiesum, T, K);
    if (s != KRUX_OK) return s;
    if ((s = check_geno(c, geno, M, ld_geno, K)) != KRUX_OK) return s;
    if (mode < KRUX_MODE_HITS || mode > KRUX_MODE_SUMS)
        return fail(c, KRUX_ERR_ARG, "mode %d", mode);
    if (precision < KRUX_PREC_FP16 || precision > KRUX_PREC_FP64)
        return fail(c, KRUX_ERR_ARG, "precision %d", precision);
    if (mode == KRUX_MODE_HITS) {
        if (!valid_p(p_c)) return fail(c, KRUX_ERR_ARG, "p_c = %g not in (0, 1]", p_c);
        if (!n_hits) return fail(c, KRUX_ERR_ARG, "n_hits is NULL");
        if (hit_capacity < 0) return fail(c, KRUX_ERR_ARG, "hit_capacity < 0");
        if (hit_capacity > 0 && !hits) return fail(c, KRUX_ERR_ARG, "hits is NULL");
        if (snp_base < 0 || snp_base + M > INT32_MAX)
            return fail(c, KRUX_ERR_ARG, "snp_base + M outside int32");
    } else if (mode == KRUX_MODE_FULL) {
        if (T * M > 0 && (!H || !p)) return fail(c, KRUX_ERR_ARG, "H/p is NULL");
    } else {
        if (T * M > 0 && !sums) return fail(c, KRUX_ERR_ARG, "sums is NULL");
    }
    if (precision == KRUX_PREC_FP64 && c->capturing)
        return fail(c, KRUX_ERR_UNSUPPORTED, "the fp64 comparator cannot be captured");
    if (precision == KRUX_PREC_FP64)
        return kx_fp64_test(c, ranks2, tiesum, T, K, geno, M, ld_geno, snp_base, p_c, mode, hits,
                            hit_capacity, n_hits, min_p, H, p, sums, st);
    Variant v;
    if ((s = choose_variant(c, K, precision, &v)) != KRUX_OK) return s;
    HIP_TRY(c, hipSetDevice(c->device));

    SnpSide sn;
    if ((s = pack_snps(c, geno, M, ld_geno, K, v.form == kx::DIAG, row_bytes(v), st, &sn)) != KRUX_OK) return s;
    Columns col;
    if ((s = expand_columns(c, v, sn, tile_shape_for(c, K, precision), st, &col)) != KRUX_OK)
        return s;
    NanSide ns;
    if ((s = flag_nan(c, ranks2, T, K, st, &ns)) != KRUX_OK) return s;
    RankSide rk;
    if ((s = prep_ranks(c, v, ranks2, tiesum, T, K, nullptr, nullptr, nullptr, T, S_A, S_THETA,
                        S_ROWV, st, &rk, S_AH, ns.flag)) != KRUX_OK)
        return s;

    kx::ScanArgs a{};
    a.A = rk.A; a.theta = rk.theta; a.row_v = rk.row_v; a.d_nrows = nullptr; a.n_rows = T;
    a.T = std::max<int64_t>(T, 1); a.tiesum = tiesum; a.ranks2 = ranks2; a.perms = nullptr;
    a.G = sn.G; a.gstride = sn.gstride; a.info = sn.info; a.tile_flags = sn.flags;
    a.mpos = sn.mpos;
    a.M = M; a.n_snp_tiles = sn.n_snp_tiles; a.K = K;
    apply_tuning(c, K, precision, v, T, sn.n_snp_tiles, &a);
    a.snp_base = snp_base;

    if (mode != KRUX_MODE_HITS) {
        a.H_out = H; a.p_out = p; a.sums_out = sums;
        set_screen(&a, 1.0);
        set_levels(&a, nullptr, 0);
        int64_t items = scan_items(v, T, a.n_snp_tiles, a.tiles_per_range);
        if (items <= 0) return KRUX_OK;
        int grid = (int)std::min<int64_t>(items, (int64_t)INT32_MAX);
        a.want_flag = -1;
        const int km = mode == KRUX_MODE_FULL ? kx::FULL : kx::SUMS;
        if ((s = launch_scan(c, a, v, col, rk.A_hi, kx::MISS3, km, grid, st)) != KRUX_OK) return s;
        return run_nan_traits(c, a, ns, 1, km, st);
    }

    int64_t cap = hit_capacity;
    kx::HitRec* stage = (kx::HitRec*)ws(c, S_STAGE, (size_t)std::max<int64_t>(cap, 1) * 24, &s);
    unsigned long long* nh = (unsigned long long*)ws(c, S_NHITS, 256, &s);
    unsigned long long* minp = (unsigned long long*)ws(c, S_MINP, (size_t)std::max<int64_t>(T, 1) * 8, &s);
    if (s != KRUX_OK) return s;
    HIP_TRY(c, kx_launch_fill_u64(nh, 1, 0ull, st));
    if (min_p) HIP_TRY(c, kx_launch_fill_u64(minp, T, 0x3FF0000000000000ull, st));
    a.hits = stage; a.hit_cap = cap; a.n_hits = nh;
    a.minp_bits = min_p ? minp : nullptr;
    a.counts = nullptr;
    set_levels(&a, &p_c, 1);
    // With min_p requested, the screen admits every pair with p below
    // p_screen >= p_c (hits are still only the pairs beyond H_c(p_c)); p_screen
    // is set so that a row of M SNPs almost surely has an exact candidate, and
    // the few rows without one get the looser passes of resolve_min_p.
    const double p_screen = min_p ? screen_level_for_min_p(p_c, M, K) : p_c;
    set_screen(&a, p_screen);
    a.cand_cap = pair_limit(candidate_capacity(T, M, p_screen), c->cand_limit);
    if ((s = run_screen(c, a, v, col, rk.A_hi, st, T, true)) != KRUX_OK) return s;
    if ((s = run_nan_traits(c, a, ns, 1, kx::SCREEN, st)) != KRUX_OK) return s;
    if (min_p && T > 0) {
        if ((s = resolve_min_p(c, a, v, col, ranks2, tiesum, T, K, nullptr, T, p_screen, M,
                               ns.flag, st)) != KRUX_OK)
            return s;
        HIP_TRY(c, kx_launch_bits_to_double(minp, T, min_p, st));
    }
    // deterministic order of the hit list
    return sort_stage(c, stage, nh, cap, hits, n_hits, T, snp_base + M, st);
}

}  // namespace

// ---------------------------------------------------------------------------
// internal hooks used by other translation units
// ---------------------------------------------------------------------------
krux_status kx_fail(krux_ctx* c, krux_status s, const char* msg) { return fail(c, s, "%s", msg); }
void* kx_ws(krux_ctx* c, int slot, size_t bytes, krux_status* st) { return ws(c, slot, bytes, st); }
void** kx_blas_handle(krux_ctx* c) { return &c->blas; }
int kx_ctx_device(krux_ctx* c) { return c->device; }
double kx_threshold_of(double p_c, int df) { return threshold_of(p_c, df); }
int kx_slot_f64_r() { return S_F64_R; }
int kx_slot_f64_i() { return S_F64_I; }
int kx_slot_f64_s() { return S_F64_S; }
int kx_slot_minp() { return S_MINP; }
int kx_slot_stage() { return S_STAGE; }
int kx_slot_nhits() { return S_NHITS; }
int kx_slot_keys() { return S_KEYS; }
int kx_slot_idx() { return S_IDX; }
int kx_slot_sort_tmp() { return S_SORT_TMP; }

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

krux_status krux_create(krux_ctx** out, int device) {
    if (!out) return fail(nullptr, KRUX_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
        return fail(nullptr, KRUX_ERR_HIP, "no HIP device");
    if (device < 0 || device >= n) return fail(nullptr, KRUX_ERR_ARG, "device %d of %d", device, n);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, KRUX_ERR_HIP, "hipSetDevice");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(nullptr, KRUX_ERR_HIP, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, KRUX_ERR_UNSUPPORTED, "device %d is %s, not gfx950", device,
                    prop.gcnArchName);
    krux_ctx* c = new krux_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    // the static scratch of krux_test_noalloc on this device (null if the
    // lookup failed; that entry point then reports the error)
    hipError_t serr = hipSuccess;
    c->noalloc_scratch = scratch_address(device, &serr);
    std::snprintf(c->arch, sizeof c->arch, "%.6s", prop.gcnArchName);
    *out = c;
    return KRUX_OK;
}

krux_status krux_timer_start(krux_ctx* c) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    c->timing = true;
    c->ev_used = 0;
    return KRUX_OK;
}

krux_status krux_timer_read(krux_ctx* c, double* total_ms, int64_t* launches) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (!total_ms || !launches) return fail(c, KRUX_ERR_ARG, "NULL output");
    double tot = 0.0;
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        HIP_TRY(c, hipEventSynchronize(c->ev[i + 1]));
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)(c->ev_used / 2);
    c->timing = false;
    c->ev_used = 0;
    return KRUX_OK;
}

krux_status krux_test_noalloc(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum,
                              int64_t T, int32_t K, const int8_t* geno, int64_t M,
                              int64_t ld_geno, int64_t snp_base, double p_c, int32_t mode,
                              int32_t precision, krux_hit* hits, int64_t hit_capacity,
                              int64_t* n_hits, double* min_p, double* H, double* p,
                              int32_t* sums, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (precision == KRUX_PREC_FP64)
        return fail(c, KRUX_ERR_UNSUPPORTED, "the fp64 comparator allocates (rocBLAS); use "
                    "krux_test");
    if (!c->noalloc_scratch) {
        hipError_t e = hipSuccess;
        (void)scratch_address(c->device, &e);
        return fail(c, KRUX_ERR_HIP, "no static scratch on device %d: %s", c->device,
                    hipGetErrorString(e));
    }
    hipStream_t st = (hipStream_t)stream;
    krux_status s = begin_call(c, st);
    if (s != KRUX_OK) return s;
    // screened-pair buffers of a few MB (pairs beyond them are evaluated in
    // the scan kernels), no event timing; restored on every return
    struct Restore {
        krux_ctx* c;
        int64_t cand, mcand;
        bool timing;
        ~Restore() {
            c->arena = 0;
            c->cand_limit = cand;
            c->mcand_limit = mcand;
            c->timing = timing;
        }
    } restore{c, c->cand_limit, c->mcand_limit, c->timing};
    c->cand_limit = pair_limit(1 << 18, restore.cand);
    c->mcand_limit = pair_limit(1 << 16, restore.mcand);
    c->timing = false;
    auto pass = [&](int arena) {
        c->arena = arena;
        c->arena_base = (uint8_t*)c->noalloc_scratch;
        c->arena_cap = KRUX_NOALLOC_SCRATCH_BYTES;
        c->arena_used = 0;
        std::fill(c->arena_len, c->arena_len + S_N_SLOTS, (size_t)0);
        return test_impl(c, ranks2, tiesum, T, K, geno, M, ld_geno, snp_base, p_c, mode,
                         precision, hits, hit_capacity, n_hits, min_p, H, p, sums, st);
    };
    // the host side once without launches gives the scratch layout; a call
    // that needs more than the static array is refused before any launch
    if ((s = pass(1)) != KRUX_OK) return s;
    if (c->arena_used > c->arena_cap)
        return fail(c, KRUX_ERR_UNSUPPORTED, "the call needs %zu bytes of scratch, more than the "
                    "%zu bytes of the static array (use krux_test, or a smaller SNP slice)",
                    c->arena_used, c->arena_cap);
    return pass(2);
}

krux_status krux_set_pair_buffer_limits(krux_ctx* c, int64_t candidates, int64_t missing_pairs) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (candidates < 0 || missing_pairs < 0) return fail(c, KRUX_ERR_ARG, "negative limit");
    c->cand_limit = candidates;
    c->mcand_limit = missing_pairs;
    return KRUX_OK;
}

void krux_destroy(krux_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    kx_fp64_release(c);
    for (auto& b : c->bufs)
        if (b.p) (void)hipFree(b.p);
    for (void* p : c->retired) (void)hipFree(p);
    delete c;
}

const char* krux_last_error(const krux_ctx* c) {
    if (c) return c->err.empty() ? g_err_null.c_str() : c->err.c_str();
    return g_err_noctx.empty() ? g_err_null.c_str() : g_err_noctx.c_str();
}

krux_status krux_threshold(double p_c, int32_t df, double* H_c) {
    if (!H_c) return fail(nullptr, KRUX_ERR_ARG, "H_c is NULL");
    if (!valid_p(p_c)) return fail(nullptr, KRUX_ERR_ARG, "p_c = %g not in (0, 1]", p_c);
    if (df < 1 || df > 2) return fail(nullptr, KRUX_ERR_UNSUPPORTED, "df = %d", df);
    *H_c = threshold_of(p_c, df);
    return KRUX_OK;
}

krux_status krux_rank(krux_ctx* c, const float* expr, int64_t T, int32_t K, int64_t ld_expr,
                      int16_t* ranks2, int64_t* tiesum, int32_t* nvalid, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (T < 0) return fail(c, KRUX_ERR_ARG, "T < 0");
    if (K < 1 || K > KRUX_MAX_K_RANK)
        return fail(c, KRUX_ERR_UNSUPPORTED, "K = %d outside [1, %d]", K, KRUX_MAX_K_RANK);
    if (ld_expr < K) return fail(c, KRUX_ERR_SHAPE, "ld_expr < K");
    if (T > 0 && (!expr || !ranks2 || !tiesum)) return fail(c, KRUX_ERR_ARG, "NULL array");
    if (T == 0) return KRUX_OK;
    krux_status s = begin_call(c, (hipStream_t)stream);
    if (s != KRUX_OK) return s;
    HIP_TRY(c, kx_launch_rank(expr, T, K, ld_expr, ranks2, tiesum, nvalid, 1 << 30,
                              (hipStream_t)stream));
    return KRUX_OK;
}

krux_status krux_test(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                      int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno, int64_t snp_base,
                      double p_c, int32_t mode, int32_t precision, krux_hit* hits,
                      int64_t hit_capacity, int64_t* n_hits, double* min_p, double* H, double* p,
                      int32_t* sums, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    krux_status s = begin_call(c, (hipStream_t)stream);
    if (s != KRUX_OK) return s;
    return test_impl(c, ranks2, tiesum, T, K, geno, M, ld_geno, snp_base, p_c, mode, precision,
                     hits, hit_capacity, n_hits, min_p, H, p, sums, (hipStream_t)stream);
}

namespace {

// Permuted-data scan: counts per threshold, per-row minimum p and/or the
// hit list at the first threshold (rows perm * T + trait).
krux_status permute_impl(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                         int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno,
                         const int32_t* perms, int32_t P, const double* p_cs, int32_t n_thr,
                         int64_t* counts, double* min_p, krux_hit* hits, int64_t hit_capacity,
                         int64_t* n_hits, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    krux_status s = check_ranks(c, ranks2, tiesum, T, K);
    if (s != KRUX_OK) return s;
    if ((s = check_geno(c, geno, M, ld_geno, K)) != KRUX_OK) return s;
    if ((s = begin_call(c, (hipStream_t)stream)) != KRUX_OK) return s;
    if (P < 1 || !perms) return fail(c, KRUX_ERR_ARG, "need P >= 1 permutations");
    if (n_thr < 1 || n_thr > kx::kMaxLevels || !p_cs)
        return fail(c, KRUX_ERR_ARG, "n_thr must be in [1, %d]", kx::kMaxLevels);
    for (int i = 0; i < n_thr; ++i)
        if (!valid_p(p_cs[i])) return fail(c, KRUX_ERR_ARG, "p_cs[%d] = %g", i, p_cs[i]);
    if ((int64_t)P * T > INT32_MAX / 2) return fail(c, KRUX_ERR_UNSUPPORTED, "P * T too large");
    Variant v;
    if ((s = choose_variant(c, K, KRUX_PREC_FP16, &v)) != KRUX_OK) return s;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t V = (int64_t)P * T;
    SnpSide sn;
    if ((s = pack_snps(c, geno, M, ld_geno, K, v.form == kx::DIAG, row_bytes(v), st, &sn)) != KRUX_OK) return s;
    Columns col;
    if ((s = expand_columns(c, v, sn, tile_shape_for(c, K, KRUX_PREC_FP16), st, &col)) != KRUX_OK)
        return s;
    NanSide ns;
    if ((s = flag_nan(c, ranks2, T, K, st, &ns)) != KRUX_OK) return s;
    RankSide rk;
    if ((s = prep_ranks(c, v, ranks2, tiesum, T, K, perms, nullptr, nullptr, V, S_A, S_THETA,
                        S_ROWV, st, &rk, S_AH, ns.flag)) != KRUX_OK)
        return s;
    unsigned long long* minp =
        (unsigned long long*)ws(c, S_MINP, (size_t)std::max<int64_t>(V, 1) * 8, &s);
    if (s != KRUX_OK) return s;
    if (counts)
        HIP_TRY(c, kx_launch_fill_u64((unsigned long long*)counts, (int64_t)P * n_thr, 0ull, st));
    kx::HitRec* stage = nullptr;
    unsigned long long* nh = nullptr;
    if (n_hits) {
        stage = (kx::HitRec*)ws(c, S_STAGE, (size_t)std::max<int64_t>(hit_capacity, 1) * 24, &s);
        nh = (unsigned long long*)ws(c, S_NHITS, 256, &s);
        if (s != KRUX_OK) return s;
        HIP_TRY(c, kx_launch_fill_u64(nh, 1, 0ull, st));
    }
    if (min_p) HIP_TRY(c, kx_launch_fill_u64(minp, V, 0x3FF0000000000000ull, st));
    kx::ScanArgs a{};
    a.A = rk.A; a.theta = rk.theta; a.row_v = rk.row_v; a.d_nrows = nullptr; a.n_rows = V;
    a.T = std::max<int64_t>(T, 1); a.tiesum = tiesum; a.ranks2 = ranks2; a.perms = perms;
    a.G = sn.G; a.gstride = sn.gstride; a.info = sn.info; a.tile_flags = sn.flags;
    a.mpos = sn.mpos;
    a.M = M; a.n_snp_tiles = sn.n_snp_tiles; a.K = K;
    apply_tuning(c, K, KRUX_PREC_FP16, v, V, sn.n_snp_tiles, &a);
    a.hits = stage; a.hit_cap = n_hits ? hit_capacity : 0; a.n_hits = nh;
    a.counts = (unsigned long long*)counts;
    a.minp_bits = min_p ? minp : nullptr;
    set_levels(&a, p_cs, n_thr);
    double loosest = *std::max_element(p_cs, p_cs + n_thr);
    if (min_p) loosest = screen_level_for_min_p(loosest, M, K);
    set_screen(&a, loosest);
    a.cand_cap = pair_limit(candidate_capacity(V, M, loosest), c->cand_limit);
    if ((s = run_screen(c, a, v, col, rk.A_hi, st, V, true)) != KRUX_OK) return s;
    if ((s = run_nan_traits(c, a, ns, P, kx::SCREEN, st)) != KRUX_OK) return s;
    if (min_p && V > 0) {
        if ((s = resolve_min_p(c, a, v, col, ranks2, tiesum, T, K, perms, V, loosest, M, ns.flag,
                               st)) != KRUX_OK)
            return s;
        HIP_TRY(c, kx_launch_bits_to_double(minp, V, min_p, st));
    }
    if (n_hits) return sort_stage(c, stage, nh, hit_capacity, hits, n_hits, V, M, st);
    return KRUX_OK;
}

}  // namespace

krux_status krux_permute(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                         int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno,
                         const int32_t* perms, int32_t P, const double* p_cs, int32_t n_thr,
                         int64_t* counts, double* min_p, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (!counts) return fail(c, KRUX_ERR_ARG, "counts is NULL");
    return permute_impl(c, ranks2, tiesum, T, K, geno, M, ld_geno, perms, P, p_cs, n_thr, counts,
                        min_p, nullptr, 0, nullptr, stream);
}

krux_status krux_permute_hits(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum,
                              int64_t T, int32_t K, const int8_t* geno, int64_t M,
                              int64_t ld_geno, const int32_t* perms, int32_t P, double p_c,
                              krux_hit* hits, int64_t hit_capacity, int64_t* n_hits,
                              void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (!n_hits) return fail(c, KRUX_ERR_ARG, "n_hits is NULL");
    if (hit_capacity < 0) return fail(c, KRUX_ERR_ARG, "hit_capacity < 0");
    if (hit_capacity > 0 && !hits) return fail(c, KRUX_ERR_ARG, "hits is NULL");
    if (hit_capacity > (int64_t)UINT32_MAX) return fail(c, KRUX_ERR_ARG, "hit_capacity too large");
    return permute_impl(c, ranks2, tiesum, T, K, geno, M, ld_geno, perms, P, &p_c, 1, nullptr,
                        nullptr, hits, hit_capacity, n_hits, stream);
}

krux_status krux_fdr_curve(krux_ctx* c, const krux_hit* real, const int64_t* n_real,
                           int64_t real_capacity, const krux_hit* perm, const int64_t* n_perm,
                           int64_t perm_capacity, int32_t P, double* fdr, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (P < 1) return fail(c, KRUX_ERR_ARG, "P must be >= 1");
    if (real_capacity < 0 || perm_capacity < 0) return fail(c, KRUX_ERR_ARG, "capacity < 0");
    if (!n_real || !n_perm) return fail(c, KRUX_ERR_ARG, "n_real / n_perm is NULL");
    if ((real_capacity > 0 && (!real || !fdr)) || (perm_capacity > 0 && !perm))
        return fail(c, KRUX_ERR_ARG, "hit list or fdr is NULL");
    krux_status s = begin_call(c, (hipStream_t)stream);
    if (s != KRUX_OK) return s;
    const int64_t big = std::max<int64_t>(std::max(real_capacity, perm_capacity), 1);
    const size_t tmp_bytes = kx_sort_keys_tmp_bytes(big);
    unsigned long long* kr = (unsigned long long*)ws(c, S_KEYS, (size_t)std::max<int64_t>(real_capacity, 1) * 16, &s);
    unsigned long long* kp = (unsigned long long*)ws(c, S_IDX, (size_t)std::max<int64_t>(perm_capacity, 1) * 16, &s);
    void* tmp = ws(c, S_SORT_TMP, tmp_bytes, &s);
    if (s != KRUX_OK) return s;
    HIP_TRY(c, kx_fdr_curve((const kx::HitRec*)real, n_real, real_capacity,
                            (const kx::HitRec*)perm, n_perm, perm_capacity, P, kr, kp, tmp,
                            tmp_bytes, fdr, (hipStream_t)stream));
    return KRUX_OK;
}

// Hits of one scan with SNPs grouped by missing-genotype pattern (Handling
// missing values): each group of at least min_group SNPs with the same
// missing samples Q becomes a complete sub-problem over the other K - |Q|
// samples (ranks recomputed over them by ranking the gathered ranks); the
// remaining SNPs form one more sub-problem over all K samples.  The
// sub-problems' hits are mapped back to SNP indices and sorted together, and
// their per-trait minima merged.  Results equal krux_test's.
krux_status krux_test_grouped(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum,
                              int64_t T, int32_t K, const int8_t* geno, int64_t M,
                              int64_t ld_geno, int64_t snp_base, double p_c, int32_t precision,
                              int64_t min_group, krux_hit* hits, int64_t hit_capacity,
                              int64_t* n_hits, double* min_p, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    krux_status s = check_ranks(c, ranks2, tiesum, T, K);
    if (s != KRUX_OK) return s;
    if ((s = check_geno(c, geno, M, ld_geno, K)) != KRUX_OK) return s;
    if (!valid_p(p_c)) return fail(c, KRUX_ERR_ARG, "p_c = %g not in (0, 1]", p_c);
    if (precision < KRUX_PREC_FP16 || precision > KRUX_PREC_FP64)
        return fail(c, KRUX_ERR_ARG, "precision %d", precision);
    if (!n_hits) return fail(c, KRUX_ERR_ARG, "n_hits is NULL");
    if (hit_capacity < 0 || (hit_capacity > 0 && !hits))
        return fail(c, KRUX_ERR_ARG, "hits / hit_capacity");
    if (hit_capacity > (int64_t)UINT32_MAX) return fail(c, KRUX_ERR_ARG, "hit_capacity too large");
    if (min_group < 1) return fail(c, KRUX_ERR_ARG, "min_group < 1");
    if ((s = begin_call(c, st, false)) != KRUX_OK) return s;
    auto plain = [&]() {
        return test_impl(c, ranks2, tiesum, T, K, geno, M, ld_geno, snp_base, p_c, KRUX_MODE_HITS,
                         precision, hits, hit_capacity, n_hits, min_p, nullptr, nullptr, nullptr,
                         st);
    };
    if (M == 0 || T == 0) return plain();
    HIP_TRY(c, hipSetDevice(c->device));
    const int grid = c->n_cu * 8;

    // 1. pattern keys; their runs in sorted order give the patterns shared
    //    by at least min_group SNPs (G of them, keys ascending)
    const size_t tmpb = kx_group_tmp_bytes(M);
    uint64_t* keys = (uint64_t*)ws(c, S_G_KEYS, (size_t)M * 28 + 256, &s);
    void* gtmp = ws(c, S_G_EXPR, std::max(tmpb, (size_t)T * K * 4), &s);
    if (s != KRUX_OK) return s;
    uint64_t* sorted = keys + M;
    uint64_t* uniq = keys + 2 * M;
    uint32_t* runc = (uint32_t*)(keys + 3 * M);
    uint32_t* nrun = runc + M;
    HIP_TRY(c, kx_launch_miss_keys(geno, M, ld_geno, K, keys, grid, st));
    HIP_TRY(c, kx_group_runs(keys, M, sorted, uniq, runc, nrun, gtmp, tmpb, st));
    uint32_t n_runs = 0;
    HIP_TRY(c, hipMemcpyAsync(&n_runs, nrun, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    std::vector<uint64_t> uk(n_runs);
    std::vector<uint32_t> uc(n_runs);
    if (n_runs) {
        HIP_TRY(c, hipMemcpyAsync(uk.data(), uniq, (size_t)n_runs * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipMemcpyAsync(uc.data(), runc, (size_t)n_runs * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
    }
    std::vector<uint64_t> big;
    std::vector<int64_t> off(1, 0);
    for (uint32_t r = 0; r < n_runs; ++r)
        if (uk[r] != 0 && (int64_t)uc[r] >= min_group) {
            big.push_back(uk[r]);
            off.push_back(off.back() + uc[r]);
        }
    const int G = (int)big.size();
    if (G == 0) return plain();
    off.push_back(M);                                  // the rest: [off[G], M)

    // 2. every SNP into its part; each group's pattern from one member,
    //    every member checked against it (a key collision sends the whole
    //    call to the ungrouped path)
    int32_t* d_snps = (int32_t*)ws(c, S_G_SNPS, (size_t)M * 4 + 256, &s);
    int64_t* d_off = (int64_t*)ws(c, S_G_SAMPLES, (size_t)(G + 2) * 8 + (size_t)G * K * 4 + 256, &s);
    int32_t* d_smp = (int32_t*)(d_off + G + 2);
    uint64_t* d_big = (uint64_t*)ws(c, S_G_QMASK, (size_t)G * 8 + (size_t)G * K + 256, &s);
    uint8_t* d_q = (uint8_t*)(d_big + G);
    unsigned long long* cnt = (unsigned long long*)ws(c, S_G_CNT, 256, &s);
    if (s != KRUX_OK) return s;
    HIP_TRY(c, hipMemcpyAsync(d_big, big.data(), (size_t)G * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipMemcpyAsync(d_off, off.data(), (size_t)(G + 2) * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(c, kx_launch_fill_u64(cnt, 3, 0ull, st));  // bad, stored, total
    int32_t* pid = (int32_t*)sorted;                   // the sorted keys are no longer needed
    HIP_TRY(c, kx_group_parts(keys, M, d_big, G, pid, pid + M, (int32_t*)uniq, d_snps, gtmp, tmpb,
                              grid, st));
    HIP_TRY(c, kx_launch_pattern_mask(geno, ld_geno, K, d_snps, d_off, G, d_q, grid, st));
    for (int gi = 0; gi < G; ++gi)
        HIP_TRY(c, kx_launch_check_pattern(geno, ld_geno, K, d_snps + off[gi],
                                           off[gi + 1] - off[gi], d_q + (int64_t)gi * K, cnt,
                                           grid, st));
    std::vector<uint8_t> qmask_h((size_t)G * K);
    unsigned long long bad = 0;
    HIP_TRY(c, hipMemcpyAsync(qmask_h.data(), d_q, qmask_h.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(&bad, cnt, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (bad) return plain();
    std::vector<int32_t> smp_all;
    std::vector<int64_t> smp_off;
    std::vector<int> kp_of;
    for (int gi = 0; gi < G; ++gi) {
        smp_off.push_back((int64_t)smp_all.size());
        for (int k = 0; k < K; ++k)
            if (!qmask_h[(size_t)gi * K + k]) smp_all.push_back(k);
        kp_of.push_back((int)(smp_all.size() - smp_off.back()));
    }
    if (!smp_all.empty()) {
        HIP_TRY(c, hipMemcpyAsync(d_smp, smp_all.data(), smp_all.size() * 4,
                                  hipMemcpyHostToDevice, st));
        HIP_TRY(c, hipStreamSynchronize(st));         // smp_all is pageable host memory
    }

    // 3. the sub-problems
    const int64_t cap = hit_capacity;
    kx::HitRec* stage = (kx::HitRec*)ws(c, S_G_STAGE, (size_t)std::max<int64_t>(cap, 1) * 24, &s);
    kx::HitRec* phits = (kx::HitRec*)ws(c, S_G_PHITS, (size_t)std::max<int64_t>(cap, 1) * 24, &s);
    int64_t* pn = (int64_t*)ws(c, S_G_PN, 256, &s);
    double* acc = min_p ? (double*)ws(c, S_G_MINP, (size_t)T * 8, &s) : nullptr;
    double* pmin = min_p ? (double*)ws(c, S_G_PMINP, (size_t)T * 8, &s) : nullptr;
    int8_t* gsub = (int8_t*)ws(c, S_G_GENO, (size_t)M * K, &s);
    float* xsub = (float*)gtmp;
    int16_t* rsub = (int16_t*)ws(c, S_G_R, (size_t)T * K * 2, &s);
    int64_t* tsub = (int64_t*)ws(c, S_G_TS, (size_t)T * 8, &s);
    if (s != KRUX_OK) return s;
    if (min_p) HIP_TRY(c, kx_launch_fill_u64((unsigned long long*)acc, T, 0x3FF0000000000000ull, st));
    for (int part = 0; part <= G; ++part) {
        const bool grp = part < G;
        const int64_t n = off[part + 1] - off[part];
        if (n == 0) continue;
        const int32_t* snps = d_snps + off[part];
        const int Kp = grp ? kp_of[part] : K;
        const int16_t* r2 = ranks2;
        const int64_t* ts = tiesum;
        const int32_t* S = nullptr;
        if (grp) {
            if (Kp == 0) continue;                 // no sample left: H = 0, p = 1, no hit
            S = d_smp + smp_off[part];
            HIP_TRY(c, kx_launch_gather_rank_cols(ranks2, T, K, S, Kp, xsub, grid, st));
            HIP_TRY(c, kx_launch_rank(xsub, T, Kp, Kp, rsub, tsub, nullptr, 1 << 30, st));
            r2 = rsub;
            ts = tsub;
        }
        HIP_TRY(c, kx_launch_gather_geno(geno, ld_geno, snps, n, S, Kp, gsub, grid, st));
        if ((s = test_impl(c, r2, ts, T, Kp, gsub, n, Kp, 0, p_c, KRUX_MODE_HITS, precision,
                           (krux_hit*)phits, cap, pn, pmin, nullptr, nullptr, nullptr, st)) !=
            KRUX_OK)
            return s;
        HIP_TRY(c, kx_launch_append_hits(phits, pn, cap, snps, snp_base, stage, cnt + 1, cnt + 2,
                                         grid, st));
        if (min_p) HIP_TRY(c, kx_launch_min_merge(pmin, acc, T, grid, st));
    }
    if ((s = sort_stage(c, stage, cnt + 1, cap, hits, n_hits, T, snp_base + M, st)) != KRUX_OK)
        return s;
    HIP_TRY(c, kx_launch_set_counts(n_hits, cnt + 2, cnt + 1, cap, st));
    if (min_p) HIP_TRY(c, hipMemcpyAsync(min_p, acc, (size_t)T * 8, hipMemcpyDeviceToDevice, st));
    return KRUX_OK;
}

namespace {

// Upper chi-square tail for any df on the host (the closed forms of
// Q(df/2, H/2), as in the multi-allelic kernel), and its threshold on H.
double host_chi2_upper(double H, int df) {
    if (df <= 0) return 1.0;
    const double x = 0.5 * H;
    if (df % 2 == 0) {
        double term = 1.0, total = 1.0;
        for (int k = 1; k < df / 2; ++k) {
            term *= x / k;
            total += term;
        }
        return std::exp(-x) * total;
    }
    double total = std::erfc(std::sqrt(x));
    if (df > 1) {
        double term = std::sqrt(x) / 0.88622692545275801365;   // Gamma(3/2)
        double sum = term;
        for (int k = 2; k <= (df - 1) / 2; ++k) {
            term *= x / (k - 0.5);
            sum += term;
        }
        total += std::exp(-x) * sum;
    }
    return total;
}

double threshold_any_df(double p_c, int df) {
    uint64_t lo, hi;
    double d0 = 0.0, d1 = 8192.0;
    std::memcpy(&lo, &d0, 8);
    std::memcpy(&hi, &d1, 8);
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        double h;
        std::memcpy(&h, &mid, 8);
        if (host_chi2_upper(h, df) >= p_c) lo = mid; else hi = mid;
    }
    double r;
    std::memcpy(&r, &lo, 8);
    return r;
}

}  // namespace

// Multi-allelic markers: classes 0..n_classes-1, exact per pair on the GPU
// without the GEMM (HITS or FULL).
krux_status krux_test_multi(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                            int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno,
                            int32_t n_classes, int64_t snp_base, double p_c, int32_t mode,
                            krux_hit* hits, int64_t hit_capacity, int64_t* n_hits,
                            double* min_p, double* H, double* p, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    krux_status s = check_ranks(c, ranks2, tiesum, T, K);
    if (s != KRUX_OK) return s;
    if ((s = check_geno(c, geno, M, ld_geno, K)) != KRUX_OK) return s;
    if (K > 2048) return fail(c, KRUX_ERR_UNSUPPORTED, "K = %d above 2048", K);
    if (n_classes < 2 || n_classes > kx::kMaxClasses)
        return fail(c, KRUX_ERR_ARG, "n_classes = %d not in [2, %d]", n_classes, kx::kMaxClasses);
    if (mode != KRUX_MODE_HITS && mode != KRUX_MODE_FULL)
        return fail(c, KRUX_ERR_ARG, "mode %d (HITS or FULL)", mode);
    hipStream_t st = (hipStream_t)stream;
    if ((s = begin_call(c, st)) != KRUX_OK) return s;
    kx::MultiArgs a{};
    a.ranks2 = ranks2; a.tiesum = tiesum; a.T = T; a.K = K; a.M = M; a.snp_base = snp_base;
    a.G = n_classes;
    a.pstride = (K + 31) & ~31;
    a.record_hits = 1;
    if (mode == KRUX_MODE_HITS) {
        if (!valid_p(p_c)) return fail(c, KRUX_ERR_ARG, "p_c = %g not in (0, 1]", p_c);
        if (!n_hits) return fail(c, KRUX_ERR_ARG, "n_hits is NULL");
        if (hit_capacity < 0 || (hit_capacity > 0 && !hits))
            return fail(c, KRUX_ERR_ARG, "hits / hit_capacity");
        if (hit_capacity > (int64_t)UINT32_MAX)
            return fail(c, KRUX_ERR_ARG, "hit_capacity too large");
        if (snp_base < 0 || snp_base + M > INT32_MAX)
            return fail(c, KRUX_ERR_ARG, "snp_base + M outside int32");
        for (int df = 1; df < n_classes; ++df) a.hc[df] = threshold_any_df(p_c, df);
    } else if (T * M > 0 && (!H || !p)) {
        return fail(c, KRUX_ERR_ARG, "H / p is NULL");
    }
    kx::HitRec* stage = nullptr;
    unsigned long long* nh = nullptr;
    if (mode == KRUX_MODE_HITS) {
        stage = (kx::HitRec*)ws(c, S_STAGE, (size_t)std::max<int64_t>(hit_capacity, 1) * 24, &s);
        nh = (unsigned long long*)ws(c, S_NHITS, 256, &s);
        if (s != KRUX_OK) return s;
        HIP_TRY(c, kx_launch_fill_u64(nh, 1, 0ull, st));
        a.hits = stage; a.hit_cap = hit_capacity; a.n_hits = nh;
        if (min_p && T > 0) {
            a.minp_bits = (unsigned long long*)ws(c, S_MINP, (size_t)T * 8, &s);
            if (s != KRUX_OK) return s;
            HIP_TRY(c, kx_launch_fill_u64(a.minp_bits, T, 0x3FF0000000000000ull, st));
        }
    } else {
        a.H_out = H; a.p_out = p;
    }
    if (T > 0 && M > 0) {
        uint8_t* packed = (uint8_t*)ws(c, S_G_GENO, (size_t)M * a.pstride, &s);
        kx::MultiInfo* info = (kx::MultiInfo*)ws(c, S_MINFO, (size_t)M * sizeof(kx::MultiInfo), &s);
        int32_t* any_missing = (int32_t*)ws(c, S_MFLAG, 256, &s);
        if (s != KRUX_OK) return s;
        HIP_TRY(c, kx_launch_multi_pack(geno, ld_geno, M, K, n_classes, a.pstride, packed,
                                        c->n_cu * 8, st));
        HIP_TRY(c, kx_launch_multi_info(packed, a.pstride, M, K, n_classes, info, any_missing,
                                        c->n_cu * 8, st));
        a.packed = packed;
        a.info = info;
        a.any_missing = any_missing;
        const int64_t nb = (M + 63) / 64;
        const int lane_grid = (int)std::min<int64_t>((T * nb + 3) / 4, (int64_t)c->n_cu * 8);
        // complete pairs of K <= 128 with at most five classes take the MFMA
        // screen; every other pair is evaluated per lane
        const bool gemm = mode == KRUX_MODE_HITS && K <= 128 && n_classes <= 5;
        if (!gemm) {
            HIP_TRY(c, kx_launch_multi(&a, n_classes, mode == KRUX_MODE_FULL ? kx::FULL : kx::SCREEN,
                                       lane_grid, st));
        } else {
            NanSide ns;
            if ((s = flag_nan(c, ranks2, T, K, st, &ns)) != KRUX_OK) return s;
            const Variant v{kx::F16, (int)ceil_div(K, 16), kx::DIAG, false, false};
            RankSide rk;
            if ((s = prep_ranks(c, v, ranks2, tiesum, T, K, nullptr, nullptr, nullptr, T, S_A,
                                S_THETA, S_ROWV, st, &rk, S_AH, ns.flag)) != KRUX_OK)
                return s;
            a.A = rk.A; a.theta = rk.theta; a.row_v = rk.row_v; a.n_rows = T;
            a.n_snp_tiles = ceil_div(M, kx::kTile);
            a.tiles_per_range = trait_range(v, T, a.n_snp_tiles, c->n_cu);
            a.nan_flag = ns.flag;
            a.n_nan = ns.n;
            const double p_screen = min_p ? screen_level_for_min_p(p_c, M, K) : p_c;
            for (int df = 1; df < n_classes; ++df) {
                // 1/H_c(df) capped: at p_screen = 1 (H_c = 0) every pair with
                // a non-zero class sum passes, and no 0 * inf appears
                const double h = threshold_any_df(p_screen, df);
                a.inv_hc[df] = (float)std::min(1.0 / std::max(h, 1e-300), 1e30);
            }
            a.cand_cap = pair_limit(candidate_capacity(T, M, p_screen), c->cand_limit);
            a.cand = (kx::MultiCand*)ws(c, S_CAND, (size_t)a.cand_cap * sizeof(kx::MultiCand), &s);
            a.n_cand = (unsigned long long*)ws(c, S_NCAND, 256, &s);   // cleared by prep
            if (s != KRUX_OK) return s;
            const int64_t items = ceil_div(ceil_div(T, kx::kTile), a.tiles_per_range) *
                                  ceil_div(a.n_snp_tiles, kx::kWavesPerBlock);
            hipEvent_t ev[2] = {nullptr, nullptr};
            if (c->timing) {
                while (c->ev.size() < c->ev_used + 2) {
                    hipEvent_t e;
                    HIP_TRY(c, hipEventCreate(&e));
                    c->ev.push_back(e);
                }
                ev[0] = c->ev[c->ev_used];
                ev[1] = c->ev[c->ev_used + 1];
                c->ev_used += 2;
                HIP_TRY(c, hipEventRecord(ev[0], st));
            }
            HIP_TRY(c, kx_launch_multi_mfma(&a, n_classes, (int)ceil_div(K, 16),
                                            (int)std::min<int64_t>(items, INT32_MAX), st));
            if (ev[1]) HIP_TRY(c, hipEventRecord(ev[1], st));
            HIP_TRY(c, kx_launch_multi_exact(&a, n_classes, c->n_cu * 8, st));
            // pairs of traits with a NaN value and of SNPs with a removed code
            a.only_incomplete = 1;
            HIP_TRY(c, kx_launch_multi(&a, n_classes, kx::SCREEN, lane_grid, st));
            a.only_incomplete = 0;
            if (a.minp_bits) {
                // traits whose smallest evaluated p is not below the screen
                // level: every pair of theirs, minimum p only
                int32_t* list = (int32_t*)ws(c, S_LIST_A, (size_t)T * 4, &s);
                int32_t* cnt = (int32_t*)ws(c, S_COUNT_A, 256, &s);
                if (s != KRUX_OK) return s;
                const double bound = p_screen * (1.0 - 1e-12);
                unsigned long long limit;
                std::memcpy(&limit, &bound, 8);
                HIP_TRY(c, kx_launch_list_unresolved(a.minp_bits, limit, nullptr, nullptr, T, list,
                                                     cnt, st));
                a.trait_list = list;
                a.n_list = cnt;
                a.record_hits = 0;
                HIP_TRY(c, kx_launch_multi(&a, n_classes, kx::SCREEN, lane_grid, st));
            }
        }
    }
    if (mode == KRUX_MODE_HITS) {
        if (a.minp_bits) HIP_TRY(c, kx_launch_bits_to_double(a.minp_bits, T, min_p, st));
        return sort_stage(c, stage, nh, hit_capacity, hits, n_hits, T, snp_base + M, st);
    }
    return KRUX_OK;
}

krux_status krux_test_batched(krux_ctx* c, const krux_cohort* co, int32_t n, int64_t M,
                              double p_c, int32_t precision, void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (n < 0 || (n > 0 && !co)) return fail(c, KRUX_ERR_ARG, "cohorts");
    krux_status s0 = begin_call(c, (hipStream_t)stream);
    if (s0 != KRUX_OK) return s0;
    for (int i = 0; i < n; ++i) {
        krux_status s = test_impl(c, co[i].ranks2, co[i].tiesum, co[i].T, co[i].K, co[i].geno, M,
                                  co[i].ld_geno, 0, p_c, KRUX_MODE_HITS, precision, co[i].hits,
                                  co[i].hit_capacity, co[i].n_hits, co[i].min_p, nullptr, nullptr,
                                  nullptr, (hipStream_t)stream);
        if (s != KRUX_OK) return s;
    }
    return KRUX_OK;
}

// ---------------------------------------------------------------- autotuning
namespace {

const char* prec_name(int p) {
    return p == KRUX_PREC_FP16 ? "fp16" : p == KRUX_PREC_INT8 ? "int8" : "fp64";
}

// Candidate configurations of the kernel family serving (K, precision).
std::vector<Tuning> tuning_candidates(const Variant& v) {
    std::vector<Tuning> out;
    if (!v.tiled) {
        for (int ring = 0; ring <= 4; ++ring)
            for (int kb : {640, 1280, 2560, 5120}) {
                Tuning t;
                t.ring = ring;
                t.range_kb = kb;
                out.push_back(t);
            }
    } else {
        for (int shape = 0; shape <= 3; ++shape)
            for (int g = 0; g <= 1; ++g) {
                Tuning t;
                t.grouped = g;
                t.shape = shape;
                out.push_back(t);
            }
    }
    return out;
}

// One line of the cache file: {"arch": "gfx950", "K": 102, "precision": "fp16",
// "mode": "hits", "ring": 0, "range_kb": 2560, "grouped": -1, "shape": -1, "ms": 3.41}
bool parse_tuning_line(const char* line, const char* arch, int* K, int* prec, Tuning* t) {
    char a[32] = {0}, p[16] = {0}, m[16] = {0};
    int k = 0, ring = -1, kb = 0, grouped = -1, shape = -1;
    double ms = 0.0;
    const int n = std::sscanf(line,
                              " {\"arch\": \"%31[^\"]\", \"K\": %d, \"precision\": \"%15[^\"]\", "
                              "\"mode\": \"%15[^\"]\", \"ring\": %d, \"range_kb\": %d, "
                              "\"grouped\": %d, \"shape\": %d, \"ms\": %lf",
                              a, &k, p, m, &ring, &kb, &grouped, &shape, &ms);
    if (n != 9 || std::strcmp(a, arch) != 0 || std::strcmp(m, "hits") != 0) return false;
    if (std::strcmp(p, "fp16") == 0) *prec = KRUX_PREC_FP16;
    else if (std::strcmp(p, "int8") == 0) *prec = KRUX_PREC_INT8;
    else return false;
    *K = k;
    t->ring = ring; t->range_kb = kb; t->grouped = grouped; t->shape = shape; t->ms = ms;
    return true;
}

}  // namespace

krux_status krux_autotune(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                          int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno,
                          int32_t precision, const char* cache_path, double* best_ms,
                          void* stream) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    krux_status s = check_ranks(c, ranks2, tiesum, T, K);
    if (s != KRUX_OK) return s;
    if ((s = check_geno(c, geno, M, ld_geno, K)) != KRUX_OK) return s;
    if (precision != KRUX_PREC_FP16 && precision != KRUX_PREC_INT8)
        return fail(c, KRUX_ERR_UNSUPPORTED, "only the MFMA paths are tuned");
    if (T <= 0 || M <= 0) return fail(c, KRUX_ERR_ARG, "empty tuning input");
    Variant v;
    if ((s = choose_variant(c, K, precision, &v)) != KRUX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = begin_call(c, st, false)) != KRUX_OK) return s;
    const int64_t cap = 1 << 16;
    krux_hit* hits = (krux_hit*)ws(c, S_TUNE_HITS, (size_t)cap * sizeof(krux_hit), &s);
    int64_t* nh = (int64_t*)ws(c, S_TUNE_N, 256, &s);
    if (s != KRUX_OK) return s;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    const std::pair<int, int> key{K, precision};
    const bool had = c->tuned.count(key) != 0;
    const Tuning before = had ? c->tuned[key] : Tuning();
    Tuning best;
    best.ms = -1.0;
    krux_status err = KRUX_OK;
    for (const Tuning& cand : tuning_candidates(v)) {
        c->tuned[key] = cand;
        auto run = [&]() {
            return test_impl(c, ranks2, tiesum, T, K, geno, M, ld_geno, 0, 1e-5, KRUX_MODE_HITS,
                             precision, hits, cap, nh, nullptr, nullptr, nullptr, nullptr, st);
        };
        if ((err = run()) != KRUX_OK) break;                 // warmup (grows buffers)
        if (hipEventRecord(e0, st) != hipSuccess) { err = fail(c, KRUX_ERR_HIP, "event"); break; }
        const int reps = 3;
        for (int r = 0; r < reps && err == KRUX_OK; ++r) err = run();
        if (err != KRUX_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            err = fail(c, KRUX_ERR_HIP, "event");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        Tuning t = cand;
        t.ms = ms / reps;
        if (best.ms < 0.0 || t.ms < best.ms) best = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != KRUX_OK) {
        if (had) c->tuned[key] = before; else c->tuned.erase(key);
        return err;
    }
    c->tuned[key] = best;
    if (best_ms) *best_ms = best.ms;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(c, KRUX_ERR_ARG, "cannot open %s", cache_path);
        std::fprintf(f,
                     "{\"arch\": \"%s\", \"K\": %d, \"precision\": \"%s\", \"mode\": \"hits\", "
                     "\"ring\": %d, \"range_kb\": %d, \"grouped\": %d, \"shape\": %d, "
                     "\"ms\": %.6f}\n",
                     c->arch, K, prec_name(precision), best.ring, best.range_kb, best.grouped,
                     best.shape, best.ms);
        std::fclose(f);
    }
    return KRUX_OK;
}

krux_status krux_load_tuning(krux_ctx* c, const char* cache_path) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    if (!cache_path) return fail(c, KRUX_ERR_ARG, "cache_path is NULL");
    FILE* f = std::fopen(cache_path, "r");
    if (!f) return fail(c, KRUX_ERR_ARG, "cannot open %s", cache_path);
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        int K = 0, prec = 0;
        Tuning t;
        if (parse_tuning_line(line, c->arch, &K, &prec, &t)) c->tuned[{K, prec}] = t;  // later lines win
    }
    std::fclose(f);
    return KRUX_OK;
}

krux_status krux_tuning_of(krux_ctx* c, int32_t K, int32_t precision, int32_t* ring,
                           int32_t* range_kb, int32_t* grouped, int32_t* shape) {
    if (!c) return fail(nullptr, KRUX_ERR_ARG, "ctx is NULL");
    Tuning t;
    auto it = c->tuned.find({K, precision});
    if (it != c->tuned.end()) t = it->second;
    if (ring) *ring = t.ring;
    if (range_kb) *range_kb = t.range_kb;
    if (grouped) *grouped = t.grouped;
    if (shape) *shape = t.shape;
    return KRUX_OK;
}

}  // extern "C"
