// kx_host.h -- host-side declarations shared by the translation units of the
// library (launchers defined next to their kernels, context hooks in api.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/krux.h"
#include "kx_common.h"

namespace kx {
struct PrepArgs;
struct ScanArgs;
struct TiledArgs;
struct MultiArgs;
struct MultiInfo;
}

extern "C" {
hipError_t kx_launch_rank(const float* expr, int64_t T, int K, int64_t ld, int16_t* ranks2,
                          int64_t* tiesum, int32_t* nvalid, int max_blocks, hipStream_t st);
hipError_t kx_launch_pack(const int8_t* geno, int64_t M, int64_t ld, int K, int64_t m_pad,
                          int gstride, int diag_ok, int8_t* gp, kx::SnpInfo* info,
                          int32_t* tile_flags, int16_t* mpos, int grid, hipStream_t st);
hipError_t kx_launch_prep(const kx::PrepArgs* a, int is_i8, int grid, hipStream_t st);
hipError_t kx_launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
hipError_t kx_launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v,
                              hipStream_t st);
hipError_t kx_launch_list_unresolved(const unsigned long long* minp_bits,
                                     unsigned long long limit_bits, const int32_t* rows_in,
                                     const int32_t* d_n_in, int64_t n_in_max, int32_t* rows_out,
                                     int32_t* d_n_out, hipStream_t st);
hipError_t kx_launch_bits_to_double(const unsigned long long* bits, int64_t n, double* out,
                                    hipStream_t st);
hipError_t kx_launch_scan(const kx::ScanArgs* a, int elem, int ks, int form, int mode, int grid,
                          hipStream_t st);
hipError_t kx_launch_exact(const kx::ScanArgs* a, int grid, hipStream_t st);
hipError_t kx_launch_flag_nan(const int16_t* ranks2, int64_t T, int K, uint8_t* flag,
                              int32_t* list, int32_t* n_list, int grid, hipStream_t st);
hipError_t kx_launch_nan_traits(const kx::ScanArgs* a, const int32_t* list, const int32_t* n_list,
                                int P, int mode, int grid, hipStream_t st);
hipError_t kx_launch_tiled_f16(const kx::ScanArgs* a, const kx::TiledArgs* ta, int form, int mode,
                               int grid, hipStream_t st);
hipError_t kx_launch_tiled_i8(const kx::ScanArgs* a, const kx::TiledArgs* ta, int form, int mode,
                              int grid, hipStream_t st);
hipError_t kx_launch_expand_f16(const int8_t* G, int gstride, const kx::SnpInfo* info,
                                int64_t n_tiles_pad, int ks, int form, void* Bf, int grid,
                                hipStream_t st);
hipError_t kx_launch_expand_i8(const int8_t* G, int gstride, const kx::SnpInfo* info,
                               int64_t n_tiles_pad, int ks, int form, void* Bf, int grid,
                               hipStream_t st);
size_t kx_sort_tmp_bytes(int64_t cap);
hipError_t kx_sort_hits(const kx::HitRec* stage, const unsigned long long* n_hits, int64_t cap,
                        unsigned long long* keys, uint32_t* idx, void* tmp, size_t tmp_bytes,
                        kx::HitRec* out, int64_t* n_out, int trait_bits, int snp_bits,
                        hipStream_t st);
hipError_t kx_launch_miss_keys(const int8_t* geno, int64_t M, int64_t ld, int K, uint64_t* key,
                               int grid, hipStream_t st);
size_t kx_group_tmp_bytes(int64_t M);
hipError_t kx_group_runs(const uint64_t* key, int64_t M, uint64_t* sorted, uint64_t* uniq,
                         uint32_t* counts, uint32_t* n_runs, void* tmp, size_t tmp_bytes,
                         hipStream_t st);
hipError_t kx_group_parts(const uint64_t* key, int64_t M, const uint64_t* big, int G,
                          int32_t* pid, int32_t* pid_sorted, int32_t* idx, int32_t* list,
                          void* tmp, size_t tmp_bytes, int grid, hipStream_t st);
hipError_t kx_launch_pattern_mask(const int8_t* geno, int64_t ld, int K, const int32_t* list,
                                  const int64_t* off, int G, uint8_t* qmask, int grid,
                                  hipStream_t st);
hipError_t kx_launch_check_pattern(const int8_t* geno, int64_t ld, int K, const int32_t* snps,
                                   int64_t n, const uint8_t* qmask, unsigned long long* bad,
                                   int grid, hipStream_t st);
hipError_t kx_launch_gather_rank_cols(const int16_t* ranks2, int64_t T, int K, const int32_t* S,
                                      int Kp, float* out, int grid, hipStream_t st);
hipError_t kx_launch_gather_geno(const int8_t* geno, int64_t ld, const int32_t* rows, int64_t n,
                                 const int32_t* S, int Kp, int8_t* out, int grid, hipStream_t st);
hipError_t kx_launch_append_hits(const kx::HitRec* part, const int64_t* part_n, int64_t cap,
                                 const int32_t* snp_map, int64_t snp_base, kx::HitRec* stage,
                                 unsigned long long* stored, unsigned long long* total, int grid,
                                 hipStream_t st);
hipError_t kx_launch_min_merge(const double* part, double* acc, int64_t n, int grid,
                               hipStream_t st);
hipError_t kx_launch_set_counts(int64_t* n_out, const unsigned long long* total,
                                unsigned long long* stored, int64_t cap, hipStream_t st);
hipError_t kx_launch_multi_pack(const int8_t* geno, int64_t ld, int64_t M, int K, int G,
                                int stride, uint8_t* out, int grid, hipStream_t st);
hipError_t kx_launch_multi_info(const uint8_t* packed, int pstride, int64_t M, int K, int G,
                                kx::MultiInfo* info, int32_t* any_missing, int grid,
                                hipStream_t st);
hipError_t kx_launch_multi_exact(const kx::MultiArgs* a, int n_classes, int grid, hipStream_t st);
hipError_t kx_launch_multi_mfma(const kx::MultiArgs* a, int n_classes, int ks, int grid,
                                hipStream_t st);
hipError_t kx_launch_multi(const kx::MultiArgs* a, int n_classes, int mode, int grid,
                           hipStream_t st);
size_t kx_sort_keys_tmp_bytes(int64_t cap);
hipError_t kx_fdr_curve(const kx::HitRec* real, const int64_t* n_real, int64_t real_cap,
                        const kx::HitRec* perm, const int64_t* n_perm, int64_t perm_cap, int P,
                        unsigned long long* keys_r, unsigned long long* keys_p, void* tmp,
                        size_t tmp_bytes, double* fdr, hipStream_t st);
}

// context hooks (api.cpp)
krux_status kx_fail(krux_ctx* c, krux_status s, const char* msg);
void* kx_ws(krux_ctx* c, int slot, size_t bytes, krux_status* st);
void** kx_blas_handle(krux_ctx* c);
int kx_ctx_device(krux_ctx* c);
double kx_threshold_of(double p_c, int df);
int kx_slot_f64_r();
int kx_slot_f64_i();
int kx_slot_f64_s();
int kx_slot_minp();
int kx_slot_stage();
int kx_slot_nhits();
int kx_slot_keys();
int kx_slot_idx();
int kx_slot_sort_tmp();

// fp64 comparator (fp64.hip)
krux_status kx_fp64_test(krux_ctx* c, const int16_t* ranks2, const int64_t* tiesum, int64_t T,
                         int32_t K, const int8_t* geno, int64_t M, int64_t ld_geno,
                         int64_t snp_base, double p_c, int32_t mode, krux_hit* hits,
                         int64_t hit_capacity, int64_t* n_hits, double* min_p, double* H,
                         double* p, int32_t* sums, hipStream_t st);
void kx_fp64_release(krux_ctx* c);
