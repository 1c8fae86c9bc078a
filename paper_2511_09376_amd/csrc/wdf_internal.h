// Internal declarations shared by the host code and the static kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wdf_dev.h"

namespace wdf {

hipError_t launch_hist_generic(const Group *groups, const PathNode *path, int64_t n_groups, const float *B,
                               int64_t m, int64_t ldb, uint32_t *hist, hipStream_t s);
hipError_t launch_explain_generic(const Group *groups, const PathNode *path, int64_t n_groups, const float *tab,
                                  const float *X, int64_t n, int64_t ldx, float *phi, int64_t ldphi, int F,
                                  hipStream_t s);
hipError_t launch_patterns(const Group *groups, const PathNode *path, int64_t n_groups, const float *X,
                           int64_t n, int64_t ldx, uint32_t *out, hipStream_t s);
hipError_t launch_columns(const Group *groups, const PathNode *path, int64_t n_groups, const uint32_t *hist,
                          const double *freq, const double *freq_r, double scale, const int64_t *class_off, double *H,
                          hipStream_t s);
// The FP64 products of up to kGemmMaxClasses distinct-feature classes in one
// launch: class i owns waves [c[i].wave0, c[i].wave0 + its 32x32 blocks).
// K is a power of two; for K >= 16, M and H rows must be 16-byte aligned.
constexpr int kGemmMaxClasses = 8;
struct GemmClass {
  const double *M;  // R x K, row-major
  const double *H;  // ncols x K
  double *S;        // ncols x R
  int R, K, ncols, wave0;
};
struct GemmBatch {
  GemmClass c[kGemmMaxClasses];
  int n;
};
// 32x32 output blocks (waves) of one class
inline int gemm_waves(int R, int ncols) { return ((R + 31) / 32) * ((ncols + 31) / 32); }
hipError_t launch_gemm_f64(const GemmBatch &batch, int waves, hipStream_t s);
hipError_t launch_expand(const Group *groups, const PathNode *path, int64_t n_groups, const int64_t *s_class_off,
                         const double *S, float *tab, double *tab64, hipStream_t s);
hipError_t launch_base(const Group *groups, int64_t n_groups, const uint32_t *hist, const double *freq,
                       const double *freq_r, double scale, double *out, hipStream_t s);
hipError_t launch_pd_freq(const Group *groups, int64_t n_groups, const double *ratio, const double *ratio_r,
                          double *freq, double *freq_r, hipStream_t s);
hipError_t launch_quantize(const float *X, int64_t n, int64_t ldx, int F, const float *thr_pad, const int2 *meta,
                           int wide, int words, uint32_t *codes, int64_t ldc, hipStream_t s);
hipError_t launch_expand_iv(const Group *groups, const PathNode *path, int64_t n_groups, const int64_t *iv_off,
                            const int64_t *s_class_off, const double *S, float *tab, hipStream_t s);
hipError_t launch_ivtab(const IvUnit *units, int64_t n_units, const float *tab, float *t2, hipStream_t s);
// patterns of every group into pat (n_groups * n bytes)
hipError_t launch_patterns_u8(const Group *groups, const PathNode *path, int64_t n_groups, const float *X, int64_t n,
                              int64_t ldx, uint8_t *pat, hipStream_t s);
// patterns of every group into pat (n_groups * n bytes), then the interaction kernel
hipError_t launch_explain_iv(const Group *groups, const PathNode *path, int64_t n_groups, const int32_t *item_off,
                             const int2 *items, const float *tab, const float *X, int64_t n, int64_t ldx, uint8_t *pat,
                             float *out, int64_t ldo, int F, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_xtab(const XUnit *units, int64_t n_units, const float *tab, float *xtab, hipStream_t s);
// device address, on the current device, of the library's scratch array
// (WDF_NOALLOC_SCRATCH_BYTES bytes) used by the entry points that allocate nothing
hipError_t scratch_address(void **out);

}  // namespace wdf
