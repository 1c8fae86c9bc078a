// Static kernels: the generic (data-driven) pattern, histogram and gather path,
// the MFMA contraction of coefficient matrices with background histograms,
// and the small bookkeeping kernels around it.  Model-specialised versions of
// the pattern/histogram/gather kernels are generated at load time (wdf_jit.cpp).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wdf.h"
#include "wdf_dev.h"
#include "wdf_internal.h"

namespace wdf {

// Def. Decision Tree: split(c) is True iff c_f < theta (True goes left); a
// NaN value takes the node's default direction.
__device__ __forceinline__ bool goes_left(float x, float thr, uint8_t dl) {
  return (x != x) ? (dl != 0) : (x < thr);
}

// Def. Decision Pattern along a group's path; the root's bit is the MSB.
__device__ __forceinline__ uint32_t group_pattern(const Group &g, const PathNode *__restrict__ path,
                                                  const float *__restrict__ X, int64_t ldx, int64_t r) {
  uint32_t p = 0;
  for (int k = 0; k < g.depth; ++k) {
    const PathNode nd = path[g.path_off + k];
    const float x = X[(int64_t)nd.feat * ldx + r];
    const bool left = goes_left(x, nd.thr, nd.dl);
    p = (p << 1) | ((left == (nd.dir == 0)) ? 1u : 0u);
  }
  return p;
}

// ---------------------------------------------------------------------------
// Generic path
// ---------------------------------------------------------------------------

constexpr int kGroupsPerBlock = 64;

__global__ __launch_bounds__(256) void k_hist_generic(const Group *__restrict__ groups,
                                                      const PathNode *__restrict__ path, int64_t n_groups,
                                                      const float *__restrict__ B, int64_t m, int64_t ldb,
                                                      uint32_t *__restrict__ hist) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= m) return;
  const int64_t g0 = (int64_t)blockIdx.y * kGroupsPerBlock;
  const int64_t g1 = g0 + kGroupsPerBlock < n_groups ? g0 + kGroupsPerBlock : n_groups;
  for (int64_t gi = g0; gi < g1; ++gi) {
    const Group g = groups[gi];
    const uint32_t p = group_pattern(g, path, B, ldb, r);
    atomicAdd(&hist[g.hist_off + p], 1u);
  }
}

__global__ __launch_bounds__(256) void k_explain_generic(const Group *__restrict__ groups,
                                                         const PathNode *__restrict__ path, int64_t n_groups,
                                                         const float *__restrict__ tab,
                                                         const float *__restrict__ X, int64_t n, int64_t ldx,
                                                         float *__restrict__ phi, int64_t ldphi, int F) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  for (int f = 0; f < F; ++f) phi[(int64_t)f * ldphi + r] = 0.f;
  for (int64_t gi = 0; gi < n_groups; ++gi) {
    const Group g = groups[gi];
    if (g.depth == 0) continue;
    const uint32_t p = group_pattern(g, path, X, ldx, r);
    const float *t = tab + g.tab_off + p;
    for (int k = 0; k < g.depth; ++k) {
      const PathNode nd = path[g.path_off + k];
      if (!nd.first) continue;
      float *dst = phi + (int64_t)nd.feat * ldphi + r;
      *dst += t[(int64_t)k << g.depth];
    }
  }
}

__global__ __launch_bounds__(256) void k_patterns(const Group *__restrict__ groups,
                                                  const PathNode *__restrict__ path, int64_t n_groups,
                                                  const float *__restrict__ X, int64_t n, int64_t ldx,
                                                  uint32_t *__restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const int64_t gi = blockIdx.y;
  out[gi * n + r] = group_pattern(groups[gi], path, X, ldx, r);
}

// ---------------------------------------------------------------------------
// Contraction: columns, MFMA product, expansion into the gather tables
// ---------------------------------------------------------------------------

// Merge a path pattern over its distinct features: the merged bit of a feature
// is the AND of the bits of all path positions carrying it (a repeated feature
// acts as one node whose condition is the intersection of the conditions).
__device__ __forceinline__ uint32_t merge_pattern(const PathNode *__restrict__ pn, int d, int dp, uint32_t p) {
  uint32_t merged = (1u << dp) - 1u;
  for (int k = 0; k < d; ++k) {
    const uint32_t bit = (p >> (d - 1 - k)) & 1u;
    if (!bit) merged &= ~(1u << (dp - 1 - pn[k].merge));
  }
  return merged;
}

// H_{d'}[col][p'] = w * scale * sum over patterns p merging to p' of count[p];
// the right leaf of a pair sees count[p ^ 1] (its pattern is the left's with
// the last bit flipped).  `counts` is uint32 (background) or double
// frequencies (path-dependent: freq for the left or single leaf, freq_r for
// the right leaf of a pair, each indexed by that leaf's own pattern).
__global__ __launch_bounds__(256) void k_columns(const Group *__restrict__ groups,
                                                 const PathNode *__restrict__ path,
                                                 const uint32_t *__restrict__ hist,
                                                 const double *__restrict__ freq, const double *__restrict__ freq_r,
                                                 double scale, const int64_t *__restrict__ class_off,
                                                 double *__restrict__ H) {
  __shared__ uint32_t acc[2 * 256];  // merged counts of the left and right leaf (d' <= 8)
  const Group g = groups[blockIdx.x];
  if (g.depth == 0) return;
  const int d = g.depth, dp = g.dprime;
  const uint32_t K = 1u << dp;
  const PathNode *pn = path + g.path_off;
  double *Hc = H + class_off[dp];
  if (dp < d && hist) {
    // repeated features: scatter the integer counts onto their merged
    // patterns (integer adds: exact in any order, so the result is
    // deterministic), then weight
    for (uint32_t i = threadIdx.x; i < 2 * K; i += blockDim.x) acc[i] = 0u;
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < (1u << d); p += blockDim.x) {
      const uint32_t c = hist[g.hist_off + p];
      if (!c) continue;
      atomicAdd(&acc[merge_pattern(pn, d, dp, p)], c);
      if (g.col_r >= 0) atomicAdd(&acc[K + merge_pattern(pn, d, dp, p ^ 1u)], c);
    }
    __syncthreads();
    for (uint32_t pp = threadIdx.x; pp < K; pp += blockDim.x) {
      Hc[(int64_t)g.col_l * K + pp] = (double)acc[pp] * (double)g.w_l * scale;
      if (g.col_r >= 0) Hc[(int64_t)g.col_r * K + pp] = (double)acc[K + pp] * (double)g.w_r * scale;
    }
    return;
  }
  for (uint32_t pp = threadIdx.x; pp < K; pp += blockDim.x) {
    double sl = 0.0, sr = 0.0;
    if (dp == d) {
      // no repeated feature: the merge only permutes the bits, so exactly one
      // pattern p merges to pp (and p ^ 1 for the right leaf)
      uint32_t p = 0;
      for (int k = 0; k < d; ++k) p |= ((pp >> (dp - 1 - pn[k].merge)) & 1u) << (d - 1 - k);
      sl = hist ? (double)hist[g.hist_off + p] : freq[g.hist_off + p];
      if (g.col_r >= 0) sr = hist ? (double)hist[g.hist_off + (p ^ 1u)] : freq_r[g.hist_off + p];
    } else {
      for (uint32_t p = 0; p < (1u << d); ++p) {
        const double c = hist ? (double)hist[g.hist_off + p] : freq[g.hist_off + p];
        if (merge_pattern(pn, d, dp, p) == pp) sl += c;
        if (g.col_r >= 0) {
          if (hist && merge_pattern(pn, d, dp, p ^ 1u) == pp) sr += c;
          if (!hist && merge_pattern(pn, d, dp, p) == pp) sr += freq_r[g.hist_off + p];
        }
      }
    }
    Hc[(int64_t)g.col_l * K + pp] = sl * (double)g.w_l * scale;
    if (g.col_r >= 0) Hc[(int64_t)g.col_r * K + pp] = sr * (double)g.w_r * scale;
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// S[col][r] = sum_k M[r][k] * H[col][k]  (M: R x K row-major, H: ncols x K)
// for every distinct-feature class of the batch, in one launch.  One wave per
// 32x32 block of a class's output: 2 x 2 tiles of 16x16, each on
// v_mfma_f64_16x16x4f64 over K, so that each A and B fragment feeds two
// MFMAs.  The waves of a class are consecutive (c[i].wave0 on), the row blocks
// of one column block adjacent, so the four waves of a block share their B
// lines in the CU's cache.
//
// K >= 16 (a power of two, operand rows 128-byte aligned): the sum over K is
// taken in blocks of 16, where lane group q (lanes 16q..16q+15) supplies
// k = k0 + 4q + s to the MFMA of step s = 0..3 (the same permutation of k for
// A and B).  A lane's four values are then contiguous: two 16-byte loads per
// operand and tile, and the four lane groups of a row read one whole 128-byte
// line.  Rows or columns past the class's edge read row 0 instead; they only
// reach outputs that are not stored.  Smaller K (d' <= 3) keeps the plain
// order k = k0 + q with zeros past K.
__device__ __forceinline__ void gemm_store(const GemmClass &c, int br, int bc, int lane, const v4d (&acc)[2][2]) {
  // in tile (x, y), output element (row 4*t + lane/16, column lane%16) sits in acc[x][y][t]
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int ccol = bc * 32 + 16 * y + (lane & 15);
      const int rbase = br * 32 + 16 * x + (lane >> 4);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int rr = rbase + 4 * t;
        if (rr < c.R && ccol < c.ncols) c.S[(int64_t)ccol * c.R + rr] = acc[x][y][t];
      }
    }
}

__device__ __forceinline__ void gemm_wave_small(const GemmClass &c, int br, int bc, int lane) {
  const int i = lane & 15, kq = lane >> 4;
  const int arow[2] = {br * 32 + i, br * 32 + 16 + i};
  const int bcol[2] = {bc * 32 + i, bc * 32 + 16 + i};
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < c.K; k0 += 4) {
    const int kk = k0 + kq;
    double a[2], b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      a[h] = (arow[h] < c.R && kk < c.K) ? c.M[(int64_t)arow[h] * c.K + kk] : 0.0;
      b[h] = (bcol[h] < c.ncols && kk < c.K) ? c.H[(int64_t)bcol[h] * c.K + kk] : 0.0;
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
  }
  gemm_store(c, br, bc, lane, acc);
}

// fragments of one block of 16 k values: [tile][pair of k]
struct GemmFrag {
  double2 a[2][2], b[2][2];
};

__device__ __forceinline__ void gemm_load(GemmFrag &f, const double2 *const (&pa)[2], const double2 *const (&pb)[2],
                                          int k2) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    f.a[h][0] = pa[h][k2];
    f.a[h][1] = pa[h][k2 + 1];
    f.b[h][0] = pb[h][k2];
    f.b[h][1] = pb[h][k2 + 1];
  }
}

__device__ __forceinline__ void gemm_mfma16(const GemmFrag &f, v4d (&acc)[2][2]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const double av = (s & 1) ? f.a[x][s >> 1].y : f.a[x][s >> 1].x;
        const double bv = (s & 1) ? f.b[y][s >> 1].y : f.b[y][s >> 1].x;
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[x][y], 0, 0, 0);
      }
}

__device__ __forceinline__ void gemm_wave_wide(const GemmClass &c, int br, int bc, int lane) {
  const int i = lane & 15, kq = lane >> 4;
  const double2 *pa[2], *pb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = br * 32 + 16 * h + i, col = bc * 32 + 16 * h + i;
    pa[h] = (const double2 *)(c.M + (int64_t)(r < c.R ? r : 0) * c.K + 4 * kq);
    pb[h] = (const double2 *)(c.H + (int64_t)(col < c.ncols ? col : 0) * c.K + 4 * kq);
  }
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
  // two fragment buffers: one block's loads are in flight while the other's
  // MFMAs run (indices in double2 units: a block of 16 k is 8 of them).  The
  // loads are unconditional, so that the waits count only the older buffer's;
  // past the end of K they re-read the current block, and those values are
  // not used.
  GemmFrag f0, f1;
  const int K2 = c.K / 2;
  gemm_load(f0, pa, pb, 0);
  for (int k2 = 0; k2 < K2; k2 += 16) {
    const bool second = k2 + 8 < K2;
    gemm_load(f1, pa, pb, second ? k2 + 8 : k2);
    gemm_mfma16(f0, acc);
    gemm_load(f0, pa, pb, k2 + 16 < K2 ? k2 + 16 : k2);
    if (second) gemm_mfma16(f1, acc);
  }
  gemm_store(c, br, bc, lane, acc);
}

__global__ __launch_bounds__(256) void k_gemm_f64(const GemmBatch batch) {
  const int lane = threadIdx.x & 63;
  const int wave = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // this wave's class (constant indices only: the batch stays in kernel arguments)
  GemmClass c = batch.c[0];
#pragma unroll
  for (int k = 1; k < kGemmMaxClasses; ++k)
    if (k < batch.n && wave >= batch.c[k].wave0) c = batch.c[k];
  const int w = wave - c.wave0;
  const int blocks_r = (c.R + 31) >> 5, blocks_c = (c.ncols + 31) >> 5;
  if (w >= blocks_r * blocks_c) return;  // uniform per wave
  const int br = w % blocks_r, bc = w / blocks_r;
  if (c.K >= 16) gemm_wave_wide(c, br, bc, lane);
  else gemm_wave_small(c, br, bc, lane);
}

// tab[g][k][p] = S_l[merge(k)][g(p)] + S_r[merge(k)][g(p ^ 1)] at the first
// position of each feature on the path, 0 at later repeats.
__global__ __launch_bounds__(256) void k_expand(const Group *__restrict__ groups,
                                                const PathNode *__restrict__ path,
                                                const int64_t *__restrict__ s_class_off,
                                                const double *__restrict__ S, float *__restrict__ tab,
                                                double *__restrict__ tab64) {
  const Group g = groups[blockIdx.x];
  if (g.depth == 0) return;
  const int d = g.depth, dp = g.dprime;
  const int64_t K = 1 << dp, R = (int64_t)dp * K;
  const PathNode *pn = path + g.path_off;
  const double *Sc = S + s_class_off[dp];
  const int total = d << d;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int k = idx >> d;
    const uint32_t p = (uint32_t)(idx & ((1 << d) - 1));
    double v = 0.0;
    if (pn[k].first) {
      const int64_t row = (int64_t)pn[k].merge * K;
      v = Sc[(int64_t)g.col_l * R + row + merge_pattern(pn, d, dp, p)];
      if (g.col_r >= 0) v += Sc[(int64_t)g.col_r * R + row + merge_pattern(pn, d, dp, p ^ 1u)];
    }
    tab[g.tab_off + idx] = (float)v;
    if (tab64) tab64[g.tab_off + idx] = v;
  }
}

// Base value: sum over groups of w_l * c[all ones] + w_r * c[all ones ^ 1]
// (path-dependent: w_l * freq[all ones] + w_r * freq_r[all ones]), times
// scale; one block, fixed reduction order (deterministic).
__global__ __launch_bounds__(256) void k_base(const Group *__restrict__ groups, int64_t n_groups,
                                              const uint32_t *__restrict__ hist,
                                              const double *__restrict__ freq, const double *__restrict__ freq_r,
                                              double scale, double *__restrict__ out) {
  __shared__ double part[256];
  double s = 0.0;
  for (int64_t gi = threadIdx.x; gi < n_groups; gi += 256) {
    const Group g = groups[gi];
    const uint32_t all = (1u << g.depth) - 1u;
    const double cl = hist ? (double)hist[g.hist_off + all] : freq[g.hist_off + all];
    s += (double)g.w_l * cl;
    if (g.col_r >= 0) {
      const double cr = hist ? (double)hist[g.hist_off + (all ^ 1u)] : freq_r[g.hist_off + all];
      s += (double)g.w_r * cr;
    }
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0] * scale;
}

// Section 8: freq[p] = prod over the leaf's path positions of r (bit 1) or
// 1 - r (bit 0), r = cover(next node on the path) / cover(node); one block per
// group.  The right leaf of a pair gets its own vector along its own path
// (freq_r, the last ratio ratio_r[group]): with cover(parent) = 0 both last
// ratios are 0 and the right leaf's is not 1 minus the left's.
__global__ __launch_bounds__(256) void k_pd_freq(const Group *__restrict__ groups, const double *__restrict__ ratio,
                                                 const double *__restrict__ ratio_r, double *__restrict__ freq,
                                                 double *__restrict__ freq_r) {
  const Group g = groups[blockIdx.x];
  const int d = g.depth;
  const double *r = ratio + g.path_off;
  for (uint32_t p = threadIdx.x; p < (1u << d); p += blockDim.x) {
    double v = 1.0, vr = 1.0;
    for (int k = 0; k < d; ++k) {
      const bool bit = ((p >> (d - 1 - k)) & 1u) != 0;
      const double rk = k + 1 < d || g.col_r < 0 ? r[k] : ratio_r[blockIdx.x];
      v *= bit ? r[k] : 1.0 - r[k];
      vr *= bit ? rk : 1.0 - rk;
    }
    freq[g.hist_off + p] = v;
    if (g.col_r >= 0) freq_r[g.hist_off + p] = vr;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_hist_generic(const Group *groups, const PathNode *path, int64_t n_groups, const float *B,
                               int64_t m, int64_t ldb, uint32_t *hist, hipStream_t s) {
  if (m <= 0 || n_groups <= 0) return hipSuccess;
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)((n_groups + kGroupsPerBlock - 1) / kGroupsPerBlock));
  hipLaunchKernelGGL(k_hist_generic, grid, dim3(256), 0, s, groups, path, n_groups, B, m, ldb, hist);
  return hipGetLastError();
}

hipError_t launch_explain_generic(const Group *groups, const PathNode *path, int64_t n_groups, const float *tab,
                                  const float *X, int64_t n, int64_t ldx, float *phi, int64_t ldphi, int F,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_explain_generic, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, groups, path,
                     n_groups, tab, X, n, ldx, phi, ldphi, F);
  return hipGetLastError();
}

hipError_t launch_patterns(const Group *groups, const PathNode *path, int64_t n_groups, const float *X,
                           int64_t n, int64_t ldx, uint32_t *out, hipStream_t s) {
  if (n <= 0 || n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_patterns, dim3((unsigned)((n + 255) / 256), (unsigned)n_groups), dim3(256), 0, s, groups,
                     path, n_groups, X, n, ldx, out);
  return hipGetLastError();
}

hipError_t launch_columns(const Group *groups, const PathNode *path, int64_t n_groups, const uint32_t *hist,
                          const double *freq, const double *freq_r, double scale, const int64_t *class_off, double *H,
                          hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_columns, dim3((unsigned)n_groups), dim3(256), 0, s, groups, path, hist, freq, freq_r, scale,
                     class_off, H);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const GemmBatch &batch, int waves, hipStream_t s) {
  if (waves <= 0 || batch.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, batch);
  return hipGetLastError();
}

hipError_t launch_expand(const Group *groups, const PathNode *path, int64_t n_groups, const int64_t *s_class_off,
                         const double *S, float *tab, double *tab64, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)n_groups), dim3(256), 0, s, groups, path, s_class_off, S, tab,
                     tab64);
  return hipGetLastError();
}

hipError_t launch_base(const Group *groups, int64_t n_groups, const uint32_t *hist, const double *freq,
                       const double *freq_r, double scale, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_base, dim3(1), dim3(256), 0, s, groups, n_groups, hist, freq, freq_r, scale, out);
  return hipGetLastError();
}

hipError_t launch_pd_freq(const Group *groups, int64_t n_groups, const double *ratio, const double *ratio_r,
                          double *freq, double *freq_r, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pd_freq, dim3((unsigned)n_groups), dim3(256), 0, s, groups, ratio, ratio_r, freq, freq_r);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Threshold ranks for the model-specialised kernels
// ---------------------------------------------------------------------------

// codes[w * ldc + r]: ranks of the features packed in word w of row r.  The
// rank of x among the sorted distinct thresholds T_f of its feature is
// #{t in T_f : t <= x}, so that x < T_f[j] exactly when rank <= j.  A NaN gets
// the code with only the top bit set (0x80 / 0x8000): it compares below every
// rank as a signed number and above every rank as an unsigned one, which the
// kernels use to send it to the node's default side.
// One block: one word, kQuantRows rows; one thread runs the (up to four)
// searches of a row's word side by side.  Each used feature's thresholds are
// padded with NaN to 2^c entries (c = meta[f].y, offset meta[f].x), so its
// search takes exactly c steps in every lane and never leaves the feature's
// block: NaN never compares <= x.  The word's blocks are contiguous and are
// staged in LDS when they fit.
constexpr int kQuantRows = 2048;
constexpr int kQuantLds = 4096;

// the rows of one block; T is the word's thresholds (LDS or global memory),
// off[k] the block of its k-th feature inside T
__device__ __forceinline__ void quantize_rows(const float *__restrict__ T, const int (&off)[4], const int (&c)[4],
                                              int cmax, const float *__restrict__ X, int64_t r0, int64_t r1,
                                              int64_t ldx, int f0, int nf, int bits, uint32_t *__restrict__ out) {
  const uint32_t nan_code = 1u << (bits - 1);
  // two rows per thread and iteration (r and r + 256; the second re-reads the
  // first when past the end and is not stored), so that their loads and
  // searches overlap
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 512) {
    const int64_t rb = r + 256 < r1 ? r + 256 : r;
    float x[2][4];
    int p[2][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[0][k] = k < nf ? X[(int64_t)(f0 + k) * ldx + r] : 0.f;
      x[1][k] = k < nf ? X[(int64_t)(f0 + k) * ldx + rb] : 0.f;
      p[0][k] = p[1][k] = 0;
    }
    for (int sidx = cmax - 1; sidx >= 0; --sidx) {
      // the searches load unconditionally (a feature past its last step
      // re-reads its own first threshold and ignores it), so the loads overlap
      const int step = 1 << sidx;
      float t[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 4; ++k) t[h][k] = T[sidx < c[k] ? off[k] + p[h][k] + step - 1 : off[k]];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 4; ++k) p[h][k] += (sidx < c[k] && t[h][k] <= x[h][k]) ? step : 0;
    }
    uint32_t word[2] = {0u, 0u};
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < nf) word[h] |= (x[h][k] != x[h][k] ? nan_code : (uint32_t)p[h][k]) << (k * bits);
    out[r] = word[0];
    if (rb != r) out[rb] = word[1];
  }
}

// The same for four consecutive rows per thread: X and the codes are read and
// written with 16-byte accesses (row offsets, ldx and ldc multiples of four,
// 16-byte aligned bases), and a thread runs sixteen searches side by side.
// The last one to three rows of the matrix go through the row-wise loop.
__device__ __forceinline__ void quantize_rows4(const float *__restrict__ T, const int (&off)[4], const int (&c)[4],
                                               int cmax, const float *__restrict__ X, int64_t r0, int64_t r1,
                                               int64_t ldx, int f0, int nf, int bits, uint32_t *__restrict__ out) {
  const uint32_t nan_code = 1u << (bits - 1);
  const int64_t rw = r0 + ((r1 - r0) & ~(int64_t)3);  // end of the whole groups of four
  for (int64_t r = r0 + 4 * (int64_t)threadIdx.x; r < rw; r += 4 * 256) {
    float x[4][4];  // [feature][row]
    int p[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // features past the word's last re-read its first; their ranks are not used
      const float4 v = *(const float4 *)(X + (int64_t)(f0 + (k < nf ? k : 0)) * ldx + r);
      x[k][0] = v.x;
      x[k][1] = v.y;
      x[k][2] = v.z;
      x[k][3] = v.w;
#pragma unroll
      for (int j = 0; j < 4; ++j) p[k][j] = 0;
    }
    for (int sidx = cmax - 1; sidx >= 0; --sidx) {
      const int step = 1 << sidx;
      float t[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) t[k][j] = T[sidx < c[k] ? off[k] + p[k][j] + step - 1 : off[k]];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) p[k][j] += (sidx < c[k] && t[k][j] <= x[k][j]) ? step : 0;
    }
    uint32_t word[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k < nf) word[j] |= (x[k][j] != x[k][j] ? nan_code : (uint32_t)p[k][j]) << (k * bits);
    *(uint4 *)(out + r) = make_uint4(word[0], word[1], word[2], word[3]);
  }
  if (rw < r1) quantize_rows(T, off, c, cmax, X, rw, r1, ldx, f0, nf, bits, out);
}

__global__ __launch_bounds__(256) void k_quantize(const float *__restrict__ X, int64_t n, int64_t ldx, int F,
                                                  const float *__restrict__ thr_pad, const int2 *__restrict__ meta,
                                                  int wide, uint32_t *__restrict__ codes, int64_t ldc, int vec4) {
  __shared__ float st[kQuantLds];
  const int w = blockIdx.y;
  const int per = wide ? 2 : 4, bits = wide ? 16 : 8;
  const int f0 = w * per, nf = min(F - f0, per);
  int off[4], c[4];
  int lo = 0x7fffffff, hi = 0, cmax = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int2 mk = k < nf ? meta[f0 + k] : make_int2(0, 0);
    off[k] = mk.x;
    c[k] = mk.y;
    if (mk.y > 0) {
      lo = min(lo, mk.x);
      hi = max(hi, mk.x + (1 << mk.y));
      cmax = max(cmax, mk.y);
    }
  }
  if (cmax == 0) lo = hi = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) off[k] = c[k] > 0 ? off[k] - lo : 0;
  uint32_t *out = codes + (int64_t)w * ldc;
  const int64_t r0 = (int64_t)blockIdx.x * kQuantRows;
  const int64_t r1 = r0 + kQuantRows < n ? r0 + kQuantRows : n;
  if (hi - lo <= kQuantLds) {
    for (int i = threadIdx.x; i < hi - lo; i += 256) st[i] = thr_pad[lo + i];
    __syncthreads();
    if (vec4) quantize_rows4(st, off, c, cmax, X, r0, r1, ldx, f0, nf, bits, out);
    else quantize_rows(st, off, c, cmax, X, r0, r1, ldx, f0, nf, bits, out);
  } else {
    if (vec4) quantize_rows4(thr_pad + lo, off, c, cmax, X, r0, r1, ldx, f0, nf, bits, out);
    else quantize_rows(thr_pad + lo, off, c, cmax, X, r0, r1, ldx, f0, nf, bits, out);
  }
}

hipError_t launch_quantize(const float *X, int64_t n, int64_t ldx, int F, const float *thr_pad, const int2 *meta,
                           int wide, int words, uint32_t *codes, int64_t ldc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int vec4 = ldx % 4 == 0 && ldc % 4 == 0 && ((uintptr_t)X & 15u) == 0 && ((uintptr_t)codes & 15u) == 0;
  hipLaunchKernelGGL(k_quantize, dim3((unsigned)((n + kQuantRows - 1) / kQuantRows), (unsigned)words), dim3(256), 0, s,
                     X, n, ldx, F, thr_pad, meta, wide, codes, ldc, vec4);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interaction values (Section 3): tables per pair of path positions
// ---------------------------------------------------------------------------

// index of the unordered pair (a, b), a < b, among n positions
__device__ __forceinline__ int pair_index(int a, int b, int n) { return a * (2 * n - a - 1) / 2 + (b - a - 1); }

// tab_iv[iv_off[g] + q * 2^d + p] for the pair q = (k1, k2), k1 < k2, of path
// positions: the contraction product of the pair of distinct features at
// (merge(k1), merge(k2)) for the left leaf's merged pattern, plus the right
// leaf's for p ^ 1; 0 unless both positions are their feature's first.
__global__ __launch_bounds__(256) void k_expand_iv(const Group *__restrict__ groups,
                                                   const PathNode *__restrict__ path,
                                                   const int64_t *__restrict__ iv_off,
                                                   const int64_t *__restrict__ s_class_off,
                                                   const double *__restrict__ S, float *__restrict__ tab) {
  const int gi = blockIdx.x;
  const Group g = groups[gi];
  if (g.depth < 2) return;
  const int d = g.depth, dp = g.dprime;
  const int64_t K = 1 << dp, R = (int64_t)(dp * (dp - 1) / 2) * K;
  const PathNode *pn = path + g.path_off;
  const double *Sc = S + s_class_off[dp];
  const int total = (d * (d - 1) / 2) << d;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int q = idx >> d;
    const uint32_t p = (uint32_t)(idx & ((1 << d) - 1));
    int k1 = 0, rest = q;  // decode q = pair_index(k1, k2, d)
    while (rest >= d - 1 - k1) rest -= d - 1 - k1, ++k1;
    const int k2 = k1 + 1 + rest;
    double v = 0.0;
    if (pn[k1].first && pn[k2].first) {
      const int u = min((int)pn[k1].merge, (int)pn[k2].merge), w = max((int)pn[k1].merge, (int)pn[k2].merge);
      const int64_t row = (int64_t)pair_index(u, w, dp) * K;
      v = Sc[(int64_t)g.col_l * R + row + merge_pattern(pn, d, dp, p)];
      if (g.col_r >= 0) v += Sc[(int64_t)g.col_r * R + row + merge_pattern(pn, d, dp, p ^ 1u)];
    }
    tab[iv_off[gi] + idx] = (float)v;
  }
}

// Interleaved interaction tables (IvUnit): value column k of a unit (its
// partner k, 0 past the last partner) at raw index r is the pair table of
// (i, partner k) at pattern r ^ mask, stored at slot ivunit_slot(r) of the
// column's plane; the rounding pad after the last plane is zeroed.
__global__ __launch_bounds__(256) void k_ivtab(const IvUnit *__restrict__ units, const float *__restrict__ tab,
                                               float *__restrict__ t2) {
  const IvUnit u = units[blockIdx.x];
  const int d = u.depth, E = 1 << d;
  const int nq = ivunit_quads(u.cnt), w = ivunit_tail(u.cnt);
  const int cols = 4 * nq + w, total = (int)ivunit_floats(u);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    if (idx >= cols * E) {
      t2[u.dst + idx] = 0.f;
      continue;
    }
    const int k = idx >> d, r = idx & (E - 1);
    const int s = (int)ivunit_slot((uint32_t)r);
    const int64_t at = k < 4 * nq ? (int64_t)(k >> 2) * 4 * E + 4 * s + (k & 3) : (int64_t)4 * nq * E + w * s + (k - 4 * nq);
    t2[u.dst + at] = k < u.cnt ? tab[u.src + ((int64_t)u.q[k] << d) + (r ^ (int)u.mask)] : 0.f;
  }
}

hipError_t launch_ivtab(const IvUnit *units, int64_t n_units, const float *tab, float *t2, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ivtab, dim3((unsigned)n_units), dim3(256), 0, s, units, tab, t2);
  return hipGetLastError();
}

// Patterns of every group for every row, one byte each (depth <= 8):
// pat[g * n + r].  Computed once per call, read by every feature's wave.
__global__ __launch_bounds__(256) void k_patterns_u8(const Group *__restrict__ groups,
                                                     const PathNode *__restrict__ path, const float *__restrict__ X,
                                                     int64_t n, int64_t ldx, uint8_t *__restrict__ pat) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const int64_t gi = blockIdx.y;
  pat[gi * n + r] = (uint8_t)group_pattern(groups[gi], path, X, ldx, r);
}

hipError_t launch_patterns_u8(const Group *groups, const PathNode *path, int64_t n_groups, const float *X, int64_t n,
                              int64_t ldx, uint8_t *pat, hipStream_t s) {
  if (n <= 0 || n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_patterns_u8, dim3((unsigned)((n + 255) / 256), (unsigned)n_groups), dim3(256), 0, s, groups,
                     path, X, n, ldx, pat);
  return hipGetLastError();
}


// Interaction values of consumer rows: one wave = 64 rows and one feature i
// (blockIdx.y).  The wave walks the work list of i: items (offset of the pair
// table of (i, j) for one group, group << 16 | j), sorted by j, a multiple of
// 8 of them.  Eight items at a time: the rows' patterns of the eight groups
// (loaded while the previous eight are summed), then the eight table entries.
// A register sums the entries of one j (a run of the sorted list); when j
// changes, the sum is stored to iv[(i * F + j) * ldo + r] and the columns that
// have no items (the diagonal among them) get 0.  The lists are uniform
// across the wave, so they are read through the scalar cache, and j is a
// scalar: the run tests are branches of the wave, not of lanes.
__global__ __launch_bounds__(256) void k_explain_iv(const int32_t *__restrict__ item_off,
                                                    const int2 *__restrict__ items,
                                                    const float *__restrict__ tab, const uint8_t *__restrict__ pat,
                                                    int64_t n, float *__restrict__ out, int64_t ldo, int F) {
  constexpr int U = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int i = blockIdx.y;
  const int64_t row = ((int64_t)blockIdx.x * waves + wave) * 64 + lane;
  const int64_t rr = row < n ? row : n - 1;
  const bool live = row < n;
  float *o = out + (int64_t)i * F * ldo + row;
  const int k0 = item_off[i], nch = (item_off[i + 1] - k0) / U;
  int2 it[U];
  uint32_t p[U];
  if (nch) {
#pragma unroll
    for (int u = 0; u < U; ++u) it[u] = items[k0 + u];
#pragma unroll
    for (int u = 0; u < U; ++u) p[u] = pat[(int64_t)((uint32_t)it[u].y >> 16) * n + rr];
  }
  int cur = 0;  // first column not yet stored
  int rj = -1;  // column of the current run
  float run = 0.f;
  for (int c = 0; c < nch; ++c) {
    float v[U];
    int jv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = tab[(int64_t)it[u].x + p[u]];
      jv[u] = it[u].y & 0xffff;
    }
    if (c + 1 < nch) {
#pragma unroll
      for (int u = 0; u < U; ++u) it[u] = items[k0 + (c + 1) * U + u];
#pragma unroll
      for (int u = 0; u < U; ++u) p[u] = pat[(int64_t)((uint32_t)it[u].y >> 16) * n + rr];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (jv[u] != rj) {
        if (rj >= 0) {
          if (live) o[(int64_t)rj * ldo] = run;
          cur = rj + 1;
        }
        for (; cur < jv[u]; ++cur)
          if (live) o[(int64_t)cur * ldo] = 0.f;
        rj = jv[u];
        run = 0.f;
      }
      run += v[u];
    }
  }
  if (rj >= 0) {
    if (live) o[(int64_t)rj * ldo] = run;
    cur = rj + 1;
  }
  for (; cur < F; ++cur)
    if (live) o[(int64_t)cur * ldo] = 0.f;
}

hipError_t launch_expand_iv(const Group *groups, const PathNode *path, int64_t n_groups, const int64_t *iv_off,
                            const int64_t *s_class_off, const double *S, float *tab, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_iv, dim3((unsigned)n_groups), dim3(256), 0, s, groups, path, iv_off, s_class_off, S,
                     tab);
  return hipGetLastError();
}

hipError_t launch_explain_iv(const Group *groups, const PathNode *path, int64_t n_groups, const int32_t *item_off,
                             const int2 *items, const float *tab, const float *X, int64_t n, int64_t ldx, uint8_t *pat,
                             float *out, int64_t ldo, int F, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n_groups > 0) {
    hipLaunchKernelGGL(k_patterns_u8, dim3((unsigned)((n + 255) / 256), (unsigned)n_groups), dim3(256), 0, s, groups,
                       path, X, n, ldx, pat);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int waves = 4;
  const int64_t blocks = (n + 64 * waves - 1) / (64 * waves);
  hipLaunchKernelGGL(k_explain_iv, dim3((unsigned)blocks, (unsigned)F), dim3(64 * waves), 0, s, item_off, items, tab,
                     pat, n, out, ldo, F);
  return hipGetLastError();
}

// Explain tables from the gather tables: each unit re-indexed by raw splits
// and laid out in float4 planes; quads built from their two pair tables.  For a quad of pair depth d, entry I (d+1 bits:
// prefix, s_a, s_aL, s_aR) has the left pair pattern (prefix, s_a, s_aL) and
// the right pair pattern (prefix, !s_a, s_aR); value v < d-1 sums both pairs
// at path position v, v = d-1 is the left pair's last position, v = d the
// right pair's.
__global__ __launch_bounds__(256) void k_xtab(const XUnit *__restrict__ units, const float *__restrict__ tab,
                                              float *__restrict__ xtab) {
  const XUnit u = units[blockIdx.x];
  const int d = u.depth, P = 1 << d;
  const int E = 1 << (d + u.quad), planes = (u.nv + 3) / 4;
  const float *tl = tab + u.src_l, *tr = tab + u.src_r;
  for (int i = threadIdx.x; i < planes * E * 4; i += blockDim.x) {
    const int v = (i / (4 * E)) * 4 + (i & 3), I = (i / 4) % E;
    // entry I sits at slot xunit_slot(I) of its plane (a bijection on [0, E)
    // that spreads entries over the LDS bank groups)
    const int slot = (i / (4 * E)) * 4 * E + 4 * xunit_slot(u, I) + (i & 3);
    float val = 0.f;
    if (v < u.nv) {
      if (!u.quad) {
        val = tl[v * P + (I ^ (int)u.mask)];
      } else {
        // raw splits: the node and its left child go left on the left pair's
        // path, the node goes right and its right child left on the right pair's
        const int prefix = (I >> 3) ^ (int)u.mask, sa = (I >> 2) & 1, sl = (I >> 1) & 1, sr = I & 1;
        const int pl = (prefix << 2) | (sa << 1) | sl;
        const int pr = (prefix << 2) | ((1 - sa) << 1) | sr;
        if (v < d - 1) val = tl[v * P + pl] + tr[v * P + pr];
        else if (v == d - 1) val = tl[(d - 1) * P + pl];
        else val = tr[(d - 1) * P + pr];
      }
    }
    xtab[u.dst + slot] = val;
  }
}

// p[0, n) = v: a kernel rather than a memset node, so that captured graphs
// hold kernels only
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Scratch of the entry points that allocate nothing (wdf_explain_iv_noalloc):
// one array per device, each device that loads the library holding its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: host code passes the address that
// scratch_address() returns on the current device, never the name itself.
static __device__ __align__(256) uint8_t scratch[WDF_NOALLOC_SCRATCH_BYTES];

hipError_t scratch_address(void **out) { return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)); }

hipError_t launch_xtab(const XUnit *units, int64_t n_units, const float *tab, float *xtab, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xtab, dim3((unsigned)n_units), dim3(256), 0, s, units, tab, xtab);
  return hipGetLastError();
}

}  // namespace wdf
