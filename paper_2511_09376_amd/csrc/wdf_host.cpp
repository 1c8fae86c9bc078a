// Host side of the C ABI declared in include/wdf.h: ensemble validation and
// layout, coefficient matrices in double precision, background summaries and
// the explain dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "wdf.h"
#include "wdf_dev.h"
#include "wdf_internal.h"
#include "wdf_impl.h"

using namespace wdf;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

namespace wdf {
int set_error(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
int hip_error(hipError_t e, const char *what) {
  return set_error(WDF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace wdf

extern "C" const char *wdf_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------

namespace wdf {

DevBuf::~DevBuf() { reset(); }
void DevBuf::reset() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}
int DevBuf::alloc(size_t n) {
  reset();
  if (n == 0) return WDF_OK;
  hipError_t e = hipMalloc(&ptr, n);
  if (e != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    return set_error(WDF_E_OOM, "hipMalloc(%zu bytes): %s", n, hipGetErrorString(e));
  }
  bytes = n;
  return WDF_OK;
}

int ws_reserve(DevBuf &buf, size_t bytes) {
  if (buf.bytes >= bytes && buf.ptr) return WDF_OK;
  return buf.alloc(std::max<size_t>(bytes, 256));
}

}  // namespace wdf

// Copy a host vector into a fresh device buffer.  The copy completes before
// return, so the vector may be a temporary.
template <class T>
static int upload(DevBuf &buf, const std::vector<T> &v, hipStream_t s) {
  int rc = buf.alloc(v.size() * sizeof(T));
  if (rc) return rc;
  if (!v.empty()) {
    HIP_TRY(hipMemcpyAsync(buf.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return WDF_OK;
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

extern "C" int wdf_create(int device, wdf_ctx **out) {
  if (!out) return set_error(WDF_E_INVALID_ARG, "wdf_create: out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count)
    return set_error(WDF_E_INVALID_ARG, "wdf_create: device %d out of range (%d devices)", device, count);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(WDF_E_UNSUPPORTED, "wdf_create: device %d is %s; this library is built for gfx950", device,
                     prop.gcnArchName);
  std::unique_ptr<wdf_ctx> c(new (std::nothrow) wdf_ctx());
  if (!c) return set_error(WDF_E_OOM, "wdf_create: out of host memory");
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  // the device address of the scratch array of the no-alloc entry points,
  // resolved once per context with its device current
  HIP_TRY(scratch_address(&c->scratch));
  HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  *out = c.release();
  return WDF_OK;
}

extern "C" void wdf_destroy(wdf_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

// ---------------------------------------------------------------------------
// Coefficient matrices (Section 5 four rules, Formulas shap_simplified_formula
// and banzhaf_simplified_formula), for a path of d distinct features
// ---------------------------------------------------------------------------

static double binomial(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * double(n - k + i) / double(i);
  return r;
}

// M[(k * 2^d + pc) * 2^d + pb] = value of the feature at path position k for the
// cube of the pattern pair (pc, pb) with leaf weight 1.  A (0,0) position makes
// the cube unsatisfiable (all zero); (1,0) gives a positive literal, (0,1) a
// negated one, (1,1) no literal.
static void build_coef_matrix(int d, int values, std::vector<double> &M) {
  const int P = 1 << d;
  M.assign((size_t)d * P * P, 0.0);
  for (int pc = 0; pc < P; ++pc) {
    for (int pb = 0; pb < P; ++pb) {
      if (((~pc) & (~pb)) & (P - 1)) continue;  // some position with (0,0)
      const int pos = __builtin_popcount(pc & ~pb & (P - 1));
      const int neg = __builtin_popcount(~pc & pb & (P - 1));
      const int s = pos + neg;
      if (s == 0) continue;
      double cp, cn;
      if (values == WDF_BANZHAF) {
        cp = std::ldexp(1.0, -(s - 1));
        cn = -cp;
      } else {
        cp = pos ? 1.0 / (double(pos) * binomial(s, pos)) : 0.0;
        cn = neg ? -1.0 / (double(neg) * binomial(s, neg)) : 0.0;
      }
      for (int k = 0; k < d; ++k) {
        const int bit = d - 1 - k;
        const int c = (pc >> bit) & 1, b = (pb >> bit) & 1;
        double v = 0.0;
        if (c && !b) v = cp;
        else if (!c && b) v = cn;
        M[((size_t)k * P + pc) * P + pb] = v;
      }
    }
  }
}

// Interaction coefficients (Section 3): M[(q * 2^d + pc) * 2^d + pb] for the
// pair q = (u, v), u < v, of distinct-feature positions: with the cube of
// (pc, pb) built by the same four rules, a = |S+|, b = |S-|, s = a + b, and u, v
// both in the cube: Shapley (Table table_shap_iv) 1/((a-1) C(s-1, a-1)) when
// both are positive, 1/((b-1) C(s-1, b-1)) when both are negated, and
// -1/(a C(s-1, a)) (= -1/(b C(s-1, b))) when the signs differ; Banzhaf
// (Formula banzhaf_simplified_formula_interactions) +-1/2^(s-2), + for equal
// signs.  0 when u or v is not in the cube or the cube is false.
static void build_iv_matrix(int d, int kind, std::vector<double> &M) {
  const int P = 1 << d, Q = d * (d - 1) / 2;
  M.assign((size_t)Q * P * P, 0.0);
  for (int pc = 0; pc < P; ++pc) {
    for (int pb = 0; pb < P; ++pb) {
      if (((~pc) & (~pb)) & (P - 1)) continue;
      const int posm = pc & ~pb & (P - 1), negm = ~pc & pb & (P - 1);
      const int a = __builtin_popcount(posm), b = __builtin_popcount(negm), s = a + b;
      if (s < 2) continue;
      int q = 0;
      for (int u = 0; u < d; ++u) {
        for (int v = u + 1; v < d; ++v, ++q) {
          const int bu = 1 << (d - 1 - u), bv = 1 << (d - 1 - v);
          const bool iu = (posm | negm) & bu, iv = (posm | negm) & bv;
          if (!iu || !iv) continue;
          const bool pu = posm & bu, pv = posm & bv;
          double c;
          if (kind == 1) {
            c = std::ldexp(pu == pv ? 1.0 : -1.0, -(s - 2));
          } else if (pu && pv) {
            c = 1.0 / (double(a - 1) * binomial(s - 1, a - 1));
          } else if (!pu && !pv) {
            c = 1.0 / (double(b - 1) * binomial(s - 1, b - 1));
          } else {
            c = -1.0 / (double(a) * binomial(s - 1, a));
          }
          M[((size_t)q * P + pc) * P + pb] = c;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Model
// ---------------------------------------------------------------------------

int wdf::validate_and_layout(const wdf_model_desc *d, wdf_model *M) {
  if (d->n_trees < 1) return set_error(WDF_E_INVALID_ARG, "model: n_trees must be >= 1");
  if (d->n_features < 1) return set_error(WDF_E_INVALID_ARG, "model: n_features must be >= 1");
  if (d->n_features > WDF_MAX_FEATURES)
    return set_error(WDF_E_UNSUPPORTED, "model: %d features exceeds the limit %d", d->n_features, WDF_MAX_FEATURES);
  if (!d->node_offset || !d->feature || !d->left || !d->right || !d->threshold || !d->value || !d->default_left)
    return set_error(WDF_E_INVALID_ARG, "model: a required array is NULL");
  if (d->node_offset[0] != 0) return set_error(WDF_E_INVALID_ARG, "model: node_offset[0] must be 0");
  const int T = d->n_trees;
  for (int t = 0; t < T; ++t)
    if (d->node_offset[t + 1] <= d->node_offset[t])
      return set_error(WDF_E_INVALID_ARG, "model: tree %d has no nodes", t);
  const int64_t N = d->node_offset[T];
  M->n_trees = T;
  M->n_features = d->n_features;
  M->n_nodes = N;
  M->feature.assign(d->feature, d->feature + N);
  M->left.assign(d->left, d->left + N);
  M->right.assign(d->right, d->right + N);
  M->threshold.assign(d->threshold, d->threshold + N);
  M->value.assign(d->value, d->value + N);
  M->default_left.assign(d->default_left, d->default_left + N);
  M->node_offset.assign(d->node_offset, d->node_offset + T + 1);
  M->has_cover = d->cover != nullptr;
  if (M->has_cover) M->cover.assign(d->cover, d->cover + N);

  // structure checks: every non-root node has exactly one parent, every node is
  // reachable from the root, features in range, paths within the depth limit
  for (int t = 0; t < T; ++t) {
    const int64_t base = d->node_offset[t], nn = d->node_offset[t + 1] - base;
    std::vector<int> parents((size_t)nn, 0), depth((size_t)nn, -1);
    for (int64_t i = 0; i < nn; ++i) {
      const int32_t f = d->feature[base + i], l = d->left[base + i], r = d->right[base + i];
      if (f < 0) {
        if (l != -1 || r != -1)
          return set_error(WDF_E_INVALID_ARG, "model: tree %d node %lld is a leaf with children", t, (long long)i);
        continue;
      }
      if (f >= d->n_features)
        return set_error(WDF_E_INVALID_ARG, "model: tree %d node %lld has feature %d >= n_features %d", t,
                         (long long)i, f, d->n_features);
      if (std::isnan(d->threshold[base + i]))
        return set_error(WDF_E_INVALID_ARG, "model: tree %d node %lld has a NaN threshold", t, (long long)i);
      if (l <= 0 || r <= 0 || l >= nn || r >= nn || l == r)
        return set_error(WDF_E_INVALID_ARG, "model: tree %d node %lld has invalid children (%d, %d)", t,
                         (long long)i, l, r);
      parents[(size_t)l]++;
      parents[(size_t)r]++;
    }
    for (int64_t i = 1; i < nn; ++i)
      if (parents[(size_t)i] != 1)
        return set_error(WDF_E_INVALID_ARG, "model: tree %d node %lld has %d parents", t, (long long)i,
                         parents[(size_t)i]);
    if (parents[0] != 0) return set_error(WDF_E_INVALID_ARG, "model: tree %d root has a parent", t);
    std::vector<int64_t> queue{0};
    depth[0] = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
      const int64_t i = queue[h];
      if (d->feature[base + i] < 0) continue;
      for (int32_t c : {d->left[base + i], d->right[base + i]}) {
        if (depth[(size_t)c] >= 0) return set_error(WDF_E_INVALID_ARG, "model: tree %d has a cycle", t);
        depth[(size_t)c] = depth[(size_t)i] + 1;
        if (depth[(size_t)c] > WDF_MAX_DEPTH)
          return set_error(WDF_E_UNSUPPORTED, "model: tree %d has a path with more than %d inner nodes", t,
                           WDF_MAX_DEPTH);
        queue.push_back(c);
      }
    }
    if ((int64_t)queue.size() != nn)
      return set_error(WDF_E_INVALID_ARG, "model: tree %d has %lld nodes unreachable from the root", t,
                       (long long)(nn - (int64_t)queue.size()));
  }

  // groups in depth-first order per tree
  M->tree_group_off.assign(1, 0);
  for (int t = 0; t < T; ++t) {
    const int64_t base = d->node_offset[t];
    int64_t path_nodes[WDF_MAX_DEPTH + 1];
    uint8_t path_dirs[WDF_MAX_DEPTH + 1];
    auto emit = [&](int dep, int64_t leaf_l, int64_t leaf_r) {
      Group g{};
      g.tree = t;
      g.depth = dep;
      g.path_off = (int32_t)M->path.size();
      g.w_l = d->value[leaf_l];
      g.w_r = leaf_r >= 0 ? d->value[leaf_r] : 0.f;
      g.col_l = -1;
      g.col_r = leaf_r >= 0 ? 0 : -1;  // real columns assigned below
      int32_t feats[WDF_MAX_DEPTH];
      int dp = 0;
      for (int k = 0; k < dep; ++k) {
        const int64_t nd = path_nodes[k];
        PathNode pn{};
        pn.thr = d->threshold[nd];
        pn.feat = d->feature[nd];
        pn.dl = d->default_left[nd] ? 1 : 0;
        pn.dir = path_dirs[k];
        int found = -1;
        for (int q = 0; q < dp; ++q)
          if (feats[q] == pn.feat) found = q;
        if (found < 0) {
          feats[dp] = pn.feat;
          pn.merge = (uint8_t)dp++;
          pn.first = 1;
        } else {
          pn.merge = (uint8_t)found;
          pn.first = 0;
        }
        M->path.push_back(pn);
        M->path_nodes.push_back(nd);
      }
      g.dprime = dp;
      M->groups.push_back(g);
      M->group_leaf_l.push_back(leaf_l);
      M->group_leaf_r.push_back(leaf_r);
    };
    // depth-first; a pair's pattern is its left leaf's (last direction 0)
    std::function<void(int64_t, int)> visit = [&](int64_t local, int dep) {
      const int64_t g = base + local;
      if (d->feature[g] < 0) {
        if (dep == 0) emit(0, g, -1);  // a tree that is a single leaf
        return;
      }
      path_nodes[dep] = g;
      const int64_t l = base + d->left[g], r = base + d->right[g];
      const bool ll = d->feature[l] < 0, rl = d->feature[r] < 0;
      if (ll && rl) {
        path_dirs[dep] = 0;
        emit(dep + 1, l, r);
      } else {
        if (ll) { path_dirs[dep] = 0; emit(dep + 1, l, -1); }
        if (rl) { path_dirs[dep] = 1; emit(dep + 1, r, -1); }
      }
      if (!ll) { path_dirs[dep] = 0; visit(d->left[g], dep + 1); }
      if (!rl) { path_dirs[dep] = 1; visit(d->right[g], dep + 1); }
    };
    visit(0, 0);
    M->tree_group_off.push_back((int64_t)M->groups.size());
  }

  // histogram / table offsets and contraction columns per class
  int64_t h = 0, tb = 0;
  for (auto &g : M->groups) {
    g.hist_off = h;
    g.tab_off = tb;
    h += (int64_t)1 << g.depth;
    tb += (((int64_t)g.depth << g.depth) + 3) & ~(int64_t)3;  // 16-byte aligned tables
    if (g.depth > 0) {
      ClassInfo &c = M->cls[g.dprime];
      g.col_l = c.ncols++;
      g.col_r = (g.col_r >= 0) ? c.ncols++ : -1;
    } else {
      g.col_l = -1;
      g.col_r = -1;
    }
  }
  M->hist_size = h;
  M->tab_size = tb;
  int64_t ho = 0, so = 0;
  for (int dp = 0; dp <= WDF_MAX_DEPTH; ++dp) {
    ClassInfo &c = M->cls[dp];
    c.h_off = ho;
    c.s_off = so;
    // classes start on 128-byte lines: the contraction reads column rows of
    // 2^d' doubles with 16-byte loads
    ho = (ho + ((int64_t)c.ncols << dp) + 15) & ~(int64_t)15;
    so += (int64_t)c.ncols * dp << dp;
  }
  M->h_total = ho;
  M->s_total = so;
  return WDF_OK;
}

static int upload_model(wdf_model *M) {
  hipStream_t s = M->ctx->stream;
  int rc;
  if ((rc = upload(M->d_groups, M->groups, s))) return rc;
  if ((rc = upload(M->d_path, M->path, s))) return rc;
  std::vector<int64_t> hoff(WDF_MAX_DEPTH + 1), soff(WDF_MAX_DEPTH + 1);
  for (int dp = 0; dp <= WDF_MAX_DEPTH; ++dp) {
    hoff[(size_t)dp] = M->cls[dp].h_off;
    soff[(size_t)dp] = M->cls[dp].s_off;
  }
  if ((rc = upload(M->d_hclass_off, hoff, s))) return rc;
  if ((rc = upload(M->d_sclass_off, soff, s))) return rc;
  for (int values = 0; values < 2; ++values) {
    for (int dp = 1; dp <= WDF_MAX_DEPTH; ++dp) {
      if (M->cls[dp].ncols == 0) continue;
      std::vector<double> coef;
      build_coef_matrix(dp, values, coef);
      if ((rc = upload(M->d_coef[values][dp], coef, s))) return rc;
    }
  }
  if (M->has_cover) {
    // cover ratio of every path position: cover(next node) / cover(node)
    std::vector<double> ratio(M->path.size(), 0.0);
    for (size_t gi = 0; gi < M->groups.size(); ++gi) {
      const Group &g = M->groups[gi];
      for (int k = 0; k < g.depth; ++k) {
        const int64_t nd = M->path_nodes[(size_t)g.path_off + k];
        const int64_t base = M->node_offset[(size_t)g.tree];
        int64_t nx;
        if (k + 1 < g.depth) nx = M->path_nodes[(size_t)g.path_off + k + 1];
        else nx = M->path[(size_t)g.path_off + k].dir ? base + M->right[(size_t)nd] : base + M->left[(size_t)nd];
        const double cn = M->cover[(size_t)nd];
        ratio[(size_t)g.path_off + k] = cn > 0 ? M->cover[(size_t)nx] / cn : 0.0;
      }
    }
    if ((rc = upload(M->d_ratio, ratio, s))) return rc;
    // the right leaf of a pair: its last ratio cover(right leaf) / cover(parent),
    // 0 when no training row reached the parent (then it is not 1 minus the
    // left leaf's, which is 0 as well)
    std::vector<double> ratio_r(std::max<size_t>(M->groups.size(), 1), 0.0);
    for (size_t gi = 0; gi < M->groups.size(); ++gi) {
      const Group &g = M->groups[gi];
      if (g.col_r < 0 || g.depth == 0) continue;
      const double cp = M->cover[(size_t)M->path_nodes[(size_t)g.path_off + (size_t)g.depth - 1]];
      ratio_r[gi] = cp > 0 ? M->cover[(size_t)M->group_leaf_r[gi]] / cp : 0.0;
    }
    if ((rc = upload(M->d_ratio_r, ratio_r, s))) return rc;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return WDF_OK;
}

extern "C" int wdf_model_load(wdf_ctx *ctx, const wdf_model_desc *desc, int kernel, wdf_model **out) {
  if (!ctx || !desc || !out) return set_error(WDF_E_INVALID_ARG, "wdf_model_load: NULL argument");
  *out = nullptr;
  const bool quads = (kernel & WDF_KERNEL_PAIRS) == 0;
  kernel &= ~WDF_KERNEL_PAIRS;
  if (kernel < WDF_KERNEL_AUTO || kernel > WDF_KERNEL_SPECIALISED)
    return set_error(WDF_E_INVALID_ARG, "wdf_model_load: unknown kernel choice %d", kernel);
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<wdf_model> M(new (std::nothrow) wdf_model());
  if (!M) return set_error(WDF_E_OOM, "wdf_model_load: out of host memory");
  M->ctx = ctx;
  M->device = ctx->device;
  int rc;
  try {
    if ((rc = validate_and_layout(desc, M.get()))) return rc;
  } catch (const std::bad_alloc &) {
    return set_error(WDF_E_OOM, "wdf_model_load: out of host memory");
  }
  if ((rc = upload_model(M.get()))) return rc;
  if (kernel != WDF_KERNEL_GENERIC) {
    M->jp.quad_depth = quads ? WDF_MAX_DEPTH : 0;
    rc = jit_build(M.get());
    if (rc != WDF_OK) {
      if (kernel == WDF_KERNEL_SPECIALISED) return rc;
      M->jit.reset();  // AUTO: keep the generic kernels
    }
  }
  *out = M.release();
  return WDF_OK;
}

extern "C" void wdf_model_destroy(wdf_model *model) {
  if (!model) return;
  (void)hipSetDevice(model->device);
  delete model;
}

extern "C" int wdf_model_specialised(const wdf_model *model) { return (model && model->jit) ? 1 : 0; }

extern "C" int wdf_bg_specialised(const wdf_bg *bg) {
  if (!bg) return 0;
  return (bg->iv ? bg->iv_spec : bg->model->jit != nullptr) ? 1 : 0;
}

extern "C" int64_t wdf_model_groups(const wdf_model *model, int32_t *tree, int32_t *depth, int64_t *leaf_left,
                                    int64_t *leaf_right, int64_t *hist_offset, int64_t *table_offset) {
  if (!model) return set_error(WDF_E_INVALID_ARG, "wdf_model_groups: NULL model");
  const size_t G = model->groups.size();
  for (size_t i = 0; i < G; ++i) {
    const Group &g = model->groups[i];
    if (tree) tree[i] = g.tree;
    if (depth) depth[i] = g.depth;
    if (leaf_left) leaf_left[i] = model->group_leaf_l[i];
    if (leaf_right) leaf_right[i] = model->group_leaf_r[i];
    if (hist_offset) hist_offset[i] = g.hist_off;
    if (table_offset) table_offset[i] = g.tab_off;
  }
  return (int64_t)G;
}

// ---------------------------------------------------------------------------
// Background summary: patterns -> histograms -> MFMA contraction -> tables
// ---------------------------------------------------------------------------

// NULL selects the HIP null stream, which orders with every blocking stream
// (torch's default stream is the null stream).
static hipStream_t pick_stream(wdf_ctx *, void *s) { return (hipStream_t)s; }

// Interaction layout and coefficient matrices, prepared once per model and
// kind (the caller holds the model's workspace lock).
// Host side of the interaction layout: table offsets, the generic kernel's
// work lists (ioff, items) and the specialised kernel's units.  Needs no GPU.
static int iv_layout_host(wdf_model *M, std::vector<int32_t> &ioff, std::vector<int32_t> &items) {
  const size_t G = M->groups.size();
  M->iv_off.assign(G, 0);
  int64_t off = 0;
  for (size_t g = 0; g < G; ++g) {
    const int d = M->groups[g].depth;
    M->iv_off[g] = off;
    off += ((((int64_t)d * (d - 1) / 2) << d) + 3) & ~(int64_t)3;
  }
  M->iv_tab_size = off;
  int64_t so = 0;
  for (int dp = 0; dp <= WDF_MAX_DEPTH; ++dp) {
    M->s_iv_class_off[dp] = so;
    so += (int64_t)M->cls[dp].ncols * (dp * (dp - 1) / 2) << dp;
  }
  M->s_iv_total = so;
  // Work lists of the interaction kernel, one per feature i: for every
  // group where i and another feature j both have a first occurrence on the
  // path, one item (offset of the pair table of (i, j) in the interaction
  // tables, group << 16 | j), sorted by j, then group.  Each list is padded
  // to a multiple of 8 items with items of its last j that read the zero
  // block after the tables.
  const int F = M->n_features;
  if (M->iv_tab_size + 256 >= ((int64_t)1 << 31))
    return set_error(WDF_E_UNSUPPORTED, "interaction tables of %lld floats exceed 2^31", (long long)M->iv_tab_size);
  if (G > 65535 || F > 65535)
    return set_error(WDF_E_UNSUPPORTED, "interaction values: %zu groups or %d features exceed 65535", G, F);
  std::vector<std::vector<std::array<int32_t, 3>>> lists((size_t)F);  // (j, group, table offset)
  for (size_t g = 0; g < G; ++g) {
    const Group &gr = M->groups[g];
    const int d = gr.depth;
    for (int k1 = 0; k1 < d; ++k1) {
      const PathNode &a = M->path[(size_t)gr.path_off + k1];
      if (!a.first) continue;
      for (int k2 = 0; k2 < d; ++k2) {
        const PathNode &b = M->path[(size_t)gr.path_off + k2];
        if (k2 == k1 || !b.first) continue;
        const int u = std::min(k1, k2), v = std::max(k1, k2);
        const int q = u * (2 * d - u - 1) / 2 + (v - u - 1);
        lists[(size_t)a.feat].push_back({b.feat, (int32_t)g, (int32_t)(M->iv_off[g] + ((int64_t)q << d))});
      }
    }
  }
  ioff.assign((size_t)F + 1, 0);
  items.clear();
  for (int f = 0; f < F; ++f) {
    auto &l = lists[(size_t)f];
    std::sort(l.begin(), l.end());
    for (const auto &e : l) items.insert(items.end(), {e[2], (int32_t)((uint32_t)e[1] << 16 | (uint32_t)e[0])});
    if (!l.empty())
      while ((items.size() / 2) % 8) items.insert(items.end(), {(int32_t)M->iv_tab_size, l.back()[0]});
    ioff[(size_t)f + 1] = (int32_t)(items.size() / 2);
  }
  if (items.empty()) items.assign(2, 0);
  // Units of the interleaved tables (specialised kernel): per feature i,
  // one per group where i has a first occurrence and a partner, in group
  // order; a feature's units are contiguous in the tables.
  std::vector<std::vector<IvUnit>> ufeat((size_t)F);
  std::vector<std::vector<std::array<int32_t, 7>>> upart((size_t)F);
  for (size_t g = 0; g < G; ++g) {
    const Group &gr = M->groups[g];
    const int d = gr.depth;
    for (int k1 = 0; k1 < d; ++k1) {
      const PathNode &a = M->path[(size_t)gr.path_off + k1];
      if (!a.first) continue;
      IvUnit u{};
      std::array<int32_t, 7> js{};
      u.src = M->iv_off[g];
      u.depth = d;
      u.group = (int32_t)g;
      for (int k = 0; k < d; ++k)
        if (M->path[(size_t)gr.path_off + k].dir) u.mask |= 1u << (d - 1 - k);
      for (int k2 = 0; k2 < d; ++k2) {
        const PathNode &b = M->path[(size_t)gr.path_off + k2];
        if (k2 == k1 || !b.first) continue;
        const int lo = std::min(k1, k2), hi = std::max(k1, k2);
        js[(size_t)u.cnt] = b.feat;
        u.q[u.cnt++] = lo * (2 * d - lo - 1) / 2 + (hi - lo - 1);
      }
      if (u.cnt > 0) {
        ufeat[(size_t)a.feat].push_back(u);
        upart[(size_t)a.feat].push_back(js);
      }
    }
  }
  M->iv_units.clear();
  M->iv_unit_partners.clear();
  M->iv_unit_off.assign((size_t)F + 1, 0);
  int64_t dst = 0;
  for (int f = 0; f < F; ++f) {
    for (size_t k = 0; k < ufeat[(size_t)f].size(); ++k) {
      IvUnit &u = ufeat[(size_t)f][k];
      u.dst = dst;
      dst += ivunit_floats(u);
      M->iv_units.push_back(u);
      M->iv_unit_partners.push_back(upart[(size_t)f][k]);
    }
    M->iv_unit_off[(size_t)f + 1] = (int32_t)M->iv_units.size();
  }
  M->iv_units_size = dst;
  return WDF_OK;
}

static int prepare_iv(wdf_model *M, int kind) {
  hipStream_t s = M->ctx->stream;
  int rc;
  if (!M->iv_layout) {
    std::vector<int32_t> ioff, items;
    if ((rc = iv_layout_host(M, ioff, items))) return rc;
    if ((rc = upload(M->d_iv_units, M->iv_units.empty() ? std::vector<IvUnit>(1) : M->iv_units, s))) return rc;
    std::vector<int64_t> soff(M->s_iv_class_off, M->s_iv_class_off + WDF_MAX_DEPTH + 1);
    if ((rc = upload(M->d_iv_off, M->iv_off.empty() ? std::vector<int64_t>(1, 0) : M->iv_off, s))) return rc;
    if ((rc = upload(M->d_siv_class_off, soff, s))) return rc;
    if ((rc = upload(M->d_iv_item_off, ioff, s))) return rc;
    if ((rc = upload(M->d_iv_items, items, s))) return rc;
    M->iv_layout = true;
  }
  if (!M->iv_coef_ready[kind]) {
    for (int dp = 2; dp <= WDF_MAX_DEPTH; ++dp) {
      if (M->cls[dp].ncols == 0) continue;
      std::vector<double> coef;
      build_iv_matrix(dp, kind, coef);
      if ((rc = upload(M->d_coef_iv[kind][dp], coef, s))) return rc;
    }
    M->iv_coef_ready[kind] = true;
  }
  return WDF_OK;
}

// Table storage of a summary, zeroed once (the padding between tables, and the
// 256 floats after the interaction tables that padding items read, are never
// written again).
static int alloc_tables(wdf_model *M, wdf_bg *bg, hipStream_t s) {
  int rc;
  const int64_t n = bg->iv ? M->iv_tab_size + 256 : M->tab_size;
  if ((rc = bg->d_tab.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(float)))) return rc;
  HIP_TRY(hipMemsetAsync(bg->d_tab.ptr, 0, bg->d_tab.bytes, s));
  if (M->jit && !bg->iv) {
    if ((rc = bg->d_xtab.alloc((size_t)std::max<int64_t>(M->jp.xtab_size, 1) * sizeof(float)))) return rc;
    HIP_TRY(hipMemsetAsync(bg->d_xtab.ptr, 0, bg->d_xtab.bytes, s));
  }
  if (bg->iv_spec) {
    if ((rc = bg->d_xtab.alloc((size_t)std::max<int64_t>(M->iv_units_size, 1) * sizeof(float)))) return rc;
    HIP_TRY(hipMemsetAsync(bg->d_xtab.ptr, 0, bg->d_xtab.bytes, s));
  }
  return WDF_OK;
}

// The MFMA products S = M_{d'} H_{d'} of every distinct-feature class d'
// (Section 7 steps (e)-(f)), all classes in one FP64 GEMM launch.  *flops
// (when given) receives their floating-point operations, 2 R K per column.
static_assert(kGemmMaxClasses >= WDF_MAX_DEPTH, "one launch holds every class d' = 1..WDF_MAX_DEPTH");
static int enqueue_gemms(wdf_model *M, const wdf_bg *bg, const double *H, double *S, hipStream_t s, double *flops) {
  double f = 0.0;
  GemmBatch batch{};
  int waves = 0;
  for (int dp = bg->iv ? 2 : 1; dp <= WDF_MAX_DEPTH; ++dp) {
    const ClassInfo &c = M->cls[dp];
    if (c.ncols == 0) continue;
    const int K = 1 << dp, R = (bg->iv ? dp * (dp - 1) / 2 : dp) * K;
    const double *coef = bg->iv ? M->d_coef_iv[bg->values - WDF_SHAPLEY_IV][dp].as<double>()
                                : M->d_coef[bg->values][dp].as<double>();
    double *Sc = S + (bg->iv ? M->s_iv_class_off[dp] : c.s_off);
    batch.c[batch.n++] = GemmClass{coef, H + c.h_off, Sc, R, K, c.ncols, waves};
    waves += gemm_waves(R, c.ncols);
    f += 2.0 * (double)R * (double)K * (double)c.ncols;
  }
  HIP_TRY(launch_gemm_f64(batch, waves, s));
  if (flops) *flops = f;
  return WDF_OK;
}

// Columns, MFMA products per class, expansion into the gather tables (and the
// explain tables), base value into *base: kernel launches only.
static int enqueue_contract(wdf_model *M, wdf_bg *bg, const uint32_t *hist, const double *freq, double scale,
                            double *H, double *S, double *base, hipStream_t s) {
  const int64_t G = (int64_t)M->groups.size();
  const double *freq_r = freq ? freq + M->hist_size : nullptr;  // right leaves' own frequencies
  HIP_TRY(launch_columns(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), G, hist, freq, freq_r, scale,
                         M->d_hclass_off.as<int64_t>(), H, s));
  if (bg->iv) {  // pair products per class, then pair tables
    int rc;
    if ((rc = enqueue_gemms(M, bg, H, S, s, nullptr))) return rc;
    HIP_TRY(launch_expand_iv(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), G, M->d_iv_off.as<int64_t>(),
                             M->d_siv_class_off.as<int64_t>(), S, bg->d_tab.as<float>(), s));
    if (bg->iv_spec)  // interleaved tables of the specialised interaction kernel
      HIP_TRY(launch_ivtab(M->d_iv_units.as<IvUnit>(), (int64_t)M->iv_units.size(), bg->d_tab.as<float>(),
                           bg->d_xtab.as<float>(), s));
    HIP_TRY(launch_base(M->d_groups.as<Group>(), G, hist, freq, freq_r, hist ? 1.0 / (double)bg->m : 1.0, base, s));
    return WDF_OK;
  }
  int rc;
  if ((rc = enqueue_gemms(M, bg, H, S, s, nullptr))) return rc;
  HIP_TRY(launch_expand(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), G, M->d_sclass_off.as<int64_t>(), S,
                        bg->d_tab.as<float>(), nullptr, s));
  if (M->jit)  // explain tables of the specialised kernel
    HIP_TRY(launch_xtab(M->jp.d_xunits.as<XUnit>(), (int64_t)M->jp.xunits.size(), bg->d_tab.as<float>(),
                        bg->d_xtab.as<float>(), s));
  HIP_TRY(launch_base(M->d_groups.as<Group>(), G, hist, freq, freq_r, hist ? 1.0 / (double)bg->m : 1.0, base, s));
  return WDF_OK;
}

// Summary of a new background: tables allocated, contraction with the model's
// shared workspace, base value copied to the host, stream synchronised.
static int contract(wdf_model *M, wdf_bg *bg, const uint32_t *hist, const double *freq, double scale,
                    hipStream_t s) {
  DevBuf &H = M->ws_H, &S = M->ws_S, &base = M->ws_base;
  int rc;
  if ((rc = ws_reserve(H, (size_t)std::max<int64_t>(M->h_total, 1) * sizeof(double)))) return rc;
  if ((rc = ws_reserve(S, (size_t)std::max<int64_t>(bg->iv ? M->s_iv_total : M->s_total, 1) * sizeof(double))))
    return rc;
  if ((rc = ws_reserve(base, sizeof(double)))) return rc;
  if ((rc = alloc_tables(M, bg, s))) return rc;
  if ((rc = enqueue_contract(M, bg, hist, freq, scale, H.as<double>(), S.as<double>(), base.as<double>(), s)))
    return rc;
  HIP_TRY(hipMemcpyAsync(&bg->base, base.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return WDF_OK;
}

extern "C" int wdf_background_load(wdf_model *M, const float *B, int64_t m, int64_t ldb, int b_on_device,
                                   int values, void *hip_stream, wdf_bg **out) {
  if (!M || !B || !out) return set_error(WDF_E_INVALID_ARG, "wdf_background_load: NULL argument");
  *out = nullptr;
  if (m < 1 || ldb < m) return set_error(WDF_E_INVALID_ARG, "wdf_background_load: need m >= 1 and ldb >= m");
  if (m > 0xFFFFFFFFll) return set_error(WDF_E_UNSUPPORTED, "wdf_background_load: m exceeds uint32 counts");
  if (values < WDF_SHAPLEY || values > WDF_BANZHAF_IV)
    return set_error(WDF_E_INVALID_ARG, "wdf_background_load: unknown value kind %d", values);
  HIP_TRY(hipSetDevice(M->ctx->device));
  hipStream_t s = pick_stream(M->ctx, hip_stream);
  std::unique_ptr<wdf_bg> bg(new (std::nothrow) wdf_bg());
  if (!bg) return set_error(WDF_E_OOM, "wdf_background_load: out of host memory");
  std::lock_guard<std::mutex> ws_lock(M->ws_mu);
  bg->model = M;
  bg->device = M->device;
  bg->m = m;
  bg->values = values;
  bg->iv = values >= WDF_SHAPLEY_IV;
  if (bg->iv) {
    int rc_iv;
    if ((rc_iv = prepare_iv(M, values - WDF_SHAPLEY_IV))) return rc_iv;
    if (M->jit) {  // the specialised interaction kernels; the generic one when they cannot be built
      rc_iv = jit_build_iv(M);
      if (rc_iv == WDF_E_OOM || rc_iv == WDF_E_DEVICE) return rc_iv;
      bg->iv_spec = rc_iv == WDF_OK;
    }
  }
  int rc;
  DevBuf Bcopy;
  const float *Bd = B;
  if (!b_on_device) {
    if ((rc = Bcopy.alloc((size_t)M->n_features * (size_t)m * sizeof(float)))) return rc;
    HIP_TRY(hipMemcpy2DAsync(Bcopy.ptr, (size_t)m * sizeof(float), B, (size_t)ldb * sizeof(float),
                             (size_t)m * sizeof(float), (size_t)M->n_features, hipMemcpyHostToDevice, s));
    Bd = Bcopy.as<float>();
    ldb = m;
  }
  if ((rc = bg->d_hist.alloc((size_t)std::max<int64_t>(M->hist_size, 1) * sizeof(uint32_t)))) return rc;
  HIP_TRY(hipMemsetAsync(bg->d_hist.ptr, 0, bg->d_hist.bytes, s));
  if (M->jit) {
    if ((rc = ws_reserve(M->ws_codes, (size_t)M->jp.words * (size_t)m * sizeof(uint32_t)))) return rc;
    if ((rc = jit_hist(M, Bd, m, ldb, bg->d_hist.as<uint32_t>(), M->ws_codes.as<uint32_t>(), s))) return rc;
  } else {
    HIP_TRY(launch_hist_generic(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), (int64_t)M->groups.size(), Bd,
                                m, ldb, bg->d_hist.as<uint32_t>(), s));
  }
  if ((rc = contract(M, bg.get(), bg->d_hist.as<uint32_t>(), nullptr, 1.0 / (double)m, s))) return rc;
  ++M->n_bg;
  *out = bg.release();
  return WDF_OK;
}

// Private workspace of in-place refreshes.
static int ensure_refresh_workspace(wdf_bg *bg) {
  wdf_model *M = bg->model;
  int rc;
  if (M->jit && !bg->own_codes.ptr &&
      (rc = bg->own_codes.alloc((size_t)M->jp.words * (size_t)bg->m * sizeof(uint32_t))))
    return rc;
  if (!bg->own_H.ptr && (rc = bg->own_H.alloc((size_t)std::max<int64_t>(M->h_total, 1) * sizeof(double)))) return rc;
  if (!bg->own_S.ptr &&
      (rc = bg->own_S.alloc((size_t)std::max<int64_t>(bg->iv ? M->s_iv_total : M->s_total, 1) * sizeof(double))))
    return rc;
  if (!bg->d_base.ptr) {
    // seeded with the load's base value, so that the value read back from the
    // device is valid before the first refresh has run
    if ((rc = bg->d_base.alloc(sizeof(double)))) return rc;
    HIP_TRY(hipMemcpy(bg->d_base.ptr, &bg->base, sizeof(double), hipMemcpyHostToDevice));
  }
  return WDF_OK;
}

// The launches of a refresh: histograms cleared by a kernel, recounted,
// contracted; nothing else.
static int enqueue_refresh(wdf_bg *bg, const float *B, int64_t ldb, hipStream_t s) {
  wdf_model *M = bg->model;
  const int64_t m = bg->m;
  int rc;
  HIP_TRY(launch_fill_u32(bg->d_hist.as<uint32_t>(), std::max<int64_t>(M->hist_size, 1), 0u, s));
  if (M->jit) {
    if ((rc = jit_hist(M, B, m, ldb, bg->d_hist.as<uint32_t>(), bg->own_codes.as<uint32_t>(), s))) return rc;
  } else {
    HIP_TRY(launch_hist_generic(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), (int64_t)M->groups.size(), B, m,
                                ldb, bg->d_hist.as<uint32_t>(), s));
  }
  return enqueue_contract(M, bg, bg->d_hist.as<uint32_t>(), nullptr, 1.0 / (double)m, bg->own_H.as<double>(),
                          bg->own_S.as<double>(), bg->d_base.as<double>(), s);
}

static int check_refresh(const wdf_bg *bg, const float *B, int64_t ldb, const char *who) {
  if (!bg || !B) return set_error(WDF_E_INVALID_ARG, "%s: NULL argument", who);
  if (bg->pathdep) return set_error(WDF_E_INVALID_ARG, "%s: a path-dependent summary has no background", who);
  if (ldb < bg->m) return set_error(WDF_E_INVALID_ARG, "%s: need ldb >= m", who);
  return WDF_OK;
}

extern "C" int wdf_background_refresh(wdf_bg *bg, const float *B, int64_t ldb, void *hip_stream) {
  int rc;
  if ((rc = check_refresh(bg, B, ldb, "wdf_background_refresh"))) return rc;
  HIP_TRY(hipSetDevice(bg->device));
  if ((rc = ensure_refresh_workspace(bg))) return rc;
  if ((rc = enqueue_refresh(bg, B, ldb, pick_stream(bg->model->ctx, hip_stream)))) return rc;
  bg->base_on_device = true;
  return WDF_OK;
}

// ---------------------------------------------------------------------------
// HIP graphs: refresh + explain recorded once, replayed
// ---------------------------------------------------------------------------

extern "C" int wdf_graph_create(wdf_bg *bg, const float *B, int64_t ldb, const float *X, int64_t n, int64_t ldx,
                                float *phi, int64_t ldphi, wdf_graph **out) {
  if (!bg || !out) return set_error(WDF_E_INVALID_ARG, "wdf_graph_create: NULL argument");
  *out = nullptr;
  int rc;
  if (B && (rc = check_refresh(bg, B, ldb, "wdf_graph_create"))) return rc;
  if (n < 0 || (n > 0 && (!X || !phi || ldx < n || ldphi < n)))
    return set_error(WDF_E_INVALID_ARG, "wdf_graph_create: need X, phi and 0 <= n <= ldx, ldphi");
  if (!B && n == 0) return set_error(WDF_E_INVALID_ARG, "wdf_graph_create: nothing to record");
  HIP_TRY(hipSetDevice(bg->device));
  if (B && (rc = ensure_refresh_workspace(bg))) return rc;
  std::unique_ptr<wdf_graph> g(new (std::nothrow) wdf_graph());
  if (!g) return set_error(WDF_E_OOM, "wdf_graph_create: out of host memory");
  g->bg = bg;
  g->device = bg->device;
  HIP_TRY(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
  auto fail = [&](int code) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipStreamDestroy(g->stream);
    return code;
  };
  hipError_t e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail(hip_error(e, "hipStreamBeginCapture"));
  rc = WDF_OK;
  if (B) rc = enqueue_refresh(bg, B, ldb, g->stream);
  if (!rc && n > 0) rc = wdf_explain(bg, X, n, ldx, phi, ldphi, g->stream);
  e = hipStreamEndCapture(g->stream, &g->graph);
  if (rc) return fail(rc);
  if (e != hipSuccess) return fail(hip_error(e, "hipStreamEndCapture"));
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return fail(hip_error(e, "hipGraphInstantiate"));
  if (B) bg->base_on_device = true;  // the base value is read from the device from now on
  *out = g.release();
  return WDF_OK;
}

extern "C" int wdf_graph_launch(wdf_graph *g, void *hip_stream) {
  if (!g) return set_error(WDF_E_INVALID_ARG, "wdf_graph_launch: NULL graph");
  HIP_TRY(hipSetDevice(g->device));
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
  return WDF_OK;
}

extern "C" void wdf_graph_destroy(wdf_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

extern "C" int wdf_pathdep_load(wdf_model *M, int values, void *hip_stream, wdf_bg **out) {
  if (!M || !out) return set_error(WDF_E_INVALID_ARG, "wdf_pathdep_load: NULL argument");
  *out = nullptr;
  if (!M->has_cover) return set_error(WDF_E_INVALID_ARG, "wdf_pathdep_load: the model was loaded without covers");
  if (values != WDF_SHAPLEY && values != WDF_BANZHAF)
    return set_error(WDF_E_INVALID_ARG, "wdf_pathdep_load: value kind %d (interaction kinds need a background)",
                     values);
  HIP_TRY(hipSetDevice(M->ctx->device));
  hipStream_t s = pick_stream(M->ctx, hip_stream);
  std::unique_ptr<wdf_bg> bg(new (std::nothrow) wdf_bg());
  if (!bg) return set_error(WDF_E_OOM, "wdf_pathdep_load: out of host memory");
  std::lock_guard<std::mutex> ws_lock(M->ws_mu);
  bg->model = M;
  bg->device = M->device;
  bg->m = 0;
  bg->values = values;
  bg->iv = values >= WDF_SHAPLEY_IV;
  if (bg->iv) {
    int rc_iv;
    if ((rc_iv = prepare_iv(M, values - WDF_SHAPLEY_IV))) return rc_iv;
    if (M->jit) {  // the specialised interaction kernels; the generic one when they cannot be built
      rc_iv = jit_build_iv(M);
      if (rc_iv == WDF_E_OOM || rc_iv == WDF_E_DEVICE) return rc_iv;
      bg->iv_spec = rc_iv == WDF_OK;
    }
  }
  bg->pathdep = true;
  int rc;
  // frequencies of the left (or single) leaves, then those of the right leaves
  if ((rc = bg->d_hist.alloc((size_t)std::max<int64_t>(2 * M->hist_size, 1) * sizeof(double)))) return rc;
  HIP_TRY(launch_pd_freq(M->d_groups.as<Group>(), (int64_t)M->groups.size(), M->d_ratio.as<double>(),
                         M->d_ratio_r.as<double>(), bg->d_hist.as<double>(), bg->d_hist.as<double>() + M->hist_size,
                         s));
  if ((rc = contract(M, bg.get(), nullptr, bg->d_hist.as<double>(), 1.0, s))) return rc;
  ++M->n_bg;
  *out = bg.release();
  return WDF_OK;
}

extern "C" void wdf_bg_destroy(wdf_bg *bg) {
  if (!bg) return;
  (void)hipSetDevice(bg->device);
  --bg->model->n_bg;
  delete bg;
}

extern "C" int wdf_base_value(const wdf_bg *bg, double *out) {
  if (!bg || !out) return set_error(WDF_E_INVALID_ARG, "wdf_base_value: NULL argument");
  if (bg->base_on_device) {  // refreshed: the caller has synchronised the refresh's stream
    HIP_TRY(hipSetDevice(bg->device));
    HIP_TRY(hipMemcpy(out, bg->d_base.ptr, sizeof(double), hipMemcpyDeviceToHost));
    return WDF_OK;
  }
  *out = bg->base;
  return WDF_OK;
}

// ---------------------------------------------------------------------------
// Explain
// ---------------------------------------------------------------------------

extern "C" int wdf_explain(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *phi, int64_t ldphi,
                           void *hip_stream) {
  if (!bg) return set_error(WDF_E_INVALID_ARG, "wdf_explain: NULL summary");
  if (n < 0 || ldx < n || ldphi < n) return set_error(WDF_E_INVALID_ARG, "wdf_explain: need 0 <= n <= ldx, ldphi");
  if (n == 0) return WDF_OK;
  if (!X || !phi) return set_error(WDF_E_INVALID_ARG, "wdf_explain: NULL X or phi");
  if (bg->iv) return set_error(WDF_E_INVALID_ARG, "wdf_explain: an interaction summary: use wdf_explain_iv");
  wdf_model *M = bg->model;
  hipStream_t s = pick_stream(M->ctx, hip_stream);
  if (M->jit) return jit_explain(bg, X, n, ldx, phi, ldphi, s);
  HIP_TRY(launch_explain_generic(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), (int64_t)M->groups.size(),
                                 bg->d_tab.as<float>(), X, n, ldx, phi, ldphi, M->n_features, s));
  return WDF_OK;
}

extern "C" int64_t wdf_explain_iv_workspace(const wdf_bg *bg, int64_t n) {
  if (!bg || n < 0) return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv_workspace: NULL summary or n < 0");
  return std::max<int64_t>((int64_t)bg->model->groups.size() * iv_pattern_stride(n), 1);
}

extern "C" int wdf_explain_iv(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *iv, int64_t ldiv,
                              void *workspace, size_t workspace_bytes, void *hip_stream) {
  if (!bg) return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv: NULL summary");
  if (!bg->iv) return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv: not an interaction summary");
  if (n < 0 || ldx < n || ldiv < n) return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv: need 0 <= n <= ldx, ldiv");
  if (n == 0) return WDF_OK;
  if (!X || !iv) return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv: NULL X or iv");
  wdf_model *M = bg->model;
  const int64_t G = (int64_t)M->groups.size();
  if (G > 65535) return set_error(WDF_E_UNSUPPORTED, "wdf_explain_iv: %lld groups exceeds 65535", (long long)G);
  const int64_t need = wdf_explain_iv_workspace(bg, n);
  if (!workspace || (int64_t)workspace_bytes < need)
    return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv: workspace of %zu bytes, need %lld", workspace_bytes,
                     (long long)need);
  if ((uintptr_t)workspace % 16)
    return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv: workspace not 16-byte aligned");
  hipStream_t s = pick_stream(M->ctx, hip_stream);
  if (bg->iv_spec) return jit_explain_iv(bg, X, ldx, (uint8_t *)workspace, n, iv, ldiv, s);
  HIP_TRY(launch_explain_iv(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), G, M->d_iv_item_off.as<int32_t>(),
                            M->d_iv_items.as<int2>(), bg->d_tab.as<float>(), X, n, ldx, (uint8_t *)workspace, iv, ldiv,
                            M->n_features, s));
  return WDF_OK;
}

extern "C" int wdf_explain_iv_noalloc(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *iv,
                                      int64_t ldiv, void *hip_stream) {
  if (!bg) return set_error(WDF_E_INVALID_ARG, "wdf_explain_iv_noalloc: NULL summary");
  const int64_t need = wdf_explain_iv_workspace(bg, n);
  if (need < 0) return (int)need;
  if (need > (int64_t)WDF_NOALLOC_SCRATCH_BYTES)
    return set_error(WDF_E_INVALID_ARG,
                     "wdf_explain_iv_noalloc: %lld rows need %lld bytes of pattern scratch, above the library's "
                     "%lld (explain at most %lld rows per call, or pass a workspace to wdf_explain_iv)",
                     (long long)n, (long long)need, (long long)WDF_NOALLOC_SCRATCH_BYTES,
                     (long long)((int64_t)WDF_NOALLOC_SCRATCH_BYTES /
                                 std::max<int64_t>((int64_t)bg->model->groups.size(), 1) / 512 * 512));
  // the pattern kernel writes every byte the interaction kernels read, so
  // the scratch needs no clearing between calls
  return wdf_explain_iv(bg, X, n, ldx, iv, ldiv, bg->model->ctx->scratch, WDF_NOALLOC_SCRATCH_BYTES, hip_stream);
}

extern "C" int wdf_debug_time_contraction(const wdf_bg *bg, int reps, void *hip_stream, double *flops, float *ms) {
  if (!bg || !flops || !ms || reps < 1)
    return set_error(WDF_E_INVALID_ARG, "wdf_debug_time_contraction: NULL argument or reps < 1");
  wdf_model *M = bg->model;
  HIP_TRY(hipSetDevice(bg->device));
  hipStream_t s = pick_stream(M->ctx, hip_stream);
  // private columns and products: the summary's own state is left untouched
  DevBuf H, S;
  int rc;
  if ((rc = H.alloc((size_t)std::max<int64_t>(M->h_total, 1) * sizeof(double)))) return rc;
  if ((rc = S.alloc((size_t)std::max<int64_t>(bg->iv ? M->s_iv_total : M->s_total, 1) * sizeof(double)))) return rc;
  const bool counts = !bg->pathdep;
  HIP_TRY(launch_columns(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), (int64_t)M->groups.size(),
                         counts ? bg->d_hist.as<uint32_t>() : nullptr, counts ? nullptr : bg->d_hist.as<double>(),
                         counts ? nullptr : bg->d_hist.as<double>() + M->hist_size, counts ? 1.0 / (double)bg->m : 1.0,
                         M->d_hclass_off.as<int64_t>(), H.as<double>(), s));
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    return hip_error(e, "hipEventCreate");
  }
  rc = enqueue_gemms(M, bg, H.as<double>(), S.as<double>(), s, flops);  // warm-up
  if (!rc && (e = hipEventRecord(a, s)) != hipSuccess) rc = hip_error(e, "hipEventRecord");
  for (int r = 0; !rc && r < reps; ++r) rc = enqueue_gemms(M, bg, H.as<double>(), S.as<double>(), s, flops);
  if (!rc && (e = hipEventRecord(b, s)) != hipSuccess) rc = hip_error(e, "hipEventRecord");
  if (!rc && (e = hipEventSynchronize(b)) != hipSuccess) rc = hip_error(e, "hipEventSynchronize");
  float t = 0.f;
  if (!rc && (e = hipEventElapsedTime(&t, a, b)) != hipSuccess) rc = hip_error(e, "hipEventElapsedTime");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  *ms = t / (float)reps;
  return WDF_OK;
}

// ---------------------------------------------------------------------------
// Debug / parity
// ---------------------------------------------------------------------------

extern "C" int wdf_debug_patterns(const wdf_model *M, const float *X, int64_t n, int64_t ldx, uint32_t *out,
                                  void *hip_stream) {
  if (!M || (!X && n) || (!out && n)) return set_error(WDF_E_INVALID_ARG, "wdf_debug_patterns: NULL argument");
  if (n < 0 || ldx < n) return set_error(WDF_E_INVALID_ARG, "wdf_debug_patterns: need 0 <= n <= ldx");
  HIP_TRY(hipSetDevice(M->ctx->device));
  hipStream_t s = pick_stream(M->ctx, hip_stream);
  HIP_TRY(launch_patterns(M->d_groups.as<Group>(), M->d_path.as<PathNode>(), (int64_t)M->groups.size(), X, n, ldx,
                          out, s));
  HIP_TRY(hipStreamSynchronize(s));
  return WDF_OK;
}

extern "C" int64_t wdf_debug_histograms(const wdf_bg *bg, uint32_t *host_out, int64_t cap) {
  if (!bg) return set_error(WDF_E_INVALID_ARG, "wdf_debug_histograms: NULL summary");
  if (bg->pathdep) return set_error(WDF_E_INVALID_ARG, "wdf_debug_histograms: path-dependent summary has no counts");
  const int64_t n = bg->model->hist_size;
  if (host_out) {
    if (cap < n) return set_error(WDF_E_INVALID_ARG, "wdf_debug_histograms: capacity %lld < %lld", (long long)cap,
                                  (long long)n);
    HIP_TRY(hipSetDevice(bg->model->ctx->device));
    HIP_TRY(hipMemcpy(host_out, bg->d_hist.ptr, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost));
  }
  return n;
}

extern "C" int64_t wdf_debug_tables(const wdf_bg *bg, float *host_out, int64_t cap) {
  if (!bg) return set_error(WDF_E_INVALID_ARG, "wdf_debug_tables: NULL summary");
  const int64_t n = bg->iv ? bg->model->iv_tab_size : bg->model->tab_size;
  if (host_out) {
    if (cap < n) return set_error(WDF_E_INVALID_ARG, "wdf_debug_tables: capacity %lld < %lld", (long long)cap,
                                  (long long)n);
    HIP_TRY(hipSetDevice(bg->model->ctx->device));
    HIP_TRY(hipMemcpy(host_out, bg->d_tab.ptr, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
  }
  return n;
}

extern "C" int64_t wdf_debug_coef_matrix(int dprime, int values, double *out, int64_t cap) {
  if (dprime < 1 || dprime > WDF_MAX_DEPTH) return set_error(WDF_E_INVALID_ARG, "wdf_debug_coef_matrix: dprime %d", dprime);
  if (values < WDF_SHAPLEY || values > WDF_BANZHAF_IV)
    return set_error(WDF_E_INVALID_ARG, "wdf_debug_coef_matrix: value kind %d", values);
  std::vector<double> M;
  try {
    if (values >= WDF_SHAPLEY_IV) {
      if (dprime < 2) return 0;
      build_iv_matrix(dprime, values - WDF_SHAPLEY_IV, M);
    } else {
      build_coef_matrix(dprime, values, M);
    }
  } catch (const std::bad_alloc &) {
    return set_error(WDF_E_OOM, "wdf_debug_coef_matrix: out of host memory");
  }
  if (out && cap >= (int64_t)M.size()) std::memcpy(out, M.data(), M.size() * sizeof(double));
  return (int64_t)M.size();
}

extern "C" int64_t wdf_debug_iv_source(const wdf_model_desc *desc, char *out, int64_t cap) {
  if (!desc) return set_error(WDF_E_INVALID_ARG, "wdf_debug_iv_source: NULL desc");
  try {
    wdf_model M;
    int rc = validate_and_layout(desc, &M);
    if (rc) return rc;
    std::vector<int32_t> ioff, items;
    if ((rc = iv_layout_host(&M, ioff, items))) return rc;
    std::string src;
    if ((rc = jit_iv_source(&M, src))) return rc;
    if (out && cap > (int64_t)src.size()) std::memcpy(out, src.c_str(), src.size() + 1);
    return (int64_t)src.size();
  } catch (const std::bad_alloc &) {
    return set_error(WDF_E_OOM, "wdf_debug_iv_source: out of host memory");
  }
}

extern "C" int64_t wdf_debug_specialised_source(const wdf_model_desc *desc, int kernel, int do_compile, char *out,
                                                int64_t cap) {
  if (!desc) return set_error(WDF_E_INVALID_ARG, "wdf_debug_specialised_source: NULL desc");
  try {
    wdf_model M;
    int rc = validate_and_layout(desc, &M);
    if (rc) return rc;
    M.jp.quad_depth = (kernel & WDF_KERNEL_PAIRS) == 0 ? WDF_MAX_DEPTH : 0;
    std::string src;
    if ((rc = jit_source(&M, do_compile != 0, src))) return rc;
    if (out && cap > (int64_t)src.size()) std::memcpy(out, src.c_str(), src.size() + 1);
    return (int64_t)src.size();
  } catch (const std::bad_alloc &) {
    return set_error(WDF_E_OOM, "wdf_debug_specialised_source: out of host memory");
  }
}
