// Internal state behind the opaque handles of include/wdf.h.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <atomic>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "wdf.h"
#include "wdf_dev.h"

namespace wdf {

int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);

// return the library error for a failed HIP call
#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_error(e_, #expr);  \
  } while (0)

struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf();
  int alloc(size_t n);
  void reset();
  template <class T>
  T *as() const { return static_cast<T *>(ptr); }
};

struct JitPart;    // one compiled program of model-specialised kernels (wdf_jit.cpp)
struct JitModule;  // the histogram and explain programs of a model (wdf_jit.cpp)

// Largest histogram block the generated kernel can be compiled for (its
// launch bound; a launch may use any multiple of 64 threads up to the bound).
constexpr int kHistMaxThreads = 1024;

// Layout of the model-specialised kernels (wdf_jit.cpp).
struct JitPlan {
  int wide = 0;                 // 0: 8-bit threshold ranks, 1: 16-bit
  int per_word = 4;             // ranks packed per 32-bit word
  int words = 0;                // words per row
  std::vector<float> thr;       // sorted distinct thresholds, feature after feature
  std::vector<int32_t> thr_off; // n_features + 1
  std::vector<int32_t> rank;    // per node: index of its threshold among its feature's
  int hist_bound = kHistMaxThreads;     // launch bound the histogram kernel is compiled for
  int hist_bound_cap = kHistMaxThreads; // lowered when the kernel spilled registers at a larger bound
  int nt_hist = 0, nt_explain = 512;    // threads per block (histogram: a launch-time choice, 0 = the bound)
  int explain_bpc = 1;           // explain blocks per CU sharing the LDS (512 / bpc threads each)
  int hist_cap = 32768;         // uint32 counters per histogram chunk (LDS)
  int stage_floats_max = 40960; // table floats per explain stage (LDS, double-buffered; capped by what fits)
  int stage_floats = 12288;     // the same after room for the thresholds
  std::vector<float> thr_pad;   // used features' thresholds, NaN-padded to powers of two
  std::vector<int32_t> thr_pad_off, thr_steps;  // per feature: offset in thr_pad, search steps
  std::vector<std::pair<int64_t, int64_t>> hist_chunks;    // group ranges
  std::vector<std::pair<int64_t, int64_t>> explain_stages; // group ranges
  std::vector<uint32_t> perm;   // histogram bin of every LDS slot (absolute offsets)
  std::vector<XUnit> xunits;    // explain-table units in group order
  std::vector<int64_t> unit_g0; // first group of every unit (plus a final G)
  int64_t xtab_size = 0;
  int quad_depth = WDF_MAX_DEPTH;  // pair groups of depth <= this merge into quads (0: pair tables only)
  bool thr_in_lds = true;       // thresholds searched in LDS (else in global memory)
  int hist_rounds = 2;          // histogram blocks per CU over the whole launch
  std::vector<int32_t> pad_meta;  // per feature: thr_pad offset, steps (the quantizer's view)
  DevBuf d_pad_meta, d_perm, d_thr_pad, d_xunits;
};

// Per-class contraction shape: paths with dprime distinct features.
struct ClassInfo {
  int ncols = 0;          // leaf columns in this class
  int64_t h_off = 0;      // offset (doubles) of this class in the column buffer
  int64_t s_off = 0;      // offset (doubles) of this class in the product buffer
};

}  // namespace wdf

struct wdf_ctx {
  int device = 0;
  int n_cu = 0;
  hipStream_t stream = nullptr;
  void *scratch = nullptr;  // this device's address of the no-alloc scratch array
  std::mutex jit_mu;
  std::map<std::string, std::shared_ptr<wdf::JitPart>> jit_cache;  // by generated source
};

struct wdf_model {
  wdf_ctx *ctx = nullptr;
  int device = 0;
  int n_trees = 0, n_features = 0;
  int64_t n_nodes = 0;
  std::vector<int64_t> node_offset;
  std::vector<int32_t> feature, left, right;
  std::vector<float> threshold, value;
  std::vector<uint8_t> default_left;
  std::vector<double> cover;
  bool has_cover = false;

  // layout
  std::vector<wdf::Group> groups;
  std::vector<wdf::PathNode> path;
  std::vector<int64_t> path_nodes;       // global node index of each PathNode
  std::vector<int64_t> group_leaf_l, group_leaf_r;
  std::vector<int64_t> tree_group_off;   // groups of tree t: [off[t], off[t+1])
  int64_t hist_size = 0, tab_size = 0;
  wdf::ClassInfo cls[WDF_MAX_DEPTH + 1];
  int64_t h_total = 0, s_total = 0;

  // device copies
  wdf::DevBuf d_groups, d_path, d_hclass_off, d_sclass_off, d_ratio, d_ratio_r;
  wdf::DevBuf d_coef[2][WDF_MAX_DEPTH + 1];  // [values][dprime]

  // model-specialised kernels
  std::shared_ptr<wdf::JitModule> jit;
  wdf::JitPlan jp;

  // workspace of background summaries (threshold codes, contraction columns
  // and products), grown on demand and reused; ws_mu serialises summaries of
  // one model
  std::mutex ws_mu;
  wdf::DevBuf ws_codes, ws_H, ws_S, ws_base;

  std::atomic<int> n_bg{0};  // live background summaries (their tables follow the current plan)

  // interaction values (prepared at the first summary of an interaction kind):
  // per group the offset of its pair tables, per class the offset of its
  // products, per feature the list of its first occurrences with their
  // partner features and pair-table offsets
  bool iv_layout = false;
  std::vector<int64_t> iv_off;
  int64_t iv_tab_size = 0, s_iv_total = 0;
  int64_t s_iv_class_off[WDF_MAX_DEPTH + 1] = {};
  wdf::DevBuf d_iv_off, d_siv_class_off, d_iv_item_off, d_iv_items;
  // interleaved interaction tables of the specialised interaction kernel:
  // units grouped by feature (iv_unit_off[i] .. iv_unit_off[i + 1])
  std::vector<wdf::IvUnit> iv_units;
  std::vector<std::array<int32_t, 7>> iv_unit_partners;  // partner features of each unit
  std::vector<int32_t> iv_unit_off;
  int64_t iv_units_size = 0;   // floats
  wdf::DevBuf d_iv_units;
  bool iv_coef_ready[2] = {false, false};
  wdf::DevBuf d_coef_iv[2][WDF_MAX_DEPTH + 1];  // [Shapley/Banzhaf][dprime]
};

struct wdf_bg {
  wdf_model *model = nullptr;
  int device = 0;
  int64_t m = 0;
  int values = WDF_SHAPLEY;
  bool iv = false;      // an interaction kind: pair tables in d_tab, no explain tables
  bool pathdep = false;
  double base = 0.0;
  wdf::DevBuf d_hist;   // uint32 counts (background) or double frequencies (path-dependent: the left or
                        // single leaves' [hist_size], then the right leaves' [hist_size])
  wdf::DevBuf d_tab;    // float gather tables
  wdf::DevBuf d_xtab;   // explain tables of the specialised kernel (quads merged), or the
                        // interleaved interaction tables (iv_spec)
  bool iv_spec = false; // interaction summary explained by the specialised kernel
  // private workspace of in-place refreshes (allocated by the first one):
  // threshold ranks, contraction columns and products, the base value
  wdf::DevBuf own_codes, own_H, own_S, d_base;
  bool base_on_device = false;  // a refresh wrote the base value to d_base
};

struct wdf_graph {
  wdf_bg *bg = nullptr;
  int device = 0;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace wdf {
// Model-specialised kernels (wdf_jit.cpp).
int jit_build(wdf_model *M);
// compile (in parallel) and cache the programs (source, kernel name) not yet cached
int jit_compile_all(wdf_model *M, const std::vector<std::pair<std::string, std::string>> &progs);
// the explain-kernel source of the model's current plan (plans the model)
int jit_explain_source(wdf_model *M, std::string &src);
const char *jit_explain_name(const wdf_model *M);
// the specialised interaction kernel (compiled on first use; WDF_E_UNSUPPORTED
// when the model is too large for it)
int jit_build_iv(wdf_model *M);
int jit_iv_source(wdf_model *M, std::string &src);  // interaction and pattern kernels (plans the model)
// patterns of the consumer rows into the workspace pat, then the interaction kernels
// Row stride of the interaction kernels' pattern workspace: n rounded up to
// a multiple of 512 (whole blocks of 16-byte pieces for every row block).
inline int64_t iv_pattern_stride(int64_t n) { return (n + 511) / 512 * 512; }
int jit_explain_iv(const wdf_bg *bg, const float *X, int64_t ldx, uint8_t *pat, int64_t n, float *iv, int64_t ldiv,
                   hipStream_t s);
int jit_source(wdf_model *M, bool do_compile, std::string &src);
int validate_and_layout(const wdf_model_desc *d, wdf_model *M);
// background histograms; `codes` holds P.words * m words of threshold ranks
int jit_hist(wdf_model *M, const float *B, int64_t m, int64_t ldb, uint32_t *hist, uint32_t *codes, hipStream_t s);
// grid of the specialised histogram kernel for m background rows
struct HistLaunch {
  int64_t blocks = 0, chunks = 0, threads = 0, tiles_per_block = 0, ntiles = 0;
};
HistLaunch hist_launch(const wdf_model *M, int64_t m);
// Grow a workspace buffer to at least `bytes` (contents are not kept).
int ws_reserve(DevBuf &buf, size_t bytes);
int jit_explain(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *phi, int64_t ldphi, hipStream_t s);
}  // namespace wdf
