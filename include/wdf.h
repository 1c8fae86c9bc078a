/*
 * wdf.h: C ABI of the MI355X (gfx950) Background-SHAP library.
 *
 * The library computes, for every consumer row c and feature i, the
 * Background (interventional) Shapley value
 *     phi_i(c) = Shapley value of v(S) = (1/|B|) sum_b f(c_S, b_rest)
 * of a decision-tree ensemble f, by the WOODELF decomposition of arXiv
 * 2511.09376 (Section 7, Formula eq:bg_shap_derivation; Alg. 3):
 *   1. decision patterns of every background row at every leaf
 *      (Def. Decision Pattern, Alg. 1),
 *   2. their per-leaf histogram vc[l][p_b] (Section 7 step (d)),
 *   3. s_{l,i} = w_l * M_{l,i} * f_l with the pattern-to-coefficient matrix
 *      M built from the four rules (Section 5, Alg. 2) and the linear-time
 *      formula (Formula shap_simplified_formula), as a dense matrix product,
 *   4. phi_i(c) = sum_l s_{l,i}[P[l][c]] (Section 7 step (g)).
 * Sibling leaves share one table indexed by the left leaf's pattern
 * (Section 9.1, improvement 3).  The same machinery gives Banzhaf values
 * (Formula banzhaf_simplified_formula) and Path-Dependent SHAP (Section 8).
 *
 * Conventions
 *   - A row goes left at an inner node iff x[feature] < threshold (float32
 *     compare, Def. Decision Tree); a NaN feature value goes to the side
 *     named by the node's default_left byte.
 *   - Matrices are column-major float32: element (feature f, row r) of X is
 *     X[f * ldx + r].  phi uses the same layout with ldphi.
 *   - Every function returns WDF_OK (0) or a negative error code; the text of
 *     the last error on the calling thread is returned by wdf_last_error().
 *     No C++ exception crosses this boundary.
 *   - Handles are owned by the library and freed by the matching destroy call.
 *     A context is bound to one HIP device.  Calls taking a `hip_stream`
 *     enqueue on it; NULL means the HIP null (legacy default) stream.
 *     Loads, refreshes, debug copies and graph calls make the context's
 *     device current on the calling thread; wdf_explain and wdf_explain_iv
 *     do not (their launch path stays short), so call them with that device
 *     current and a stream that belongs to it.
 */
#ifndef WDF_H
#define WDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WDF_OK = 0,
  WDF_E_INVALID_ARG = -1,   /* null pointer, bad size, malformed ensemble */
  WDF_E_UNSUPPORTED = -2,   /* a path deeper than WDF_MAX_DEPTH, too many features */
  WDF_E_OOM = -3,           /* device or host allocation failed */
  WDF_E_DEVICE = -4,        /* a HIP call failed; the HIP error text is in wdf_last_error() */
  WDF_E_BUSY = -5,          /* serving queue full */
  WDF_E_TIMEOUT = -6,       /* wait timed out */
  WDF_E_COMPILE = -7        /* runtime specialisation of a kernel failed */
};

#define WDF_MAX_DEPTH 8       /* inner nodes on any root-to-leaf path */
#define WDF_MAX_FEATURES 65535          /* features of a model (columns of X and B) */
#define WDF_MAX_SPECIALISED_FEATURES 4096 /* the specialised kernels' limit (their rank words
                                             cover every feature); larger models run the
                                             generic kernels */

/* Values computed from the cube of a (consumer, background) pattern pair. */
enum {
  WDF_SHAPLEY = 0,          /* Formula shap_simplified_formula */
  WDF_BANZHAF = 1,          /* Formula banzhaf_simplified_formula */
  WDF_SHAPLEY_IV = 2,       /* interaction values: Def. shap_iv_def, Table table_shap_iv */
  WDF_BANZHAF_IV = 3        /* Def. banzhaf_iv_def, Formula banzhaf_simplified_formula_interactions */
};

/* Kernel choice for the pattern, histogram and gather steps. */
enum {
  WDF_KERNEL_AUTO = 0,      /* model-specialised kernels when they compile, else generic */
  WDF_KERNEL_GENERIC = 1,   /* data-driven kernels that walk each leaf path */
  WDF_KERNEL_SPECIALISED = 2,/* kernels compiled for this ensemble at load time (hipRTC) */
  /* Flag, OR-ed into AUTO or SPECIALISED: the specialised gather reads every
   * sibling pair from its own table (d values at 2^d entries) instead of
   * merging the two pairs below a node into one "quad" table (d + 1 values at
   * 2^(d+1) entries), the default.  Results are the same sums in another
   * order. */
  WDF_KERNEL_PAIRS = 16
};

typedef struct wdf_ctx wdf_ctx;
typedef struct wdf_model wdf_model;
typedef struct wdf_bg wdf_bg;

/* Last error message of the calling thread ("" when none).  The pointer stays
 * valid until the next wdf call on the same thread. */
const char *wdf_last_error(void);

/* Create a context on HIP device `device`: the library's handle for one
 * gfx950 device and its private stream.  *out receives the handle, owned by
 * the caller until wdf_destroy.  Destroy the context's models and summaries
 * before the context: wdf_destroy frees only the context itself.
 * Errors: INVALID_ARG (NULL out, no such device), UNSUPPORTED (not gfx950),
 * OOM, DEVICE. */
int wdf_create(int device, wdf_ctx **out);
void wdf_destroy(wdf_ctx *ctx);

/* Ensemble description: host arrays, trees concatenated; node indices in
 * left/right are local to the tree (0 = the tree's first node = its root).
 * Leaves have feature = -1 and left = right = -1.  (Def. Decision Tree.) */
typedef struct {
  int32_t n_trees;
  int32_t n_features;
  const int64_t *node_offset;   /* n_trees + 1 entries, node_offset[0] = 0 */
  const int32_t *feature;       /* split feature, -1 for leaves */
  const int32_t *left;          /* local index of the left child, -1 for leaves */
  const int32_t *right;         /* local index of the right child, -1 for leaves */
  const float *threshold;       /* x < threshold goes left; not NaN (+-inf allowed) */
  const float *value;           /* leaf value w_l (ignored for inner nodes) */
  const uint8_t *default_left;  /* NaN direction: nonzero = left */
  const double *cover;          /* training rows reaching each node (Section 8); may be NULL */
} wdf_model_desc;

/* Validate and copy an ensemble (Def. Decision Tree; the caller may free its
 * arrays on return), extract its root-to-leaf paths (the cubes of the tree's
 * WDNF form, Formula model_to_wdnf_equation), pair sibling leaves, build the
 * pattern-to-coefficient matrices in double precision (Section 5's four rules
 * valued by Formula shap_simplified_formula or banzhaf_simplified_formula,
 * one matrix per distinct-feature count; Alg. 2) and upload everything to the
 * context's device.  `kernel` is one of WDF_KERNEL_AUTO, _GENERIC,
 * _SPECIALISED, optionally OR-ed with WDF_KERNEL_PAIRS; with AUTO or
 * SPECIALISED the pattern/histogram/gather kernels are generated for this
 * ensemble and compiled with hipRTC (cached per source).
 * A model with more than WDF_MAX_SPECIALISED_FEATURES features runs the
 * generic kernels (AUTO), or is refused with UNSUPPORTED (SPECIALISED).
 * Errors: INVALID_ARG (cycles, bad child or feature index, a NaN threshold,
 * n_features < 1), UNSUPPORTED (a path with more than WDF_MAX_DEPTH inner
 * nodes, more than WDF_MAX_FEATURES features), COMPILE (SPECIALISED only),
 * OOM, DEVICE. */
int wdf_model_load(wdf_ctx *ctx, const wdf_model_desc *desc, int kernel, wdf_model **out);
void wdf_model_destroy(wdf_model *model);

/* Per-group description of the model's layout (for tests and tools).  A group
 * is a pair of sibling leaves or a single leaf whose sibling is an inner node;
 * its root-to-leaf path is the cube of the tree's WDNF form (Formula
 * model_to_wdnf_equation), shared by both siblings but for the last literal.
 * Any array may be NULL; a non-NULL array is host memory of at least as many
 * entries as there are groups (call once with all NULL to learn the count).
 * Returns the number of groups (>= 0) or INVALID_ARG (NULL model). */
int64_t wdf_model_groups(const wdf_model *model, int32_t *tree, int32_t *depth, int64_t *leaf_left,
                         int64_t *leaf_right, int64_t *hist_offset, int64_t *table_offset);

/* 1 when the model runs the specialised kernels, 0 for the generic ones or a
 * NULL model.  Never fails. */
int wdf_model_specialised(const wdf_model *model);

/* Summarise a background set: decision patterns of every row at every group,
 * exact uint32 histograms, then (MFMA) the tables
 *     t_q[k][p] = (w_l/m) (M h_l)[p] + (w_r/m) (M h_r)[p ^ 1]
 * for the values selected by `values` (WDF_SHAPLEY / WDF_BANZHAF), and the base
 * value mean_b f(b).  With WDF_SHAPLEY_IV / WDF_BANZHAF_IV the tables are per
 * pair of path positions instead (C(d,2) tables of 2^d entries per group,
 * from coefficient matrices of the same four-rule cubes valued by the
 * interaction formulas of Section 3), for wdf_explain_iv.  B is column-major (B[f * ldb + r]), m >= 1 rows, on the
 * device when b_on_device is nonzero, else on the host (copied in).  Work is
 * enqueued on `hip_stream` (NULL = the HIP null stream) and the call
 * returns after it finishes, so B may be freed on return.  The summary owns
 * all device state that wdf_explain needs (histograms, tables, workspace).
 * The first interaction summary of a model with specialised kernels also
 * generates and compiles the model's interaction kernels (tens of seconds for
 * 100 depth-6 trees); when they cannot be built (a model too large for them,
 * a failed compile) the summary uses the generic interaction kernel
 * (wdf_bg_specialised tells which).
 * Errors: INVALID_ARG, UNSUPPORTED (interaction kinds: more than 65535 groups
 * or features), OOM, DEVICE. */
int wdf_background_load(wdf_model *model, const float *B, int64_t m, int64_t ldb, int b_on_device,
                        int values, void *hip_stream, wdf_bg **out);

/* Path-Dependent variant (Section 8, Formula eq:path_dependent_estimation):
 * the background histogram is replaced by the cover-product frequency of every
 * pattern; the model must have been loaded with covers.  Same output handle.
 * WDF_SHAPLEY or WDF_BANZHAF only. */
int wdf_pathdep_load(wdf_model *model, int values, void *hip_stream, wdf_bg **out);

void wdf_bg_destroy(wdf_bg *bg);

/* 1 when the summary is explained by model-specialised kernels (Shapley and
 * Banzhaf values: the model's; interaction values: the model's interaction
 * kernels, which very large models do without), 0 for the generic ones or a
 * NULL summary. */
int wdf_bg_specialised(const wdf_bg *bg);

/* Explain consumer rows against a summary (Section 7 step (g); Alg. 3): each
 * row's decision pattern at every group (Def. Decision Pattern) selects one
 * entry of each of the group's tables, and the entries add up per feature.
 * phi[f * ldphi + r] = value of feature f for consumer row r, r < n.  X and phi
 * are device pointers (column-major), n >= 0, ldx >= n, ldphi >= n.  Every
 * feature row of phi in [0, n_features) is written (exact 0.0 for features no
 * path uses).  Asynchronous on `hip_stream`; the caller keeps X and phi alive
 * until the stream reaches this work.  Allocates nothing; read-only on bg, so
 * concurrent calls on different streams are safe.
 * Errors: INVALID_ARG, DEVICE. */
int wdf_explain(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *phi, int64_t ldphi,
                void *hip_stream);

/* Interaction values phi_{i,j} (i != j) of consumer rows, for a summary
 * loaded with WDF_SHAPLEY_IV or WDF_BANZHAF_IV (Section 3; by linearity the
 * Background game's interaction values are the per-cube formulas summed over
 * leaves and background rows, as for Shapley values, Section 7).  X: device
 * [F][ldx >= n]; iv: device [F * F][ldiv >= n], iv[(i * F + j) * ldiv + r]
 * for consumer r, symmetric in (i, j), diagonal 0.  The rows' patterns of
 * every group go to `workspace` (device memory of at least
 * wdf_explain_iv_workspace(bg, n) bytes, 16-byte aligned, owned by the
 * caller, not shared by overlapping calls); then one lane per (row, feature
 * i) adds the pair tables of i's partners j, selected by those patterns, into
 * registers and stores row i of each row's matrix (kernels generated for the
 * model, which stream each feature's tables and the rows' patterns through
 * LDS, or a generic kernel walking i's (group, j) work list sorted by j).
 * Asynchronous on hip_stream; allocates nothing.
 * Errors: INVALID_ARG (NULL, sizes, small or misaligned workspace, summary
 * not of an interaction kind), UNSUPPORTED (more than 65535 groups), DEVICE. */
int wdf_explain_iv(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *iv, int64_t ldiv,
                   void *workspace, size_t workspace_bytes, void *hip_stream);
/* Workspace bytes wdf_explain_iv needs for n rows (one byte per group and
 * row, the rows rounded up to a multiple of 512; at least 1).
 * Errors: INVALID_ARG (NULL summary, n < 0). */
int64_t wdf_explain_iv_workspace(const wdf_bg *bg, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * interaction values as wdf_explain_iv, same arguments and layout, with the
 * rows' patterns kept in the library's own scratch array instead of a caller
 * workspace.  The array is a file-scope device array of
 * WDF_NOALLOC_SCRATCH_BYTES bytes that every device the library runs on holds
 * until the process ends; the call allocates nothing and calls no allocating
 * routine.  n rows need wdf_explain_iv_workspace(bg, n) bytes of it (one per
 * group and row, rows in blocks of 512): larger calls fail with INVALID_ARG and the row limit in
 * wdf_last_error().  All calls on one device share its array, which keeps the
 * last call's patterns (every byte read is written first, so nothing needs
 * clearing): calls that overlap on one device (different streams, or before
 * the previous call's work has run) race and give wrong values; order them on
 * one stream.  Errors: as wdf_explain_iv, and INVALID_ARG above the limit. */
#define WDF_NOALLOC_SCRATCH_BYTES (32u << 20)
int wdf_explain_iv_noalloc(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *iv, int64_t ldiv,
                           void *hip_stream);

/* mean_b f(b) in double precision (Appendix B.1 efficiency: sum_i phi_i(c) =
 * f(c) - base).  For a path-dependent summary: the cover-weighted mean.  After
 * a refresh (below) the value is read from the device: synchronise the
 * refresh's stream first.  *out is host memory.
 * Errors: INVALID_ARG (NULL argument), DEVICE. */
int wdf_base_value(const wdf_bg *bg, double *out);

/* Recompute a background summary in place from new background rows: the same
 * count m as at load, device pointer B [F][ldb >= m], column-major.  The same
 * steps as wdf_background_load (threshold ranks, exact histograms, MFMA
 * contraction, tables, base value; Section 7 steps (d)-(f)), enqueued on
 * hip_stream as kernel launches only: no allocation after the first call (which
 * allocates the summary's private workspace), no host copy, no
 * synchronisation, so the call can be captured into a HIP graph.  The caller
 * keeps B alive until the stream has run the work, and does not run explains
 * of this summary concurrently with a refresh.
 * Errors: INVALID_ARG (NULL, ldb < m, path-dependent summary), OOM, DEVICE. */
int wdf_background_refresh(wdf_bg *bg, const float *B, int64_t ldb, void *hip_stream);

/* A whole step recorded once into a HIP graph and replayed: the refresh of bg
 * from B (skipped when B is NULL) followed by wdf_explain of X into phi
 * (skipped when n == 0).  All pointers and sizes are fixed at creation; the
 * caller changes the contents of B and X between launches and keeps every
 * buffer alive while the graph exists.  Launches on one summary must not
 * overlap.  Errors: INVALID_ARG, OOM, DEVICE. */
typedef struct wdf_graph wdf_graph;
int wdf_graph_create(wdf_bg *bg, const float *B, int64_t ldb, const float *X, int64_t n, int64_t ldx, float *phi,
                     int64_t ldphi, wdf_graph **out);
int wdf_graph_launch(wdf_graph *g, void *hip_stream);
void wdf_graph_destroy(wdf_graph *g);

/* ---- debug / parity (not on the hot path) ------------------------------- */

/* Decision patterns (Def. Decision Pattern, group orientation: the left leaf
 * of a pair, the leaf itself for a single) of n device rows:
 * out[g * n + r], uint32, device pointer of at least n * groups entries;
 * X device [F][ldx >= n].  Synchronous.
 * Errors: INVALID_ARG (NULL, n < 0, ldx < n), DEVICE. */
int wdf_debug_patterns(const wdf_model *model, const float *X, int64_t n, int64_t ldx, uint32_t *out,
                       void *hip_stream);
/* Time the MFMA contraction of a summary (Section 7 steps (e)-(f)): the
 * FP64 GEMM launches S = M_{d'} H_{d'}, one per distinct-feature class, run
 * `reps` times on hip_stream (after one untimed run) from the summary's
 * current histograms, into private buffers (the summary is not changed).
 * *ms receives the average time of one contraction (all classes), *flops its
 * floating-point operations (2 R K per leaf column of a class with R x K
 * coefficients).  Allocates its buffers; synchronises.  For measurement.
 * Errors: INVALID_ARG (NULL, reps < 1), OOM, DEVICE. */
int wdf_debug_time_contraction(const wdf_bg *bg, int reps, void *hip_stream, double *flops, float *ms);

/* Copy the uint32 histograms (Section 7 step (d); cap entries of host
 * memory) / the float tables (step (f)) to the host.  With host_out NULL,
 * only the entry count is returned.  Returns the number of entries, or
 * INVALID_ARG (NULL summary, cap too small, a path-dependent summary for the
 * histograms) or DEVICE. */
int64_t wdf_debug_histograms(const wdf_bg *bg, uint32_t *host_out, int64_t cap);
int64_t wdf_debug_tables(const wdf_bg *bg, float *host_out, int64_t cap);

/* The library's coefficient matrix for d' = dprime distinct path features
 * (1..8) and a value kind, as built on the host (no device needed):
 * WDF_SHAPLEY / WDF_BANZHAF: M[(k * 2^d' + pc) * 2^d' + pb], the value of the
 * feature at position k for the cube of the pattern pair (pc, pb) (Section 5's
 * four rules; position 0 is the patterns' most significant bit);
 * WDF_SHAPLEY_IV / WDF_BANZHAF_IV: M[(q * 2^d' + pc) * 2^d' + pb] for the q-th
 * position pair (u, v), u < v, in lexicographic order.  Returns the entry
 * count; copies into out when cap allows.  For tests. */
int64_t wdf_debug_coef_matrix(int dprime, int values, double *out, int64_t cap);

/* Model-specialised kernels without a device: lay out the ensemble, write the
 * generated HIP source (returned in out, NUL-terminated, when cap is large
 * enough; the return value is the source length) and, with compile != 0, also
 * compile it for gfx950 with hipRTC (COMPILE on failure, the log in
 * wdf_last_error()).  `kernel` takes the flags of wdf_model_load (only
 * WDF_KERNEL_PAIRS matters here).  For tools and tests; needs no GPU. */
int64_t wdf_debug_specialised_source(const wdf_model_desc *desc, int kernel, int compile, char *out, int64_t cap);

/* Generated source of the model's specialised interaction-value kernels
 * (wdf_explain_iv on a summary of a model with specialised kernels): the
 * consumer patterns of every group (Def. Decision Pattern) into the
 * workspace, and the kernels that add the pair tables of Table table_shap_iv /
 * Formula banzhaf_simplified_formula_interactions, laid out per (group,
 * feature) and interleaved by pattern.  Same buffer convention as
 * wdf_debug_specialised_source; needs no GPU.  The source is written
 * whatever the model's size (loads fall back to the generic kernel above
 * 400k table loads and adds).  Errors: as for model validation (INVALID_ARG,
 * UNSUPPORTED), UNSUPPORTED for more than 65535 groups or features or a
 * feature with more than 32767 distinct thresholds, OOM. */
int64_t wdf_debug_iv_source(const wdf_model_desc *desc, char *out, int64_t cap);

/* ---- autotuning --------------------------------------------------------- */

/* Launch configurations measured by wdf_model_autotune (times in ms, -1 when
 * not measured). */
typedef struct {
  int quads;                  /* chosen explain gather: the sibling pairs of depth <= quads are merged
                                 into quad tables, 0 = pair tables only (WDF_MAX_DEPTH: all) */
  int explain_rows;           /* chosen explain tile: 512 (one block per CU, all of the LDS) or 256
                                 rows per block (two per CU, half of it each) */
  int hist_rounds;            /* chosen histogram grid: blocks per CU over the launch */
  int hist_threads;           /* chosen histogram block: 512, 768 or 1024 threads (at most the
                                 launch bound the model's histogram kernel was compiled for) */
  float explain_ms[WDF_MAX_DEPTH + 1];  /* explain time per quads value, 512-row tiles */
  float explain_rows_ms[2];   /* explain time with the chosen gather: [0] 512-row, [1] 256-row tiles */
  float hist_ms[3][9];        /* histogram time with [512, 768, 1024 threads][hist_rounds = 1..8] */
} wdf_tuning;

/* Measure the model's specialised kernels on the caller's data and keep the
 * fastest configuration for later calls: the explain gather (pair tables
 * only, quads for the sibling pairs of depth <= 6 when deeper ones exist, or
 * quads for all), the explain tile (512 or 256 rows per
 * block) - compile-time choices, each variant generated, compiled once (the
 * candidates in parallel) and cached - and the histogram grid and block size
 * (launch-time choices).  B [F][ldb] (m rows) and X [F][ldx] (n rows) are
 * device pointers; a sample of a few hundred thousand rows is enough.  Runs
 * and synchronises on hip_stream.  No summary of the model may exist during
 * the call (summaries hold tables laid out for the gather in use).
 * Errors: INVALID_ARG (NULL, sizes, summaries exist), UNSUPPORTED (the model
 * runs the generic kernels), COMPILE, OOM, DEVICE. */
int wdf_model_autotune(wdf_model *model, const float *B, int64_t m, int64_t ldb, const float *X, int64_t n,
                       int64_t ldx, void *hip_stream, wdf_tuning *out);

/* Apply a launch configuration measured earlier (by wdf_model_autotune, in
 * this process or another, and kept by the caller) without measuring again:
 * t->quads selects the explain gather (sibling pairs of depth <= quads merged
 * into quads, 0 pair tables only, -1 the current one), t->explain_rows the
 * explain tile (512 or 256 rows, 0 the current one; each variant is
 * compiled once and cached), t->hist_threads (a multiple of 64 in
 * [64, the launch bound the model's histogram kernel was compiled for]) and
 * t->hist_rounds (1..64 blocks per CU over the launch) the histogram grid.
 * The time fields are ignored.  No summary of the model may exist during the
 * call.  The histograms are exact counts in any grid; the gathers and tiles
 * add the same table values, the gathers in another order (phi agrees to
 * rounding).
 * Errors: INVALID_ARG (NULL, a field out of range, summaries exist),
 * UNSUPPORTED (the model runs the generic kernels), COMPILE, OOM, DEVICE. */
int wdf_model_set_tuning(wdf_model *model, const wdf_tuning *t);

/* Grid of the model's specialised histogram kernel (Section 7 step (d)) for a
 * summary of m background rows in the current launch configuration, as the
 * next load or refresh of m rows will launch it.  launch (host, 6 entries):
 * [0] blocks per chunk, [1] chunks (groups whose counters share one LDS
 * histogram), [2] threads per block, [3] 64-row tiles per block, [4] tiles in
 * all (the last one ragged when 64 does not divide m), [5] tiles counted by
 * the busiest wave (wave w of a block takes the block's tiles w, w + waves,
 * ...).  chunk_group (host, chunks + 1 entries, may be NULL): chunk c counts
 * the groups [chunk_group[c], chunk_group[c + 1]).  Returns the chunk count.
 * For tests; needs no device work.  Errors: INVALID_ARG (NULL model or
 * launch, m < 1, capacity below chunks + 1), UNSUPPORTED (generic kernels). */
int64_t wdf_debug_hist_launch(const wdf_model *model, int64_t m, int64_t *launch, int64_t *chunk_group,
                              int64_t cap);

/* ---- serving: continuous batching of explain requests ------------------- */

typedef struct wdf_server wdf_server;

typedef struct {
  uint64_t submitted, completed, rejected;
  uint64_t batches;           /* device launches */
  uint64_t rows;              /* rows explained */
  double p50_ms, p99_ms, mean_ms, max_ms;  /* submit -> result on host, over the most
                                            * recent 1048576 completed requests */
  double busy_ms;             /* device time of all batches, copy-in start to copy-out end */
  double copy_in_ms, explain_ms, copy_out_ms;  /* busy_ms split into its three parts */
  double pack_ms, unpack_ms;  /* host time packing requests into the slots' staging and
                                 unpacking results (on the copy threads) */
  double active_ms;           /* first submission to the latest completion */
  int slots;                  /* batch slots the server holds */
  int64_t batch_rows;         /* rows per batch slot */
} wdf_stats;

/* Server configuration. */
typedef struct {
  size_t mem_budget;  /* bytes of staging the server may hold: each batch slot takes
                         4 * n_features * batch_rows * 4 (pinned host and device, X and phi);
                         the server creates as many slots as fit, at most four */
  int max_rows;       /* largest request, in rows (>= 1) */
  int batch_rows;     /* rows per batch slot, max_rows .. 2^24; 0: max(max_rows, 65536) */
  int queue_cap;      /* queued requests beyond which submit returns BUSY (>= 1) */
  int flags;          /* WDF_SERVE_ONE_PER_LAUNCH, WDF_SERVE_START_PAUSED */
  int copy_threads;   /* host threads that pack and unpack batches (0: 4; at most 64) */
} wdf_server_config;

/* A server keeps bg resident and owns a worker thread, copy threads and up to
 * four batch slots, each with pinned host staging and device buffers for
 * batch_rows rows of X and phi, a stream and events; the slots it creates are
 * those that fit in cfg->mem_budget.  Queued requests of 1..max_rows rows are
 * admitted FIFO as slots free up: a batch packs the oldest requests that fit
 * in batch_rows rows, is copied in, explained (wdf_explain) and copied out on
 * its slot's stream, so batches of different slots overlap on the device and
 * with the packing of the next batch.  With WDF_SERVE_ONE_PER_LAUNCH the server
 * is the plain form: one slot of max_rows rows, one request per launch, each
 * copied in, explained and copied out before the next.  Each result is
 * bit-identical to wdf_explain on the same rows alone.  The server must be
 * destroyed before bg.  Errors: INVALID_ARG (NULL, budget below one slot,
 * sizes out of range), OOM, DEVICE. */
#define WDF_SERVE_ONE_PER_LAUNCH 1
#define WDF_SERVE_START_PAUSED 2   /* admit nothing until wdf_server_pause(srv, 0) */
int wdf_server_create(const wdf_bg *bg, const wdf_server_config *cfg, wdf_server **out);
/* Stop (paused != 0) or resume admitting queued requests into batches.
 * Batches already launched complete; submissions keep queueing while paused
 * (up to queue_cap).  Errors: INVALID_ARG (NULL server). */
int wdf_server_pause(wdf_server *srv, int paused);
/* Enqueue n rows of host X (column-major, ldx >= n); phi_host receives
 * [n_features][n] column-major float32 when the ticket completes.  Both stay
 * owned by the caller and must remain valid until wdf_server_wait has returned
 * for the ticket (the rows are read when the request enters a batch).
 * Errors: INVALID_ARG (n outside 1..max_rows), BUSY (queue full). */
int wdf_server_submit(wdf_server *srv, const float *X_host, int64_t n, int64_t ldx, float *phi_host,
                      uint64_t *ticket);
/* Wait until the ticket completes (timeout_ms < 0: forever).  A return other
 * than TIMEOUT releases the ticket, so wait on every ticket until it does
 * (the server holds each ticket's entry until then); a released ticket is
 * unknown afterwards.  Errors: TIMEOUT, INVALID_ARG (unknown ticket), or the
 * error of the ticket's batch (DEVICE). */
int wdf_server_wait(wdf_server *srv, uint64_t ticket, int timeout_ms);
/* Counters since creation and latency percentiles (nearest rank) into *out
 * (host memory).  Errors: INVALID_ARG (NULL argument). */
int wdf_server_stats(wdf_server *srv, wdf_stats *out);
/* Explain the requests still queued, stop the worker and free the server.
 * No other call on srv may run concurrently or follow. */
void wdf_server_destroy(wdf_server *srv);

#ifdef __cplusplus
}
#endif
#endif
