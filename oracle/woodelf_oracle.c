/*
 * Test infrastructure only: the FP64 CPU oracle for Background SHAP on
 * decision-tree ensembles.  Nothing in the product path may link or call
 * this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no code, header or table with the GPU
 * library.
 *
 * What it computes, and from which passage of the paper (arXiv 2511.09376,
 * "From Decision Trees to Boolean Logic: A Fast and Unified SHAP Algorithm"):
 *
 *   wo_predict              model output, Def. Decision Tree (Section 4)
 *   wo_leaf_info            root-to-leaf paths (Def. Root-to-Leaf Path, Section 4)
 *   wo_patterns             Def. Decision Pattern, walked per leaf (not Alg. 1's BFS)
 *   wo_histograms           the value counts vc[l][p_b] of Section 7, step (d)
 *   wo_wdnf_eval            Def. PB Function and WDNF (Section 2)
 *   wo_wdnf_values          Formula shap_simplified_formula / banzhaf_simplified_formula
 *                           (Sections 2-3), contradictory cubes removed first
 *   wo_wdnf_bruteforce      Formula PB_shap / PB_banzhaf (Appendix B): the exponential
 *                           definitions over all assignments
 *   wo_bg_fourrule          Formula trival_bg (Section 7): for every consumer c,
 *                           background row b and leaf l, the cube d_l[P[l][c]][P[l][b]]
 *                           built by the four rules of Section 5, valued by the
 *                           simplified formula, averaged over B
 *   wo_bg_walk              the same sum, visiting only the leaves whose cube is
 *                           satisfiable (a depth-first walk applying the four rules
 *                           node by node); identical result, faster
 *   wo_bg_bruteforce        Formula eq:s (Section 1.1) on the Background-SHAP game:
 *                           v(S) = mean over b of the model on (c_S, b_rest)
 *   wo_map_patterns_to_cube Alg. 2 (MapPatternsToCube) for one path
 *   wo_woodelf_tables       Alg. 3 steps 2-3: M_{l,i}[p_c][p_b] from Alg. 2 and the
 *                           value function, s_{l,i} = w_l * M_{l,i} * f_l
 *   wo_pd_freq              Formula eq:path_dependent_estimation (Section 8)
 *   wo_wdnf_iv_values       interaction values of a WDNF: Table table_shap_iv (Shapley)
 *                           and Formula banzhaf_simplified_formula_interactions (Banzhaf)
 *   wo_wdnf_iv_bruteforce   the same from the definitions (Def. shap_iv_def: phi_{j|i=1}
 *                           - phi_{j|i=0}; Def. banzhaf_iv_def) over all assignments
 *   wo_bg_iv_walk           Background interaction values: the depth-first walk with
 *                           every satisfiable cube valued by the interaction formulas
 *   wo_bg_iv_bruteforce     the same from the definitions on the Background-SHAP game
 *
 * Readings of the paper taken here (the paper is silent on them):
 *   - a missing (NaN) feature value follows the node's default direction;
 *   - a pattern's most significant bit belongs to the root (Alg. 1 shifts left
 *     at every level; the Section 8 example reads pattern 5 = 101 from the root);
 *   - |S+| and |S-| count distinct features, so a feature repeated on a path is
 *     credited once (set union in Alg. 2);
 *   - an empty cube adds to the prediction and nothing to any value.
 *
 * All arithmetic is in double precision.  Thresholds and features are float32
 * inputs; promoting both to double preserves every comparison.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WO_MAXD 64

typedef struct {
  int32_t n_trees;
  int32_t n_features;
  const int64_t *node_offset; /* n_trees + 1 */
  const int32_t *feature;     /* -1 for leaves */
  const int32_t *left;        /* tree-local child index, -1 for leaves */
  const int32_t *right;
  const float *threshold;
  const float *value;
  const uint8_t *default_left;
  const double *cover;        /* may be NULL unless path-dependent frequencies are asked for */
} wo_model;

typedef struct {
  int depth;                 /* number of inner nodes on the path */
  int64_t leaf;              /* global node index of the leaf */
  int64_t nodes[WO_MAXD];    /* global node indices n_1 .. n_depth */
  uint8_t dir[WO_MAXD];      /* 0: path continues to the left child, 1: right */
} wo_path;

enum { WO_SHAPLEY = 0, WO_BANZHAF = 1 };

/* ------------------------------------------------------------------------ */
/* Trees                                                                     */
/* ------------------------------------------------------------------------ */

/* Def. Decision Tree: split(c) is True iff c_f < theta; True goes left.
 * A missing value takes the node's default direction. */
static int goes_left(const wo_model *M, int64_t node, double x) {
  if (isnan(x)) return M->default_left[node] != 0;
  return x < (double)M->threshold[node];
}

static double tree_predict(const wo_model *M, int t, const double *x) {
  int64_t base = M->node_offset[t];
  int64_t nd = base;
  while (M->feature[nd] >= 0) {
    int l = goes_left(M, nd, x[M->feature[nd]]);
    nd = base + (l ? M->left[nd] : M->right[nd]);
  }
  return (double)M->value[nd];
}

static void load_row(const float *X, int64_t ld, int64_t row, int F, double *x) {
  for (int f = 0; f < F; ++f) x[f] = (double)X[(int64_t)f * ld + row];
}

/* Enumerate root-to-leaf paths of tree t in node order of the leaves. */
static int64_t collect_paths(const wo_model *M, int t, wo_path *out) {
  int64_t base = M->node_offset[t], end = M->node_offset[t + 1];
  int64_t count = 0;
  for (int64_t nd = base; nd < end; ++nd) {
    if (M->feature[nd] >= 0) continue;
    /* climb to the root by searching parents (trees are small) */
    int64_t chain[WO_MAXD + 1];
    uint8_t dirs[WO_MAXD + 1];
    int depth = 0;
    int64_t cur = nd;
    while (cur != base) {
      int64_t parent = -1;
      uint8_t d = 0;
      for (int64_t p = base; p < end; ++p) {
        if (M->feature[p] < 0) continue;
        if (base + M->left[p] == cur) { parent = p; d = 0; break; }
        if (base + M->right[p] == cur) { parent = p; d = 1; break; }
      }
      if (parent < 0 || depth >= WO_MAXD) return -1;
      chain[depth] = parent;
      dirs[depth] = d;
      ++depth;
      cur = parent;
    }
    if (out) {
      wo_path *P = &out[count];
      P->depth = depth;
      P->leaf = nd;
      for (int i = 0; i < depth; ++i) { /* reverse: root first */
        P->nodes[i] = chain[depth - 1 - i];
        P->dir[i] = dirs[depth - 1 - i];
      }
    }
    ++count;
  }
  return count;
}

/* Def. Decision Pattern: bit i is 1 iff the row continues along the path at
 * n_i.  Bit of n_1 (the root) is the most significant. */
static uint64_t path_pattern(const wo_model *M, const wo_path *P, const double *x) {
  uint64_t p = 0;
  for (int i = 0; i < P->depth; ++i) {
    int64_t nd = P->nodes[i];
    int l = goes_left(M, nd, x[M->feature[nd]]);
    int follows = (l && P->dir[i] == 0) || (!l && P->dir[i] == 1);
    p = (p << 1) | (uint64_t)follows;
  }
  return p;
}

static int path_bit(const wo_path *P, uint64_t p, int i) {
  return (int)((p >> (P->depth - 1 - i)) & 1u);
}

/* ------------------------------------------------------------------------ */
/* Coefficients of one weighted cube                                        */
/* ------------------------------------------------------------------------ */

static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
  return r;
}

/* Formula shap_simplified_formula: +1/(|S+| C(|S|,|S+|)) for a positive
 * literal, -1/(|S-| C(|S|,|S-|)) for a negated one.  Formula
 * banzhaf_simplified_formula: +-1/2^(|S|-1). */
static double cube_coef(int kind, int a, int b, int positive) {
  int s = a + b;
  if (kind == WO_BANZHAF) return (positive ? 1.0 : -1.0) / ldexp(1.0, s - 1);
  if (positive) return 1.0 / ((double)a * binom(s, a));
  return -1.0 / ((double)b * binom(s, b));
}

static int set_has(const int32_t *s, int n, int32_t f) {
  for (int i = 0; i < n; ++i)
    if (s[i] == f) return 1;
  return 0;
}

/* The four rules of Section 5 applied along a path to the pattern pair
 * (pc, pb).  Returns 0 when the cube is bottom (some (0,0) position) or
 * contradictory (a feature both positive and negated); else 1 with the
 * distinct positive and negated features. */
static int four_rule_cube(const wo_model *M, const wo_path *P, uint64_t pc, uint64_t pb,
                          int32_t *sp, int *na, int32_t *sm, int *nb) {
  *na = 0;
  *nb = 0;
  for (int i = 0; i < P->depth; ++i) {
    int c = path_bit(P, pc, i), b = path_bit(P, pb, i);
    int32_t f = M->feature[P->nodes[i]];
    if (c && !b) {
      if (!set_has(sp, *na, f)) sp[(*na)++] = f;
    } else if (!c && b) {
      if (!set_has(sm, *nb, f)) sm[(*nb)++] = f;
    } else if (!c && !b) {
      return 0;
    }
  }
  for (int i = 0; i < *na; ++i)
    if (set_has(sm, *nb, sp[i])) return 0;
  return 1;
}

static void credit_cube(int kind, double w, const int32_t *sp, int na, const int32_t *sm, int nb,
                        double *phi) {
  if (na + nb == 0) return;
  if (na) {
    double c = w * cube_coef(kind, na, nb, 1);
    for (int i = 0; i < na; ++i) phi[sp[i]] += c;
  }
  if (nb) {
    double c = w * cube_coef(kind, na, nb, 0);
    for (int i = 0; i < nb; ++i) phi[sm[i]] += c;
  }
}

/* Interaction value of the ordered pair (i, j), i != j, both literals of one
 * cube with a positive and b negated distinct features (s = a + b):
 * Table table_shap_iv for Shapley, Formula
 * banzhaf_simplified_formula_interactions for Banzhaf.  pi, pj: 1 when the
 * literal of i (j) is positive. */
static double cube_iv_coef(int kind, int a, int b, int pi, int pj) {
  int s = a + b;
  if (kind == WO_BANZHAF) return (pi == pj ? 1.0 : -1.0) / ldexp(1.0, s - 2);
  if (pi && pj) return 1.0 / ((double)(a - 1) * binom(s - 1, a - 1));
  if (!pi && !pj) return 1.0 / ((double)(b - 1) * binom(s - 1, b - 1));
  if (pj) return -1.0 / ((double)a * binom(s - 1, a)); /* i negated, j positive */
  return -1.0 / ((double)b * binom(s - 1, b));         /* i positive, j negated */
}

/* iv[i * F + j] += w * coefficient, for every ordered pair of the cube's literals */
static void credit_cube_iv(int kind, double w, const int32_t *sp, int na, const int32_t *sm, int nb, int F,
                           double *iv) {
  int32_t lit[2 * WO_MAXD];
  int pos[2 * WO_MAXD];
  int n = 0;
  for (int k = 0; k < na; ++k) lit[n] = sp[k], pos[n++] = 1;
  for (int k = 0; k < nb; ++k) lit[n] = sm[k], pos[n++] = 0;
  for (int x = 0; x < n; ++x)
    for (int y = 0; y < n; ++y)
      if (x != y) iv[(int64_t)lit[x] * F + lit[y]] += w * cube_iv_coef(kind, na, nb, pos[x], pos[y]);
}

/* ------------------------------------------------------------------------ */
/* Threading helper                                                          */
/* ------------------------------------------------------------------------ */

typedef void (*row_fn)(void *ctx, int64_t row);
typedef struct {
  row_fn fn;
  void *ctx;
  int64_t n;
  int64_t next;
  pthread_mutex_t mu;
} pool_t;

static void *pool_worker(void *arg) {
  pool_t *P = (pool_t *)arg;
  for (;;) {
    pthread_mutex_lock(&P->mu);
    int64_t r = P->next++;
    pthread_mutex_unlock(&P->mu);
    if (r >= P->n) break;
    P->fn(P->ctx, r);
  }
  return NULL;
}

static void parallel_rows(int64_t n, int threads, row_fn fn, void *ctx) {
  pool_t P;
  P.fn = fn;
  P.ctx = ctx;
  P.n = n;
  P.next = 0;
  pthread_mutex_init(&P.mu, NULL);
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if (threads == 1 || n <= 1) {
    pool_worker(&P);
  } else {
    pthread_t th[256];
    for (int i = 0; i < threads; ++i) pthread_create(&th[i], NULL, pool_worker, &P);
    for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
  }
  pthread_mutex_destroy(&P.mu);
}

/* ------------------------------------------------------------------------ */
/* Predictions, paths, patterns, histograms                                  */
/* ------------------------------------------------------------------------ */

int wo_predict(const wo_model *M, const float *X, int64_t n, int64_t ldx, double *out) {
  double *x = (double *)malloc(sizeof(double) * (size_t)M->n_features);
  if (!x) return -1;
  for (int64_t r = 0; r < n; ++r) {
    load_row(X, ldx, r, M->n_features, x);
    double s = 0.0;
    for (int t = 0; t < M->n_trees; ++t) s += tree_predict(M, t, x);
    out[r] = s;
  }
  free(x);
  return 0;
}

/* Number of leaves in the ensemble; when the arrays are given, the global node
 * index and path depth of every leaf, trees in order, leaves in node order. */
int64_t wo_leaf_info(const wo_model *M, int64_t *leaf_node, int32_t *leaf_depth, int32_t *leaf_tree) {
  int64_t total = 0;
  for (int t = 0; t < M->n_trees; ++t) {
    int64_t nl = collect_paths(M, t, NULL);
    if (nl < 0) return -1;
    if (leaf_node) {
      wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)nl);
      collect_paths(M, t, paths);
      for (int64_t j = 0; j < nl; ++j) {
        leaf_node[total + j] = paths[j].leaf;
        leaf_depth[total + j] = paths[j].depth;
        leaf_tree[total + j] = t;
      }
      free(paths);
    }
    total += nl;
  }
  return total;
}

/* Path features of one leaf (global leaf order as wo_leaf_info). */
int wo_leaf_path(const wo_model *M, int64_t leaf_index, int32_t *features, uint8_t *dirs,
                 int64_t *nodes) {
  int64_t seen = 0;
  for (int t = 0; t < M->n_trees; ++t) {
    int64_t nl = collect_paths(M, t, NULL);
    if (leaf_index < seen + nl) {
      wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)nl);
      collect_paths(M, t, paths);
      wo_path *P = &paths[leaf_index - seen];
      for (int i = 0; i < P->depth; ++i) {
        if (features) features[i] = M->feature[P->nodes[i]];
        if (dirs) dirs[i] = P->dir[i];
        if (nodes) nodes[i] = P->nodes[i];
      }
      int d = P->depth;
      free(paths);
      return d;
    }
    seen += nl;
  }
  return -1;
}

/* out[leaf * n + row] = decision pattern of `row` at `leaf` (global leaf order). */
int wo_patterns(const wo_model *M, const float *X, int64_t n, int64_t ldx, uint32_t *out) {
  double *x = (double *)malloc(sizeof(double) * (size_t)M->n_features);
  int64_t lbase = 0;
  for (int t = 0; t < M->n_trees; ++t) {
    int64_t nl = collect_paths(M, t, NULL);
    wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)nl);
    collect_paths(M, t, paths);
    for (int64_t r = 0; r < n; ++r) {
      load_row(X, ldx, r, M->n_features, x);
      for (int64_t j = 0; j < nl; ++j) out[(lbase + j) * n + r] = (uint32_t)path_pattern(M, &paths[j], x);
    }
    free(paths);
    lbase += nl;
  }
  free(x);
  return 0;
}

/* Value counts: hist[hist_off[leaf] + p] = #{b : P[leaf][b] = p}, with
 * hist_off[leaf+1] - hist_off[leaf] = 2^depth(leaf).  hist is zeroed here.
 * Every background row is walked along every leaf's path (Def. Decision
 * Pattern).  With threads > 1 the rows are split into contiguous ranges, each
 * counted into its own integer histogram; the ranges' counts are then added.
 * Integer counts are exact, so the result is the same for any thread count. */
typedef struct {
  const wo_model *M;
  const float *B;
  int64_t ldb, r0, r1, n_leaves, bins;
  const wo_path *paths;       /* every leaf of every tree, in global leaf order */
  const int64_t *hist_off;
  uint64_t *out;              /* this range's histogram, bins entries */
} hist_range_t;

/* rows in blocks of 64, so that each leaf's path is read once per block */
static void *hist_range(void *arg) {
  hist_range_t *H = (hist_range_t *)arg;
  const int F = H->M->n_features;
  double *x = (double *)malloc(sizeof(double) * (size_t)F * 64);
  memset(H->out, 0, sizeof(uint64_t) * (size_t)H->bins);
  for (int64_t r0 = H->r0; r0 < H->r1; r0 += 64) {
    const int64_t nb = H->r1 - r0 < 64 ? H->r1 - r0 : 64;
    for (int64_t i = 0; i < nb; ++i) load_row(H->B, H->ldb, r0 + i, F, x + (size_t)i * (size_t)F);
    for (int64_t j = 0; j < H->n_leaves; ++j)
      for (int64_t i = 0; i < nb; ++i)
        H->out[H->hist_off[j] + (int64_t)path_pattern(H->M, &H->paths[j], x + (size_t)i * (size_t)F)] += 1;
  }
  free(x);
  return NULL;
}

int wo_histograms(const wo_model *M, const float *B, int64_t m, int64_t ldb, uint64_t *hist,
                  const int64_t *hist_off, int threads) {
  int64_t nl = 0;
  for (int t = 0; t < M->n_trees; ++t) nl += collect_paths(M, t, NULL);
  wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)(nl > 0 ? nl : 1));
  int64_t lbase = 0;
  for (int t = 0; t < M->n_trees; ++t) lbase += collect_paths(M, t, paths + lbase);
  const int64_t bins = hist_off[nl];
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if ((int64_t)threads > m) threads = m > 0 ? (int)m : 1;
  hist_range_t R[256];
  uint64_t *part = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(bins > 0 ? bins : 1) * (size_t)threads);
  for (int i = 0; i < threads; ++i) {
    R[i].M = M;
    R[i].B = B;
    R[i].ldb = ldb;
    R[i].r0 = m * i / threads;
    R[i].r1 = m * (i + 1) / threads;
    R[i].n_leaves = nl;
    R[i].bins = bins;
    R[i].paths = paths;
    R[i].hist_off = hist_off;
    R[i].out = part + (size_t)i * (size_t)bins;
  }
  if (threads == 1) {
    hist_range(&R[0]);
  } else {
    pthread_t th[256];
    for (int i = 0; i < threads; ++i) pthread_create(&th[i], NULL, hist_range, &R[i]);
    for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
  }
  for (int64_t k = 0; k < bins; ++k) {
    uint64_t c = 0;
    for (int i = 0; i < threads; ++i) c += part[(size_t)i * (size_t)bins + (size_t)k];
    hist[k] = c;
  }
  free(part);
  free(paths);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* WDNF formulas (Sections 2, 3 and Appendix B)                              */
/* ------------------------------------------------------------------------ */

/* lits[k * max_lits + j]: +(v+1) for literal x_v, -(v+1) for its negation, 0 for padding. */
static int cube_satisfied(const int32_t *lits, int max_lits, const uint8_t *x) {
  for (int j = 0; j < max_lits; ++j) {
    int32_t L = lits[j];
    if (L == 0) continue;
    int v = (L > 0 ? L : -L) - 1;
    if (L > 0 && !x[v]) return 0;
    if (L < 0 && x[v]) return 0;
  }
  return 1;
}

double wo_wdnf_eval(int n_cubes, const double *w, const int32_t *lits, int max_lits, const uint8_t *x) {
  double s = 0.0;
  for (int k = 0; k < n_cubes; ++k)
    if (cube_satisfied(lits + (int64_t)k * max_lits, max_lits, x)) s += w[k];
  return s;
}

/* Simplified linear-time formulas; contradictory cubes are removed first. */
int wo_wdnf_values(int n_vars, int n_cubes, const double *w, const int32_t *lits, int max_lits,
                   int kind, double *out) {
  for (int v = 0; v < n_vars; ++v) out[v] = 0.0;
  int32_t sp[WO_MAXD], sm[WO_MAXD];
  for (int k = 0; k < n_cubes; ++k) {
    int na = 0, nb = 0;
    const int32_t *c = lits + (int64_t)k * max_lits;
    for (int j = 0; j < max_lits; ++j) {
      int32_t L = c[j];
      if (L == 0) continue;
      int32_t v = (L > 0 ? L : -L) - 1;
      if (L > 0) { if (!set_has(sp, na, v)) sp[na++] = v; }
      else { if (!set_has(sm, nb, v)) sm[nb++] = v; }
    }
    int bad = 0;
    for (int i = 0; i < na; ++i)
      if (set_has(sm, nb, sp[i])) bad = 1;
    if (bad) continue;
    credit_cube(kind, w[k], sp, na, sm, nb, out);
  }
  return 0;
}

/* Exponential definitions (Formulas PB_shap, PB_banzhaf) over all 2^n assignments. */
int wo_wdnf_bruteforce(int n_vars, int n_cubes, const double *w, const int32_t *lits, int max_lits,
                       int kind, double *out) {
  if (n_vars > 24) return -1;
  uint8_t x[32];
  int64_t N = (int64_t)1 << n_vars;
  double *F = (double *)malloc(sizeof(double) * (size_t)N);
  for (int64_t a = 0; a < N; ++a) {
    for (int v = 0; v < n_vars; ++v) x[v] = (uint8_t)((a >> v) & 1);
    F[a] = wo_wdnf_eval(n_cubes, w, lits, max_lits, x);
  }
  for (int i = 0; i < n_vars; ++i) {
    double s = 0.0;
    for (int64_t a = 0; a < N; ++a) {
      if ((a >> i) & 1) continue;
      int size = __builtin_popcountll((unsigned long long)a);
      double wt = kind == WO_BANZHAF ? 1.0 / ldexp(1.0, n_vars - 1)
                                     : 1.0 / ((double)n_vars * binom(n_vars - 1, size));
      s += wt * (F[a | ((int64_t)1 << i)] - F[a]);
    }
    out[i] = s;
  }
  free(F);
  return 0;
}

/* Interaction values of a WDNF by the per-cube formulas; out[i * n + j]. */
int wo_wdnf_iv_values(int n_vars, int n_cubes, const double *w, const int32_t *lits, int max_lits, int kind,
                      double *out) {
  for (int64_t v = 0; v < (int64_t)n_vars * n_vars; ++v) out[v] = 0.0;
  int32_t sp[WO_MAXD], sm[WO_MAXD];
  for (int k = 0; k < n_cubes; ++k) {
    int na = 0, nb = 0;
    const int32_t *c = lits + (int64_t)k * max_lits;
    for (int j = 0; j < max_lits; ++j) {
      int32_t L = c[j];
      if (L == 0) continue;
      int32_t v = (L > 0 ? L : -L) - 1;
      if (L > 0) { if (!set_has(sp, na, v)) sp[na++] = v; }
      else { if (!set_has(sm, nb, v)) sm[nb++] = v; }
    }
    int bad = 0;
    for (int i = 0; i < na; ++i)
      if (set_has(sm, nb, sp[i])) bad = 1;
    if (bad) continue;
    credit_cube_iv(kind, w[k], sp, na, sm, nb, n_vars, out);
  }
  return 0;
}

/* The interaction definitions over a table of game values g[S] (S a bitmask
 * of n players):
 *   Shapley (Def. shap_iv_def): phi_{j|i=1} - phi_{j|i=0}, each a Shapley value
 *     of j in the game on the other n - 1 players with i fixed;
 *   Banzhaf (Def. banzhaf_iv_def): E[g | i,j in S] + E[g | i,j not in S]
 *     - E[g | i in S, j not] - E[g | j in S, i not], S uniform.
 * out[i * n + j], diagonal 0. */
static void iv_from_game(int n, const double *g, int kind, double *out) {
  int64_t N = (int64_t)1 << n;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      if (i != j) {
        int64_t bi = (int64_t)1 << i, bj = (int64_t)1 << j;
        /* sum over T subset of the players other than i and j */
        double e11 = 0, e00 = 0, e10 = 0, e01 = 0;
        for (int64_t T = 0; T < N; ++T) {
          if (T & (bi | bj)) continue;
          if (kind == WO_BANZHAF) {
            e11 += g[T | bi | bj];
            e00 += g[T];
            e10 += g[T | bi];
            e01 += g[T | bj];
          } else {
            /* Shapley value of j in an (n-1)-player game: weight of coalition T
             * (|T| players besides j) is 1 / ((n-1) C(n-2, |T|)) */
            int t = __builtin_popcountll((unsigned long long)T);
            double wt = 1.0 / ((double)(n - 1) * binom(n - 2, t));
            double with_i = g[T | bi | bj] - g[T | bi];   /* i always participates */
            double without_i = g[T | bj] - g[T];          /* i always missing */
            s += wt * (with_i - without_i);
          }
        }
        if (kind == WO_BANZHAF) {
          double cnt = ldexp(1.0, n - 2); /* subsets T per conditional expectation */
          s = (e11 + e00 - e10 - e01) / cnt;
        }
      }
      out[(int64_t)i * n + j] = s;
    }
  }
}

/* Interaction values of a WDNF from the definitions over all 2^n assignments. */
int wo_wdnf_iv_bruteforce(int n_vars, int n_cubes, const double *w, const int32_t *lits, int max_lits, int kind,
                          double *out) {
  if (n_vars > 20 || n_vars < 2) return -1;
  uint8_t x[32];
  int64_t N = (int64_t)1 << n_vars;
  double *F = (double *)malloc(sizeof(double) * (size_t)N);
  for (int64_t a = 0; a < N; ++a) {
    for (int v = 0; v < n_vars; ++v) x[v] = (uint8_t)((a >> v) & 1);
    F[a] = wo_wdnf_eval(n_cubes, w, lits, max_lits, x);
  }
  iv_from_game(n_vars, F, kind, out);
  free(F);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Background SHAP: Formula trival_bg with the four rules                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  const wo_model *M;
  const float *C;
  int64_t ldc;
  int64_t m;
  int kind;
  int64_t nl;
  const wo_path *paths;
  const uint64_t *pb; /* [leaf][m] background patterns of the current tree */
  double *phi;        /* [F][n] accumulated */
  int64_t ldphi;
} fourrule_ctx;

static void fourrule_row(void *vctx, int64_t r) {
  fourrule_ctx *X = (fourrule_ctx *)vctx;
  const wo_model *M = X->M;
  int F = M->n_features;
  double *x = (double *)malloc(sizeof(double) * (size_t)F);
  double *acc = (double *)calloc((size_t)F, sizeof(double));
  load_row(X->C, X->ldc, r, F, x);
  int32_t sp[WO_MAXD], sm[WO_MAXD];
  for (int64_t j = 0; j < X->nl; ++j) {
    const wo_path *P = &X->paths[j];
    uint64_t pc = path_pattern(M, P, x);
    double w = (double)M->value[P->leaf] / (double)X->m;
    for (int64_t b = 0; b < X->m; ++b) {
      int na, nb;
      if (!four_rule_cube(M, P, pc, X->pb[j * X->m + b], sp, &na, sm, &nb)) continue;
      credit_cube(X->kind, w, sp, na, sm, nb, acc);
    }
  }
  for (int f = 0; f < F; ++f) X->phi[(int64_t)f * X->ldphi + r] += acc[f];
  free(acc);
  free(x);
}

/* phi[f * ldphi + r] = Background value of feature f for consumer r. */
int wo_bg_fourrule(const wo_model *M, const float *C, int64_t n, int64_t ldc, const float *B,
                   int64_t m, int64_t ldb, int kind, double *phi, int64_t ldphi, int threads) {
  int F = M->n_features;
  for (int f = 0; f < F; ++f)
    for (int64_t r = 0; r < n; ++r) phi[(int64_t)f * ldphi + r] = 0.0;
  double *x = (double *)malloc(sizeof(double) * (size_t)F);
  for (int t = 0; t < M->n_trees; ++t) {
    int64_t nl = collect_paths(M, t, NULL);
    wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)nl);
    collect_paths(M, t, paths);
    uint64_t *pb = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nl * m));
    for (int64_t b = 0; b < m; ++b) {
      load_row(B, ldb, b, F, x);
      for (int64_t j = 0; j < nl; ++j) pb[j * m + b] = path_pattern(M, &paths[j], x);
    }
    fourrule_ctx ctx = {M, C, ldc, m, kind, nl, paths, pb, phi, ldphi};
    parallel_rows(n, threads, fourrule_row, &ctx);
    free(pb);
    free(paths);
  }
  free(x);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Background SHAP: depth-first walk over satisfiable cubes                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  const wo_model *M;
  const double *c, *b;
  int kind;
  double scale;
  double *phi;
  int64_t base;
  double *iv; /* when set: interaction values [F][F] instead of phi */
} walk_state;

/* At an inner node with feature f (c and b take directions gc, gb):
 *  f already positive in the cube -> only gc can keep the cube satisfiable;
 *  f already negated             -> only gb can;
 *  gc == gb                      -> rule 3 on that child, rule 4 on the other;
 *  gc != gb                      -> rule 1 toward gc, rule 2 toward gb. */
static void walk(walk_state *S, int64_t nd, int32_t *sp, int na, int32_t *sm, int nb) {
  const wo_model *M = S->M;
  int32_t f = M->feature[nd];
  if (f < 0) {
    if (S->iv)
      credit_cube_iv(S->kind, S->scale * (double)M->value[nd], sp, na, sm, nb, M->n_features, S->iv);
    else
      credit_cube(S->kind, S->scale * (double)M->value[nd], sp, na, sm, nb, S->phi);
    return;
  }
  int64_t lc = S->base + M->left[nd], rc = S->base + M->right[nd];
  int64_t gc = goes_left(M, nd, S->c[f]) ? lc : rc;
  int64_t gb = goes_left(M, nd, S->b[f]) ? lc : rc;
  if (set_has(sp, na, f)) {
    walk(S, gc, sp, na, sm, nb);
  } else if (set_has(sm, nb, f)) {
    walk(S, gb, sp, na, sm, nb);
  } else if (gc == gb) {
    walk(S, gc, sp, na, sm, nb);
  } else {
    sp[na] = f;
    walk(S, gc, sp, na + 1, sm, nb);
    sm[nb] = f;
    walk(S, gb, sp, na, sm, nb + 1);
  }
}

/* Formula trival_bg averages over the background rows.  A task is one
 * consumer row and one contiguous range ("part") of the background: it sums
 * the row's cube values over that range into its own accumulator.  With at
 * least as many rows as threads there is one part per row; with fewer rows
 * the background is cut into enough parts to give every thread work.  The
 * parts of a row are then added in range order, so the result depends only
 * on the part count, never on the thread schedule. */
typedef struct {
  const wo_model *M;
  const float *C;
  int64_t ldc;
  const float *B;
  int64_t m, ldb;
  int kind;
  int iv;          /* interaction values ([F][F] per row) instead of phi */
  int64_t parts;   /* background ranges per consumer row */
  int64_t width;   /* accumulator entries per task: F, or F * F */
  double *acc;     /* [n][parts][width] */
} walkrows_ctx;

static void walk_task(void *vctx, int64_t task) {
  walkrows_ctx *X = (walkrows_ctx *)vctx;
  const wo_model *M = X->M;
  const int F = M->n_features;
  const int64_t r = task / X->parts, part = task % X->parts;
  const int64_t k0 = X->m * part / X->parts, k1 = X->m * (part + 1) / X->parts;
  double *c = (double *)malloc(sizeof(double) * (size_t)F);
  double *b = (double *)malloc(sizeof(double) * (size_t)F);
  double *acc = X->acc + (size_t)task * (size_t)X->width;
  load_row(X->C, X->ldc, r, F, c);
  int32_t sp[WO_MAXD], sm[WO_MAXD];
  walk_state S = {M, c, b, X->kind, 1.0 / (double)X->m, X->iv ? NULL : acc, 0, X->iv ? acc : NULL};
  for (int64_t k = k0; k < k1; ++k) {
    load_row(X->B, X->ldb, k, F, b);
    for (int t = 0; t < M->n_trees; ++t) {
      S.base = M->node_offset[t];
      walk(&S, S.base, sp, 0, sm, 0);
    }
  }
  free(b);
  free(c);
}

static int walk_rows(const wo_model *M, const float *C, int64_t n, int64_t ldc, const float *B, int64_t m,
                     int64_t ldb, int kind, int iv, double *out, int64_t ldo, int threads) {
  const int F = M->n_features;
  if (threads < 1) threads = 1;
  int64_t parts = 1;
  if (n > 0 && n < threads) parts = (threads + n - 1) / n;
  if (parts > m) parts = m > 0 ? m : 1;
  const int64_t width = iv ? (int64_t)F * F : F;
  double *acc = (double *)calloc((size_t)(n * parts * width > 0 ? n * parts * width : 1), sizeof(double));
  if (!acc) return -1;
  walkrows_ctx ctx = {M, C, ldc, B, m, ldb, kind, iv, parts, width, acc};
  parallel_rows(n * parts, threads, walk_task, &ctx);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t q = 0; q < width; ++q) {
      double v = 0.0;
      for (int64_t p = 0; p < parts; ++p) v += acc[((size_t)r * (size_t)parts + (size_t)p) * (size_t)width + (size_t)q];
      out[q * ldo + r] = v;
    }
  free(acc);
  return 0;
}

int wo_bg_walk(const wo_model *M, const float *C, int64_t n, int64_t ldc, const float *B, int64_t m,
               int64_t ldb, int kind, double *phi, int64_t ldphi, int threads) {
  return walk_rows(M, C, n, ldc, B, m, ldb, kind, 0, phi, ldphi, threads);
}

/* Background interaction values: iv[(i * F + j) * ldphi + r] for consumer r,
 * the pair (i, j) of features, diagonal 0. */
int wo_bg_iv_walk(const wo_model *M, const float *C, int64_t n, int64_t ldc, const float *B, int64_t m,
                  int64_t ldb, int kind, double *iv, int64_t ldphi, int threads) {
  return walk_rows(M, C, n, ldc, B, m, ldb, kind, 1, iv, ldphi, threads);
}

/* ------------------------------------------------------------------------ */
/* Background SHAP by coalition enumeration (Formula eq:s)                   */
/* ------------------------------------------------------------------------ */

typedef struct {
  const wo_model *M;
  const float *C;
  int64_t ldc;
  const float *B;
  int64_t m, ldb;
  int kind;
  double *phi;
  int64_t ldphi;
} brute_ctx;

static void brute_row(void *vctx, int64_t r) {
  brute_ctx *X = (brute_ctx *)vctx;
  const wo_model *M = X->M;
  int F = M->n_features;
  int64_t N = (int64_t)1 << F;
  double *c = (double *)malloc(sizeof(double) * (size_t)F);
  double *b = (double *)malloc(sizeof(double) * (size_t)F);
  double *h = (double *)malloc(sizeof(double) * (size_t)F);
  double *v = (double *)calloc((size_t)N, sizeof(double));
  load_row(X->C, X->ldc, r, F, c);
  for (int64_t k = 0; k < X->m; ++k) {
    load_row(X->B, X->ldb, k, F, b);
    for (int64_t S = 0; S < N; ++S) {
      for (int f = 0; f < F; ++f) h[f] = ((S >> f) & 1) ? c[f] : b[f];
      double s = 0.0;
      for (int t = 0; t < M->n_trees; ++t) s += tree_predict(M, t, h);
      v[S] += s;
    }
  }
  for (int64_t S = 0; S < N; ++S) v[S] /= (double)X->m;
  for (int i = 0; i < F; ++i) {
    double s = 0.0;
    for (int64_t S = 0; S < N; ++S) {
      if ((S >> i) & 1) continue;
      int size = __builtin_popcountll((unsigned long long)S);
      double wt = X->kind == WO_BANZHAF ? 1.0 / ldexp(1.0, F - 1)
                                        : 1.0 / ((double)F * binom(F - 1, size));
      s += wt * (v[S | ((int64_t)1 << i)] - v[S]);
    }
    X->phi[(int64_t)i * X->ldphi + r] = s;
  }
  free(v);
  free(h);
  free(b);
  free(c);
}

static void iv_brute_row(void *vctx, int64_t r) {
  brute_ctx *X = (brute_ctx *)vctx;
  const wo_model *M = X->M;
  int F = M->n_features;
  int64_t N = (int64_t)1 << F;
  double *c = (double *)malloc(sizeof(double) * (size_t)F);
  double *b = (double *)malloc(sizeof(double) * (size_t)F);
  double *h = (double *)malloc(sizeof(double) * (size_t)F);
  double *v = (double *)calloc((size_t)N, sizeof(double));
  double *out = (double *)malloc(sizeof(double) * (size_t)F * (size_t)F);
  load_row(X->C, X->ldc, r, F, c);
  for (int64_t k = 0; k < X->m; ++k) {
    load_row(X->B, X->ldb, k, F, b);
    for (int64_t S = 0; S < N; ++S) {
      for (int f = 0; f < F; ++f) h[f] = ((S >> f) & 1) ? c[f] : b[f];
      double s = 0.0;
      for (int t = 0; t < M->n_trees; ++t) s += tree_predict(M, t, h);
      v[S] += s;
    }
  }
  for (int64_t S = 0; S < N; ++S) v[S] /= (double)X->m;
  iv_from_game(F, v, X->kind, out);
  for (int64_t q = 0; q < (int64_t)F * F; ++q) X->phi[q * X->ldphi + r] = out[q];
  free(out);
  free(v);
  free(h);
  free(b);
  free(c);
}

/* Interaction values from their definitions on the Background-SHAP game
 * (F <= 20); layout as wo_bg_iv_walk. */
int wo_bg_iv_bruteforce(const wo_model *M, const float *C, int64_t n, int64_t ldc, const float *B, int64_t m,
                        int64_t ldb, int kind, double *iv, int64_t ldphi, int threads) {
  if (M->n_features > 20 || M->n_features < 2) return -1;
  brute_ctx ctx = {M, C, ldc, B, m, ldb, kind, iv, ldphi};
  parallel_rows(n, threads, iv_brute_row, &ctx);
  return 0;
}

int wo_bg_bruteforce(const wo_model *M, const float *C, int64_t n, int64_t ldc, const float *B,
                     int64_t m, int64_t ldb, int kind, double *phi, int64_t ldphi, int threads) {
  if (M->n_features > 20) return -1;
  brute_ctx ctx = {M, C, ldc, B, m, ldb, kind, phi, ldphi};
  parallel_rows(n, threads, brute_row, &ctx);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 and Alg. 3 steps 2-3                                               */
/* ------------------------------------------------------------------------ */

/* Alg. 2 for a path with features feat[0..d-1].  Every reachable pattern pair
 * (pc, pb) receives a cube; the result lists 3^d entries.  Cubes are kept as
 * position masks: bit i of pos_mask / neg_mask set when the literal comes
 * from path position i (rule 1 / rule 2).  Returns the entry count. */
int64_t wo_map_patterns_to_cube(int d, uint32_t *pc, uint32_t *pb, uint32_t *pos_mask, uint32_t *neg_mask) {
  if (d > 16) return -1;
  int64_t cap = 1;
  for (int i = 0; i < d; ++i) cap *= 3;
  uint32_t *a_pc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap), *a_pb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
  uint32_t *a_p = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap), *a_n = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
  uint32_t *b_pc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap), *b_pb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
  uint32_t *b_p = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap), *b_n = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
  int64_t cnt = 1;
  a_pc[0] = 0; a_pb[0] = 0; a_p[0] = 0; a_n[0] = 0;
  for (int i = 0; i < d; ++i) {
    int64_t nc = 0;
    for (int64_t e = 0; e < cnt; ++e) {
      /* (1,0): add f; (0,1): add not f; (1,1): unchanged; (0,0) never stored */
      b_pc[nc] = 2 * a_pc[e] + 1; b_pb[nc] = 2 * a_pb[e] + 0; b_p[nc] = a_p[e] | (1u << i); b_n[nc] = a_n[e]; ++nc;
      b_pc[nc] = 2 * a_pc[e] + 0; b_pb[nc] = 2 * a_pb[e] + 1; b_p[nc] = a_p[e]; b_n[nc] = a_n[e] | (1u << i); ++nc;
      b_pc[nc] = 2 * a_pc[e] + 1; b_pb[nc] = 2 * a_pb[e] + 1; b_p[nc] = a_p[e]; b_n[nc] = a_n[e]; ++nc;
    }
    uint32_t *t;
    t = a_pc; a_pc = b_pc; b_pc = t;
    t = a_pb; a_pb = b_pb; b_pb = t;
    t = a_p; a_p = b_p; b_p = t;
    t = a_n; a_n = b_n; b_n = t;
    cnt = nc;
  }
  if (pc) {
    memcpy(pc, a_pc, sizeof(uint32_t) * (size_t)cnt);
    memcpy(pb, a_pb, sizeof(uint32_t) * (size_t)cnt);
    memcpy(pos_mask, a_p, sizeof(uint32_t) * (size_t)cnt);
    memcpy(neg_mask, a_n, sizeof(uint32_t) * (size_t)cnt);
  }
  free(a_pc); free(a_pb); free(a_p); free(a_n);
  free(b_pc); free(b_pb); free(b_p); free(b_n);
  return cnt;
}

/* Alg. 3 steps 2-3 for every leaf:
 *   M_{l,i}[pc][pb] = v(d_l[pc][pb])_i (leaf weight 1), from Alg. 2 and the
 *   value function of `kind`; s_{l,i} = w_l * M_{l,i} * f_l.
 * freq[hist_off[l] + pb] is f_l (already normalised).  Output
 * s_out[s_off[l] + k * 2^d + pc] holds s_{l,i} for the feature i at path
 * position k when k is the first position carrying i, and 0 at later
 * positions carrying the same feature (so each feature appears once), with
 * s_off[l] = sum over earlier leaves of depth * 2^depth. */
int wo_woodelf_tables(const wo_model *M, const double *freq, const int64_t *hist_off, int kind,
                      double *s_out) {
  int64_t lbase = 0, sbase = 0;
  for (int t = 0; t < M->n_trees; ++t) {
    int64_t nl = collect_paths(M, t, NULL);
    wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)nl);
    collect_paths(M, t, paths);
    for (int64_t j = 0; j < nl; ++j) {
      const wo_path *P = &paths[j];
      int d = P->depth;
      int64_t np = (int64_t)1 << d;
      double *s = s_out + sbase;
      for (int64_t e = 0; e < (int64_t)d * np; ++e) s[e] = 0.0;
      if (d > 0) {
        int64_t ne = wo_map_patterns_to_cube(d, NULL, NULL, NULL, NULL);
        uint32_t *pc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ne), *pb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ne);
        uint32_t *pm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ne), *nm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ne);
        wo_map_patterns_to_cube(d, pc, pb, pm, nm);
        /* feature of each position and the first position carrying it */
        int32_t feat[WO_MAXD];
        int first[WO_MAXD];
        for (int k = 0; k < d; ++k) {
          feat[k] = M->feature[P->nodes[k]];
          first[k] = k;
          for (int q = 0; q < k; ++q)
            if (feat[q] == feat[k]) { first[k] = q; break; }
        }
        const double *f = freq + hist_off[lbase + j];
        double w = (double)M->value[P->leaf];
        for (int64_t e = 0; e < ne; ++e) {
          /* sets of distinct features; Alg. 2 positions were pushed MSB-first,
           * so position mask bit i is path position i */
          int32_t sp[WO_MAXD], sm[WO_MAXD];
          int na = 0, nb = 0;
          for (int k = 0; k < d; ++k) {
            if ((pm[e] >> k) & 1u) { if (!set_has(sp, na, feat[k])) sp[na++] = feat[k]; }
            if ((nm[e] >> k) & 1u) { if (!set_has(sm, nb, feat[k])) sm[nb++] = feat[k]; }
          }
          int bad = 0;
          for (int i = 0; i < na; ++i)
            if (set_has(sm, nb, sp[i])) bad = 1;
          if (bad || na + nb == 0) continue;
          double fb = f[pb[e]];
          if (fb == 0.0) continue;
          for (int k = 0; k < d; ++k) {
            if (first[k] != k) continue;
            double v = 0.0;
            if (set_has(sp, na, feat[k])) v = cube_coef(kind, na, nb, 1);
            else if (set_has(sm, nb, feat[k])) v = cube_coef(kind, na, nb, 0);
            else continue;
            s[(int64_t)k * np + pc[e]] += w * v * fb;
          }
        }
        free(pc); free(pb); free(pm); free(nm);
      }
      sbase += (int64_t)d * np;
    }
    free(paths);
    lbase += nl;
  }
  return 0;
}

/* Formula eq:path_dependent_estimation: for every leaf,
 * freq[hist_off[l] + p] = prod_i (r_i if bit i of p is 1 else 1 - r_i) with
 * r_i = cover(n_{i+1}) / cover(n_i) along the path. */
int wo_pd_freq(const wo_model *M, const int64_t *hist_off, double *freq) {
  if (!M->cover) return -1;
  int64_t lbase = 0;
  for (int t = 0; t < M->n_trees; ++t) {
    int64_t nl = collect_paths(M, t, NULL);
    wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)nl);
    collect_paths(M, t, paths);
    int64_t base = M->node_offset[t];
    for (int64_t j = 0; j < nl; ++j) {
      const wo_path *P = &paths[j];
      int d = P->depth;
      double r[WO_MAXD];
      for (int i = 0; i < d; ++i) {
        int64_t nd = P->nodes[i];
        int64_t nx = (i + 1 < d) ? P->nodes[i + 1] : P->leaf;
        (void)base;
        r[i] = M->cover[nd] > 0 ? M->cover[nx] / M->cover[nd] : 0.0;
      }
      for (int64_t p = 0; p < ((int64_t)1 << d); ++p) {
        double v = 1.0;
        for (int i = 0; i < d; ++i) v *= path_bit(P, (uint64_t)p, i) ? r[i] : 1.0 - r[i];
        freq[hist_off[lbase + j] + p] = v;
      }
    }
    free(paths);
    lbase += nl;
  }
  return 0;
}

/* Path-dependent game by coalition enumeration: v(S) = sum over leaves of
 * w_l * prod_i g_i with g_i = 1[c follows the path at n_i] when the node's
 * feature is in S, else the cover ratio r_i; values by Formula eq:s (or the
 * Banzhaf definition). */
int wo_pd_bruteforce(const wo_model *M, const float *C, int64_t n, int64_t ldc, int kind, double *phi,
                     int64_t ldphi) {
  int F = M->n_features;
  if (F > 20 || !M->cover) return -1;
  int64_t N = (int64_t)1 << F;
  double *c = (double *)malloc(sizeof(double) * (size_t)F);
  double *v = (double *)malloc(sizeof(double) * (size_t)N);
  for (int64_t r = 0; r < n; ++r) {
    load_row(C, ldc, r, F, c);
    for (int64_t S = 0; S < N; ++S) v[S] = 0.0;
    for (int t = 0; t < M->n_trees; ++t) {
      int64_t nl = collect_paths(M, t, NULL);
      wo_path *paths = (wo_path *)malloc(sizeof(wo_path) * (size_t)nl);
      collect_paths(M, t, paths);
      for (int64_t j = 0; j < nl; ++j) {
        const wo_path *P = &paths[j];
        uint64_t pc = path_pattern(M, P, c);
        for (int64_t S = 0; S < N; ++S) {
          double g = (double)M->value[P->leaf];
          for (int i = 0; i < P->depth && g != 0.0; ++i) {
            int64_t nd = P->nodes[i];
            int64_t nx = (i + 1 < P->depth) ? P->nodes[i + 1] : P->leaf;
            if ((S >> M->feature[nd]) & 1) g *= path_bit(P, pc, i) ? 1.0 : 0.0;
            else g *= M->cover[nd] > 0 ? M->cover[nx] / M->cover[nd] : 0.0;
          }
          v[S] += g;
        }
      }
      free(paths);
    }
    for (int i = 0; i < F; ++i) {
      double s = 0.0;
      for (int64_t S = 0; S < N; ++S) {
        if ((S >> i) & 1) continue;
        int size = __builtin_popcountll((unsigned long long)S);
        double wt = kind == WO_BANZHAF ? 1.0 / ldexp(1.0, F - 1) : 1.0 / ((double)F * binom(F - 1, size));
        s += wt * (v[S | ((int64_t)1 << i)] - v[S]);
      }
      phi[(int64_t)i * ldphi + r] = s;
    }
  }
  free(v);
  free(c);
  return 0;
}
