// Model-specialised kernels.
//
// For a given ensemble this file writes the pattern/histogram kernel and the
// pattern/gather kernel as straight-line HIP code in which every node's
// feature, threshold rank and default direction, every table offset and every
// output feature is a compile-time constant, then compiles them with hipRTC
// for gfx950.  A row's threshold ranks (8 or 16 bits per feature, packed in
// 32-bit words) and its phi accumulators live in registers with static
// indices; one node costs a byte-select compare and an add-with-carry that
// shifts the path pattern (Alg. 1: P[left] = 2 P + split, P[right] = P[left] ^ 1).
// Gather tables stream through LDS in double-buffered stages with direct
// global-to-LDS loads.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "wdf.h"
#include "wdf_dev.h"
#include "wdf_impl.h"
#include "wdf_internal.h"

namespace wdf {

struct JitPart {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  ~JitPart() {
    if (mod) (void)hipModuleUnload(mod);
  }
};

constexpr int kIvSideStreams = 3;  // streams besides the caller's that run interaction kernels

struct JitModule {
  std::shared_ptr<JitPart> hist_part, explain_part;
  std::vector<std::shared_ptr<JitPart>> iv_parts;  // programs of the interaction and pattern kernels
  hipFunction_t hist = nullptr, explain = nullptr;
  std::vector<hipFunction_t> iv;  // interaction kernels, features [c * 4, c * 4 + 4)
  hipFunction_t patterns = nullptr;  // all groups' patterns of consumer rows, for the interaction kernels
  // the interaction kernels of one chunk of rows run on the caller's stream
  // and these (created with the kernels, default priority), forked from and
  // joined back to the caller's stream by events; iv_mu orders the enqueues
  // of calls from several host threads
  hipStream_t iv_side[kIvSideStreams] = {};
  hipEvent_t iv_fork = nullptr, iv_join[kIvSideStreams] = {};
  std::mutex iv_mu;
  ~JitModule() {
    for (hipStream_t &x : iv_side)
      if (x) (void)hipStreamDestroy(x);
    if (iv_fork) (void)hipEventDestroy(iv_fork);
    for (hipEvent_t &x : iv_join)
      if (x) (void)hipEventDestroy(x);
  }
};

namespace {

// ---------------------------------------------------------------------------
// Plan: threshold ranks, histogram chunks, explain stages
// ---------------------------------------------------------------------------

// The fold of an explain-table unit (XUnit::fold_a, fold_b): slot shifts
// that spread the entries rows tend to read together over the 16 groups of
// LDS banks one 16-lane phase of a 16-byte read spans.  With the model's
// covers, each index bit (a raw split, MSB first) is 1 with probability
// cover(left child) / cover(node), the splits taken as independent; the fold
// kept minimises the sum over bank groups of the squared probability mass in
// the group (the chance that two reads hit one group, up to a term no fold
// changes).  Shifts come from ancestors' patterns: at least 1 for a group, 2
// for a quad (whose index has no register for I >> 1).  Without covers, or on
// a tie: shifts 3 and 6 where below the index width.
void choose_fold(const wdf_model *M, XUnit &u, int64_t tree, const std::vector<int64_t> &nodes) {
  const int bits = u.depth + u.quad;
  u.fold_a = bits > 3 ? 3 : 0;
  u.fold_b = bits > 6 ? 6 : 0;
  if (!M->has_cover || bits <= 4) return;  // up to 16 entries sit in distinct groups whatever the fold
  const int E = 1 << bits;
  const int64_t base = M->node_offset[(size_t)tree];
  std::vector<double> P((size_t)E, 1.0);
  for (int k = 0; k < bits; ++k) {
    const int64_t nd = nodes[(size_t)k];
    const double c = M->cover[(size_t)nd];
    const double pl = c > 0 ? M->cover[(size_t)(base + M->left[(size_t)nd])] / c : 0.5;
    for (int I = 0; I < E; ++I) P[(size_t)I] *= ((I >> (bits - 1 - k)) & 1) ? pl : 1.0 - pl;
  }
  auto cost = [&](int a, int b) {
    double grp[16] = {};
    for (int I = 0; I < E; ++I) grp[(I ^ (a ? I >> a : 0) ^ (b ? I >> b : 0)) & 15] += P[(size_t)I];
    double c = 0.0;
    for (double x : grp) c += x * x;
    return c;
  };
  double best = cost(u.fold_a, u.fold_b);
  const int lo = u.quad ? 2 : 1;
  for (int a = lo; a < bits; ++a)
    for (int b = 0; b < bits; ++b) {
      if (b != 0 && b <= a) continue;
      const double c = cost(a, b);
      if (c < best * (1.0 - 1e-9)) best = c, u.fold_a = a, u.fold_b = b;
    }
}

int make_plan(wdf_model *M) {
  JitPlan &P = M->jp;
  const int F = M->n_features;
  // a row's threshold ranks are packed for every feature (feature f in word
  // f / per_word), so the rank words, the background codes and the generated
  // code grow with F
  if (F > WDF_MAX_SPECIALISED_FEATURES)
    return set_error(WDF_E_UNSUPPORTED, "specialised kernels: %d features exceeds %d", F, WDF_MAX_SPECIALISED_FEATURES);
  std::vector<std::vector<float>> per(F);
  for (int64_t i = 0; i < M->n_nodes; ++i) {
    const int32_t f = M->feature[(size_t)i];
    if (f < 0) continue;
    const float t = M->threshold[(size_t)i];
    if (std::isnan(t)) return set_error(WDF_E_UNSUPPORTED, "specialised kernels: NaN threshold at node %lld", (long long)i);
    per[(size_t)f].push_back(t);
  }
  size_t maxk = 0;
  P.thr.clear();
  P.thr_off.assign((size_t)F + 1, 0);
  for (int f = 0; f < F; ++f) {
    auto &v = per[(size_t)f];
    std::sort(v.begin(), v.end());
    // distinct values; -0.0 and +0.0 compare equal and count once
    std::vector<float> u;
    for (float t : v)
      if (u.empty() || !(u.back() == t)) u.push_back(t);
    maxk = std::max(maxk, u.size());
    P.thr.insert(P.thr.end(), u.begin(), u.end());
    P.thr_off[(size_t)f + 1] = (int32_t)P.thr.size();
  }
  if (maxk <= 127) {
    P.wide = 0;
    P.per_word = 4;
  } else if (maxk <= 32767) {
    P.wide = 1;
    P.per_word = 2;
  } else {
    return set_error(WDF_E_UNSUPPORTED, "specialised kernels: a feature has %zu distinct thresholds", maxk);
  }
  P.words = (F + P.per_word - 1) / P.per_word;
  P.rank.assign((size_t)M->n_nodes, -1);
  for (int64_t i = 0; i < M->n_nodes; ++i) {
    const int32_t f = M->feature[(size_t)i];
    if (f < 0) continue;
    const float *b = P.thr.data() + P.thr_off[(size_t)f];
    const float *e = P.thr.data() + P.thr_off[(size_t)f + 1];
    P.rank[(size_t)i] = (int32_t)(std::lower_bound(b, e, M->threshold[(size_t)i]) - b);
  }
  // histogram chunks: consecutive groups whose counters fit the LDS budget,
  // filled to about the same size so that every chunk is about the same work
  P.hist_chunks.clear();
  const int64_t G = (int64_t)M->groups.size();
  int64_t total = 0;
  for (const Group &g : M->groups) total += (int64_t)1 << g.depth;
  const int64_t n_chunks = std::max<int64_t>(1, (total + P.hist_cap - 1) / P.hist_cap);
  const int64_t target = (total + n_chunks - 1) / n_chunks;
  for (int64_t g = 0; g < G;) {
    int64_t a = g, size = 0;
    while (g < G && size + ((int64_t)1 << M->groups[(size_t)g].depth) <= P.hist_cap &&
           (size < target || g == a)) {
      size += (int64_t)1 << M->groups[(size_t)g].depth;
      ++g;
    }
    if (g == a) return set_error(WDF_E_UNSUPPORTED, "specialised kernels: histogram chunk too small");
    P.hist_chunks.push_back({a, g});
  }
  // LDS slot of every histogram bin: bin p of a group of depth d sits at
  // slot s with lanes of a half-wave on distinct banks (see CountGen); perm
  // maps a slot back to its bin.  Below a right turn at path position k < 6
  // the histogram kernel keeps the left child's lane masks, so there a lane
  // counts the bin of the lane with bit k flipped: the group's bins are
  // XOR-permuted by its right turns (bit reversed, as lane bits map to
  // pattern bits).
  P.perm.assign((size_t)M->hist_size, 0);
  for (const Group &g : M->groups) {
    const int d = g.depth, dl = std::min(d, 6);
    uint32_t flip = 0;  // right turns at positions k < 6, as pattern bits of the lane part
    for (int k = 0; k < dl; ++k)
      if (M->path[(size_t)g.path_off + k].dir) flip |= 1u << (dl - 1 - k);
    for (uint32_t s = 0; s < (1u << d); ++s) {
      uint32_t p;
      if (d < 6) {
        p = s ^ flip;
      } else {
        const uint32_t lo = s & 63u, j = s >> 6;
        const uint32_t v = ((lo << 1) | (lo >> 5)) & 63u;  // undo the rotate-right of the lane part
        p = ((v ^ flip) << (d - 6)) | j;
      }
      P.perm[(size_t)(g.hist_off + s)] = (uint32_t)(g.hist_off + p);
    }
  }
  // thresholds of every used feature, padded with NaN to a power of two, for
  // the rank search inside the explain kernel (NaN never compares <= x)
  std::vector<char> used((size_t)F, 0);
  for (const PathNode &pn : M->path) used[(size_t)pn.feat] = 1;
  P.thr_pad.clear();
  P.thr_pad_off.assign((size_t)F, -1);
  P.thr_steps.assign((size_t)F, 0);
  for (int f = 0; f < F; ++f) {
    if (!used[(size_t)f]) continue;
    const int K = P.thr_off[(size_t)f + 1] - P.thr_off[(size_t)f];
    int c = 0;
    while ((1 << c) <= K) ++c;  // 2^c > K: c steps of a branch-free search
    P.thr_pad_off[(size_t)f] = (int32_t)P.thr_pad.size();
    P.thr_steps[(size_t)f] = c;
    for (int i = 0; i < (1 << c); ++i)
      P.thr_pad.push_back(i < K ? P.thr[(size_t)(P.thr_off[(size_t)f] + i)] : std::nanf(""));
  }
  while (P.thr_pad.size() % 4) P.thr_pad.push_back(std::nanf(""));
  // LDS: two table stages fill the 160 KB of a workgroup; the thresholds
  // borrow the stage buffers while the ranks are searched (more thresholds
  // than the buffers hold are searched in global memory)
  const int64_t lds_floats = 160 * 1024 / 4;
  P.nt_explain = 512 / P.explain_bpc;
  // histogram launch bound: 1024 threads leave 128 VGPRs, enough for two
  // tiles of up to 32 words (current and prefetched) and the masks of paths
  // of up to six positions; otherwise 512 (256 VGPRs)
  int max_depth = 0;
  for (const Group &g : M->groups) max_depth = std::max(max_depth, g.depth);
  P.hist_bound = std::min(P.hist_bound_cap, max_depth <= 6 && P.words <= 32 ? kHistMaxThreads : 512);
  if (P.nt_hist <= 0 || P.nt_hist > P.hist_bound) P.nt_hist = P.hist_bound;
  const int64_t room = lds_floats / P.explain_bpc / 2 / 4 * 4;
  P.stage_floats = (int)std::min<int64_t>(P.stage_floats_max, room);
  P.thr_in_lds = (int64_t)P.thr_pad.size() <= 2 * (int64_t)P.stage_floats;
  int max_table = 0;
  for (const Group &g : M->groups) max_table = std::max(max_table, 4 * ((g.depth + 3) / 4) << g.depth);
  if (P.stage_floats < max_table)
    return set_error(WDF_E_UNSUPPORTED, "specialised kernels: %zu thresholds leave too little LDS for the tables",
                     P.thr_pad.size());
  // explain-table units: a pair group and the next pair group form a quad
  // when their pair nodes are the left and right children of one node
  P.xunits.clear();
  P.unit_g0.clear();
  int64_t xoff = 0;
  for (int64_t g = 0; g < G;) {
    const Group &ga = M->groups[(size_t)g];
    bool quad = false;
    if (ga.depth <= P.quad_depth && g + 1 < G && ga.depth >= 2 && ga.col_r >= 0) {
      const Group &gb = M->groups[(size_t)g + 1];
      if (gb.depth == ga.depth && gb.col_r >= 0 && gb.tree == ga.tree) {
        const size_t la = (size_t)ga.path_off + (size_t)ga.depth, lb = (size_t)gb.path_off + (size_t)gb.depth;
        quad = M->path_nodes[la - 2] == M->path_nodes[lb - 2] && M->path[la - 2].dir == 0 && M->path[lb - 2].dir == 1;
      }
    }
    XUnit u{};
    u.src_l = ga.tab_off;
    u.src_r = quad ? M->groups[(size_t)g + 1].tab_off : -1;
    u.dst = xoff;
    u.depth = ga.depth;
    u.quad = quad ? 1 : 0;
    u.nv = ga.depth + u.quad;
    if (quad && xunit_floats(u) > P.stage_floats) {
      quad = false;
      u.src_r = -1;
      u.quad = 0;
      u.nv = ga.depth;
    }
    u.mask = 0;
    for (int k = 0; k < (quad ? ga.depth - 2 : ga.depth); ++k)
      u.mask = (u.mask << 1) | M->path[(size_t)ga.path_off + (size_t)k].dir;
    {
      // the nodes of the index bits: the group's path (and for a quad the
      // right pair's node last)
      std::vector<int64_t> nodes;
      for (int k = 0; k < ga.depth; ++k) nodes.push_back(M->path_nodes[(size_t)ga.path_off + (size_t)k]);
      if (quad) {
        const Group &gb = M->groups[(size_t)g + 1];
        nodes.push_back(M->path_nodes[(size_t)gb.path_off + (size_t)gb.depth - 1]);
      }
      choose_fold(M, u, ga.tree, nodes);
    }
    xoff += xunit_floats(u);
    P.xunits.push_back(u);
    P.unit_g0.push_back(g);
    g += quad ? 2 : 1;
  }
  P.unit_g0.push_back(G);
  P.xtab_size = xoff;
  // explain stages: consecutive units whose tables fit one LDS buffer (stored
  // as group ranges; a stage never splits a quad)
  P.explain_stages.clear();
  const int64_t U = (int64_t)P.xunits.size();
  auto unit_end = [&](int64_t u) { return P.xunits[(size_t)u].dst + xunit_floats(P.xunits[(size_t)u]); };
  for (int64_t u = 0; u < U;) {
    const int64_t a = u, t0 = P.xunits[(size_t)u].dst;
    while (u < U && unit_end(u) - t0 <= P.stage_floats) ++u;
    if (u == a) return set_error(WDF_E_UNSUPPORTED, "specialised kernels: explain stage too small");
    P.explain_stages.push_back({P.unit_g0[(size_t)a], P.unit_g0[(size_t)u]});
  }
  return WDF_OK;
}

// ---------------------------------------------------------------------------
// Source generation
// ---------------------------------------------------------------------------

const char *kPreamble = R"(
typedef unsigned int u32;
typedef long long i64;
// Node test on a threshold rank: t = rank - (j + 1) is negative exactly when
// rank <= j, i.e. when the row goes left (TU: rank unsigned, so a NaN goes
// right; TS: rank sign-extended, so a NaN goes left).  The caller shifts t's
// sign bit into the pattern with alignbit: P' = 2 P + split.  j + 1 <= 64 is
// an inline constant of the instruction (TU/TS); larger ones come in an SGPR
// (TUX/TSX).  Tests share no register, so independent ones interleave.
#define TU(t, w, sel, j1) asm("v_sub_u32_sdwa %0, %1, " #j1 " src0_sel:" sel " src1_sel:DWORD" : "=v"(t) : "v"(w))
#define TS(t, w, sel, j1) asm("v_sub_u32_sdwa %0, sext(%1), " #j1 " src0_sel:" sel " src1_sel:DWORD" : "=v"(t) : "v"(w))
#define TUX(t, w, sel, j1) asm("v_sub_u32_sdwa %0, %1, %2 src0_sel:" sel " src1_sel:DWORD" : "=v"(t) : "v"(w), "s"(j1))
#define TSX(t, w, sel, j1) asm("v_sub_u32_sdwa %0, sext(%1), %2 src0_sel:" sel " src1_sel:DWORD" : "=v"(t) : "v"(w), "s"(j1))
)";

// the explain kernel is named by its gather, so that profiles tell the variants apart
const char *explain_kernel_name(const JitPlan &P) { return P.quad_depth > 0 ? "wdf_explain_quads" : "wdf_explain_pairs"; }

struct TreeIndex {
  // per global node: group indices hanging off it, and the group range below it
  std::vector<int64_t> pair_of, single_l, single_r, gmin, gmax;
  std::vector<int64_t> quad_of;  // unit index when the node roots a quad
  std::vector<int64_t> root_leaf_group;  // per tree, -1 if the root is inner
};

TreeIndex index_tree_groups(const wdf_model *M) {
  TreeIndex ix;
  const size_t N = (size_t)M->n_nodes;
  ix.pair_of.assign(N, -1);
  ix.single_l.assign(N, -1);
  ix.single_r.assign(N, -1);
  ix.gmin.assign(N, INT64_MAX);
  ix.gmax.assign(N, -1);
  ix.root_leaf_group.assign((size_t)M->n_trees, -1);
  ix.quad_of.assign(N, -1);
  for (size_t u = 0; u < M->jp.xunits.size(); ++u) {
    if (!M->jp.xunits[u].quad) continue;
    const Group &g = M->groups[(size_t)M->jp.unit_g0[u]];
    ix.quad_of[(size_t)M->path_nodes[(size_t)g.path_off + (size_t)g.depth - 2]] = (int64_t)u;
  }
  for (size_t g = 0; g < M->groups.size(); ++g) {
    const Group &gr = M->groups[g];
    if (gr.depth == 0) {
      ix.root_leaf_group[(size_t)gr.tree] = (int64_t)g;
      continue;
    }
    const size_t last = (size_t)gr.path_off + (size_t)gr.depth - 1;
    const int64_t parent = M->path_nodes[last];
    if (gr.col_r >= 0) ix.pair_of[(size_t)parent] = (int64_t)g;
    else if (M->path[last].dir == 0) ix.single_l[(size_t)parent] = (int64_t)g;
    else ix.single_r[(size_t)parent] = (int64_t)g;
    for (int k = 0; k < gr.depth; ++k) {
      const size_t nd = (size_t)M->path_nodes[(size_t)gr.path_off + k];
      ix.gmin[nd] = std::min<int64_t>(ix.gmin[nd], (int64_t)g);
      ix.gmax[nd] = std::max<int64_t>(ix.gmax[nd], (int64_t)g);
    }
  }
  return ix;
}

struct Gen {
  const wdf_model *M;
  const TreeIndex &ix;
  std::ostringstream o;
  int64_t a = 0, b = 0;  // group range being emitted
  std::function<void(int64_t g, const std::string &p)> on_group;

  std::string sel(int f) const {
    const JitPlan &P = M->jp;
    const int s = f % P.per_word;
    if (P.wide) return s ? "\"WORD_1\"" : "\"WORD_0\"";
    static const char *B[4] = {"\"BYTE_0\"", "\"BYTE_1\"", "\"BYTE_2\"", "\"BYTE_3\""};
    return B[s];
  }

  std::function<void(int64_t unit, const std::string &p)> on_quad;  // null: no quads
  std::function<void()> on_tree_end;                                 // before a tree's block closes

  void test(int64_t nd, const std::string &pout, const std::string &pin) {
    const int f = M->feature[(size_t)nd];
    const int j1 = M->jp.rank[(size_t)nd] + 1;
    const char *mac = M->default_left[(size_t)nd] ? (j1 <= 64 ? "TS(" : "TSX(") : (j1 <= 64 ? "TU(" : "TUX(");
    o << "u32 " << pout << "; { u32 t_; " << mac << "t_, w" << f / M->jp.per_word << ", " << sel(f) << ", " << j1
      << "); " << pout << " = __builtin_amdgcn_alignbit(" << pin << ", t_, 31); }\n";
  }

  // depth-first over the nodes whose subtree holds groups of [a, b)
  // pattern variables of the current node's ancestors and itself: chain[k]
  // holds the raw splits of the first k + 1 nodes of the path
  std::vector<std::string> chain;
  struct ChainPush {
    std::vector<std::string> &c;
    ChainPush(std::vector<std::string> &c_, const std::string &v) : c(c_) { c.push_back(v); }
    ~ChainPush() { c.pop_back(); }
  };

  // Table slot of a unit's index `idx` of `bits` bits: the explain tables store
  // entry I at I ^ (I >> a) ^ (I >> b) (a bijection; the unit's fold, 0 for
  // no term), which spreads entries over the groups of LDS banks.  I >> k is
  // the pattern of an ancestor, already in a register, so the slot costs one
  // three-input XOR.
  std::string slot(const std::string &idx, int bits, int a, int b) {
    std::vector<std::string> t{idx};
    for (int k : {a, b})
      if (k) t.push_back(chain[(size_t)(bits - k - 1)]);
    if (t.size() == 1) return idx;
    const std::string v = "z" + idx;
    if (t.size() == 2) o << "const u32 " << v << " = " << t[0] << " ^ " << t[1] << ";\n";
    else o << "const u32 " << v << " = __builtin_amdgcn_bitop3_b32(" << t[0] << ", " << t[1] << ", " << t[2] << ", 0x96);\n";
    return v;
  }

  void node(int64_t nd, const std::string &pin) {
    if (!(ix.gmin[(size_t)nd] < b && ix.gmax[(size_t)nd] >= a)) return;
    const std::string pl = "p" + std::to_string(nd);
    test(nd, pl, pin);
    ChainPush push(chain, pl);
    const int64_t base = M->node_offset[(size_t)M->groups[(size_t)ix.gmin[(size_t)nd]].tree];
    const int64_t L = base + M->left[(size_t)nd], R = base + M->right[(size_t)nd];
    if (on_quad && ix.quad_of[(size_t)nd] >= 0) {
      // quad: index = ((2 P + s_a) * 2 + s_left) * 2 + s_right
      const std::string il = "i" + std::to_string(nd), iq = "I" + std::to_string(nd);
      test(L, il, pl);
      test(R, iq, il);
      on_quad(ix.quad_of[(size_t)nd], iq);
      return;
    }
    auto in = [&](int64_t g) { return g >= a && g < b; };
    if (ix.pair_of[(size_t)nd] >= 0) {
      if (in(ix.pair_of[(size_t)nd])) on_group(ix.pair_of[(size_t)nd], pl);
      return;
    }
    // patterns carry raw splits: both children extend the same prefix
    if (ix.single_l[(size_t)nd] >= 0 && in(ix.single_l[(size_t)nd])) on_group(ix.single_l[(size_t)nd], pl);
    if (ix.single_r[(size_t)nd] >= 0 && in(ix.single_r[(size_t)nd])) on_group(ix.single_r[(size_t)nd], pl);
    if (M->feature[(size_t)L] >= 0) node(L, pl);
    if (M->feature[(size_t)R] >= 0) node(R, pl);
  }

  // every tree touching [a, b)
  void range(int64_t ga, int64_t gb) {
    a = ga;
    b = gb;
    const int t0 = M->groups[(size_t)ga].tree, t1 = M->groups[(size_t)gb - 1].tree;
    for (int t = t0; t <= t1; ++t) {
      const int64_t root = M->node_offset[(size_t)t];
      if (M->feature[(size_t)root] < 0) continue;
      // `live` is always 1; the branch only splits the code into one basic
      // block per tree, which keeps instruction selection time linear
      o << "if (live) {\n";
      node(root, "zero");
      if (on_tree_end) on_tree_end();
      o << "}\n";
    }
  }
};

std::vector<int> used_words(const wdf_model *M, const TreeIndex &ix, int64_t a, int64_t b) {
  std::vector<char> u((size_t)M->jp.words, 0);
  for (int64_t g = a; g < b; ++g) {
    const Group &gr = M->groups[(size_t)g];
    for (int k = 0; k < gr.depth; ++k)
      u[(size_t)(M->path[(size_t)gr.path_off + k].feat / M->jp.per_word)] = 1;
  }
  (void)ix;
  std::vector<int> out;
  for (int w = 0; w < M->jp.words; ++w)
    if (u[(size_t)w]) out.push_back(w);
  return out;
}

// Background histograms by wave-wide masks.  A node's compare yields a 64-bit
// mask of the rows (lanes) that go left.  After the compares the lanes change
// role: lane L stands for the pattern whose bit at path position i is bit i
// of L (positions 0..5; deeper positions are enumerated as replicas).  Its
// accumulator is the mask of rows that follow the path with exactly its bits,
// the AND over the path of (mask XOR E) where E = all ones when the lane's bit
// is 0; a popcount then gives that pattern's count for the 64 rows, added to
// the LDS histogram without conflicts (every lane owns one bin).
struct CountGen {
  static constexpr int64_t kLdsHalf = 16384;  // 64 KiB of u32 histogram slots
  const wdf_model *M;
  const TreeIndex &ix;
  std::ostringstream &o;
  int64_t a = 0, b = 0, h0 = 0;
  int uid = 0;
  struct Half { std::string lo, hi; };
  using Acc = std::vector<Half>;

  std::string sel(int f) const {
    const JitPlan &P = M->jp;
    const int s = f % P.per_word;
    if (P.wide) return s ? "\"WORD_1\"" : "\"WORD_0\"";
    static const char *B[4] = {"\"BYTE_0\"", "\"BYTE_1\"", "\"BYTE_2\"", "\"BYTE_3\""};
    return B[s];
  }
  bool in(int64_t g) const { return g >= a && g < b; }
  bool sub(int64_t nd) const { return ix.gmin[(size_t)nd] < b && ix.gmax[(size_t)nd] >= a; }

  // Lane L counts the pattern whose bits at positions 0..5 are L's bits 0..5
  // (deeper positions: replica j).  Its LDS slot is the lane part reversed
  // into pattern order and rotated right by one bit, plus 64 j, so the 32
  // lanes of each half-wave add to 32 distinct banks; groups shorter than six
  // positions use only their first 2^d lanes.
  void group(int64_t g, int d, const Acc &acc) {
    const int64_t off = M->groups[(size_t)g].hist_off - h0;
    for (size_t j = 0; j < acc.size(); ++j) {
      const std::string c = "c" + std::to_string(uid++);
      o << "{ const u32 " << c << " = __builtin_popcount(" << acc[j].lo << ") + __builtin_popcount(" << acc[j].hi
        << ");";
      if (d < 6) o << " if (lane < " << (1 << d) << "u)";
      // slots past the first 64 KiB index from hb*, so that the byte offset
      // stays within the 16-bit offset field of ds_add
      const int64_t slot = off + 64 * (int64_t)j;
      if (slot >= kLdsHalf)
        o << " atomicAdd(&lh[" << (slot - kLdsHalf) << " + hb" << std::min(d, 6) << "], " << c << "); }\n";
      else
        o << " atomicAdd(&lh[" << slot << " + adr" << std::min(d, 6) << "], " << c << "); }\n";
    }
  }

  void node(int64_t nd, int level, const Acc &acc) {
    if (!sub(nd)) return;
    const int f = M->feature[(size_t)nd];
    const int id = uid++;
    const std::string S = "S" + std::to_string(id);
    const int j = M->jp.rank[(size_t)nd];
    const char *mac = M->default_left[(size_t)nd] ? (j <= 64 ? "NDMS(" : "NDMSX(") : (j <= 64 ? "NDM(" : "NDMX(");
    o << "u64 " << S << "; " << mac << S << ", w" << f / M->jp.per_word << ", " << sel(f) << ", " << j << ");\n";
    const std::string sl = "sl" + std::to_string(id), sh = "sh" + std::to_string(id);
    o << "const u32 " << sl << " = (u32)" << S << ", " << sh << " = (u32)(" << S << " >> 32);\n";
    const int64_t base = M->node_offset[(size_t)M->groups[(size_t)ix.gmin[(size_t)nd]].tree];
    const int64_t L = base + M->left[(size_t)nd], R = base + M->right[(size_t)nd];
    const bool pair = ix.pair_of[(size_t)nd] >= 0 && in(ix.pair_of[(size_t)nd]);
    const bool need_l = pair || (ix.single_l[(size_t)nd] >= 0 && in(ix.single_l[(size_t)nd])) ||
                        (M->feature[(size_t)L] >= 0 && sub(L));
    const bool need_r = (ix.single_r[(size_t)nd] >= 0 && in(ix.single_r[(size_t)nd])) ||
                        (M->feature[(size_t)R] >= 0 && sub(R));
    Acc left, right;
    auto var = [&](const char *tag, size_t r, int h) {
      return std::string(tag) + std::to_string(id) + "_" + std::to_string(r) + (h ? "h" : "l");
    };
    if (level < 6) {
      // one three-input op per half: acc & (S ^ E) (truth table 0x60).  The
      // right child's masks, acc & ~(S ^ E), are the left child's in the lane
      // with bit `level` flipped, so the right subtree keeps the left masks
      // and its groups' bins are permuted instead (perm, built with the plan)
      const std::string E = "E" + std::to_string(level);
      for (size_t r = 0; r < acc.size(); ++r) {
        if (need_l || need_r) {
          left.push_back({var("L", r, 0), var("L", r, 1)});
          o << "const u32 " << left.back().lo << " = __builtin_amdgcn_bitop3_b32(" << acc[r].lo << ", " << sl << ", " << E
            << ", 0x60), " << left.back().hi << " = __builtin_amdgcn_bitop3_b32(" << acc[r].hi << ", " << sh << ", "
            << E << ", 0x60);\n";
        }
      }
      right = left;
    } else {
      // deeper positions: both values of the bit, as replicas 2r (bit 0) and 2r+1 (bit 1)
      for (size_t r = 0; r < acc.size(); ++r) {
        const Half one{var("A", r, 0), var("A", r, 1)}, zer{var("Z", r, 0), var("Z", r, 1)};
        o << "const u32 " << one.lo << " = " << acc[r].lo << " & " << sl << ", " << one.hi << " = " << acc[r].hi
          << " & " << sh << ";\n";
        o << "const u32 " << zer.lo << " = " << acc[r].lo << " & ~" << sl << ", " << zer.hi << " = " << acc[r].hi
          << " & ~" << sh << ";\n";
        left.push_back(zer);   // left child: following means going left (split true)
        left.push_back(one);
        right.push_back(one);  // right child: following means split false
        right.push_back(zer);
      }
    }
    const int d = level + 1;
    if (pair) {
      group(ix.pair_of[(size_t)nd], d, left);
      return;
    }
    if (ix.single_l[(size_t)nd] >= 0 && in(ix.single_l[(size_t)nd])) group(ix.single_l[(size_t)nd], d, left);
    if (ix.single_r[(size_t)nd] >= 0 && in(ix.single_r[(size_t)nd])) group(ix.single_r[(size_t)nd], d, right);
    if (M->feature[(size_t)L] >= 0) node(L, level + 1, left);
    if (M->feature[(size_t)R] >= 0) node(R, level + 1, right);
  }

  void range(int64_t ga, int64_t gb) {
    a = ga;
    b = gb;
    const int t0 = M->groups[(size_t)ga].tree, t1 = M->groups[(size_t)gb - 1].tree;
    for (int t = t0; t <= t1; ++t) {
      const int64_t root = M->node_offset[(size_t)t];
      if (M->feature[(size_t)root] < 0) continue;
      // `live` is always 1; the branch only splits the code into one basic
      // block per tree, which keeps instruction selection time linear
      o << "if (live) {\n";
      node(root, 0, Acc{{"vl", "vh"}});
      o << "}\n";
    }
  }
};

std::string gen_hist(const wdf_model *M, const TreeIndex &ix) {
  const JitPlan &P = M->jp;
  std::ostringstream o;
  CountGen gen{M, ix, o};
  int maxd = 0;
  for (const Group &g : M->groups) maxd = std::max(maxd, g.depth);
  o << kPreamble;
  o << "typedef unsigned long long u64;\n"
    // rank <= j as a wave mask; j <= 64 is an inline constant (NDM/NDMS), larger
    // ones come in an SGPR (NDMX/NDMSX)
    << "#define NDM(S, w, sel, j) asm(\"v_cmp_le_u32_sdwa %0, %1, \" #j \" src0_sel:\" sel \" src1_sel:DWORD\" : \"=s\"(S) : \"v\"(w))\n"
    << "#define NDMS(S, w, sel, j) asm(\"v_cmp_le_i32_sdwa %0, sext(%1), \" #j \" src0_sel:\" sel \" src1_sel:DWORD\" : \"=s\"(S) : \"v\"(w))\n"
    << "#define NDMX(S, w, sel, j) asm(\"v_cmp_le_u32_sdwa %0, %1, %2 src0_sel:\" sel \" src1_sel:DWORD\" : \"=s\"(S) : \"v\"(w), \"s\"(j))\n"
    << "#define NDMSX(S, w, sel, j) asm(\"v_cmp_le_i32_sdwa %0, sext(%1), %2 src0_sel:\" sel \" src1_sel:DWORD\" : \"=s\"(S) : \"v\"(w), \"s\"(j))\n";
  o << "extern \"C\" __global__ __launch_bounds__(" << P.hist_bound
    << ") void wdf_hist_spec(const u32* __restrict__ codes, i64 ldc, i64 m, i64 tiles_per_block, u32* __restrict__ hist, const u32* __restrict__ perm, int live) {\n"
    << "  __shared__ u32 lh[" << P.hist_cap << "];\n"
    << "  const u32 lane = threadIdx.x & 63u;\n"
    << "  const int nw = blockDim.x >> 6;  // waves of the block (any multiple of 64 threads up to the bound)\n"
    << "  const i64 ntiles = (m + 63) >> 6;\n"
    << "  const i64 tb0 = (i64)blockIdx.x * tiles_per_block;\n"
    << "  i64 tb1 = tb0 + tiles_per_block; if (tb1 > ntiles) tb1 = ntiles;\n"
    << "  const u32 rev6 = __builtin_bitreverse32(lane) >> 26;\n";
  for (int l = 0; l < 6; ++l) o << "  const u32 E" << l << " = (lane >> " << l << ") & 1u ? 0u : ~0u;\n";
  for (int d = 1; d <= std::min(5, maxd); ++d) o << "  const u32 adr" << d << " = rev6 >> " << 6 - d << ";\n";
  o << "  const u32 adr6 = (rev6 >> 1) | ((rev6 & 1u) << 5);\n";
  // Bases of the second 64 KiB of the histogram: opaque to the compiler,
  // which would otherwise keep one base register per slot there.
  if (P.hist_cap > CountGen::kLdsHalf) {
    for (int d = 1; d <= 6; ++d) {
      if (d <= 5 && d > maxd) continue;
      o << "  u32 hb" << d << " = adr" << d << " + " << CountGen::kLdsHalf << "u; asm(\"\" : \"+v\"(hb" << d << "));\n";
    }
  }
  o << "  switch (blockIdx.y) {\n";
  for (size_t c = 0; c < P.hist_chunks.size(); ++c) {
    const int64_t a = P.hist_chunks[c].first, b = P.hist_chunks[c].second;
    const int64_t h0 = M->groups[(size_t)a].hist_off;
    const int64_t h1 = M->groups[(size_t)b - 1].hist_off + ((int64_t)1 << M->groups[(size_t)b - 1].depth);
    gen.h0 = h0;
    // The words of a wave's next tile are loaded while it counts the current
    // one (software pipelining; the last prefetch re-reads row m - 1).  The
    // load pointer steps by ldc and is opaque to the compiler, which would
    // otherwise hold one 64-bit base per word in scalar registers.
    const std::vector<int> ws = used_words(M, ix, a, b);
    auto load_words = [&](const char *dst, const char *row) {
      o << "      { const __attribute__((address_space(1))) u32* p_ = (const __attribute__((address_space(1))) u32*)(codes + " << row << ");";
      int prev = 0;
      for (int w : ws) {
        if (w != prev) o << " p_ += (i64)" << (w - prev) << " * ldc; asm(\"\" : \"+v\"(p_));";
        prev = w;
        o << " " << dst << w << " = *p_;";
      }
      o << " }\n";
    };
    o << "  case " << c << ": {\n"
      << "    for (int i = threadIdx.x; i < " << (h1 - h0) << "; i += blockDim.x) lh[i] = 0u;\n"
      << "    __syncthreads();\n"
      << "    i64 t = tb0 + (threadIdx.x >> 6);\n";
    for (int w : ws) o << "    u32 w" << w << " = 0u, n" << w << ";\n";
    o << "    if (t < tb1) {\n      const i64 r0 = t * 64 + lane;\n      const i64 rr0 = r0 < m ? r0 : m - 1;\n";
    load_words("w", "rr0");
    o << "    }\n"
      << "    for (; t < tb1; t += nw) {\n"
      << "      const i64 row = t * 64 + lane;\n"
      << "      const u64 V = __ballot(row < m);\n"
      << "      const u32 vl = (u32)V, vh = (u32)(V >> 32);\n"
      << "      const i64 rn = row + 64 * nw;\n"
      << "      const i64 rrn = rn < m ? rn : m - 1;\n";
    load_words("n", "rrn");
    gen.range(a, b);
    for (int w : ws) o << "      w" << w << " = n" << w << ";\n";
    o << "    }\n"
      << "    __syncthreads();\n"
      << "    for (int i = threadIdx.x; i < " << (h1 - h0)
      << "; i += blockDim.x) { const u32 v = lh[i]; if (v) atomicAdd(&hist[perm[" << h0 << " + i]], v); }\n";
    for (int64_t g = a; g < b; ++g)
      if (M->groups[(size_t)g].depth == 0)
        o << "    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&hist[" << M->groups[(size_t)g].hist_off
          << "], (u32)m);\n";
    o << "  } break;\n";
  }
  o << "  default: break;\n  }\n}\n";
  return o.str();
}

// Threshold ranks of the row (X[f * ldx + rr]) packed into the words w*, as
// the pattern code expects; thresholds from lthr (LDS) or thr.  The searches
// run step-major over batches of 16 features so that 16 independent reads
// are in flight at every step.
// nt: the row's values are read with non-temporal loads (each is read once).
void emit_rank_words(std::ostream &o, const wdf_model *M, const std::vector<char> &used, bool lds_thr,
                     bool nt = false) {
  const JitPlan &P = M->jp;
  const int F = M->n_features;
  for (int w = 0; w < P.words; ++w) o << "  u32 w" << w << ";\n";

  // threshold ranks of the row, packed as the pattern kernels expect.  The
  // searches run step-major over batches of 16 features so that 16
  // independent LDS reads are in flight at every step.
  const int bits = P.wide ? 16 : 8;
  std::vector<int> uf;
  for (int f = 0; f < F; ++f)
    if (used[(size_t)f]) uf.push_back(f);
  std::vector<char> word_open((size_t)P.words, 0);
  for (size_t b0 = 0; b0 < uf.size(); b0 += 16) {
    const size_t b1 = std::min(uf.size(), b0 + 16);
    o << "  if (live) {\n";  // one basic block per batch: its loads are not hoisted into the previous one
    int cmax = 0;
    for (size_t i = b0; i < b1; ++i) {
      const int f = uf[i];
      if (nt)
        o << "  const float x" << f << " = __builtin_nontemporal_load(&X[(i64)" << f << " * ldx + rr]); u32 r" << f
          << " = 0u;\n";
      else
        o << "  const float x" << f << " = X[(i64)" << f << " * ldx + rr]; u32 r" << f << " = 0u;\n";
      cmax = std::max(cmax, P.thr_steps[(size_t)f]);
    }
    for (int k = cmax - 1; k >= 0; --k) {
      o << " ";
      for (size_t i = b0; i < b1; ++i) {
        const int f = uf[i];
        if (P.thr_steps[(size_t)f] <= k) continue;
        o << " r" << f << " += (" << (lds_thr ? "lthr[" : "thr[") << P.thr_pad_off[(size_t)f] + (1 << k) - 1 << " + r" << f << "] <= x" << f
          << ") ? " << (1u << k) << "u : 0u;";
      }
      o << "\n";
    }
    for (size_t i = b0; i < b1; ++i) {
      const int f = uf[i], w = f / P.per_word, sft = (f % P.per_word) * bits;
      if (!word_open[(size_t)w]) {
        word_open[(size_t)w] = 1;
        o << "  w" << w << " = 0u;\n";
      }
      o << "  w" << w << " |= (x" << f << " != x" << f << " ? " << (1u << (bits - 1)) << "u : r" << f << ") << " << sft
        << ";\n";
    }
    o << "  }\n";
  }
}

// The stage-copy macro of the generated kernels (needs wbase4, the first
// piece of the thread's wave in floats).
const char *kStagePiece = R"(
// One 16-byte piece per thread and chunk of NT pieces, straight from global
// memory into LDS: piece c + thread of chunk k lands at dst + 4 (c + thread).
// The stages' sizes are constants, so the copies are unrolled: the uniform
// parts of the addresses stay in scalar registers.
#define STAGE_PIECE(src, dst, c) \
  __builtin_amdgcn_global_load_lds((const void*)(((src) + 4 * (c)) + 4u * threadIdx.x), \
                                   (__attribute__((address_space(3))) void*)((dst) + 4 * (c) + wbase4), 16, 0, 0)
)";

// The explain kernel's stage copies: buffer loads straight into LDS through
// a descriptor of the explain tables (base, size in bytes), the lane's byte
// offset in one VGPR and each piece's uniform offset in an SGPR, so that a
// copy instruction needs no vector address arithmetic.  Reads past the
// descriptor's size return zeros instead of faulting.
const char *kStagePieceBuf = R"(
#define STAGE_PIECE_B(sofs, dst, c) \
  __builtin_amdgcn_raw_ptr_buffer_load_lds(trs, (__attribute__((address_space(3))) void*)((dst) + 4 * (c) + wbase4), \
                                           16, tvoff, (sofs) + 16 * (c), 0, 0)
)";

constexpr int kGatherBatch = 4;  // explain units whose table reads are in flight together

// Unrolled copy of n16 16-byte pieces from tab + t0 to LDS at dst_off floats:
// full chunks of nt pieces unconditionally, the last one for the threads it covers.
void emit_stage_copy(std::ostream &o, int64_t t0, int64_t dst_off, int64_t n16, int nt) {
  o << "  { const float* s_ = tab + " << t0 << "; float* d_ = lds + " << dst_off << ";";
  int64_t c = 0;
  for (; c + nt <= n16; c += nt) o << " STAGE_PIECE(s_, d_, " << c << ");";
  if (c < n16) o << " if (threadIdx.x < " << (n16 - c) << "u) STAGE_PIECE(s_, d_, " << c << ");";
  o << " }\n";
}

// The same copy for the explain kernel, through its table descriptor (byte
// offsets from the start of the explain tables).
void emit_stage_copy_buf(std::ostream &o, int64_t t0, int64_t dst_off, int64_t n16, int nt) {
  o << "  { float* d_ = lds + " << dst_off << ";";
  int64_t c = 0;
  for (; c + nt <= n16; c += nt) o << " STAGE_PIECE_B(" << 4 * t0 << "u, d_, " << c << "u);";
  if (c < n16) o << " if (threadIdx.x < " << (n16 - c) << "u) STAGE_PIECE_B(" << 4 * t0 << "u, d_, " << c << "u);";
  o << " }\n";
}

std::string gen_explain(const wdf_model *M, const TreeIndex &ix) {
  const JitPlan &P = M->jp;
  const int F = M->n_features;
  Gen gen{M, ix};
  std::ostringstream &o = gen.o;
  std::vector<char> used((size_t)F, 0);
  for (const PathNode &pn : M->path) used[(size_t)pn.feat] = 1;
  o << kPreamble;
  o << "#define NT " << P.nt_explain << "\n#define SF " << P.stage_floats << "\n#define TF " << P.thr_pad.size() << "\n"
    << "#define EXPLAIN_NAME " << explain_kernel_name(P) << "\n"
    << "#define TAB_BYTES " << 4 * P.xtab_size << "  // bytes of the explain tables\n"
    << "typedef float vf4 __attribute__((ext_vector_type(4)));\n"
    << "typedef const __attribute__((address_space(3))) vf4* lvf4;  // an LDS address (32 bits)\n"
    << "// a table component that adds to no feature (a zero): used by an empty asm,\n"
    << "// so that the read stays 16 bytes wide without an instruction for it\n"
    << "#define KEEP(v) asm volatile(\"\" :: \"v\"(v))\n";
  // stage copies through a buffer descriptor while the tables' byte offsets
  // fit its 31-bit size (every realistic model), else global addresses
  const bool buf_copy = 4 * P.xtab_size <= 0x7fffffffll;
  auto copy = buf_copy ? emit_stage_copy_buf : emit_stage_copy;
  o << (buf_copy ? kStagePieceBuf : kStagePiece) << R"(// one row per lane, one tile of NT rows per block
extern "C" __global__ __launch_bounds__(NT, 2) void EXPLAIN_NAME(const float* __restrict__ X, i64 ldx,
                                                                     const float* __restrict__ tab,
                                                                     const float* __restrict__ thr,
                                                                     float* __restrict__ phi, i64 ldphi, i64 n, int live) {
  __shared__ __attribute__((aligned(16))) float lds[2 * SF];
  const u32 zero = 0u;
  const u32 wbase4 = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u) * 4u;  // the wave's first piece, in floats
  const i64 row = (i64)blockIdx.x * NT + threadIdx.x;
  const i64 rr = row < n ? row : n - 1;
)";
  if (buf_copy)
    o << "  const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc((void*)tab, (short)0, TAB_BYTES, "
         "0x00020000);\n"
      << "  const u32 tvoff = threadIdx.x * 16u;  // the lane's piece of a chunk, in bytes\n";
  const auto &S = P.explain_stages;
  // unit of every group, and the explain-table span of a stage
  std::vector<int64_t> unit_of(M->groups.size());
  for (size_t u = 0; u + 1 < P.unit_g0.size(); ++u)
    for (int64_t g = P.unit_g0[u]; g < P.unit_g0[u + 1]; ++g) unit_of[(size_t)g] = (int64_t)u;
  auto unit_size = [&](int64_t u) { return xunit_floats(P.xunits[(size_t)u]); };
  auto stage_span = [&](size_t s, int64_t &t0, int64_t &n16) {
    const int64_t ua = unit_of[(size_t)S[s].first], ub = unit_of[(size_t)S[s].second - 1];
    t0 = P.xunits[(size_t)ua].dst;
    n16 = (P.xunits[(size_t)ub].dst + unit_size(ub) - t0) / 4;
  };
  int64_t t0, n16;
  stage_span(0, t0, n16);
  // thresholds in the second stage buffer when they fit there, so that the
  // first stage loads during the rank search; else across both buffers
  const bool thr_hi = P.thr_in_lds && (int64_t)P.thr_pad.size() <= P.stage_floats;
  if (thr_hi) copy(o, t0, 0, n16, P.nt_explain);
  if (P.thr_in_lds)
    o << "  float* lthr = lds + " << (thr_hi ? P.stage_floats : 0) << ";\n"
      << "  for (int i = threadIdx.x; i < TF; i += NT) lthr[i] = thr[i];\n  __syncthreads();\n";
  emit_rank_words(o, M, used, P.thr_in_lds, true);
  for (int f = 0; f < F; ++f)
    if (used[(size_t)f]) o << "  float f" << f << " = 0.f;\n";
  if (P.thr_in_lds && !thr_hi) o << "  __syncthreads();\n";  // every wave is done with the thresholds
  if (!thr_hi) copy(o, t0, 0, n16, P.nt_explain);
  o << "  __builtin_amdgcn_s_waitcnt(0);\n  __syncthreads();\n";
  o << "  LDS_BASES\n";
  std::set<int64_t> lds_bases;  // 32 KiB steps of the LDS the gathers address from a base register
  for (size_t s = 0; s < S.size(); ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < S.size()) {
      stage_span(s + 1, t0, n16);
      copy(o, t0, (int64_t)(1 - buf) * P.stage_floats, n16, P.nt_explain);
    }
    const int64_t sbase = P.xunits[(size_t)unit_of[(size_t)S[s].first]].dst;
    // One 16-byte read per float4 plane returns four values of the entry;
    // value v adds to the feature of its path position when that position is
    // the feature's first on the path.  Components that add to no feature
    // (zeros in the tables) are kept by an empty asm (KEEP), so that no read is
    // narrowed to an 8- or 12-byte one (more LDS cycles per value on random
    // addresses) and no instruction is spent on them.  The
    // reads of kGatherBatch units are issued before their adds, with a
    // scheduling barrier between, so that that many are in flight (the
    // compiler otherwise reads, waits and adds one unit at a time).
    std::string pending;  // adds of the units whose reads are issued
    int npending = 0, greg = 0;
    auto flush = [&]() {
      if (!npending) return;
      o << "__builtin_amdgcn_sched_barrier(0);\n" << pending;
      pending.clear();
      npending = 0;
    };
    auto gather = [&](const XUnit &x, const std::string &pidx, const std::vector<const PathNode *> &pos) {
      const int64_t E = (int64_t)1 << (x.depth + x.quad);
      const std::string p = gen.slot(pidx, x.depth + x.quad, x.fold_a, x.fold_b);
      static const char *C[4] = {"x", "y", "z", "w"};
      std::ostringstream adds;
      for (int j = 0; 4 * j < x.nv; ++j) {
        bool any = false;
        for (int c = 0; c < 4 && 4 * j + c < x.nv; ++c) any = any || pos[(size_t)(4 * j + c)]->first;
        if (!any) continue;
        const std::string gv = "g" + std::to_string(greg++);
        // ds_read's offset field holds 16 bits: a unit whose last plane ends
        // past 64 KiB is addressed from the opaque base below it (lb<k>: LDS
        // byte offset k * 32 KiB), so its address stays one shift-add
        const int64_t ofs = buf * P.stage_floats + (x.dst - sbase);  // floats
        const int64_t last_end = 4 * (ofs + 4 * (int64_t)((x.nv + 3) / 4 - 1) * E + 4 * E);
        if (last_end <= 65536) {
          o << "const vf4 " << gv << " = ((const vf4*)(lds + " << ofs << ") + " << p << ")[" << j * E << "];\n";
        } else {
          const int64_t k = 4 * ofs / 32768;
          lds_bases.insert(k);
          o << "const vf4 " << gv << " = (lb" << k << " + " << (ofs - k * 8192) / 4 << " + " << p << ")[" << j * E
            << "];\n";
        }
        for (int c = 0; c < 4; ++c) {
          const bool real = 4 * j + c < x.nv && pos[(size_t)(4 * j + c)]->first;
          if (real) adds << " f" << pos[(size_t)(4 * j + c)]->feat << " += " << gv << "." << C[c] << ";";
          else adds << " KEEP(" << gv << "." << C[c] << ");";
        }
      }
      pending += adds.str() + "\n";
      if (++npending == kGatherBatch) flush();
    };
    gen.on_tree_end = flush;
    gen.on_group = [&](int64_t g, const std::string &p) {
      const Group &gr = M->groups[(size_t)g];
      std::vector<const PathNode *> pos;
      for (int k = 0; k < gr.depth; ++k) pos.push_back(&M->path[(size_t)gr.path_off + k]);
      gather(P.xunits[(size_t)unit_of[(size_t)g]], p, pos);
    };
    gen.on_quad = [&](int64_t u, const std::string &p) {
      const XUnit &x = P.xunits[(size_t)u];
      const Group &gl = M->groups[(size_t)P.unit_g0[(size_t)u]], &gr = M->groups[(size_t)P.unit_g0[(size_t)u] + 1];
      std::vector<const PathNode *> pos;
      for (int v = 0; v < x.depth; ++v) pos.push_back(&M->path[(size_t)gl.path_off + v]);
      pos.push_back(&M->path[(size_t)gr.path_off + x.depth - 1]);
      gather(x, p, pos);
    };
    o << "  {\n";
    gen.range(S[s].first, S[s].second);
    o << "  }\n";
    // keep each stage's accumulations inside the stage: without this the adds
    // sink to the final (conditional) stores and every gathered value stays live
    std::vector<char> touched((size_t)F, 0);
    for (int64_t g = S[s].first; g < S[s].second; ++g) {
      const Group &gr = M->groups[(size_t)g];
      for (int k = 0; k < gr.depth; ++k)
        if (M->path[(size_t)gr.path_off + k].first) touched[(size_t)M->path[(size_t)gr.path_off + k].feat] = 1;
    }
    for (int f = 0; f < F; ++f)
      if (touched[(size_t)f]) o << "  asm volatile(\"\" : \"+v\"(f" << f << "));\n";
    if (s + 1 < S.size()) o << "  __builtin_amdgcn_s_waitcnt(0);\n  __syncthreads();\n";
  }
  {
    // opaque base registers (the compiler would otherwise rebuild each
    // constant address past 64 KiB with an extra move)
    std::ostringstream b;
    for (int64_t k : lds_bases)
      b << "lvf4 lb" << k << " = (lvf4)(lds + " << k * 8192 << "); asm(\"\" : \"+v\"(lb" << k << "));";
    std::string body = o.str();
    const size_t at = body.find("  LDS_BASES\n");
    body.replace(at, std::strlen("  LDS_BASES\n"), "  " + b.str() + "\n");
    o.str("");
    o << body;
  }
  o << "  if (row < n) {\n";
  // phi is written once per launch and not read back: non-temporal stores
  for (int f = 0; f < F; ++f)
    o << "    __builtin_nontemporal_store(" << (used[(size_t)f] ? "f" + std::to_string(f) : "0.f") << ", &phi[" << f
      << " * ldphi + row]);\n";
  o << "  }\n}\n";
  return o.str();
}

// ---------------------------------------------------------------------------
// hipRTC
// ---------------------------------------------------------------------------

int compile(const std::string &src, std::vector<char> &code) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "wdf_spec.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return set_error(WDF_E_COMPILE, "hiprtcCreateProgram failed");
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    if (log.size() > 800) log = log.substr(0, 800);
    return set_error(WDF_E_COMPILE, "hipRTC: %s: %s", hiprtcGetErrorString(r), log.c_str());
  }
  size_t sz = 0;
  hiprtcGetCodeSize(prog, &sz);
  code.resize(sz);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return WDF_OK;
}

}  // namespace

int jit_sources(wdf_model *M, std::string &hist_src, std::string &explain_src) {
  int rc = make_plan(M);
  if (rc) return rc;
  const TreeIndex ix = index_tree_groups(M);
  hist_src = gen_hist(M, ix);
  explain_src = gen_explain(M, ix);
  return WDF_OK;
}

const char *jit_explain_name(const wdf_model *M) { return explain_kernel_name(M->jp); }

int jit_explain_source(wdf_model *M, std::string &src) {
  std::string h;
  return jit_sources(M, h, src);
}

int jit_source(wdf_model *M, bool do_compile, std::string &src) {
  std::string h, x;
  int rc = jit_sources(M, h, x);
  if (rc) return rc;
  src = h + "\n" + x.substr(std::strlen(kPreamble));
  if (do_compile) {
    std::vector<char> ch, cx;
    if ((rc = compile(h, ch)) || (rc = compile(x, cx))) return rc;
  }
  return WDF_OK;
}

// Limits beyond which the generated code would be too large to be worth it.
static const int64_t kMaxSpecialisedNodes = 200000;

namespace {

std::shared_ptr<JitPart> cached_part(wdf_model *M, const std::string &src) {
  std::lock_guard<std::mutex> lock(M->ctx->jit_mu);
  auto it = M->ctx->jit_cache.find(src);
  return it == M->ctx->jit_cache.end() ? nullptr : it->second;
}

int load_part(wdf_model *M, const std::string &src, const std::vector<char> &code, const char *name,
              std::shared_ptr<JitPart> &out) {
  auto p = std::make_shared<JitPart>();
  hipError_t e = hipModuleLoadData(&p->mod, code.data());
  if (e != hipSuccess) return hip_error(e, "hipModuleLoadData");
  if ((e = hipModuleGetFunction(&p->fn, p->mod, name)) != hipSuccess) return hip_error(e, "hipModuleGetFunction");
  std::lock_guard<std::mutex> lock(M->ctx->jit_mu);
  M->ctx->jit_cache[src] = p;
  out = p;
  return WDF_OK;
}

// register spills of a loaded kernel (its private segment), 0 if unknown
int spill_bytes(hipFunction_t fn) {
  int local = 0;
  if (hipFuncGetAttribute(&local, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn) != hipSuccess) return 0;
  return local;
}

}  // namespace

int jit_compile_all(wdf_model *M, const std::vector<std::pair<std::string, std::string>> &progs) {
  // hipRTC compiles of different programs are independent: the ones not yet
  // cached are compiled on threads of their own, then loaded on this thread
  // (which has the model's device current)
  std::vector<size_t> todo;
  for (size_t i = 0; i < progs.size(); ++i) {
    bool dup = false;
    for (size_t j : todo) dup = dup || progs[j].first == progs[i].first;
    if (!dup && !cached_part(M, progs[i].first)) todo.push_back(i);
  }
  std::vector<std::vector<char>> code(todo.size());
  std::vector<int> rcs(todo.size(), WDF_OK);
  std::vector<std::string> errs(todo.size());
  // at most as many compile threads as the host has cores (each hipRTC
  // compile holds its own copy of the compiler's state)
  const size_t nthreads =
      std::min<size_t>(todo.size(), std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency())));
  std::atomic<size_t> next{0};
  std::vector<std::thread> th;
  for (size_t t = 0; t < nthreads; ++t)
    th.emplace_back([&] {
      for (size_t k; (k = next.fetch_add(1)) < todo.size();) {
        rcs[k] = compile(progs[todo[k]].first, code[k]);
        if (rcs[k]) errs[k] = wdf_last_error();  // the error text is thread-local
      }
    });
  for (auto &t : th) t.join();
  for (size_t k = 0; k < todo.size(); ++k)
    if (rcs[k]) return set_error(rcs[k], "%s", errs[k].c_str());
  for (size_t k = 0; k < todo.size(); ++k) {
    std::shared_ptr<JitPart> part;
    const int rc = load_part(M, progs[todo[k]].first, code[k], progs[todo[k]].second.c_str(), part);
    if (rc) return rc;
  }
  return WDF_OK;
}

int jit_build(wdf_model *M) {
  if (M->n_nodes > kMaxSpecialisedNodes)
    return set_error(WDF_E_UNSUPPORTED, "specialised kernels: %lld nodes exceeds %lld", (long long)M->n_nodes,
                     (long long)kMaxSpecialisedNodes);
  std::string hsrc, xsrc;
  int rc = jit_sources(M, hsrc, xsrc);
  if (rc) return rc;
  auto mod = std::make_shared<JitModule>();
  // two programs, cached apart: variants that differ in one part (the explain
  // gather, the histogram bound) reuse the other
  if ((rc = jit_compile_all(M, {{hsrc, "wdf_hist_spec"}, {xsrc, explain_kernel_name(M->jp)}}))) return rc;
  mod->hist_part = cached_part(M, hsrc);
  mod->explain_part = cached_part(M, xsrc);
  // A histogram kernel that spills registers at its launch bound is rebuilt
  // once at 512 threads (256 VGPRs); the explain program is kept.
  if (M->jp.hist_bound > 512 && spill_bytes(mod->hist_part->fn) > 0) {
    M->jp.hist_bound_cap = 512;
    if ((rc = jit_sources(M, hsrc, xsrc))) return rc;
    mod->hist_part = cached_part(M, hsrc);
    if (!mod->hist_part) {
      std::vector<char> ch;
      if ((rc = compile(hsrc, ch))) return rc;
      if ((rc = load_part(M, hsrc, ch, "wdf_hist_spec", mod->hist_part))) return rc;
    }
  }
  mod->hist = mod->hist_part->fn;
  mod->explain = mod->explain_part->fn;
  JitPlan &P = M->jp;
  hipStream_t s = M->ctx->stream;
  // per feature: (offset in the padded thresholds, search steps); 0 steps for unused features
  P.pad_meta.assign((size_t)M->n_features * 2, 0);
  for (int f = 0; f < M->n_features; ++f)
    if (P.thr_steps[(size_t)f] > 0) {
      P.pad_meta[2 * (size_t)f] = P.thr_pad_off[(size_t)f];
      P.pad_meta[2 * (size_t)f + 1] = P.thr_steps[(size_t)f];
    }
  if ((rc = P.d_pad_meta.alloc(P.pad_meta.size() * sizeof(int32_t)))) return rc;
  hipError_t e;
  if ((e = hipMemcpyAsync(P.d_pad_meta.ptr, P.pad_meta.data(), P.pad_meta.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(e, "hipMemcpyAsync(threshold blocks)");
  if ((rc = P.d_thr_pad.alloc(std::max<size_t>(P.thr_pad.size(), 1) * sizeof(float)))) return rc;
  if (!P.thr_pad.empty() && (e = hipMemcpyAsync(P.d_thr_pad.ptr, P.thr_pad.data(), P.thr_pad.size() * sizeof(float),
                                                hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(e, "hipMemcpyAsync(padded thresholds)");
  if ((rc = P.d_xunits.alloc(std::max<size_t>(P.xunits.size(), 1) * sizeof(XUnit)))) return rc;
  if (!P.xunits.empty() && (e = hipMemcpyAsync(P.d_xunits.ptr, P.xunits.data(), P.xunits.size() * sizeof(XUnit),
                                               hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(e, "hipMemcpyAsync(units)");
  if ((rc = P.d_perm.alloc(std::max<size_t>(P.perm.size(), 1) * sizeof(uint32_t)))) return rc;
  if (!P.perm.empty() && (e = hipMemcpyAsync(P.d_perm.ptr, P.perm.data(), P.perm.size() * sizeof(uint32_t),
                                             hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(e, "hipMemcpyAsync(perm)");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  M->jit = mod;
  return WDF_OK;
}

// Interaction values, specialised: one block = kIvRows rows (one per lane)
// and one feature i (a case of the switch on blockIdx.y), two or three
// blocks per CU.  The units of i (a
// group where i has a first occurrence) are contiguous in the interleaved
// tables; they stream through a ring of LDS buffers in stages, each copied
// straight from global memory into LDS by all waves while earlier stages are
// read.  Each wave copies its own 64 rows of the units' patterns (one byte
// per row and unit, from the workspace) into a ring of its own, several
// chunks ahead: these are cold HBM reads, and no other wave reads them, so
// they need no barrier, only the wave's own wait.  Per unit and row: the
// pattern byte from LDS, one 16-byte read per four partners (and one 4- or
// 8-byte read for a last one or two), each value added into a register with
// a static index (one per partner feature of i).  Then the row's iv[i][j] for
// every j, zeros where i has no pair with j (the diagonal among them), with
// non-temporal stores.
//
// Waits are counted: the generator knows every wave's sequence of memory
// reads into LDS, and before data is used it waits until at most the number
// of copies issued after it are outstanding (vmcnt; the counter drains in
// issue order), so later prefetches stay in flight.
namespace {

int64_t iv_spec_ops(const wdf_model *M) {
  int64_t ops = 0;
  for (const IvUnit &u : M->iv_units) ops += 1 + ivunit_quads(u.cnt) + (ivunit_tail(u.cnt) > 0) + u.cnt;
  return ops;
}

constexpr int kIvRows = 256;          // rows per block of the interaction kernels (and of the
                                      // pattern workspace's blocks)
constexpr int kIvTableBufs = 2;       // table stages in LDS (copied one stage ahead)
constexpr int kIvPatChunk = 16;       // units per pattern copy: 64 lanes x 16 bytes, 4 lanes per unit
constexpr int kIvGatherBatch = 4;     // units whose table reads are issued together
constexpr int kIvPerKernel = 4;       // features per interaction kernel (compile time grows
                                      // faster than linearly with a function's size)
constexpr int kIvKernelsPerProgram = 4;  // kernels per hipRTC program (programs compile in parallel)
constexpr int64_t kIvChunkRows = 32768;  // consumer rows whose patterns all features' kernels read in turn

// Resident blocks per CU and the LDS each takes, by the largest number of
// partner accumulators among a kernel's features: three blocks (twelve waves)
// while the registers fit 168 per lane (up to 128 accumulators), else two,
// else one.  More resident blocks overlap one block's stores with another's
// table reads better.
struct IvShape {
  int blocks_per_cu;
  int table_bytes;  // one table buffer (the two stay below 64 KiB: 16-bit read offsets)
  int ring;         // pattern chunks per wave (copied ring - 1 chunks ahead)
  int pat_base() const { return kIvTableBufs * table_bytes; }
  int lds_bytes() const { return pat_base() + kIvRows / 64 * ring * 1024; }
};
const IvShape kIvShapes[3] = {{3, 20480, 3}, {2, 30720, 4}, {1, 32768, 4}};
IvShape iv_shape(int max_partners) {
  return kIvShapes[max_partners <= 128 ? 0 : max_partners <= 200 ? 1 : 2];
}
// the next shape with fewer resident blocks (for a kernel that spilled), or itself
IvShape iv_shape_fewer(const IvShape &s) {
  for (int k = 0; k < 2; ++k)
    if (kIvShapes[k].blocks_per_cu == s.blocks_per_cu) return kIvShapes[k + 1];
  return s;
}

std::string iv_kernel_name(int c) { return "wdf_iv_spec_" + std::to_string(c); }

// Stages of the units [u0, u1): consecutive units whose tables fit one buffer.
std::vector<std::pair<int, int>> iv_stages(const wdf_model *M, int u0, int u1, int table_bytes) {
  std::vector<std::pair<int, int>> st;
  for (int a = u0; a < u1;) {
    int b = a;
    int64_t tfl = 0;
    while (b < u1) {
      const int64_t t = tfl + ivunit_floats(M->iv_units[(size_t)b]);
      if (b > a && 4 * t > table_bytes) break;
      tfl = t;
      ++b;
    }
    st.emplace_back(a, b);
    a = b;
  }
  return st;
}

// Vector-memory instructions one wave issues, in order: `sure` of them
// issued by every wave, `maybe` only by some (a stage copy's last, partial
// chunk of pieces).  wait(e) emits the vmcnt wait after which copy e has
// landed: at most the sure instructions issued after e may be outstanding.
struct VmLog {
  struct Ev {
    int sure, maybe;
  };
  std::vector<Ev> ev;
  int add(int sure, int maybe) {
    ev.push_back({sure, maybe});
    return (int)ev.size() - 1;
  }
  void wait(std::ostream &o, int e) const {
    int after = 0;
    for (size_t k = (size_t)e + 1; k < ev.size(); ++k) after += ev[k].sure;
    after = std::min(after, 63);
    // s_waitcnt fields (gfx9): vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8 (all ones: no wait)
    const int imm = (after & 15) | ((after >> 4) << 14) | (7 << 4) | (15 << 8);
    o << "  __builtin_amdgcn_sched_barrier(0);\n  __builtin_amdgcn_s_waitcnt(" << imm << ");  // vmcnt(" << after
      << ")\n  __builtin_amdgcn_sched_barrier(0);\n";
  }
};

// the partner features of each feature (units' partners), and their counts
struct IvPartners {
  std::vector<std::vector<char>> of;
  std::vector<int> count;
  explicit IvPartners(const wdf_model *M) {
    const int F = M->n_features;
    of.assign((size_t)F, std::vector<char>((size_t)F, 0));
    count.assign((size_t)F, 0);
    for (int i = 0; i < F; ++i) {
      for (int k = M->iv_unit_off[(size_t)i]; k < M->iv_unit_off[(size_t)i + 1]; ++k)
        for (int s = 0; s < M->iv_units[(size_t)k].cnt; ++s)
          of[(size_t)i][(size_t)M->iv_unit_partners[(size_t)k][(size_t)s]] = 1;
      for (int j = 0; j < F; ++j) count[(size_t)i] += of[(size_t)i][(size_t)j];
    }
  }
  IvShape shape(int c, int F) const {
    const int i0 = c * kIvPerKernel, i1 = std::min(F, (c + 1) * kIvPerKernel);
    return iv_shape(*std::max_element(count.begin() + i0, count.begin() + i1));
  }
};

int iv_kernel_count(const wdf_model *M) { return (M->n_features + kIvPerKernel - 1) / kIvPerKernel; }

// types and macros of the interaction kernels
std::string gen_iv_preamble() {
  std::ostringstream o;
  // the launch configuration, recorded in the source (profiles keyed by the
  // source's hash then follow launch changes too)
  o << "// interaction kernels: rows in chunks of " << kIvChunkRows << ", " << kIvRows << "-row blocks, kernels over "
    << 1 + kIvSideStreams << " streams\n";
  o << kPreamble << kStagePiece << "typedef float vf4 __attribute__((ext_vector_type(4)));\n"
    << "typedef float vf2 __attribute__((ext_vector_type(2)));\n"
    << "typedef const __attribute__((address_space(3))) unsigned char* lu8;\n"
    << "typedef __attribute__((address_space(1))) float* gfp;  // a global address (stores stay global_store)\n"
    // (stores of iv are non-temporal: the F x F values per row stream to HBM
    // without taking the caches the table and pattern copies read through)
    // a workgroup barrier without __syncthreads' fence (which waits for every
    // outstanding read, the prefetches included: the counted waits before the
    // barrier cover what it must); the empty asm keeps memory accesses from
    // moving across it
    << "#define BARRIER() { __builtin_amdgcn_sched_barrier(0); asm volatile(\"\" ::: \"memory\"); "
       "__builtin_amdgcn_s_barrier(); asm volatile(\"\" ::: \"memory\"); __builtin_amdgcn_sched_barrier(0); }\n"
    // one wave's copy of its 64 rows of 16 units' patterns: lane L copies 16
    // rows (L % 4) of unit L / 4, group g<L / 4> (a tree of selects on the
    // bits of L / 4, not a chain of conditionals: those compile to branches)
    << "#define PAT_CHUNK(dst";
  for (int k = 0; k < kIvPatChunk; ++k) o << ", g" << k;
  o << ") { ";
  for (int k = 0; k < kIvPatChunk / 2; ++k)
    o << "const u32 a" << k << "_ = pb0 ? (u32)(g" << 2 * k + 1 << ") : (u32)(g" << 2 * k << "); ";
  for (int k = 0; k < kIvPatChunk / 4; ++k)
    o << "const u32 b" << k << "_ = pb1 ? a" << 2 * k + 1 << "_ : a" << 2 * k << "_; ";
  o << "const u32 c0_ = pb2 ? b1_ : b0_; const u32 c1_ = pb2 ? b3_ : b2_; const u32 g_ = pb3 ? c1_ : c0_; "
    << "__builtin_amdgcn_global_load_lds((const void*)(pw + g_ * 256u), "
       "(__attribute__((address_space(3))) void*)(dst), 16, 0, 0); }\n";
  return o.str();
}

// interaction kernel c (features [4c, 4c + 4)) with resident-block shape sh
std::string gen_iv_kernel(const wdf_model *M, const IvPartners &P, int c, const IvShape &sh) {
  const int F = M->n_features;
  constexpr int NW = kIvRows / 64;
  std::ostringstream o;
  static const char *C[4] = {"x", "y", "z", "w"};
  {
    const int i0 = c * kIvPerKernel, i1 = std::min(F, (c + 1) * kIvPerKernel);
    o << "extern \"C\" __global__ __launch_bounds__(" << kIvRows << ", " << sh.blocks_per_cu << ") void " << iv_kernel_name(c)
      << "(const unsigned char* __restrict__ pat, i64 n, const float* __restrict__ tab, "
         "float* __restrict__ out, i64 ldo, int live) {\n"
      << "  __shared__ __attribute__((aligned(16))) float lds[" << sh.lds_bytes() / 4 << "];\n"
      << "  const u32 lane = threadIdx.x & 63u;\n"
      << "  const u32 wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n"
      << "  const u32 wbase4 = wave * 256u;  // the wave's first table piece, in floats\n"
      << "  const i64 row0 = (i64)blockIdx.x * " << kIvRows << ", row = row0 + threadIdx.x;\n"
      << "  // the lane's share of its wave's pattern copies, and the wave's pattern ring\n"
      << "  const u32 pu = lane >> 2;\n"
      << "  const bool pb0 = (pu & 1u) != 0u, pb1 = (pu & 2u) != 0u, pb2 = (pu & 4u) != 0u, pb3 = (pu & 8u) != 0u;\n"
      << "  const unsigned char* pw = pat + (i64)blockIdx.x * " << (int64_t)M->groups.size() * 256
      << " + 64u * wave + 16u * (lane & 3u);\n"
      << "  float* const ring = lds + " << sh.pat_base() / 4 << " + wave * " << sh.ring * 256 << "u;\n"
      << "  const u32 pr = " << sh.pat_base() << "u + wave * " << sh.ring * 1024 << "u + lane;  // the lane's pattern bytes\n"
      << "  float* o = out + row;\n"
      << "  float sink = 0.f;  // unused table components (zeros)\n"
      << "  switch (blockIdx.y) {\n";
    for (int i = i0; i < i1; ++i) {
      const int u0 = M->iv_unit_off[(size_t)i], u1 = M->iv_unit_off[(size_t)i + 1];
      const int U = u1 - u0, nchunks = (U + kIvPatChunk - 1) / kIvPatChunk;
      const std::vector<char> &partner = P.of[(size_t)i];
      o << "  case " << i - c * kIvPerKernel << ": {\n";
      for (int j = 0; j < F; ++j)
        if (partner[(size_t)j]) o << "    float a" << j << " = 0.f;\n";
      const auto st = iv_stages(M, u0, u1, sh.table_bytes);
      VmLog vm;
      std::vector<int> tev(st.size(), -1), pev((size_t)nchunks, -1);
      std::vector<char> pwaited((size_t)nchunks, 0);
      auto tfloats = [&](int a, int b) {
        return M->iv_units[(size_t)b - 1].dst + ivunit_floats(M->iv_units[(size_t)b - 1]) - M->iv_units[(size_t)a].dst;
      };
      auto copy_tables = [&](size_t s) {
        const int a = st[s].first, b = st[s].second;
        const int64_t n16 = tfloats(a, b) / 4;
        emit_stage_copy(o, M->iv_units[(size_t)a].dst, (int64_t)(s % kIvTableBufs) * sh.table_bytes / 4, n16, kIvRows);
        tev[s] = vm.add((int)(n16 / kIvRows), n16 % kIvRows ? 1 : 0);
      };
      auto copy_patterns = [&](int ch) {
        o << "  PAT_CHUNK(ring + " << (ch % sh.ring) * 256;
        for (int k = 0; k < kIvPatChunk; ++k)
          o << ", " << M->iv_units[(size_t)std::min(u1 - 1, u0 + ch * kIvPatChunk + k)].group;
        o << ")\n";
        pev[(size_t)ch] = vm.add(1, 0);
      };
      // prologue: the first table stages, the first pattern chunks
      for (size_t s = 0; s + 1 < (size_t)kIvTableBufs && s < st.size(); ++s) copy_tables(s);
      int next_chunk = 0;
      for (; next_chunk < std::min(nchunks, sh.ring); ++next_chunk) copy_patterns(next_chunk);
      if (!st.empty()) {
        vm.wait(o, tev[0]);
        o << "  BARRIER();\n";
      }
      for (size_t s = 0; s < st.size(); ++s) {
        const int buf = (int)(s % kIvTableBufs);
        if (s + kIvTableBufs - 1 < st.size()) copy_tables(s + kIvTableBufs - 1);
        const int a = st[s].first, b = st[s].second;
        const int64_t sbase = M->iv_units[(size_t)a].dst;
        o << "  {\n";
        auto read_patterns = [&](int k0) {
          for (int k = k0; k < std::min(b, k0 + kIvGatherBatch); ++k) {
            const int t = k - u0, ch = t / kIvPatChunk;
            if (!pwaited[(size_t)ch]) {
              vm.wait(o, pev[(size_t)ch]);
              pwaited[(size_t)ch] = 1;
            }
            o << "  const u32 q" << k - a << " = ((lu8)lds)[pr + " << (ch % sh.ring) * 1024 + (t % kIvPatChunk) * 64
              << "u];\n";
          }
        };
        // batches of kIvGatherBatch units: the table reads of a batch are
        // issued together, then a scheduling barrier, then their adds (left to
        // itself the compiler reads, waits and adds one unit at a time)
        std::vector<char> touched((size_t)F, 0);
        std::map<int, std::string> adds_of;  // first unit of a batch -> its adds
        auto gathers = [&](int k0) {
          std::ostringstream adds;
          for (int k = k0; k < std::min(b, k0 + kIvGatherBatch); ++k) {
            const IvUnit &u = M->iv_units[(size_t)k];
            const int64_t E = (int64_t)1 << u.depth;
            const int64_t ofs = (int64_t)buf * sh.table_bytes / 4 + (u.dst - sbase);  // floats
            const int nq = ivunit_quads(u.cnt), w = ivunit_tail(u.cnt);
            const std::string q = "q" + std::to_string(k - a);
            auto add = [&](const std::string &v, int col) {
              if (col < u.cnt) {
                const int j = M->iv_unit_partners[(size_t)k][(size_t)col];
                touched[(size_t)j] = 1;
                adds << " a" << j << " += " << v << ";";
              } else {
                adds << " sink += " << v << ";";
              }
            };
            for (int pl = 0; pl < nq; ++pl) {
              const std::string g = "g" + std::to_string(k - a) + "_" + std::to_string(pl);
              o << "  const vf4 " << g << " = ((const vf4*)(lds + " << ofs + 4 * E * pl << "))[" << q << "];\n";
              for (int cc = 0; cc < 4; ++cc) add(g + "." + C[cc], 4 * pl + cc);
            }
            const std::string g = "h" + std::to_string(k - a);
            if (w == 2) {
              o << "  const vf2 " << g << " = ((const vf2*)(lds + " << ofs + 4 * E * nq << "))[" << q << "];\n";
              add(g + ".x", 4 * nq);
              add(g + ".y", 4 * nq + 1);
            } else if (w == 1) {
              o << "  const float " << g << " = (lds + " << ofs + 4 * E * nq << ")[" << q << "];\n";
              add(g, 4 * nq);
            }
            adds << "\n";
          }
          adds_of[k0] = adds.str();
        };
        constexpr int B = kIvGatherBatch;
        read_patterns(a);
        for (int k0 = a; k0 < b; k0 += B) {
          const int k1 = std::min(b, k0 + B);
          // the next batch's pattern reads, then this batch's table reads
          if (k1 < b) read_patterns(k1);
          gathers(k0);
          o << "  __builtin_amdgcn_sched_barrier(0);\n" << adds_of[k0] << "  __builtin_amdgcn_sched_barrier(0);\n";
          // the adds waited for this batch's table reads, and so for the
          // pattern reads of its units (issued before them): a chunk whose
          // units are all read frees its ring slot for the chunk sh.ring on
          while (next_chunk < nchunks && (next_chunk - sh.ring + 1) * kIvPatChunk <= k1 - u0) copy_patterns(next_chunk++);
        }
        // keep each stage's accumulations inside the stage
        for (int j = 0; j < F; ++j)
          if (touched[(size_t)j]) o << "  asm volatile(\"\" : \"+v\"(a" << j << "));\n";
        o << "  }\n";
        if (s + 1 < st.size()) {
          vm.wait(o, tev[s + 1]);
          o << "  BARRIER();\n";
        }
      }
      // the row's iv[i][j] for every j, after all reads: the stores count in
      // the same in-order counter (vmcnt) as the copies into LDS, so a store
      // issued earlier would hold up every later counted wait until HBM
      // acknowledged it.  The address steps by ldo from store to store (opaque
      // to the compiler, which otherwise forms every (i F + j) ldo product and
      // spills them)
      o << "    if (row < n) {\n      gfp p = (gfp)o + (i64)" << (int64_t)i * F << " * ldo;\n";
      for (int j = 0; j < F; ++j) {
        o << "      __builtin_nontemporal_store(" << (partner[(size_t)j] ? "a" + std::to_string(j) : std::string("0.f"))
          << ", p);";
        if (j + 1 < F) o << " p += ldo; asm volatile(\"\" : \"+v\"(p));";
        o << "\n";
      }
      o << "    }\n  } break;\n";
    }
    o << "  default: break;\n  }\n"
      << "  if (live == 2) o[0] = sink;  // never (live is 1): keeps the sink's reads whole\n}\n";
  }
  return o.str();
}

// all interaction kernels, each with the shape its partner count gives
std::string gen_iv(const wdf_model *M) {
  const IvPartners P(M);
  std::string src = gen_iv_preamble();
  for (int c = 0; c < iv_kernel_count(M); ++c) src += gen_iv_kernel(M, P, c, P.shape(c, M->n_features));
  return src;
}

// Patterns of every group for every row (Def. Decision Pattern), as raw
// splits (bit 1: the row went left, root bit first; the interaction tables
// apply the group's right turns) stored at their table slot r ^ (r >> 3) ^
// (r >> 6): one byte per (group, row), in blocks of 256 rows, all groups of
// a block together: pat[(row / 256) G 256 + g 256 + row % 256], for every row
// below ldp (a multiple of 512; rows from n on repeat row n - 1).  The
// interaction kernels copy whole 16-byte pieces, and one block's pieces come
// from one span of G x 256 bytes rather than from G rows of the workspace.
// One thread per row, the row's threshold ranks in registers, the node tests
// of all trees in straight-line code, one store per group.
constexpr int64_t kPatLdsThresholds = 16384;  // thresholds staged in LDS up to 64 KB

std::string gen_patterns(const wdf_model *M, const TreeIndex &ix) {
  const JitPlan &P = M->jp;
  const int F = M->n_features;
  const bool lds = (int64_t)P.thr_pad.size() <= kPatLdsThresholds;
  Gen gen{M, ix};
  std::ostringstream &o = gen.o;
  std::vector<char> used((size_t)F, 0);
  for (const PathNode &pn : M->path) used[(size_t)pn.feat] = 1;
  o << "extern \"C\" __global__ __launch_bounds__(256) void wdf_patterns_spec(const float* __restrict__ X, i64 ldx, "
       "const float* __restrict__ thr, unsigned char* __restrict__ pat, i64 n, i64 ldp, int live) {\n"
    << "  const u32 zero = 0u;\n"
    << "  const i64 row = (i64)blockIdx.x * 256 + threadIdx.x;\n"
    << "  const i64 rr = row < n ? row : n - 1;\n"
    << "  unsigned char* const pb = pat + (i64)blockIdx.x * " << (int64_t)M->groups.size() * 256 << " + threadIdx.x;\n";
  if (lds)
    o << "  extern __shared__ float lthr[];\n"
      << "  for (int i = threadIdx.x; i < " << P.thr_pad.size() << "; i += 256) lthr[i] = thr[i];\n"
      << "  __syncthreads();\n";
  emit_rank_words(o, M, used, lds);
  // the grid covers exactly ldp rows (the test, always true, keeps each
  // store in a block of its own: one straight-line block of all trees lets
  // the scheduler interleave them at a high register cost); the slot is
  // computed from the pattern itself (the ancestors' registers would stay
  // live across the trees)
  gen.on_group = [&](int64_t g, const std::string &p) {
    const int d = M->groups[(size_t)g].depth;
    o << "if (row < ldp) pb[" << g * 256 << "] = (unsigned char)("
      << (d > 6 ? p + " ^ (" + p + " >> 3) ^ (" + p + " >> 6)" : d > 3 ? p + " ^ (" + p + " >> 3)" : p) << ");\n";
  };
  if (!M->groups.empty()) gen.range(0, (int64_t)M->groups.size());
  o << "}\n";
  return o.str();
}

// Largest interaction model for the specialised kernel (loads and adds of all
// its units); larger ones use the generic kernel.
const int64_t kMaxIvSpecOps = 400000;

}  // namespace

int jit_iv_source(wdf_model *M, std::string &src) {
  const int rc = make_plan(M);
  if (rc) return rc;
  src = gen_iv(M) + gen_patterns(M, index_tree_groups(M));
  return WDF_OK;
}

int jit_build_iv(wdf_model *M) {
  if (!M->jit) return set_error(WDF_E_UNSUPPORTED, "specialised interaction kernel: the model runs the generic kernels");
  if (!M->jit->iv.empty()) return WDF_OK;
  if (M->iv_units.empty() || iv_spec_ops(M) > kMaxIvSpecOps)
    return set_error(WDF_E_UNSUPPORTED, "specialised interaction kernel: %lld table loads and adds exceed %lld",
                     (long long)iv_spec_ops(M), (long long)kMaxIvSpecOps);
  // programs of kIvKernelsPerProgram kernels each, and the pattern kernel,
  // compiled in parallel; a kernel that spills registers at its shape is
  // generated again with fewer resident blocks (more registers per lane)
  const IvPartners P(M);
  const int nk = iv_kernel_count(M);
  std::vector<IvShape> shapes;
  for (int c = 0; c < nk; ++c) shapes.push_back(P.shape(c, M->n_features));
  const std::string pre = gen_iv_preamble();
  const std::string pat_src = std::string(kPreamble) + gen_patterns(M, index_tree_groups(M));
  std::vector<hipFunction_t> fns((size_t)nk, nullptr);
  std::vector<std::shared_ptr<JitPart>> parts;
  for (int attempt = 0;; ++attempt) {
    std::vector<std::pair<std::string, std::string>> progs;
    for (int c0 = 0; c0 < nk; c0 += kIvKernelsPerProgram) {
      std::string src = pre;
      for (int c = c0; c < std::min(nk, c0 + kIvKernelsPerProgram); ++c) src += gen_iv_kernel(M, P, c, shapes[(size_t)c]);
      progs.push_back({src, iv_kernel_name(c0)});
    }
    progs.push_back({pat_src, "wdf_patterns_spec"});
    int rc = jit_compile_all(M, progs);
    if (rc) return rc;
    parts.clear();
    for (const auto &pr : progs) parts.push_back(cached_part(M, pr.first));
    bool again = false;
    for (int c = 0; c < nk; ++c) {
      hipError_t e = hipModuleGetFunction(&fns[(size_t)c], parts[(size_t)(c / kIvKernelsPerProgram)]->mod,
                                          iv_kernel_name(c).c_str());
      if (e != hipSuccess) return hip_error(e, "hipModuleGetFunction(interaction)");
      const IvShape fewer = iv_shape_fewer(shapes[(size_t)c]);
      if (attempt < 2 && spill_bytes(fns[(size_t)c]) > 0 && fewer.blocks_per_cu < shapes[(size_t)c].blocks_per_cu) {
        shapes[(size_t)c] = fewer;
        again = true;
      }
    }
    if (!again) break;
  }
  JitModule &J = *M->jit;
  hipError_t e = hipEventCreateWithFlags(&J.iv_fork, hipEventDisableTiming);
  for (int k = 0; k < kIvSideStreams && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&J.iv_side[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&J.iv_join[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) return hip_error(e, "interaction streams");
  J.iv_parts = parts;
  J.iv = fns;
  J.patterns = parts.back()->fn;
  return WDF_OK;
}

int jit_explain_iv(const wdf_bg *bg, const float *X, int64_t ldx, uint8_t *pat, int64_t n, float *iv, int64_t ldiv,
                   hipStream_t s) {
  const wdf_model *M = bg->model;
  if (!M->jit || M->jit->iv.empty() || !M->jit->patterns)
    return set_error(WDF_E_INVALID_ARG, "specialised interaction kernel missing");
  if (n <= 0) return WDF_OK;
  if ((uintptr_t)pat % 16) return set_error(WDF_E_INVALID_ARG, "interaction workspace not 16-byte aligned");
  JitModule &J = *M->jit;
  std::lock_guard<std::mutex> lock(J.iv_mu);
  const JitPlan &P = M->jp;
  const float *thr = P.d_thr_pad.as<float>();
  const float *t2 = bg->d_xtab.as<float>();
  const size_t lds = (int64_t)P.thr_pad.size() <= kPatLdsThresholds ? P.thr_pad.size() * sizeof(float) : 0;
  const int64_t G = (int64_t)M->groups.size();
  const int F = M->n_features;
  // Rows in chunks of kIvChunkRows: the patterns of one chunk (G bytes per
  // row) are written, then read by every feature's kernel while they are
  // still in the device's last-level cache; the chunk's kernels are spread
  // over the caller's stream and the side streams so that together they fill
  // the device.  The next chunk's patterns (on the caller's stream) go to
  // another part of the workspace, so they may overlap the side streams'
  // kernels of this chunk.
  int rc = WDF_OK;
  for (int64_t r0 = 0; r0 < n && rc == WDF_OK; r0 += kIvChunkRows) {
    int64_t m = std::min<int64_t>(kIvChunkRows, n - r0), ldp = iv_pattern_stride(m);
    const float *Xc = X + r0;
    uint8_t *pc = pat + r0 * G;
    float *ivc = iv + r0;
    int live = 1;
    void *pargs[] = {(void *)&Xc, &ldx, (void *)&thr, &pc, &m, &ldp, &live};
    hipError_t e = hipModuleLaunchKernel(J.patterns, (unsigned)(ldp / 256), 1, 1, 256, 1, 1, (unsigned)lds, s, pargs,
                                         nullptr);
    if (e == hipSuccess) e = hipEventRecord(J.iv_fork, s);
    for (int k = 0; k < kIvSideStreams && e == hipSuccess; ++k) e = hipStreamWaitEvent(J.iv_side[k], J.iv_fork, 0);
    void *args[] = {(void *)&pc, &m, (void *)&t2, &ivc, &ldiv, &live};
    const unsigned blocks = (unsigned)((m + kIvRows - 1) / kIvRows);
    for (int c = 0; c < (int)J.iv.size() && e == hipSuccess; ++c) {
      const unsigned fc = (unsigned)std::min(kIvPerKernel, F - c * kIvPerKernel);
      hipStream_t sc = c % (kIvSideStreams + 1) == 0 ? s : J.iv_side[c % (kIvSideStreams + 1) - 1];
      e = hipModuleLaunchKernel(J.iv[(size_t)c], blocks, fc, 1, kIvRows, 1, 1, 0, sc, args, nullptr);
    }
    if (e != hipSuccess) rc = hip_error(e, "interaction launches");
  }
  // the caller's stream waits for the side streams' work (also after an error)
  for (int k = 0; k < kIvSideStreams; ++k) {
    hipError_t e = hipEventRecord(J.iv_join[k], J.iv_side[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, J.iv_join[k], 0);
    if (e != hipSuccess && rc == WDF_OK) rc = hip_error(e, "interaction stream join");
  }
  return rc;
}

HistLaunch hist_launch(const wdf_model *M, int64_t m) {
  // one block per CU at a time (the LDS histogram); a whole number of rounds
  // over the CUs, split evenly between the chunks.  Wave w of a block counts
  // the block's tiles w, w + waves, w + 2 waves, ...
  const JitPlan &P = M->jp;
  HistLaunch L;
  L.chunks = (int64_t)P.hist_chunks.size();
  L.threads = P.nt_hist;
  L.ntiles = (m + 63) / 64;
  const int64_t waves = P.nt_hist / 64;
  int64_t blocks = std::max<int64_t>(1, (int64_t)P.hist_rounds * M->ctx->n_cu / L.chunks);
  blocks = std::min<int64_t>(blocks, (L.ntiles + waves - 1) / waves);
  L.tiles_per_block = (L.ntiles + blocks - 1) / blocks;
  L.blocks = (L.ntiles + L.tiles_per_block - 1) / L.tiles_per_block;
  return L;
}

int jit_hist(wdf_model *M, const float *B, int64_t m, int64_t ldb, uint32_t *hist, uint32_t *codes, hipStream_t s) {
  const JitPlan &P = M->jp;
  hipError_t e = launch_quantize(B, m, ldb, M->n_features, P.d_thr_pad.as<float>(), P.d_pad_meta.as<int2>(), P.wide,
                                 P.words, codes, m, s);
  if (e != hipSuccess) return hip_error(e, "quantize");
  const HistLaunch L = hist_launch(M, m);
  const int chunks = (int)L.chunks;
  int64_t blocks = L.blocks, tiles_per_block = L.tiles_per_block;
  const uint32_t *cp = codes;
  const uint32_t *perm = P.d_perm.as<uint32_t>();
  int64_t ldc = m;
  int live = 1;
  void *args[] = {(void *)&cp, &ldc, &m, &tiles_per_block, &hist, (void *)&perm, &live};
  e = hipModuleLaunchKernel(M->jit->hist, (unsigned)blocks, (unsigned)chunks, 1, (unsigned)P.nt_hist, 1, 1, 0, s, args,
                            nullptr);
  if (e != hipSuccess) return hip_error(e, "hipModuleLaunchKernel(hist)");
  return WDF_OK;
}

int jit_explain(const wdf_bg *bg, const float *X, int64_t n, int64_t ldx, float *phi, int64_t ldphi, hipStream_t s) {
  const wdf_model *M = bg->model;
  const JitPlan &P = M->jp;
  const float *tab = bg->d_xtab.as<float>();
  const float *thr = P.d_thr_pad.as<float>();
  int live = 1;
  void *args[] = {(void *)&X, &ldx, (void *)&tab, (void *)&thr, &phi, &ldphi, &n, &live};
  const unsigned blocks = (unsigned)((n + P.nt_explain - 1) / P.nt_explain);
  hipError_t e = hipModuleLaunchKernel(M->jit->explain, blocks, 1, 1, (unsigned)P.nt_explain, 1, 1, 0, s, args, nullptr);
  if (e != hipSuccess) return hip_error(e, "hipModuleLaunchKernel(explain)");
  return WDF_OK;
}

}  // namespace wdf
