// Autotuner of the model-specialised kernels: every candidate configuration
// is run on the caller's data and timed with HIP events; the fastest is kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "wdf.h"
#include "wdf_dev.h"
#include "wdf_impl.h"
#include "wdf_internal.h"

using namespace wdf;

namespace {

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// average duration of `reps` runs of f after one warm-up run; -1 on error
template <class Fn>
float time_runs(hipStream_t s, int reps, Fn f, int &rc) {
  Events ev;
  if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess) {
    rc = set_error(WDF_E_DEVICE, "autotune: hipEventCreate failed");
    return -1.f;
  }
  if ((rc = f())) return -1.f;
  if (hipEventRecord(ev.a, s) != hipSuccess) return rc = set_error(WDF_E_DEVICE, "autotune: event"), -1.f;
  for (int r = 0; r < reps; ++r)
    if ((rc = f())) return -1.f;
  if (hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess)
    return rc = set_error(WDF_E_DEVICE, "autotune: event"), -1.f;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ev.a, ev.b);
  return ms / (float)reps;
}

}  // namespace

extern "C" int wdf_model_autotune(wdf_model *M, const float *B, int64_t m, int64_t ldb, const float *X, int64_t n,
                                  int64_t ldx, void *hip_stream, wdf_tuning *out) {
  if (!M || !B || !X || !out) return set_error(WDF_E_INVALID_ARG, "wdf_model_autotune: NULL argument");
  if (m < 1 || ldb < m || n < 1 || ldx < n) return set_error(WDF_E_INVALID_ARG, "wdf_model_autotune: bad sizes");
  if (!M->jit) return set_error(WDF_E_UNSUPPORTED, "wdf_model_autotune: the model runs the generic kernels");
  if (M->n_bg.load() != 0)
    return set_error(WDF_E_INVALID_ARG, "wdf_model_autotune: %d background summaries of this model exist",
                     M->n_bg.load());
  HIP_TRY(hipSetDevice(M->ctx->device));
  hipStream_t s = (hipStream_t)hip_stream;
  *out = wdf_tuning{};
  for (float &t : out->explain_ms) t = -1.f;
  for (float &t : out->explain_rows_ms) t = -1.f;
  for (auto &row : out->hist_ms)
    for (float &t : row) t = -1.f;
  const int reps = 3;
  int rc = WDF_OK;

  // histogram grid and block size: launch-time choices, timed on one
  // histogram buffer
  {
    DevBuf hist, codes;
    if ((rc = hist.alloc((size_t)std::max<int64_t>(M->hist_size, 1) * sizeof(uint32_t)))) return rc;
    if ((rc = codes.alloc((size_t)M->jp.words * (size_t)m * sizeof(uint32_t)))) return rc;
    const int keep_r = M->jp.hist_rounds, keep_t = M->jp.nt_hist;
    int best_r = keep_r, best_t = keep_t;
    float best_ms = -1.f;
    const int threads[3] = {512, 768, 1024};
    static_assert(kHistMaxThreads == 1024, "the sweep covers blocks up to the largest launch bound");
    for (int ti = 0; ti < 3; ++ti) {
      if (threads[ti] > M->jp.hist_bound) continue;  // beyond the compiled launch bound
      for (int r : {1, 2, 3, 4, 6, 8}) {
        M->jp.nt_hist = threads[ti];
        M->jp.hist_rounds = r;
        const float ms = time_runs(s, reps, [&] {
          HIP_TRY(launch_fill_u32(hist.as<uint32_t>(), std::max<int64_t>(M->hist_size, 1), 0u, s));
          return jit_hist(M, B, m, ldb, hist.as<uint32_t>(), codes.as<uint32_t>(), s);
        }, rc);
        if (rc) {
          M->jp.hist_rounds = keep_r;
          M->jp.nt_hist = keep_t;
          return rc;
        }
        out->hist_ms[ti][r] = ms;
        if (best_ms < 0.f || ms < best_ms) best_ms = ms, best_r = r, best_t = threads[ti];
      }
    }
    M->jp.hist_rounds = best_r;
    M->jp.nt_hist = best_t;
    out->hist_rounds = best_r;
    out->hist_threads = best_t;
  }

  // explain gather and tile: compile-time choices.  Candidate gathers: pair
  // tables only, quads for the sibling pairs of depth <= 6 (when deeper pairs
  // exist: their quad tables are 4 to 16 times larger), and quads for all;
  // their programs are compiled in parallel, then each gets a summary of B
  // and is timed.
  DevBuf phi;
  if ((rc = phi.alloc((size_t)M->n_features * (size_t)n * sizeof(float)))) return rc;
  const int keep_q = M->jp.quad_depth, keep_bpc = M->jp.explain_bpc;
  int max_pair = 0;
  for (const Group &g : M->groups)
    if (g.col_r >= 0) max_pair = std::max(max_pair, g.depth);
  std::vector<int> qs{0};
  if (max_pair > 6) qs.push_back(6);
  if (max_pair >= 2) qs.push_back(WDF_MAX_DEPTH);
  auto restore = [&] {  // back to the plan the model had (its programs are cached)
    M->jp.quad_depth = keep_q;
    M->jp.explain_bpc = keep_bpc;
    (void)jit_build(M);
  };
  auto time_explain = [&](float &ms) {
    if ((rc = jit_build(M))) return;
    wdf_bg *bg = nullptr;
    if ((rc = wdf_background_load(M, B, m, ldb, 1, WDF_SHAPLEY, s, &bg))) return;
    ms = time_runs(s, reps, [&] { return wdf_explain(bg, X, n, ldx, phi.as<float>(), n, s); }, rc);
    wdf_bg_destroy(bg);
  };
  {
    std::vector<std::pair<std::string, std::string>> progs;
    for (int q : qs) {
      M->jp.quad_depth = q;
      M->jp.explain_bpc = 1;
      std::string src;
      if ((rc = jit_explain_source(M, src))) break;
      progs.push_back({src, jit_explain_name(M)});
    }
    if (!rc) rc = jit_compile_all(M, progs);
    if (rc) {
      restore();
      return rc;
    }
  }
  int best_q = 0;
  for (int q : qs) {
    M->jp.quad_depth = q;
    M->jp.explain_bpc = 1;
    time_explain(out->explain_ms[q]);
    if (rc) {
      restore();
      return rc;
    }
    if (out->explain_ms[q] < out->explain_ms[best_q]) best_q = q;
  }
  // the tile: one 512-row block per CU with all of the LDS, or two 256-row
  // blocks per CU with half of it each
  out->explain_rows_ms[0] = out->explain_ms[best_q];
  M->jp.quad_depth = best_q;
  M->jp.explain_bpc = 2;
  time_explain(out->explain_rows_ms[1]);
  if (rc) {
    restore();
    return rc;
  }
  M->jp.explain_bpc = out->explain_rows_ms[1] < out->explain_rows_ms[0] ? 2 : 1;
  out->quads = best_q;
  out->explain_rows = 512 / M->jp.explain_bpc;
  if ((rc = jit_build(M))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return WDF_OK;
}

extern "C" int wdf_model_set_tuning(wdf_model *M, const wdf_tuning *t) {
  if (!M || !t) return set_error(WDF_E_INVALID_ARG, "wdf_model_set_tuning: NULL argument");
  if (!M->jit) return set_error(WDF_E_UNSUPPORTED, "wdf_model_set_tuning: the model runs the generic kernels");
  if (M->n_bg.load() != 0)
    return set_error(WDF_E_INVALID_ARG, "wdf_model_set_tuning: %d background summaries of this model exist",
                     M->n_bg.load());
  if (t->quads < -1 || t->quads > WDF_MAX_DEPTH)
    return set_error(WDF_E_INVALID_ARG, "wdf_model_set_tuning: quads must be -1 .. %d", WDF_MAX_DEPTH);
  if (t->explain_rows != 0 && t->explain_rows != 512 && t->explain_rows != 256)
    return set_error(WDF_E_INVALID_ARG, "wdf_model_set_tuning: explain_rows must be 0, 256 or 512");
  if (t->hist_threads < 64 || t->hist_threads % 64 || t->hist_threads > M->jp.hist_bound)
    return set_error(WDF_E_INVALID_ARG,
                     "wdf_model_set_tuning: hist_threads %d is not a multiple of 64 in [64, %d] (the compiled bound)",
                     t->hist_threads, M->jp.hist_bound);
  if (t->hist_rounds < 1 || t->hist_rounds > 64)
    return set_error(WDF_E_INVALID_ARG, "wdf_model_set_tuning: hist_rounds %d outside [1, 64]", t->hist_rounds);
  HIP_TRY(hipSetDevice(M->ctx->device));
  const int q = t->quads >= 0 ? t->quads : M->jp.quad_depth;
  const int bpc = t->explain_rows ? 512 / t->explain_rows : M->jp.explain_bpc;
  if (q != M->jp.quad_depth || bpc != M->jp.explain_bpc) {
    const int keep_q = M->jp.quad_depth, keep_bpc = M->jp.explain_bpc;
    M->jp.quad_depth = q;
    M->jp.explain_bpc = bpc;
    int rc = jit_build(M);
    if (rc) {
      M->jp.quad_depth = keep_q;
      M->jp.explain_bpc = keep_bpc;
      (void)jit_build(M);  // the previous programs are cached
      return rc;
    }
  }
  // a rebuild re-plans the model; the launch-time choices are set after it
  M->jp.nt_hist = t->hist_threads;
  M->jp.hist_rounds = t->hist_rounds;
  return WDF_OK;
}

extern "C" int64_t wdf_debug_hist_launch(const wdf_model *M, int64_t m, int64_t *launch, int64_t *chunk_group,
                                         int64_t cap) {
  if (!M || !launch || m < 1) return set_error(WDF_E_INVALID_ARG, "wdf_debug_hist_launch: NULL argument or m < 1");
  if (!M->jit) return set_error(WDF_E_UNSUPPORTED, "wdf_debug_hist_launch: the model runs the generic kernels");
  const HistLaunch L = hist_launch(M, m);
  const int64_t waves = L.threads / 64;
  launch[0] = L.blocks;
  launch[1] = L.chunks;
  launch[2] = L.threads;
  launch[3] = L.tiles_per_block;
  launch[4] = L.ntiles;
  launch[5] = (L.tiles_per_block + waves - 1) / waves;  // tiles of the busiest wave
  if (chunk_group) {
    if (cap < L.chunks + 1)
      return set_error(WDF_E_INVALID_ARG, "wdf_debug_hist_launch: capacity %lld < %lld", (long long)cap,
                       (long long)(L.chunks + 1));
    for (int64_t c = 0; c < L.chunks; ++c) chunk_group[c] = M->jp.hist_chunks[(size_t)c].first;
    chunk_group[L.chunks] = L.chunks ? M->jp.hist_chunks[(size_t)L.chunks - 1].second : 0;
  }
  return L.chunks;
}
