"""Benchmark: Background SHAP on one MI355X.

One step is one pass of the whole path over one batch: summarise the
background (threshold ranks, exact histograms, MFMA contraction, tables, base
value) and explain every consumer row (patterns, gather-sum into phi).  The
summary's storage is allocated before timing; each step recomputes it in place
and explains, replaying two recorded HIP graphs (summary, explain) unless
--eager.  Inputs are synthetic, seeded and resident in HBM before timing
starts.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload paper|mid|uneven|small]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2511_09376_amd import synth  # noqa: E402

METRIC = "Background-SHAP rows/s (100 trees d6, 127 feat) + served p50/p99 latency"
VALU_PEAK_OPS = 256 * 64 * 2.4e9   # 32-bit lane operations per second (non-packed)
HBM_PEAK = 8.0e12                  # bytes per second

DESCRIPTIONS = {
    "paper": "paper-scale shape: 100 complete depth-6 trees, 127 features (normal/log-normal/binary/count mix, 5% NaN), 3M consumer rows x 5M background rows",
    "mid": "100 complete depth-6 trees, 127 features (mix, 5% NaN), 100k consumers x 100k background",
    "uneven": "500 pruned trees of depth 3..8, 127 features (mix, 5% NaN), 1M consumers x 1M background",
    "small": "10 complete depth-4 trees, 8 N(0,1) features, 100 x 100 rows",
}


def method_ops_per_row(ens) -> int:  # noqa: C901
    """Algorithmic operations to explain one row: per tree, one compare and two
    pattern updates per inner node plus one gather-add per (leaf group, path
    position); 381 per complete depth-6 tree."""
    total = 0
    for t in range(ens.n_trees):
        sl = ens.tree_slice(t)
        f, l, r = ens.feature[sl], ens.left[sl], ens.right[sl]
        inner = np.nonzero(f >= 0)[0]
        total += 3 * inner.size
        depth = np.zeros(f.size, np.int64)
        for i in range(f.size):          # nodes are in BFS order: parents precede children
            if f[i] >= 0:
                depth[l[i]] = depth[i] + 1
                depth[r[i]] = depth[i] + 1
        for i in inner:
            ll, rl = f[l[i]] < 0, f[r[i]] < 0
            if ll and rl:
                total += int(depth[i]) + 1
            else:
                total += (int(depth[i]) + 1) * (int(ll) + int(rl))
    return int(total)


def measured_traffic(wdf, ens, workload, gather):
    """HBM bytes per explain launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), reported
    only while the generated explain-kernel source is the one the counters
    were taken on; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"explain_{gather}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    import hashlib
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    flags = wdf.KERNEL_SPECIALISED | (wdf.KERNEL_PAIRS if gather == "pairs" else 0)
    src = wdf.specialised_source(ens, kernel=flags)
    sha = hashlib.sha1(src[src.index("#define EXPLAIN_NAME"):].encode()).hexdigest()
    if fields.get("source_sha1") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_baseline(ens, X_rows, B, seconds_hint=20.0):
    """The FP64 oracle (depth-first walk form), unchanged, on a bounded sample:
    one consumer row per host core against a prefix of the background sized to
    take about `seconds_hint` seconds.  The oracle's work is linear in the
    background size, so the measured rate is scaled to the full background."""
    import oracle
    cores = max(1, min(16, os.cpu_count() or 1))
    om = oracle.Model(ens)
    m = B.shape[1]
    probe_m = min(m, 20_000)
    t0 = time.perf_counter()
    oracle.bg_walk(om, np.ascontiguousarray(X_rows[:, :1]), np.ascontiguousarray(B[:, :probe_m]), threads=1)
    per_bg_row = (time.perf_counter() - t0) / probe_m
    m_s = int(max(1, min(m, seconds_hint / max(per_bg_row, 1e-12))))
    rows = min(cores, X_rows.shape[1])
    Xs = np.ascontiguousarray(X_rows[:, :rows])
    Bs = np.ascontiguousarray(B[:, :m_s])
    t0 = time.perf_counter()
    oracle.bg_walk(om, Xs, Bs, threads=rows)
    dt = time.perf_counter() - t0
    return {"value": rows / dt * (m_s / m), "unit": "rows/s", "cores": rows, "kind": "oracle",
            "sample": f"{rows} consumer rows (one per thread) x the first {m_s} of {m} background rows in {dt:.1f} s; "
                      f"rate scaled by {m_s}/{m} to the full background (the oracle's work is linear in it)"}


def serve_bench(wdf, ctx, loads=(0.5, 0.8), n_requests=10_000, max_rows=4096):
    """Serving: the 100-tree depth-6 model and a 100k-row background resident on
    the device; requests of log-uniform size in [1, 4096] rows arrive as a
    Poisson process at a fixed fraction of the server's saturated throughput.
    Continuous batching is compared with one request per launch at the same
    offered load.  Latency is submit -> phi on the host."""
    import torch
    w = synth.WORKLOADS["serve"]
    ens = w.ensemble()
    B = w.background()
    model = wdf.Model(ctx, ens)
    bg = wdf.Background(model, torch.from_numpy(B).cuda())
    s_sizes, s_arrival = w.seeds()[3].spawn(2)
    sizes = synth.request_sizes(n_requests, s_sizes, max_rows)
    pool = w.consumers(max_rows * 4)          # request rows are drawn from this pool
    starts = np.random.default_rng(s_arrival).integers(0, pool.shape[1] - max_rows, n_requests)
    reqs = [np.ascontiguousarray(pool[:, s:s + n]) for s, n in zip(starts, sizes)]
    outs = [np.empty_like(x) for x in reqs]
    F = model.n_features
    budget = 4 * (4 * F * max_rows * 4)

    def run(one_per_launch, rate_rows):
        srv = wdf.Server(bg, budget, max_rows, queue_cap=n_requests, one_per_launch=one_per_launch)
        gaps = np.random.default_rng(7).exponential(1.0, n_requests) if rate_rows else np.zeros(n_requests)
        mean_size = float(sizes.mean())
        if rate_rows:
            gaps *= mean_size / rate_rows
        t_arr = np.cumsum(gaps)
        tickets = []
        t0 = time.perf_counter()
        for i in range(n_requests):
            target = t0 + t_arr[i]
            while time.perf_counter() < target:
                pass
            tickets.append(srv.submit(reqs[i], outs[i]))
        for t in tickets:
            srv.wait(t)
        dt = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return {"rows_per_s": float(sizes.sum()) / dt, "requests": int(st.completed), "batches": int(st.batches),
                "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms, "max_ms": st.max_ms}

    run(False, 0)                                  # warm-up
    cap = run(False, 0)                            # saturated throughput
    out = {"workload": "100 complete depth-6 trees, 127 features, 100k background rows resident; "
                       f"{n_requests} Poisson requests, sizes log-uniform in [1, {max_rows}] (mean {sizes.mean():.0f} rows)",
           "saturated_rows_per_s": cap["rows_per_s"], "loads": []}
    for load in loads:
        rate = load * cap["rows_per_s"]
        out["loads"].append({"offered_fraction": load, "offered_rows_per_s": rate,
                             "continuous_batching": run(False, rate), "one_request_per_launch": run(True, rate)})
    bg.close()
    model.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper", choices=list(DESCRIPTIONS))
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic", "specialised", "pairs"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--values", default="shapley", choices=["shapley", "banzhaf", "shapley_iv", "banzhaf_iv"],
                    help="value kind: Shapley (default) or Banzhaf values of the same game, or their interaction "
                         "values (phi[F][F] per row, explained in consumer chunks)")
    ap.add_argument("--iv-chunk", type=int, default=1 << 18, help="consumer rows per interaction-value launch")
    ap.add_argument("--pathdep", action="store_true",
                    help="path-dependent values from node covers (no background: the summary depends on the model "
                         "only, so a step is one explain)")
    ap.add_argument("--eager", action="store_true", help="launch the step's kernels directly instead of replaying HIP graphs")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (rows shard across GPUs "
              "with no exchange, so the multi-GPU rate is the per-GPU rate times the GPU count)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_09376_amd import wdf

    if args.copy_probe:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}))
        return

    w = synth.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    ens = w.ensemble()
    X = w.consumers()
    B = w.background()
    print(f"[bench] generated {args.workload}: {ens.n_trees} trees, X {X.shape}, B {B.shape} "
          f"in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    kernel = {"auto": wdf.KERNEL_AUTO, "generic": wdf.KERNEL_GENERIC, "specialised": wdf.KERNEL_SPECIALISED,
              "pairs": wdf.KERNEL_AUTO | wdf.KERNEL_PAIRS}[args.kernel]
    ctx = wdf.Context(0)
    t0 = time.perf_counter()
    model = wdf.Model(ctx, ens, kernel)
    print(f"[bench] model loaded (specialised={model.specialised}) in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    Xd = torch.from_numpy(X).cuda()
    Bd = torch.from_numpy(B).cuda()
    phi = torch.empty_like(Xd)
    n = X.shape[1]
    stream = torch.cuda.current_stream()
    tuning = None
    if model.specialised and not args.no_autotune and not args.values.endswith("_iv"):
        t0 = time.perf_counter()
        tuning = model.autotune(Bd, Xd)        # on the workload itself: the choice transfers exactly
        print(f"[bench] autotuned in {time.perf_counter() - t0:.1f} s: {tuning}", file=sys.stderr, flush=True)
    # the summary's storage is allocated once; a step then recomputes it in
    # place from the (resident) background and explains every consumer row.
    # A path-dependent summary depends on the model only: it is built once and
    # a step is one explain.
    values = {"shapley": wdf.SHAPLEY, "banzhaf": wdf.BANZHAF, "shapley_iv": wdf.SHAPLEY_IV,
              "banzhaf_iv": wdf.BANZHAF_IV}[args.values]
    iv = values in (wdf.SHAPLEY_IV, wdf.BANZHAF_IV)
    summary_once_ms = None
    if args.pathdep:
        t0 = time.perf_counter()
        bg = wdf.Background(model, values=values, pathdep=True)
        torch.cuda.synchronize()
        summary_once_ms = (time.perf_counter() - t0) * 1e3
    else:
        bg = wdf.Background(model, Bd, values=values)
    if iv:
        # phi[F][F] per row: consumer chunks into one reused output buffer
        F = ens.n_features
        chunk = min(n, args.iv_chunk)
        out_iv = torch.empty((F, F, chunk), dtype=torch.float32, device="cuda")
        ws_iv = torch.empty(bg.iv_workspace_bytes(chunk), dtype=torch.uint8, device="cuda")
        g_bg = wdf.Graph(bg, B=Bd)

        def summarise():
            g_bg.launch(stream)

        def explain():
            for a in range(0, n, chunk):
                b = min(n, a + chunk)
                bg.explain_iv(Xd[:, a:b], out=out_iv[:, :, :b - a], stream=stream, workspace=ws_iv)
    elif args.eager:
        def summarise():
            if not args.pathdep:
                bg.refresh(Bd, stream=stream)

        def explain():
            bg.explain(Xd, out=phi, stream=stream)
    else:
        g_bg = None if args.pathdep else wdf.Graph(bg, B=Bd)  # ranks, histograms, contraction, tables
        g_ex = wdf.Graph(bg, Xd, phi)                          # one explain launch over all trees

        def summarise():
            if g_bg is not None:
                g_bg.launch(stream)

        def explain():
            g_ex.launch(stream)

    def step(ev=None):
        summarise()
        if ev is not None:
            ev[0].record(stream)
        explain()
        if ev is not None:
            ev[1].record(stream)
        return bg

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        bg = step(events[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    explain_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    value = n * args.steps / dt

    if iv:
        # the interaction launches write F * F floats per row: HBM-bound by that output
        out_bytes = 4.0 * ens.n_features ** 2 * n
        achieved = out_bytes / (explain_ms * 1e-3)
        roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK, "traffic": None,
                    "kernel": ("wdf_patterns_spec + wdf_iv_spec_*" if bg.specialised else "k_patterns_u8 + k_explain_iv"),
                    "kernel_ms": explain_ms, "bytes_per_row": 4 * ens.n_features ** 2}
    else:
        ops_row = int(method_ops_per_row(ens))
        achieved = ops_row * n / (explain_ms * 1e-3)
        gather = tuning["gather"] if tuning else ("quads" if model.specialised else None)
        traffic = measured_traffic(wdf, ens, args.workload, gather) if gather else None
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                    "frac": achieved / VALU_PEAK_OPS, "traffic": traffic,
                    "kernel": f"wdf_explain_{gather}" if gather else "k_explain_generic", "kernel_ms": explain_ms,
                    "ops_per_row": ops_row}
    base = bg.base_value
    out = {"metric": METRIC, "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": DESCRIPTIONS[args.workload], "n_consumers": int(n), "n_background": int(B.shape[1]),
                      "n_trees": ens.n_trees, "n_features": ens.n_features,
                      "kernel": "specialised" if model.specialised else "generic",
                      "launch": "eager" if args.eager else "hip_graph",
                      "values": args.values, "background": "path-dependent (covers)" if args.pathdep else "rows"},
           "roofline": roofline, "base_value": base, "tuning": tuning,
           "explain_rows_per_s": n / (explain_ms * 1e-3),
           "background_ms": ms_step - explain_ms}
    if summary_once_ms is not None:
        out["pathdep_summary_once_ms"] = summary_once_ms
    if not args.no_serve:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = serve_bench(wdf, ctx)
        sv = out["serving"]["loads"][0]["continuous_batching"]
        out["served_p50_ms"], out["served_p99_ms"] = sv["p50_ms"], sv["p99_ms"]
    if not args.no_cpu_baseline and not args.pathdep and args.values == "shapley":  # the headline method only
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ens, X[:, :64], B, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
