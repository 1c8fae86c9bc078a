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
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2511_09376_amd import synth  # noqa: E402

METRIC = "Background-SHAP rows/s (100 trees d6, 127 feat) + served p50/p99 latency"
VALU_PEAK_OPS = 256 * 64 * 2.4e9   # 32-bit lane operations per second (non-packed)
HBM_PEAK = 8.0e12                  # bytes per second
MFMA_F64_PEAK = 78.6e12            # dense FP64 matrix flops per second
# The paper's own run of this method at this shape (Section 10, KDD-Cup-99):
# 2,984,154 consumers x 4,898,431 background rows x 127 features, XGBoost
# regressor with 100 trees of depth 6, on Colab hardware.
PAPER_CONTEXT = {"cpu_s": 162.0, "gpu_s": 16.0, "cpu": "Colab CPU runtime", "gpu": "A100 (Colab), CuPy",
                 "consumers": 2984154, "background": 4898431, "features": 127, "trees": 100, "depth": 6,
                 "cpu_rows_per_s": 2984154 / 162.0, "gpu_rows_per_s": 2984154 / 16.0}

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


def measured_iv_traffic(wdf, ens, workload):
    """HBM bytes per step of the interaction kernels (pattern and interaction
    launches) from the committed counter summary, while the generated source
    is the one the counters were taken on; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"iv_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    import hashlib
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    sha = hashlib.sha1(wdf.iv_source(ens).encode()).hexdigest()
    if fields.get("source_sha1") != sha or "traffic_bytes_per_step" not in fields:
        return None
    return int(fields["traffic_bytes_per_step"])


def cpu_model_name() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads() -> int:
    """Threads for the CPU oracle: the CPUs this process may run on, at most
    16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(ens, X, B, rows, threads, kind):
    """The FP64 oracle (depth-first walk form), unchanged, on `rows` (seeded
    consumer rows) against the full background, on `threads` host threads; no
    scaling: the rate is rows over the measured wall time.  Returns the
    baseline record and the oracle's phi of those rows."""
    import oracle
    om = oracle.Model(ens)
    Xs = np.ascontiguousarray(X[:, rows])
    m = B.shape[1]
    t0 = time.perf_counter()
    ref = oracle.bg_walk(om, Xs, B, kind=kind, threads=threads)
    dt = time.perf_counter() - t0
    rec = {"value": len(rows) / dt, "unit": "rows/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(rows)} seeded consumer rows x all {m} background rows, {threads} threads, "
                     f"{dt:.1f} s wall (no scaling)",
           "seconds": dt, "rows": len(rows), "nproc": os.cpu_count(), "cpu_model": cpu_model_name()}
    return rec, ref


def run_error(got, ref, rows):
    """phi of the timed run on the oracle's rows: the maximum absolute error
    and the row-scaled error (per row, max_i |phi - ref| over max_i |ref|)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    diff = np.abs(got - ref)
    scale = np.maximum(np.abs(ref).max(axis=0), 1e-30)
    row_scaled = float((diff.max(axis=0) / scale).max())
    return {"max_abs": float(diff.max()), "row_scaled": row_scaled, "rows": int(len(rows)),
            "tolerance": 1e-5, "within_tolerance": bool(row_scaled <= 1e-5),
            "against": "FP64 oracle walk with the full background"}


def pcie_rates(F, rows=1 << 18, reps=5):
    """Pinned host <-> device copy rates (GB/s) of a [F][rows] float32 block,
    each direction alone and both at once on two streams, and what they allow
    a server that copies every row in (4 F bytes) and out (4 F bytes)."""
    import torch
    n = F * rows
    h_in = torch.empty(n, dtype=torch.float32, pin_memory=True)
    h_out = torch.empty(n, dtype=torch.float32, pin_memory=True)
    d_in = torch.empty(n, dtype=torch.float32, device="cuda")
    d_out = torch.zeros(n, dtype=torch.float32, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def both():
        with torch.cuda.stream(s1):
            d_in.copy_(h_in, non_blocking=True)
        with torch.cuda.stream(s2):
            h_out.copy_(d_out, non_blocking=True)

    bytes_ = 4 * n
    h2d = bytes_ / timed(lambda: d_in.copy_(h_in, non_blocking=True)) / 1e9
    d2h = bytes_ / timed(lambda: h_out.copy_(d_out, non_blocking=True)) / 1e9
    duplex = 2 * bytes_ / timed(both) / 1e9
    return {"h2d_gbs": h2d, "d2h_gbs": d2h, "both_directions_gbs": duplex,
            "rows_per_s_ceiling": duplex * 1e9 / (2 * 4 * F),
            "note": f"pinned copies of {bytes_ >> 20} MiB; a served row moves 4 F bytes in and 4 F bytes out"}


def serve_bench(wdf, ctx, loads=(0.5, 0.8), n_requests=10_000, max_rows=4096, batch_rows=1 << 16, copy_threads=8):
    """Serving: the 100-tree depth-6 model and a 100k-row background resident on
    the device; requests of log-uniform size in [1, 4096] rows arrive as a
    Poisson process at a fixed fraction of the server's saturated throughput.
    Continuous batching (batches of up to batch_rows rows in up to four slots,
    packed and unpacked by copy threads) is compared with the plain form, one
    request per launch, at the same offered load.  Latency is submit -> phi on
    the host."""
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
    budget = 4 * (4 * F * batch_rows * 4)

    def run(one_per_launch, rate_rows):
        srv = wdf.Server(bg, budget, max_rows, queue_cap=n_requests, one_per_launch=one_per_launch,
                         batch_rows=batch_rows, copy_threads=copy_threads)
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
        t_sub = time.perf_counter() - t0
        for t in tickets:
            srv.wait(t)
        dt = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return {"rows_per_s": float(sizes.sum()) / dt, "requests": int(st.completed), "batches": int(st.batches),
                "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms, "max_ms": st.max_ms,
                "wall_ms": dt * 1e3, "submit_ms": t_sub * 1e3, "slots": int(st.slots),
                "batch_rows": int(st.batch_rows), "device_busy_ms": st.busy_ms, "copy_in_ms": st.copy_in_ms,
                "explain_ms": st.explain_ms, "copy_out_ms": st.copy_out_ms, "pack_ms": st.pack_ms,
                "unpack_ms": st.unpack_ms}

    run(False, 0)                                  # warm-up
    cap = run(False, 0)                            # saturated throughput
    out = {"workload": "100 complete depth-6 trees, 127 features, 100k background rows resident; "
                       f"{n_requests} Poisson requests, sizes log-uniform in [1, {max_rows}] (mean {sizes.mean():.0f} rows)",
           "saturated_rows_per_s": cap["rows_per_s"], "saturated": cap, "copy_threads": copy_threads,
           "pcie": pcie_rates(F), "loads": []}
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
    ap.add_argument("--cpu-rows", type=int, default=16,
                    help="seeded consumer rows the CPU oracle explains against the full background (also the rows "
                         "on which the timed phi is checked)")
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
        # (the counters were taken with the default chunk of rows per launch)
        traffic = measured_iv_traffic(wdf, ens, args.workload) if bg.specialised and args.iv_chunk == 1 << 18 else None
        roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK, "traffic": traffic,
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
    rows_check = np.sort(np.random.default_rng(2511).choice(n, min(n, args.cpu_rows), replace=False))
    phi_rows = phi[:, torch.from_numpy(rows_check).cuda()].cpu().numpy() if not iv else None
    hbm = None
    mfma = None
    if not iv:
        alg = 2 * 4 * ens.n_features * n          # X read and phi written, once each
        hbm = {"kernel": roofline["kernel"], "algorithmic_bytes": alg, "algorithmic_gbs": alg / (explain_ms * 1e6),
               "measured_bytes": roofline["traffic"],
               "measured_gbs": (roofline["traffic"] / (explain_ms * 1e6)) if roofline["traffic"] else None,
               "peak_gbs": HBM_PEAK / 1e9}
        hbm["measured_frac"] = hbm["measured_gbs"] / hbm["peak_gbs"] if hbm["measured_gbs"] else None
        if not args.pathdep:
            c_ms, c_flops = bg.time_contraction(20, stream)
            mfma = {"kernel": "k_gemm_f64 (v_mfma_f64_16x16x4f64)", "ms_per_contraction": c_ms, "flops": c_flops,
                    "tflops": c_flops / (c_ms * 1e9), "peak_tflops": MFMA_F64_PEAK / 1e12,
                    "util": c_flops / (c_ms * 1e-3) / MFMA_F64_PEAK}
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
           "background_ms": ms_step - explain_ms, "hbm": hbm, "mfma": mfma,
           "paper_context": dict(PAPER_CONTEXT, this_run_s_per_3m_rows=3e6 / value)}
    if summary_once_ms is not None:
        out["pathdep_summary_once_ms"] = summary_once_ms
    if not args.no_serve:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = serve_bench(wdf, ctx)
        sv = out["serving"]["loads"][0]["continuous_batching"]
        out["served_p50_ms"], out["served_p99_ms"] = sv["p50_ms"], sv["p99_ms"]
    if not args.no_cpu_baseline and not args.pathdep and not iv:
        threads = host_threads()
        print(f"[bench] CPU oracle: {rows_check.size} rows x {B.shape[1]} background rows on {threads} threads",
              file=sys.stderr, flush=True)
        kind = 0 if args.values == "shapley" else 1
        out["cpu_baseline"], ref = cpu_baseline(ens, X, B, rows_check, threads, kind)
        out["error"] = run_error(phi_rows, ref, rows_check)
        print(f"[bench] oracle done in {out['cpu_baseline']['seconds']:.1f} s; row-scaled error "
              f"{out['error']['row_scaled']:.3e}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
