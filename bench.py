"""Benchmark: Background SHAP on one MI355X.

One step is one pass of the whole path over one batch: summarise the
background (patterns, exact histograms, MFMA contraction, base value) and
explain every consumer row (patterns, gather-sum into phi).  Inputs are
synthetic, seeded and resident in HBM before timing starts.  Prints one JSON
line.

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper", choices=list(DESCRIPTIONS))
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic", "specialised"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (rows shard across GPUs "
              "with no exchange, so the multi-GPU rate is the per-GPU rate times the GPU count)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_09376_amd import wdf

    w = synth.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    ens = w.ensemble()
    X = w.consumers()
    B = w.background()
    print(f"[bench] generated {args.workload}: {ens.n_trees} trees, X {X.shape}, B {B.shape} "
          f"in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    kernel = {"auto": wdf.KERNEL_AUTO, "generic": wdf.KERNEL_GENERIC, "specialised": wdf.KERNEL_SPECIALISED}[args.kernel]
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

    def step(ev=None):
        bg = wdf.Background(model, Bd)
        if ev is not None:
            ev[0].record(stream)
        bg.explain(Xd, out=phi)
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

    ops_row = int(method_ops_per_row(ens))
    achieved = ops_row * n / (explain_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                "kernel": "explain", "kernel_ms": explain_ms, "ops_per_row": ops_row}
    base = bg.base_value
    out = {"metric": METRIC, "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": DESCRIPTIONS[args.workload], "n_consumers": int(n), "n_background": int(B.shape[1]),
                      "n_trees": ens.n_trees, "n_features": ens.n_features,
                      "kernel": "specialised" if model.specialised else "generic"},
           "roofline": roofline, "base_value": base,
           "explain_rows_per_s": n / (explain_ms * 1e-3),
           "background_ms": ms_step - explain_ms}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ens, X[:, :64], B, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
