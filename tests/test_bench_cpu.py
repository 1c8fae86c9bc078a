"""CPU checks of the benchmark's host logic: the method-op count behind the
roofline figure, and the refusal of more than one GPU."""
import os
import re
import subprocess
import sys

import pytest

from paper_2511_09376_amd import synth
from tests.trees import ensemble

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_method_ops_complete_trees(bench):
    # complete depth-d tree: 2^d - 1 inner nodes (compare + two child pattern
    # updates each) and 2^(d-1) leaf pairs whose paths have d positions
    for d in (1, 2, 4, 6):
        assert bench.method_ops_per_row(_complete(d)) == 3 * (2 ** d - 1) + 2 ** (d - 1) * d
    assert bench.method_ops_per_row(_complete(6)) == 381
    assert bench.method_ops_per_row(synth.WORKLOADS["small"].ensemble()) == 10 * (3 * 15 + 8 * 4)
    assert bench.method_ops_per_row(synth.WORKLOADS["mid"].ensemble()) == 100 * 381


def test_method_ops_pruned_tree(bench):
    # root (depth 0) with a leaf on the left and a split with two leaves on the
    # right: 2 inner nodes; a single-leaf group with a 1-position path and a
    # leaf pair with a 2-position path
    ens = ensemble([("split", 0, 0.0, 0, ("leaf", 1.0), ("split", 1, 0.0, 0, ("leaf", 2.0), ("leaf", 3.0)))], 2)
    assert bench.method_ops_per_row(ens) == 3 * 2 + 1 + 2
    # a root leaf does no work
    assert bench.method_ops_per_row(ensemble([("leaf", 5.0)], 1)) == 0


def _complete(d):
    def node(k):
        return ("leaf", 1.0) if k == d else ("split", k, 0.0, 0, node(k + 1), node(k + 1))
    return ensemble([node(0)], max(d, 1))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "measures one GPU" in res.stderr and res.stdout == ""


def test_cpu_baseline_leg(bench):
    """The oracle leg of the bench line on a tiny workload: the documented keys,
    a positive rate from the measured wall time (no scaling), the thread count
    and host it used, every background row, and the oracle's phi of exactly
    the sampled rows."""
    import oracle
    w = synth.WORKLOADS["small"]
    ens, X, B = w.ensemble(), w.consumers(), w.background()
    rows = [3, 17, 99]
    out, ref = bench.cpu_baseline(ens, X, B, rows, threads=2, kind=0)
    assert {"value", "unit", "cores", "kind", "sample", "seconds", "rows", "nproc", "cpu_model"} <= set(out)
    assert out["kind"] == "oracle" and out["unit"] == "rows/s" and out["value"] > 0
    assert out["cores"] == 2 and out["rows"] == 3
    assert abs(out["value"] - 3 / out["seconds"]) <= 1e-9 * out["value"]
    assert f"all {B.shape[1]} background rows" in out["sample"] and "no scaling" in out["sample"]
    assert out["cpu_model"] and out["nproc"] >= 1
    assert ref.shape == (ens.n_features, 3)
    assert (ref == oracle.bg_walk(oracle.Model(ens), X[:, rows], B, threads=1)).all()
    assert 1 <= bench.host_threads() <= 16


def test_run_error(bench):
    """The per-run error record: maximum absolute and row-scaled error
    against the oracle's rows, and the 1e-5 gate."""
    import numpy as np
    ref = np.array([[1.0, -2.0], [0.5, 0.0]])
    got = ref + np.array([[1e-6, 0.0], [0.0, 4e-5]])
    e = bench.run_error(got, ref, [5, 6])
    assert e["rows"] == 2 and abs(e["max_abs"] - 4e-5) < 1e-15
    assert abs(e["row_scaled"] - 2e-5) < 1e-15            # row 2: 4e-5 / 2.0
    assert e["within_tolerance"] is False
    assert bench.run_error(ref, ref, [5, 6])["within_tolerance"] is True


def test_traffic_summary_matches_the_current_explain_kernel(bench):
    """The committed HBM-traffic summary was taken on the explain kernel the
    generator writes today (same source hash), so the bench line's `traffic`
    is a measurement of this kernel and not of an earlier one."""
    from paper_2511_09376_amd import wdf
    if not os.path.exists(wdf.LIB_PATH):
        pytest.skip("libwdf.so not built")
    ens = synth.WORKLOADS["paper"].ensemble()
    traffic = bench.measured_traffic(wdf, ens, "paper", "quads")
    assert traffic is not None, ("profiles/explain_quads_paper_traffic.md was taken on another explain kernel: "
                                 "measure FETCH_SIZE / WRITE_SIZE again")
    # measured bytes against the algorithmic bytes of one launch (X read,
    # phi written: 2 x 127 x 4 B per row over 3M rows, 3.05 GB): within 1.5x
    algorithmic = 2 * 127 * 4 * 3_000_000
    assert algorithmic <= traffic <= 1.5 * algorithmic


def test_traffic_summary_matches_the_current_interaction_kernels(bench):
    """The same for the interaction kernels: the committed summary was taken
    on the pattern and interaction kernels the generator writes today, and the
    measured bytes per step lie between the output alone (F x F floats per
    row) and the output plus one pattern byte per unit and row read and one
    per group and row written, with 10 % to spare."""
    from paper_2511_09376_amd import wdf
    if not os.path.exists(wdf.LIB_PATH):
        pytest.skip("libwdf.so not built")
    ens = synth.WORKLOADS["paper"].ensemble()
    traffic = bench.measured_iv_traffic(wdf, ens, "paper")
    assert traffic is not None, ("profiles/iv_paper_traffic.md was taken on other interaction kernels: "
                                 "measure FETCH_SIZE / WRITE_SIZE again")
    n, F = 3_000_000, 127
    output = 4 * F * F * n
    units = len(re.findall(r"const u32 q\d+ = ", wdf.iv_source(ens)))  # pattern reads per row
    groups = ens.n_trees * 32  # pair groups of complete depth-6 trees
    assert output <= traffic <= 1.1 * (output + (units + groups) * n)
