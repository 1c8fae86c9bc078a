"""CPU checks of the benchmark's host logic: the method-op count behind the
roofline figure, and the refusal of more than one GPU."""
import os
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
    a positive rate, the thread count it used, and a bounded sample."""
    w = synth.WORKLOADS["small"]
    ens, X, B = w.ensemble(), w.consumers(), w.background()
    out = bench.cpu_baseline(ens, X, B, seconds_hint=0.2)
    assert set(out) == {"value", "unit", "cores", "kind", "sample"}
    assert out["kind"] == "oracle" and out["unit"] == "rows/s" and out["value"] > 0
    assert 1 <= out["cores"] <= min(16, os.cpu_count() or 1, X.shape[1])
    assert "background rows" in out["sample"]


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
