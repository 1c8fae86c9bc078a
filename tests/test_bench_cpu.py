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
