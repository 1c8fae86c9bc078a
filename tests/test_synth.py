"""CPU checks of the seeded input recipe: the 127-column mix, the value
distributions and missing rate, rows regenerated alone and independent of the
thread count, and the tree shapes and covers of the named workloads."""
import numpy as np
import pytest

from paper_2511_09376_amd import synth

MIX = synth.DataSpec(127, mixed=True, nan_rate=0.05)


def test_column_mix():
    kinds = MIX.column_kinds()
    assert [int((kinds == k).sum()) for k in range(4)] == [43, 42, 21, 21]
    assert (synth.DataSpec(8, mixed=False, nan_rate=0.0).column_kinds() == 0).all()


def test_value_distributions():
    X = synth.make_matrix(MIX, 1 << 16, 12345)
    assert X.dtype == np.float32 and X.shape == (127, 1 << 16)
    nan = np.isnan(X)
    assert abs(nan.mean() - 0.05) < 1e-3
    kinds = MIX.column_kinds()
    vals = [X[kinds == k][~nan[kinds == k]] for k in range(4)]
    normal, lognormal, binary, counts = (v.astype(np.float64) for v in vals)
    assert abs(normal.mean()) < 5e-3 and abs(normal.std() - 1.0) < 5e-3
    assert (lognormal > 0).all() and abs(np.median(np.log(lognormal))) < 5e-3
    assert set(np.unique(binary)) == {0.0, 1.0} and abs(binary.mean() - 0.3) < 5e-3
    assert (counts >= 0).all() and (counts == np.round(counts)).all() and abs(counts.mean() - 3.0) < 2e-2
    assert abs(counts.var() - 3.0) < 5e-2


def test_rows_regenerate_alone_and_ignore_thread_count():
    spec = synth.DataSpec(9, mixed=True, nan_rate=0.05)
    n = 2 * synth.CHUNK_ROWS + 100                      # three chunks, the last one ragged
    full = synth.make_matrix(spec, n, 777, threads=1)
    np.testing.assert_array_equal(synth.make_matrix(spec, n, 777, threads=4), full)
    rows = np.array([0, 1, synth.CHUNK_ROWS - 1, synth.CHUNK_ROWS, 2 * synth.CHUNK_ROWS + 99, 5])
    np.testing.assert_array_equal(synth.matrix_rows(spec, n, 777, rows), full[:, rows])
    assert not np.array_equal(synth.make_matrix(spec, 100, 778), full[:, :100])


def _depths(ens, t):
    sl = ens.tree_slice(t)
    f, l, r = ens.feature[sl], ens.left[sl], ens.right[sl]
    d = np.zeros(f.size, np.int64)
    for i in range(f.size):                             # parents precede children
        if f[i] >= 0:
            d[l[i]] = d[r[i]] = d[i] + 1
    return d, f


def _check_covers(ens, t, sample_rows=4096):
    sl = ens.tree_slice(t)
    f, l, r, c = ens.feature[sl], ens.left[sl], ens.right[sl], ens.cover[sl]
    assert c[0] == sample_rows
    inner = np.nonzero(f >= 0)[0]
    np.testing.assert_array_equal(c[inner], c[l[inner]] + c[r[inner]])


@pytest.mark.parametrize("name,trees,lo,hi,complete", [("small", 10, 4, 4, True), ("mid", 100, 6, 6, True),
                                                        ("uneven", 500, 1, 8, False)])
def test_workload_trees(name, trees, lo, hi, complete):
    w = synth.WORKLOADS[name]
    ens = w.ensemble()
    assert ens.n_trees == trees and ens.n_features == w.data.n_features
    leaf_depths = []
    for t in range(trees):
        d, f = _depths(ens, t)
        leaves = d[f < 0]
        leaf_depths.append(leaves)
        assert lo <= leaves.max() <= hi
        if complete:
            assert (leaves == hi).all() and f.size == 2 ** (hi + 1) - 1
        _check_covers(ens, t)
    assert (ens.feature < ens.n_features).all() and np.isfinite(ens.threshold).all()
    assert set(np.unique(ens.default_left)) <= {0, 1}
    if w.data.nan_rate == 0:
        assert (ens.default_left[ens.feature >= 0] == 1).all()
    if not complete:
        # depth drawn from 3..8 and inner nodes pruned w.p. 0.15: shallow and
        # full-depth paths both occur
        allv = np.concatenate(leaf_depths)
        assert allv.min() == 1 and allv.max() == 8
    assert np.array_equal(w.ensemble().threshold, ens.threshold)    # seeded
