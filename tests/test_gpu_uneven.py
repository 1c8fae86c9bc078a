"""Uneven ensemble at its full size: 500 pruned trees of depth 3..8, 127
features, 1M consumers x 1M background rows, through the specialised kernels
(one explain launch over all trees, the launch the benchmark times).

At full size the checks are properties that hold at any size (histogram
invariants, efficiency against oracle predictions on sampled rows); element
parity against the oracle runs on background subsets the oracle finishes in
seconds."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2511_09376_amd import synth
from tests.gpu_util import assert_phi_close, leaf_maps

torch = pytest.importorskip("torch")
import oracle  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wdf():
    from paper_2511_09376_amd import wdf as w
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return w


@pytest.fixture(scope="module")
def uneven(wdf):
    w = synth.WORKLOADS["uneven"]
    ens = w.ensemble()
    ctx = wdf.Context(0)
    print(f"[uneven] loading {ens.n_trees} trees, {ens.feature.size} nodes", flush=True)
    model = wdf.Model(ctx, ens, wdf.KERNEL_SPECIALISED)
    X = w.consumers()
    B = w.background()
    return w, ens, ctx, model, X, B


def _predict(om, X, threads=16):
    """Oracle predictions in column chunks on host threads."""
    n = X.shape[1]
    edges = np.linspace(0, n, threads + 1).astype(np.int64)
    parts = [np.ascontiguousarray(X[:, a:b]) for a, b in zip(edges[:-1], edges[1:])]
    with ThreadPoolExecutor(threads) as ex:
        return np.concatenate(list(ex.map(lambda p: oracle.predict(om, p), parts)))


def test_uneven_full_size(wdf, uneven):
    w, ens, ctx, model, X, B = uneven
    om = oracle.Model(ens)
    m = B.shape[1]
    bg = wdf.Background(model, torch.from_numpy(B).cuda())
    phi = bg.explain(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    # histogram invariants over the full background: every group sees every
    # row once; every row reaches exactly one leaf of every tree
    groups = model.groups()
    h = bg.histograms().astype(np.int64)
    depth = groups["depth"].astype(np.int64)
    hoff = groups["hist_offset"].astype(np.int64)
    reach = np.zeros(ens.n_trees, np.int64)
    for g in range(depth.size):
        d = int(depth[g])
        hg = h[hoff[g]: hoff[g] + (1 << d)]
        assert int(hg.sum()) == m, f"group {g}: {int(hg.sum())} rows"
        allones = (1 << d) - 1
        reach[groups["tree"][g]] += int(hg[allones])
        if groups["leaf_right"][g] >= 0:
            reach[groups["tree"][g]] += int(hg[allones ^ 1])
    assert np.all(reach == m)
    # base value and efficiency on sampled rows
    base_ref = _predict(om, B).mean()
    assert abs(bg.base_value - base_ref) <= 1e-9 * max(1.0, abs(base_ref))
    rows = np.random.default_rng(3).choice(X.shape[1], 4096, replace=False)
    rows = np.concatenate([rows, [0, X.shape[1] - 1]])
    got = phi[:, torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    pred = oracle.predict(om, np.ascontiguousarray(X[:, rows]))
    eff = got.sum(0) - (pred - base_ref)
    scale = np.maximum(np.abs(got).max(0), 1.0)
    assert (np.abs(eff) / scale).max() <= 1e-4
    assert np.isfinite(phi.cpu().numpy()).all()


@pytest.mark.parametrize("kname", ["specialised", "generic"])
def test_uneven_subset_parity(wdf, uneven, kname):
    """Bit-exact histograms and phi against the oracle walk on a background
    subset (several tiles and a ragged tail), on sampled consumer rows."""
    w, ens, ctx, model, X, B = uneven
    if kname == "generic":
        model = wdf.Model(ctx, ens, wdf.KERNEL_GENERIC)
    om = oracle.Model(ens)
    Bs = np.ascontiguousarray(B[:, :8191])
    bg = wdf.Background(model, torch.from_numpy(Bs).cuda())
    groups = model.groups()
    left, _, _ = leaf_maps(om, groups)
    h = bg.histograms()
    href, off = oracle.histograms(om, Bs)
    for g in range(groups["depth"].size):
        d = int(groups["depth"][g])
        ho = int(groups["hist_offset"][g])
        np.testing.assert_array_equal(h[ho: ho + (1 << d)], href[off[left[g]]: off[left[g] + 1]])
    rows = np.random.default_rng(5).choice(X.shape[1], 16, replace=False)
    Xs = np.ascontiguousarray(X[:, rows])
    got = bg.explain(torch.from_numpy(Xs).cuda()).cpu().numpy()
    ref = oracle.bg_walk(om, Xs, Bs, threads=16)
    err = assert_phi_close(got, ref)
    print(f"uneven {kname}: row-scaled error {err:.3e}")
