"""Interaction values (Section 3) through the C ABI against the oracle: the
per-cube formulas summed by the walk, and the definitions by coalition
enumeration on small models; symmetry, zero diagonal, refresh."""
import numpy as np
import pytest

import oracle
from paper_2511_09376_amd import synth
from tests.test_gpu_parity import _edge_ensemble

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wdf():
    from paper_2511_09376_amd import wdf as w
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return w


@pytest.fixture(scope="module")
def ctx(wdf):
    return wdf.Context(0)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _iv_error(got, ref):
    """max over rows of max_{i,j} |iv - ref| / max(max_{i,j} |ref|, 1e-30); arrays [F][F][n]."""
    F = ref.shape[0]
    g = got.reshape(F * F, -1).astype(np.float64)
    r = ref.reshape(F * F, -1)
    scale = np.maximum(np.abs(r).max(0), 1e-30)
    return float((np.abs(g - r).max(0) / scale).max())


@pytest.mark.parametrize("kname", ["generic", "auto"])
@pytest.mark.parametrize("kind", ["shapley", "banzhaf"])
def test_small_iv_against_oracle(wdf, ctx, kname, kind):
    w = synth.WORKLOADS["small"]
    ens, X, B = w.ensemble(), w.consumers(), w.background()
    om = oracle.Model(ens)
    okind = oracle.SHAPLEY if kind == "shapley" else oracle.BANZHAF
    values = wdf.SHAPLEY_IV if kind == "shapley" else wdf.BANZHAF_IV
    model = wdf.Model(ctx, ens, wdf.KERNEL_GENERIC if kname == "generic" else wdf.KERNEL_AUTO)
    bg = wdf.Background(model, _cuda(B), values=values)
    got = bg.explain_iv(_cuda(X)).cpu().numpy()
    ref = oracle.bg_iv_walk(om, X, B, okind)
    err = _iv_error(got, ref)
    assert err <= 1e-5, err
    # the definitions, on a few rows (coalition enumeration over 8 features)
    rows = [0, 17, 99]
    brute = oracle.bg_iv_bruteforce(om, np.ascontiguousarray(X[:, rows]), B, okind)
    assert _iv_error(got[:, :, rows], brute) <= 1e-5
    assert np.all(got[np.arange(8), np.arange(8)] == 0)
    np.testing.assert_allclose(got, got.transpose(1, 0, 2), rtol=0, atol=1e-6 * max(1.0, np.abs(got).max()))


@pytest.mark.parametrize("n", [1, 65, 257])
def test_edge_iv(wdf, ctx, n):
    ens = _edge_ensemble()
    rng = np.random.default_rng(n)
    X = rng.normal(size=(7, n)).astype(np.float32)
    X[rng.random(X.shape) < 0.1] = np.nan
    B = rng.normal(size=(7, 33)).astype(np.float32)
    B[rng.random(B.shape) < 0.1] = np.nan
    model = wdf.Model(ctx, ens, wdf.KERNEL_AUTO)
    bg = wdf.Background(model, _cuda(B), values=wdf.SHAPLEY_IV)
    got = bg.explain_iv(_cuda(X)).cpu().numpy()
    ref = oracle.bg_iv_walk(oracle.Model(ens), X, B)
    assert _iv_error(got, ref) <= 1e-5


@pytest.mark.parametrize("kind", ["shapley", "banzhaf"])
def test_mid_iv_sampled_rows(wdf, ctx, kind):
    """Shapley (Table table_shap_iv) and Banzhaf (Formula
    banzhaf_simplified_formula_interactions) interaction values of the
    100-tree depth-6 model: sampled rows against the oracle's walk."""
    w = synth.WORKLOADS["mid"]
    ens = w.ensemble()
    B = w.background(4099)
    X = w.consumers(70)
    model = wdf.Model(ctx, ens, wdf.KERNEL_AUTO)
    values = wdf.SHAPLEY_IV if kind == "shapley" else wdf.BANZHAF_IV
    bg = wdf.Background(model, _cuda(B), values=values)
    got = bg.explain_iv(_cuda(X)).cpu().numpy()
    rows = [0, 33, 69]
    okind = oracle.SHAPLEY if kind == "shapley" else oracle.BANZHAF
    ref = oracle.bg_iv_walk(oracle.Model(ens), np.ascontiguousarray(X[:, rows]), B, kind=okind, threads=8)
    assert _iv_error(got[:, :, rows], ref) <= 1e-5
    assert np.isfinite(got).all()


def _groups_per_feature(ens):
    """Leaf groups (pairs and singles) whose path carries each feature."""
    K = np.zeros(ens.n_features, np.int64)
    for t in range(ens.n_trees):
        sl = ens.tree_slice(t)
        f, l, r = ens.feature[sl], ens.left[sl], ens.right[sl]
        parent = {}
        for i in range(len(f)):
            if f[i] >= 0:
                parent[int(l[i])] = i
                parent[int(r[i])] = i
        for i in range(len(f)):
            if f[i] >= 0 and (f[l[i]] < 0 or f[r[i]] < 0):
                feats, x = set(), i
                while True:
                    feats.add(int(f[x]))
                    if x not in parent:
                        break
                    x = parent[x]
                for a in feats:
                    K[a] += 1
    return K


def test_iv_many_groups_per_feature(wdf, ctx):
    """200 depth-4 trees over 3 of 8 features: each feature lies on more than
    a thousand group paths (long work lists, many units per feature) and has
    more than 127 distinct thresholds, so ranks are 16-bit (word selects in
    the generated pattern code)."""
    ens = synth.make_ensemble(synth.ModelSpec(200, 4, 4, 0.0, 8, feature_pool=3), synth.DataSpec(8, False, 0.0), 11)
    assert _groups_per_feature(ens).max() > 512
    assert "WORD_1" in wdf.iv_source(ens)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(8, 70)).astype(np.float32)
    B = rng.normal(size=(8, 41)).astype(np.float32)
    model = wdf.Model(ctx, ens, wdf.KERNEL_AUTO)
    bg = wdf.Background(model, _cuda(B), values=wdf.SHAPLEY_IV)
    got = bg.explain_iv(_cuda(X)).cpu().numpy()
    ref = oracle.bg_iv_walk(oracle.Model(ens), X, B, threads=8)
    assert _iv_error(got, ref) <= 1e-5


def test_iv_refresh_and_refusals(wdf, ctx):
    w = synth.WORKLOADS["small"]
    ens, X = w.ensemble(), w.consumers()
    B0, B1 = w.background(), w.background(200)[:, 100:]
    model = wdf.Model(ctx, ens, wdf.KERNEL_AUTO)
    bg = wdf.Background(model, _cuda(B0), values=wdf.SHAPLEY_IV)
    bg.refresh(_cuda(B1))
    torch.cuda.synchronize()
    fresh = wdf.Background(model, _cuda(B1), values=wdf.SHAPLEY_IV)
    np.testing.assert_array_equal(bg.tables(), fresh.tables())
    assert torch.equal(bg.explain_iv(_cuda(X)), fresh.explain_iv(_cuda(X)))
    with pytest.raises(wdf.WdfError):
        bg.explain(_cuda(X))                     # an interaction summary
    plain = wdf.Background(model, _cuda(B0))
    with pytest.raises(wdf.WdfError):
        plain.explain_iv(_cuda(X))
    with pytest.raises(wdf.WdfError):
        wdf.Background(model, values=wdf.SHAPLEY_IV, pathdep=True)
    with pytest.raises(wdf.WdfError):
        wdf.Server(bg, 1 << 28, 256, queue_cap=4)
    small = torch.empty(bg.iv_workspace_bytes(X.shape[1]) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(wdf.WdfError):
        bg.explain_iv(_cuda(X), workspace=small)
