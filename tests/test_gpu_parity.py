"""GPU parity: the HIP path against the FP64 oracle, called through the C ABI.

Integer work (patterns, histograms) must match bit for bit; phi must be within
a row-scaled error of 1e-5 (the max over features of |phi - phi_ref| divided by
the row's largest |phi_ref|), and features no split uses must be exactly 0.
"""
import numpy as np
import pytest

import oracle
from paper_2511_09376_amd import synth
from tests.gpu_util import assert_phi_close, expected_tables, leaf_maps, row_scaled_error
from tests.trees import ensemble

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def wdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_09376_amd import wdf as w
    return w


@pytest.fixture(scope="module")
def ctx(wdf):
    return wdf.Context(0)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


KERNELS = ["generic", "auto", "pairs"]


def _kernel(wdf, name):
    return {"generic": wdf.KERNEL_GENERIC, "auto": wdf.KERNEL_AUTO,
            "pairs": wdf.KERNEL_AUTO | wdf.KERNEL_PAIRS}[name]


def _load(wdf, ctx, ens, kname):
    """Load a model; with kname "auto" or "pairs" the specialised kernels must be the ones in use."""
    model = wdf.Model(ctx, ens, _kernel(wdf, kname))
    assert model.specialised == (kname != "generic"), f"kernel choice {kname}: specialised={model.specialised}"
    return model


# ---------------------------------------------------------------------------
# Small workload: everything, including coalition enumeration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kname", KERNELS)
def test_small_full_parity(wdf, ctx, kname):
    w = synth.WORKLOADS["small"]
    ens = w.ensemble()
    X, B = w.consumers(), w.background()
    om = oracle.Model(ens)
    model = _load(wdf, ctx, ens, kname)
    groups = model.groups()
    left, right, depth = leaf_maps(om, groups)

    # patterns: bit-exact against the per-leaf definition
    P = model.patterns(_cuda(X)).cpu().numpy().view(np.uint32)
    Pref = oracle.patterns(om, X)
    np.testing.assert_array_equal(P, Pref[left])

    bg = wdf.Background(model, _cuda(B))
    # histograms: bit-exact
    h = bg.histograms()
    href, off = oracle.histograms(om, B)
    for g in range(groups["depth"].size):
        d = int(groups["depth"][g])
        ho = int(groups["hist_offset"][g])
        got = h[ho: ho + (1 << d)]
        np.testing.assert_array_equal(got, href[off[left[g]]: off[left[g] + 1]])
        if right[g] >= 0:
            np.testing.assert_array_equal(got[np.arange(1 << d) ^ 1], href[off[right[g]]: off[right[g] + 1]])

    # tables: float32 of the oracle's s-vectors
    freq = href.astype(np.float64) / B.shape[1]
    t_ref = expected_tables(om, groups, freq, off, oracle.SHAPLEY)
    np.testing.assert_allclose(bg.tables(), t_ref, rtol=2e-7, atol=1e-12)

    # phi: against coalition enumeration and the oracle walk
    phi = bg.explain(_cuda(X))
    torch.cuda.synchronize()
    got = phi.cpu().numpy()
    ref = oracle.bg_bruteforce(om, X, B)
    assert_phi_close(got, ref)
    assert_phi_close(got, oracle.bg_walk(om, X, B))
    # base value and efficiency
    base_ref = oracle.predict(om, B).mean()
    assert abs(bg.base_value - base_ref) <= 1e-12 * max(1.0, abs(base_ref))
    eff = got.astype(np.float64).sum(0) - (oracle.predict(om, X) - base_ref)
    assert np.abs(eff).max() <= 1e-4


@pytest.mark.parametrize("kname", KERNELS)
@pytest.mark.parametrize("values", ["shapley", "banzhaf"])
def test_small_values_kinds(wdf, ctx, kname, values):
    w = synth.WORKLOADS["small"]
    ens = w.ensemble()
    X, B = w.consumers(), w.background()
    kind = oracle.SHAPLEY if values == "shapley" else oracle.BANZHAF
    model = _load(wdf, ctx, ens, kname)
    bg = wdf.Background(model, _cuda(B), values=kind)
    om = oracle.Model(ens)
    href, off = oracle.histograms(om, B)
    t_ref = expected_tables(om, model.groups(), href.astype(np.float64) / B.shape[1], off, kind)
    np.testing.assert_allclose(bg.tables(), t_ref, rtol=2e-7, atol=1e-12)
    got = bg.explain(_cuda(X)).cpu().numpy()
    assert_phi_close(got, oracle.bg_bruteforce(om, X, B, kind))


# ---------------------------------------------------------------------------
# Mid workload (100 depth-6 trees, 127 features, NaN): full-size run, sampled rows
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def mid():
    w = synth.WORKLOADS["mid"]
    return w, w.ensemble(), w.consumers(), w.background()


@pytest.mark.parametrize("m", [20011, 20012])
@pytest.mark.parametrize("kname", KERNELS)
def test_mid_histograms_bit_exact(wdf, ctx, mid, kname, m):
    """Several tiles and a ragged tail; a row count divisible by four (and so
    a code stride of whole 16-byte groups) takes the quantize kernel's
    four-rows-per-thread path, the other its row-wise path."""
    w, ens, X, B = mid
    Bs = np.ascontiguousarray(B[:, :m])
    om = oracle.Model(ens)
    model = _load(wdf, ctx, ens, kname)
    groups = model.groups()
    left, _, _ = leaf_maps(om, groups)
    bg = wdf.Background(model, _cuda(Bs))
    h = bg.histograms()
    href, off = oracle.histograms(om, Bs)
    for g in range(groups["depth"].size):
        d = int(groups["depth"][g])
        ho = int(groups["hist_offset"][g])
        np.testing.assert_array_equal(h[ho: ho + (1 << d)], href[off[left[g]]: off[left[g] + 1]])


@pytest.mark.parametrize("kname", KERNELS)
def test_mid_full_size_sampled_rows(wdf, ctx, mid, kname):
    w, ens, X, B = mid
    om = oracle.Model(ens)
    model = _load(wdf, ctx, ens, kname)
    bg = wdf.Background(model, _cuda(B))
    phi = bg.explain(_cuda(X))
    torch.cuda.synchronize()
    got = phi.cpu().numpy()
    # sampled rows against the oracle with the full background
    rows = np.random.default_rng(11).choice(X.shape[1], 12, replace=False)
    rows = np.concatenate([rows, [0, X.shape[1] - 1]])
    ref = oracle.bg_walk(om, np.ascontiguousarray(X[:, rows]), B, threads=8)
    err = assert_phi_close(got[:, rows], ref)
    print(f"mid sampled rows: row-scaled error {err:.3e}")
    # efficiency on every row
    base_ref = oracle.predict(om, B).mean()
    assert abs(bg.base_value - base_ref) <= 1e-9 * max(1.0, abs(base_ref))
    pred = oracle.predict(om, X)
    eff = got.astype(np.float64).sum(0) - (pred - base_ref)
    scale = np.maximum(np.abs(got).max(0), 1.0)
    assert (np.abs(eff) / scale).max() <= 1e-4
    # null players exactly zero
    used = np.unique(ens.feature[ens.feature >= 0])
    unused = np.setdiff1d(np.arange(ens.n_features), used)
    assert np.all(got[unused] == 0.0)


@pytest.mark.parametrize("kname", ["generic", "auto"])
def test_mid_banzhaf_sampled_rows(wdf, ctx, mid, kname):
    """Banzhaf values (Formula banzhaf_simplified_formula) of the 100-tree
    depth-6 model over the full 100k background: sampled rows against the
    oracle's walk with the full background; null players exactly 0."""
    w, ens, X, B = mid
    om = oracle.Model(ens)
    model = _load(wdf, ctx, ens, kname)
    bg = wdf.Background(model, _cuda(B), values=wdf.BANZHAF)
    rows = np.concatenate([np.random.default_rng(12).choice(X.shape[1], 6, replace=False), [0, X.shape[1] - 1]])
    got = bg.explain(_cuda(X[:, rows])).cpu().numpy()
    ref = oracle.bg_walk(om, np.ascontiguousarray(X[:, rows]), B, kind=oracle.BANZHAF, threads=16)
    err = assert_phi_close(got, ref)
    print(f"mid Banzhaf ({kname}): row-scaled error {err:.3e}")
    unused = np.setdiff1d(np.arange(ens.n_features), np.unique(ens.feature[ens.feature >= 0]))
    assert np.all(got[unused] == 0.0)


@pytest.mark.parametrize("kname", ["generic", "auto"])
@pytest.mark.parametrize("values", ["shapley", "banzhaf"])
def test_mid_path_dependent(wdf, ctx, mid, kname, values):
    """Path-dependent values (Section 8, Formula eq:path_dependent_estimation)
    of the 100-tree depth-6 model: the library's cover-product frequencies,
    contraction and gather against the oracle's Alg. 3 form with its own
    product-form frequencies (both pinned to coalition enumeration on the
    small model), on sampled rows; null players exactly 0."""
    w, ens, X, B = mid
    om = oracle.Model(ens)
    kind = oracle.SHAPLEY if values == "shapley" else oracle.BANZHAF
    model = _load(wdf, ctx, ens, kname)
    bg = wdf.Background(model, pathdep=True, values=kind)
    rows = np.concatenate([np.random.default_rng(13).choice(X.shape[1], 30, replace=False), [0, X.shape[1] - 1]])
    Xs = np.ascontiguousarray(X[:, rows])
    got = bg.explain(_cuda(Xs)).cpu().numpy()
    freq, off = oracle.pd_freq(om)
    ref = oracle.woodelf_phi(om, Xs, freq, off, kind)
    err = assert_phi_close(got, ref)
    print(f"mid path-dependent {values} ({kname}): row-scaled error {err:.3e}")
    unused = np.setdiff1d(np.arange(ens.n_features), np.unique(ens.feature[ens.feature >= 0]))
    assert np.all(got[unused] == 0.0)


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------

def _edge_ensemble():
    trees = [
        ("leaf", 0.75),                                             # single-leaf tree
        ("split", 0, 0.0, 1, ("leaf", 1.0), ("leaf", -2.0)),        # stump, NaN left
        # repeated feature on a path, uneven depth
        ("split", 1, 0.5, 0,
         ("split", 1, -0.5, 1, ("leaf", 3.0), ("split", 2, 0.0, 0, ("leaf", -1.0), ("leaf", 0.5))),
         ("leaf", 2.0)),
    ]
    # a depth-8 chain with a pair at the bottom
    node = ("split", 3, 0.1, 0, ("leaf", 1.0), ("leaf", -1.0))
    for k in range(7):
        node = ("split", (k % 3) + 3, 0.05 * k - 0.1, k % 2, node, ("leaf", float(k)))
    trees.append(node)
    return ensemble(trees, 7)


@pytest.mark.parametrize("kname", KERNELS)
@pytest.mark.parametrize("n", [1, 63, 64, 65, 257, 1000])
def test_edge_shapes(wdf, ctx, kname, n):
    ens = _edge_ensemble()
    rng = np.random.default_rng(n)
    X = rng.normal(size=(7, n)).astype(np.float32)
    X[rng.random(X.shape) < 0.1] = np.nan
    B = rng.normal(size=(7, 37)).astype(np.float32)
    B[rng.random(B.shape) < 0.1] = np.nan
    om = oracle.Model(ens)
    model = _load(wdf, ctx, ens, kname)
    bg = wdf.Background(model, _cuda(B))
    got = bg.explain(_cuda(X)).cpu().numpy()
    assert_phi_close(got, oracle.bg_bruteforce(om, X, B))


@pytest.mark.parametrize("kname", KERNELS)
def test_single_background_row_and_empty_explain(wdf, ctx, kname):
    ens = _edge_ensemble()
    rng = np.random.default_rng(5)
    X = rng.normal(size=(7, 40)).astype(np.float32)
    model = _load(wdf, ctx, ens, kname)
    bg = wdf.Background(model, _cuda(X[:, :1]))
    got = bg.explain(_cuda(X)).cpu().numpy()
    assert_phi_close(got, oracle.bg_bruteforce(oracle.Model(ens), X, X[:, :1]))
    assert np.all(got[:, 0] == 0.0)          # b == c gives zero
    empty = bg.explain(torch.empty((7, 0), dtype=torch.float32, device="cuda"))
    assert empty.shape == (7, 0)


@pytest.mark.parametrize("kname", KERNELS)
def test_padded_leading_dimensions(wdf, ctx, kname):
    w = synth.WORKLOADS["small"]
    ens = w.ensemble()
    X, B = w.consumers(), w.background()
    model = _load(wdf, ctx, ens, kname)
    Bp = torch.zeros((8, 160), dtype=torch.float32, device="cuda")
    Bp[:, :100] = _cuda(B)
    bg = wdf.Background(model, Bp[:, :100])
    Xp = torch.zeros((8, 128), dtype=torch.float32, device="cuda")
    Xp[:, :100] = _cuda(X)
    out = torch.full((8, 130), 7.0, dtype=torch.float32, device="cuda")
    bg.explain(Xp[:, :100], out=out[:, :100])
    got = out.cpu().numpy()
    assert_phi_close(got[:, :100], oracle.bg_walk(oracle.Model(ens), X, B))
    assert np.all(got[:, 100:] == 7.0)       # nothing written past n


@pytest.mark.parametrize("kname", KERNELS)
def test_determinism(wdf, ctx, kname):
    w = synth.WORKLOADS["small"]
    ens = w.ensemble()
    X, B = w.consumers(), w.background()
    model = _load(wdf, ctx, ens, kname)
    a = wdf.Background(model, _cuda(B))
    b = wdf.Background(model, _cuda(B))
    np.testing.assert_array_equal(a.histograms(), b.histograms())
    np.testing.assert_array_equal(a.tables(), b.tables())
    np.testing.assert_array_equal(a.explain(_cuda(X)).cpu().numpy(), a.explain(_cuda(X)).cpu().numpy())


def test_host_background_copy(wdf, ctx):
    w = synth.WORKLOADS["small"]
    ens = w.ensemble()
    X, B = w.consumers(), w.background()
    model = wdf.Model(ctx, ens)
    a = wdf.Background(model, B)              # host array, copied in by the library
    b = wdf.Background(model, _cuda(B))
    np.testing.assert_array_equal(a.histograms(), b.histograms())


# ---------------------------------------------------------------------------
# Path-dependent values (Section 8)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kname", KERNELS)
@pytest.mark.parametrize("values", ["shapley", "banzhaf"])
def test_path_dependent(wdf, ctx, kname, values):
    w = synth.WORKLOADS["small"]
    ens = w.ensemble()
    X = w.consumers()
    kind = oracle.SHAPLEY if values == "shapley" else oracle.BANZHAF
    model = _load(wdf, ctx, ens, kname)
    bg = wdf.Background(model, pathdep=True, values=kind)
    got = bg.explain(_cuda(X)).cpu().numpy()
    assert_phi_close(got, oracle.pd_bruteforce(oracle.Model(ens), X, kind))


@pytest.mark.parametrize("kname", KERNELS)
@pytest.mark.parametrize("values", ["shapley", "banzhaf"])
def test_path_dependent_zero_cover_parent(wdf, ctx, kname, values):
    """A leaf pair whose parent no training row reached: each leaf's
    frequencies along its own path (0/0 read as 0), against the path-dependent
    game by coalition enumeration."""
    from tests.test_oracle import ZERO_COVER_COVERS, ZERO_COVER_TREE, zero_cover_case
    M, C = zero_cover_case()
    kind = oracle.SHAPLEY if values == "shapley" else oracle.BANZHAF
    model = _load(wdf, ctx, ensemble([ZERO_COVER_TREE], 3, ZERO_COVER_COVERS), kname)
    bg = wdf.Background(model, pathdep=True, values=kind)
    got = bg.explain(_cuda(C)).cpu().numpy()
    assert_phi_close(got, oracle.pd_bruteforce(M, C, kind))


def test_most_features_generic(wdf, ctx):
    """The ABI's feature limit, 65535 features, with splits spread over the
    whole range: AUTO loads the generic kernels (the specialised ones take up
    to 4096 features), SPECIALISED is refused; histograms bit for bit, phi
    against the oracle walk, every feature no split uses exactly 0."""
    F = 65535
    feats = [0, 17, 4096, 40000, 65534, 31337, 65534]
    tree = lambda k: ("split", feats[k % 7], 0.1 * k, k % 2,
                      ("split", feats[(k + 1) % 7], -0.3, 0, ("leaf", 1.0 + k), ("leaf", -0.5)),
                      ("split", feats[(k + 3) % 7], 0.2, 1,
                       ("split", feats[(k + 5) % 7], 0.0, 0, ("leaf", 0.25 * k), ("leaf", 2.0)), ("leaf", -1.5)))
    ens = ensemble([tree(k) for k in range(5)], F)
    rng = np.random.default_rng(21)
    B = rng.standard_normal((F, 300)).astype(np.float32)
    X = rng.standard_normal((F, 7)).astype(np.float32)
    B[40000, ::5] = np.nan
    X[4096, 2] = np.nan
    with pytest.raises(wdf.WdfError) as e:
        wdf.Model(ctx, ens, wdf.KERNEL_SPECIALISED)
    assert e.value.code == wdf.E_UNSUPPORTED
    model = wdf.Model(ctx, ens, wdf.KERNEL_AUTO)
    assert not model.specialised
    bg = wdf.Background(model, _cuda(B))
    om = oracle.Model(ens)
    groups = model.groups()
    left, right, _ = leaf_maps(om, groups)
    h = bg.histograms()
    href, off = oracle.histograms(om, B, threads=2)
    for g in range(groups["depth"].size):
        d = int(groups["depth"][g])
        ho = int(groups["hist_offset"][g])
        np.testing.assert_array_equal(h[ho: ho + (1 << d)], href[off[left[g]]: off[left[g] + 1]])
    got = bg.explain(_cuda(X)).cpu().numpy()
    assert_phi_close(got, oracle.bg_walk(om, X, B, threads=4))
    unused = np.setdiff1d(np.arange(F), feats)
    assert np.all(got[unused] == 0.0)


# ---------------------------------------------------------------------------
# Errors cross the ABI as codes
# ---------------------------------------------------------------------------

def test_invalid_models_rejected(wdf, ctx):
    good = _edge_ensemble()
    bad_feature = ensemble([("split", 9, 0.0, 0, ("leaf", 1.0), ("leaf", 2.0))], 7)
    with pytest.raises(wdf.WdfError) as e:
        wdf.Model(ctx, bad_feature)
    assert e.value.code == wdf.E_INVALID_ARG
    node = ("leaf", 1.0)
    for k in range(9):
        node = ("split", 0, float(k), 0, node, ("leaf", 0.0))
    with pytest.raises(wdf.WdfError) as e:
        wdf.Model(ctx, ensemble([node], 1))
    assert e.value.code == wdf.E_UNSUPPORTED
    cyc = ensemble([("split", 0, 0.0, 0, ("leaf", 1.0), ("leaf", 2.0))], 1)
    cyc.left[0] = 0
    with pytest.raises(wdf.WdfError) as e:
        wdf.Model(ctx, cyc)
    assert e.value.code == wdf.E_INVALID_ARG
    m = wdf.Model(ctx, good)
    with pytest.raises(wdf.WdfError):
        wdf.Background(m, np.zeros((7, 0), np.float32))
    assert row_scaled_error(np.zeros((1, 1)), np.zeros((1, 1))) == 0.0
