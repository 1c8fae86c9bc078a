"""The 3M-consumer x 5M-background workload (100 complete depth-6 trees, 127
features) at its full size, in the launch configuration the benchmark times:
the model autotuned on the workload, one summary allocated, refreshed in
place by a replayed HIP graph, one explain launch replayed by a second graph;
and interaction values of a 256k-row chunk against the full background.
Checked on properties that hold at any size (histogram invariants over all
5M rows, efficiency on sampled rows against oracle predictions), on sampled
rows against the oracle with the full background, and bit for bit on the histograms of the first and last tree
of every histogram chunk over all 5M rows (the kernel's tile loop as
launched, dozens of tiles per wave)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2511_09376_amd import synth
from tests.gpu_util import assert_histograms_equal, assert_phi_close, chunk_trees

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wdf():
    from paper_2511_09376_amd import wdf as w
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return w


def _predict(om, X, threads=16):
    n = X.shape[1]
    edges = np.linspace(0, n, threads + 1).astype(np.int64)
    parts = [np.ascontiguousarray(X[:, a:b]) for a, b in zip(edges[:-1], edges[1:])]
    with ThreadPoolExecutor(threads) as ex:
        return np.concatenate(list(ex.map(lambda p: oracle.predict(om, p), parts)))


@pytest.fixture(scope="module")
def paper_data():
    w = synth.WORKLOADS["paper"]
    print("[paper] generating 3M x 5M", flush=True)
    return w.ensemble(), w.consumers(), w.background()


def test_paper_scale_graph_step(wdf, paper_data):
    ens, X, B = paper_data
    ctx = wdf.Context(0)
    model = wdf.Model(ctx, ens, wdf.KERNEL_SPECIALISED)
    Xd, Bd = torch.from_numpy(X).cuda(), torch.from_numpy(B).cuda()
    phi = torch.empty_like(Xd)
    print("[paper] autotune", flush=True)
    model.autotune(Bd, Xd)                       # as the benchmark does, on the workload itself
    bg = wdf.Background(model, Bd)
    g_bg, g_ex = wdf.Graph(bg, B=Bd), wdf.Graph(bg, Xd, phi)
    for _ in range(2):
        g_bg.launch()
        g_ex.launch()
    torch.cuda.synchronize()
    m = B.shape[1]
    # every group sees every background row; every row reaches one leaf per tree
    groups = model.groups()
    h = bg.histograms().astype(np.int64)
    reach = np.zeros(ens.n_trees, np.int64)
    for g in range(groups["depth"].size):
        d = int(groups["depth"][g])
        hg = h[groups["hist_offset"][g]: groups["hist_offset"][g] + (1 << d)]
        assert int(hg.sum()) == m
        full = (1 << d) - 1
        reach[groups["tree"][g]] += int(hg[full]) + (int(hg[full ^ 1]) if groups["leaf_right"][g] >= 0 else 0)
    assert np.all(reach == m)
    # the tile loop as launched (tiles per wave from the library's own grid
    # arithmetic): the first and last tree of every histogram chunk, bit for
    # bit against the oracle's per-leaf counts over all 5M rows
    L = model.hist_launch(m)
    print(f"[paper] histogram grid: {L['blocks']} blocks x {L['chunks']} chunks of {L['threads']} threads, "
          f"{L['tiles_per_block']} tiles per block, up to {L['tiles_per_wave']} per wave", flush=True)
    assert L["tiles_per_wave"] >= 4
    trees = chunk_trees(groups, L["chunk_groups"])
    print(f"[paper] oracle histograms of trees {trees}", flush=True)
    n_checked = assert_histograms_equal(groups, bg.histograms(), ens, B, trees=trees)
    print(f"[paper] {n_checked} groups bit-exact over {m} rows", flush=True)
    om = oracle.Model(ens)
    print("[paper] oracle predictions", flush=True)
    base_ref = _predict(om, B).mean()
    assert abs(bg.base_value - base_ref) <= 1e-9 * max(1.0, abs(base_ref))
    got_all = phi.cpu().numpy()
    rows = np.random.default_rng(5).choice(X.shape[1], 4096, replace=False)
    rows = np.concatenate([rows, [0, X.shape[1] - 1]])
    got = got_all[:, rows].astype(np.float64)
    pred = oracle.predict(om, np.ascontiguousarray(X[:, rows]))
    eff = got.sum(0) - (pred - base_ref)
    assert (np.abs(eff) / np.maximum(np.abs(got).max(0), 1.0)).max() <= 1e-4
    # sampled rows against the oracle with the full 5M background
    print("[paper] oracle on sampled rows", flush=True)
    few = rows[:7].tolist() + [X.shape[1] - 1]
    ref = oracle.bg_walk(om, np.ascontiguousarray(X[:, few]), B, threads=16)
    err = assert_phi_close(got_all[:, few], ref)
    print(f"[paper] row-scaled error {err:.3e}", flush=True)
    used = np.unique(ens.feature[ens.feature >= 0])
    assert np.isfinite(got_all).all()
    assert np.all(got_all[np.setdiff1d(np.arange(ens.n_features), used)] == 0)


def _iv_error(got, ref):
    """max over rows of max_{i,j} |iv - ref| / max(max_{i,j} |ref|, 1e-30); arrays [F][F][n]."""
    F = ref.shape[0]
    g = got.reshape(F * F, -1).astype(np.float64)
    r = ref.reshape(F * F, -1).astype(np.float64)
    scale = np.maximum(np.abs(r).max(0), 1e-30)
    return float((np.abs(g - r).max(0) / scale).max())


def test_paper_scale_iv_chunk(wdf, paper_data):
    """Interaction values at the full size, as the benchmark launches them: a
    summary of all 5M background rows, one 256k-row consumer chunk.  The
    oracle's interaction walk costs minutes per row against 5M background
    rows, so the full summary is checked by linearity in the background (the
    values of the whole background are the row-weighted mean of those of its
    two halves), and the formula on sampled rows of the same chunk against
    the oracle with a 20k-row background."""
    ens, X, B = paper_data
    F, m = ens.n_features, B.shape[1]
    ctx = wdf.Context(0)
    model = wdf.Model(ctx, ens, wdf.KERNEL_SPECIALISED)
    chunk, start = 1 << 18, X.shape[1] - (1 << 18) - 12345
    Xc = torch.from_numpy(np.ascontiguousarray(X[:, start:start + chunk])).cuda()
    rows = np.array([0, 1, 63, 64, 65, chunk // 2, chunk - 2, chunk - 1])
    Xr = torch.from_numpy(np.ascontiguousarray(X[:, start + rows])).cuda()

    print("[paper iv] full background", flush=True)
    Bd = torch.from_numpy(B).cuda()
    bg = wdf.Background(model, Bd, values=wdf.SHAPLEY_IV)
    assert bg.specialised
    out = bg.explain_iv(Xc)
    torch.cuda.synchronize()
    full = out[:, :, torch.from_numpy(rows).cuda()].cpu().numpy()
    del out, bg
    assert np.isfinite(full).all()
    assert np.all(full[np.arange(F), np.arange(F)] == 0)
    np.testing.assert_allclose(full, full.transpose(1, 0, 2), rtol=0, atol=1e-6 * max(1.0, np.abs(full).max()))
    h = m // 2
    parts = []
    for a, b in ((0, h), (h, m)):
        bgp = wdf.Background(model, Bd[:, a:b].contiguous(), values=wdf.SHAPLEY_IV)
        parts.append((b - a) * bgp.explain_iv(Xr).cpu().numpy().astype(np.float64))
        del bgp
    del Bd
    err = _iv_error(full, (parts[0] + parts[1]) / m)
    print(f"[paper iv] linearity in the background: {err:.3e}", flush=True)
    assert err <= 1e-5

    print("[paper iv] oracle, 20k background rows", flush=True)
    Bs = np.ascontiguousarray(B[:, :20000])
    bgs = wdf.Background(model, torch.from_numpy(Bs).cuda(), values=wdf.SHAPLEY_IV)
    sub = bgs.explain_iv(Xc)[:, :, torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = oracle.bg_iv_walk(oracle.Model(ens), np.ascontiguousarray(X[:, start + rows]), Bs, threads=8)
    err = _iv_error(sub, ref)
    print(f"[paper iv] against the oracle: {err:.3e}", flush=True)
    assert err <= 1e-5
