"""Autotuner: it measures the specialised kernels' configurations, keeps the
fastest, and results after tuning still match the oracle."""
import numpy as np
import pytest

import oracle
from paper_2511_09376_amd import synth
from tests.gpu_util import assert_phi_close

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


@pytest.mark.parametrize("workload", ["small", "mid"])
def test_autotune_then_parity(wdf, ctx, workload):
    w = synth.WORKLOADS[workload]
    ens = w.ensemble()
    m = min(w.n_background, 50021)
    B = w.background(m)
    X = w.consumers(min(w.n_consumers, 20011))
    Bd, Xd = torch.from_numpy(B).cuda(), torch.from_numpy(X).cuda()
    model = wdf.Model(ctx, ens, wdf.KERNEL_SPECIALISED)
    rep = model.autotune(Bd, Xd)
    assert rep["gather"] in ("pairs", "quads")
    assert rep["explain_ms"]["pairs"] > 0 and rep["explain_ms"]["quads"] > 0
    # the kept configurations are among the fastest measured (ties allowed)
    assert rep["explain_ms"][rep["gather"]] <= min(rep["explain_ms"].values())
    swept = {f"{nt}x{r}" for nt in (512, 768, 1024) for r in (1, 2, 3, 4, 6, 8)}
    assert {f"512x{r}" for r in (1, 2, 3, 4, 6, 8)} <= set(rep["hist_ms"]) <= swept
    kept = f"{rep['hist_threads']}x{rep['hist_rounds']}"
    assert rep["hist_ms"][kept] <= min(rep["hist_ms"].values())
    assert model.specialised
    bg = wdf.Background(model, Bd)
    phi = bg.explain(Xd).cpu().numpy()
    rows = np.random.default_rng(1).choice(X.shape[1], 6, replace=False)
    om = oracle.Model(ens)
    Bs = np.ascontiguousarray(B[:, :4096]) if workload == "mid" else B
    ref_bg = wdf.Background(model, torch.from_numpy(Bs).cuda())
    got = ref_bg.explain(torch.from_numpy(np.ascontiguousarray(X[:, rows])).cuda()).cpu().numpy()
    assert_phi_close(got, oracle.bg_walk(om, np.ascontiguousarray(X[:, rows]), Bs, threads=8))
    # efficiency on every row of the full-sample summary
    pred = oracle.predict(om, X)
    eff = phi.astype(np.float64).sum(0) - (pred - bg.base_value)
    assert (np.abs(eff) / np.maximum(np.abs(phi).max(0), 1.0)).max() <= 1e-4


def test_autotune_refusals(wdf, ctx):
    w = synth.WORKLOADS["small"]
    ens = w.ensemble()
    Bd, Xd = torch.from_numpy(w.background()).cuda(), torch.from_numpy(w.consumers()).cuda()
    model = wdf.Model(ctx, ens, wdf.KERNEL_SPECIALISED)
    bg = wdf.Background(model, Bd)
    with pytest.raises(wdf.WdfError):
        model.autotune(Bd, Xd)             # a summary exists
    bg.close()
    model.autotune(Bd, Xd)
    generic = wdf.Model(ctx, ens, wdf.KERNEL_GENERIC)
    with pytest.raises(wdf.WdfError):
        generic.autotune(Bd, Xd)
