"""In-place background refresh and HIP-graph replay of a whole step (refresh +
explain): results equal a fresh load of the same background, bit for bit, on
every replay, with eager work and synchronisations between replays."""
import numpy as np
import pytest

from paper_2511_09376_amd import synth

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


@pytest.fixture(scope="module")
def mid_data():
    w = synth.WORKLOADS["mid"]
    ens = w.ensemble()
    B = w.background(3 * 20011)
    X = w.consumers(5003)
    Bs = [torch.from_numpy(np.ascontiguousarray(B[:, k * 20011:(k + 1) * 20011])).cuda() for k in range(3)]
    return ens, Bs, torch.from_numpy(X).cuda()


def _kernel(wdf, kname):
    return {"generic": wdf.KERNEL_GENERIC, "auto": wdf.KERNEL_AUTO}[kname]


def _same_summary(a, b):
    np.testing.assert_array_equal(a.histograms(), b.histograms())
    np.testing.assert_array_equal(a.tables(), b.tables())
    assert a.base_value == b.base_value


@pytest.mark.parametrize("kname", ["auto", "generic"])
def test_refresh_equals_fresh_load(wdf, ctx, mid_data, kname):
    ens, Bs, X = mid_data
    model = wdf.Model(ctx, ens, _kernel(wdf, kname))
    bg = wdf.Background(model, Bs[0])
    for k in (1, 2, 1):
        bg.refresh(Bs[k])
        torch.cuda.synchronize()
        ref = wdf.Background(model, Bs[k])
        _same_summary(bg, ref)
        assert torch.equal(bg.explain(X), ref.explain(X))
        ref.close()


@pytest.mark.parametrize("kname", ["auto", "generic"])
def test_graph_step_replays(wdf, ctx, mid_data, kname):
    ens, Bs, X = mid_data
    model = wdf.Model(ctx, ens, _kernel(wdf, kname))
    bg = wdf.Background(model, Bs[0])
    other = wdf.Background(model, Bs[2])
    Bin = Bs[1].clone()
    phi = torch.empty_like(X)
    g = wdf.Graph(bg, X, phi, B=Bin)
    refs = {k: wdf.Background(model, Bs[k]) for k in (1, 2)}
    expect = {k: refs[k].explain(X) for k in (1, 2)}
    torch.cuda.synchronize()
    for r, k in enumerate((1, 1, 2, 1)):
        Bin.copy_(Bs[k])                      # new contents, same address
        side = other.explain(X)               # eager work between replays
        torch.cuda.synchronize()
        phi.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(phi, expect[k]), f"replay {r}"
        _same_summary(bg, refs[k])
        assert torch.isfinite(side).all()
    g.close()


def test_explain_only_graph(wdf, ctx, mid_data):
    ens, Bs, X = mid_data
    model = wdf.Model(ctx, ens, wdf.KERNEL_AUTO)
    bg = wdf.Background(model, Bs[0])
    expect = bg.explain(X)
    phi = torch.zeros_like(X)
    g = wdf.Graph(bg, X, phi)
    for _ in range(3):
        phi.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(phi, expect)
    g.close()


def test_refresh_errors(wdf, ctx, mid_data):
    ens, Bs, X = mid_data
    model = wdf.Model(ctx, ens, wdf.KERNEL_GENERIC)
    bg = wdf.Background(model, Bs[0])
    with pytest.raises(ValueError):
        bg.refresh(Bs[0][:, :100])
    pd = wdf.Background(model, pathdep=True)
    with pytest.raises(wdf.WdfError):
        pd.refresh(Bs[0])
    with pytest.raises(wdf.WdfError):
        wdf.Graph(bg)                          # nothing to record


@pytest.mark.parametrize("kname", ["auto", "generic"])
def test_base_value_before_the_first_replay(wdf, ctx, mid_data, kname):
    """A graph that refreshes the summary reads the base value (Appendix B.1
    efficiency reference) from the device from its creation on: before the
    first replay it is the load's value, after a replay the new background's."""
    ens, Bs, X = mid_data
    model = wdf.Model(ctx, ens, _kernel(wdf, kname))
    bg = wdf.Background(model, Bs[0])
    base0 = bg.base_value
    g = wdf.Graph(bg, B=Bs[1])
    assert bg.base_value == base0
    g.launch()
    torch.cuda.synchronize()
    ref = wdf.Background(model, Bs[1])
    assert bg.base_value == ref.base_value != base0
    g.close()
    ref.close()
    bg.close()
