"""The interaction-value entry point that allocates nothing
(wdf_explain_iv_noalloc: the rows' patterns in the library's own scratch
array) against the one that takes a caller workspace (wdf_explain_iv).  Both
run the same kernels, so the values must agree bit for bit, on two calls in a
row, the second with fewer and different rows (the scratch still holds the
first call's patterns).  Above the scratch's row limit the call fails with a
clear error and launches nothing."""
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


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


CASES = [("small", "specialised"), ("small", "generic"), ("mid", "generic")]


@pytest.mark.parametrize("workload,kname", CASES)
def test_noalloc_equals_workspace_entry(wdf, workload, kname):
    w = synth.WORKLOADS[workload]
    ens = w.ensemble()
    ctx = wdf.Context(0)
    kernel = wdf.KERNEL_SPECIALISED if kname == "specialised" else wdf.KERNEL_GENERIC
    model = wdf.Model(ctx, ens, kernel)
    bg = wdf.Background(model, _cuda(w.background()), values=wdf.SHAPLEY_IV)
    assert bg.specialised == (kname == "specialised")
    F = ens.n_features
    G = model.groups()["depth"].size
    n_max = wdf.NOALLOC_SCRATCH_BYTES // G // 512 * 512  # rows of the pattern workspace come in blocks of 512
    n1 = min(n_max, 12000)
    X = w.consumers(n1 + 4000)
    print(f"[no-alloc] {workload} {kname}: {G} groups, at most {n_max} rows per call", flush=True)
    # first call at up to the limit, the second smaller and on other rows
    for a, n in ((0, n1), (n1 + 123, 777)):
        Xd = _cuda(X[:, a:a + n])
        ws = torch.empty(bg.iv_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        ref = bg.explain_iv(Xd, workspace=ws)
        out = torch.full((F, F, n), float("nan"), dtype=torch.float32, device="cuda")
        bg.explain_iv_noalloc(Xd, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"rows [{a}, {a + n}): the two entry points differ"
    # one row above the limit: refused before any launch
    n_big = n_max + 1
    Xb = torch.zeros((F, n_big), dtype=torch.float32, device="cuda")
    ob = torch.zeros((F, F, n_big), dtype=torch.float32, device="cuda")
    with pytest.raises(wdf.WdfError) as e:
        bg.explain_iv_noalloc(Xb, ob)
    assert e.value.code == wdf.E_INVALID_ARG and "scratch" in str(e.value)
    assert int(torch.count_nonzero(ob)) == 0
