"""GPU tests of the serving loop: results identical alone and in a mix, admission, errors."""
import numpy as np
import pytest

from paper_2511_09376_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def served():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_09376_amd import wdf
    w = synth.WORKLOADS["serve"]
    ens = w.ensemble()
    B = w.background(20_000)
    X = w.consumers(6_000)
    ctx = wdf.Context(0)
    model = wdf.Model(ctx, ens)
    assert model.specialised
    bg = wdf.Background(model, torch.from_numpy(B).cuda())
    ref = bg.explain(torch.from_numpy(X).cuda()).cpu().numpy()
    return wdf, ctx, model, bg, X, ref


def _slot_bytes(F, batch_rows):
    return 4 * F * batch_rows * 4


@pytest.mark.parametrize("one_per_launch", [False, True])
def test_mixed_requests_match_explain(served, one_per_launch):
    wdf, ctx, model, bg, X, ref = served
    F = model.n_features
    srv = wdf.Server(bg, mem_budget=3 * _slot_bytes(F, 1024), max_rows=400, batch_rows=1024,
                     one_per_launch=one_per_launch)
    rng = np.random.default_rng(3)
    sizes = rng.integers(1, 400, size=60)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]) % (X.shape[1] - 400)
    jobs = []
    for s, n in zip(starts, sizes):
        xs = np.ascontiguousarray(X[:, s:s + n])
        out = np.empty_like(xs)
        jobs.append((srv.submit(xs, out), s, n, out, xs))
    for t, s, n, out, _ in jobs:
        srv.wait(t, timeout_ms=60_000)
        np.testing.assert_array_equal(out, ref[:, s:s + n])
    st = srv.stats()
    assert st.completed == len(jobs) and st.rows == int(sizes.sum())
    if one_per_launch:
        assert st.batches == len(jobs) and st.slots == 1      # the plain form: one request per launch
    else:
        assert st.batches <= len(jobs) and st.slots == 3
    assert abs(st.busy_ms - (st.copy_in_ms + st.explain_ms + st.copy_out_ms)) <= 1e-6 * max(1.0, st.busy_ms)
    assert st.active_ms > 0
    assert 0 < st.p50_ms <= st.p99_ms <= st.max_ms
    srv.close()


def test_request_alone_equals_request_in_mix(served):
    wdf, ctx, model, bg, X, ref = served
    F = model.n_features
    srv = wdf.Server(bg, mem_budget=2 * _slot_bytes(F, 4096), max_rows=4096, batch_rows=4096)
    a = np.ascontiguousarray(X[:, 100:357])
    alone = np.empty_like(a)
    srv.wait(srv.submit(a, alone))
    outs = []
    for k in range(20):   # the same rows among other requests
        other = np.ascontiguousarray(X[:, 1000 + 50 * k: 1000 + 50 * k + 37 + k])
        o = np.empty_like(other)
        outs.append((srv.submit(other, o), o))
        if k == 9:
            mixed = np.empty_like(a)
            tm = srv.submit(a, mixed)
    for t, _ in outs:
        srv.wait(t)
    srv.wait(tm)
    np.testing.assert_array_equal(alone, mixed)
    np.testing.assert_array_equal(alone, ref[:, 100:357])
    srv.close()


def test_server_errors(served):
    wdf, ctx, model, bg, X, ref = served
    F = model.n_features
    with pytest.raises(wdf.WdfError) as e:
        wdf.Server(bg, mem_budget=_slot_bytes(F, 4096) - 1, max_rows=4096, batch_rows=4096)
    assert e.value.code == wdf.E_INVALID_ARG
    with pytest.raises(wdf.WdfError) as e:       # a batch smaller than the largest request
        wdf.Server(bg, mem_budget=1 << 30, max_rows=4096, batch_rows=1024)
    assert e.value.code == wdf.E_INVALID_ARG
    srv = wdf.Server(bg, mem_budget=_slot_bytes(F, 64), max_rows=64, batch_rows=64)
    big = np.ascontiguousarray(X[:, :65])
    with pytest.raises(wdf.WdfError) as e:
        srv.submit(big, np.empty_like(big))
    assert e.value.code == wdf.E_INVALID_ARG
    with pytest.raises(wdf.WdfError) as e:
        srv.wait(987654321, timeout_ms=10)
    assert e.value.code == wdf.E_INVALID_ARG
    one = np.ascontiguousarray(X[:, :1])
    out = np.empty_like(one)
    srv.wait(srv.submit(one, out), timeout_ms=60_000)
    np.testing.assert_array_equal(out, ref[:, :1])
    srv.close()


def test_batches_larger_than_requests(served):
    """A batch holds many requests: the slot's capacity (batch_rows) is not the
    request cap (max_rows).  Requests queued while the server is paused are
    packed into few batches when it resumes; each result equals wdf_explain."""
    wdf, ctx, model, bg, X, ref = served
    F = model.n_features
    srv = wdf.Server(bg, mem_budget=2 * _slot_bytes(F, 4096), max_rows=1000, batch_rows=4096, paused=True,
                     copy_threads=3)
    jobs = []
    for k in range(12):
        a = 300 * k
        xs = np.ascontiguousarray(X[:, a:a + 900 + k])
        out = np.full_like(xs, np.nan)
        jobs.append((srv.submit(xs, out), a, xs.shape[1], out, xs))
    srv.pause(False)
    for t, a, n, out, _ in jobs:
        srv.wait(t, timeout_ms=60_000)
        np.testing.assert_array_equal(out, ref[:, a:a + n])
    st = srv.stats()
    assert st.batch_rows == 4096 and st.slots == 2
    assert st.batches <= 4        # four requests of 900-911 rows fit one 4096-row batch
    assert st.rows == sum(j[2] for j in jobs)
    srv.close()


def test_wait_timeout_keeps_the_ticket(served):
    """A wait that times out leaves the ticket with the library and the
    request's buffers referenced by the binding; a later blocking wait returns
    the same values as wdf_explain."""
    wdf, ctx, model, bg, X, ref = served
    F = model.n_features
    srv = wdf.Server(bg, mem_budget=_slot_bytes(F, 2048), max_rows=2048, batch_rows=2048, paused=True)
    a = np.ascontiguousarray(X[:, 10:1010])
    b = np.ascontiguousarray(X[:, 2000:2777])
    oa, ob = np.empty_like(a), np.empty_like(b)
    ta, tb = srv.submit(a, oa), srv.submit(b, ob)
    with pytest.raises(wdf.WdfError) as e:      # paused: nothing can have completed
        srv.wait(tb, timeout_ms=0)
    assert e.value.code == wdf.E_TIMEOUT
    with pytest.raises(wdf.WdfError) as e:
        srv.wait(ta, timeout_ms=20)
    assert e.value.code == wdf.E_TIMEOUT
    assert ta in srv._inflight and tb in srv._inflight
    assert srv.stats().completed == 0
    srv.pause(False)
    srv.wait(tb)
    srv.wait(ta)
    assert ta not in srv._inflight and tb not in srv._inflight
    np.testing.assert_array_equal(oa, ref[:, 10:1010])
    np.testing.assert_array_equal(ob, ref[:, 2000:2777])
    with pytest.raises(wdf.WdfError) as e:      # a released ticket is unknown
        srv.wait(ta, timeout_ms=0)
    assert e.value.code == wdf.E_INVALID_ARG
    srv.close()
