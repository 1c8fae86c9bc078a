"""The specialised histogram kernel's tile loop, bit for bit against the oracle.

Each wave of the histogram kernel counts a strided share of its block's
64-row tiles and loads the next tile's threshold ranks while it counts the
current one (Section 7 step (d): exact value counts).  These tests run that
loop the way full-size summaries run it, several tiles per wave with a ragged
last tile, in several launch configurations (block size and grid), and
compare every group's counts with the oracle's per-leaf walk (Def. Decision
Pattern).  The grid arithmetic is the library's own (wdf_debug_hist_launch),
so the asserted tiles per wave are the ones launched.
"""
import numpy as np
import pytest

from paper_2511_09376_amd import synth
from tests.gpu_util import assert_histograms_equal

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

M_ROWS = 300_007        # 4688 tiles, the last one holding 39 rows
CONFIGS = [(1024, 2), (1024, 1), (768, 3), (512, 1)]   # (threads per block, blocks per CU)


@pytest.fixture(scope="module")
def wdf():
    from paper_2511_09376_amd import wdf as w
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return w


@pytest.fixture(scope="module")
def mid(wdf):
    w = synth.WORKLOADS["mid"]
    ens = w.ensemble()
    print(f"[hist loop] mid model, {M_ROWS} background rows", flush=True)
    B = w.background(M_ROWS)
    B2 = w.consumers(M_ROWS)          # a second background of the same size, for the refresh
    ctx = wdf.Context(0)
    model = wdf.Model(ctx, ens, wdf.KERNEL_SPECIALISED)
    return ens, ctx, model, B, B2, {}


@pytest.mark.parametrize("threads,rounds", CONFIGS)
def test_mid_tile_loop_bit_exact(wdf, mid, threads, rounds):
    ens, ctx, model, B, B2, cache = mid
    model.set_tuning({"hist_threads": threads, "hist_rounds": rounds})
    L = model.hist_launch(M_ROWS)
    print(f"[hist loop] {threads} threads x {rounds} rounds: {L['blocks']} blocks x {L['chunks']} chunks, "
          f"{L['tiles_per_block']} tiles per block, up to {L['tiles_per_wave']} per wave", flush=True)
    assert L["threads"] == threads
    assert L["tiles_per_wave"] >= 4
    assert L["tiles"] * 64 > M_ROWS                      # the last tile is ragged
    # blocks cover every tile exactly once
    assert (L["blocks"] - 1) * L["tiles_per_block"] < L["tiles"] <= L["blocks"] * L["tiles_per_block"]
    groups = model.groups()
    Bd = torch.from_numpy(B).cuda()
    bg = wdf.Background(model, Bd)
    n = assert_histograms_equal(groups, bg.histograms(), ens, B, cache=cache)
    assert n == groups["depth"].size
    # the same summary recomputed in place from another background by a
    # replayed graph (the benchmark's launch)
    Bd2 = torch.from_numpy(B2).cuda()
    g = wdf.Graph(bg, B=Bd2)
    g.launch()
    torch.cuda.synchronize()
    assert_histograms_equal(groups, bg.histograms(), ens, B2, cache=cache)
    g.close()
    bg.close()


def test_mid_tile_loop_whole_groups_of_four(wdf, mid):
    """300 004 background rows: a multiple of four, so the quantize kernel
    reads the rows and writes their codes 16 bytes at a time before the same
    tile loop counts them (4688 tiles, the last one holding 36 rows)."""
    ens, ctx, model, B, B2, cache = mid
    m = M_ROWS - 3
    model.set_tuning({"hist_threads": 1024, "hist_rounds": 2})
    L = model.hist_launch(m)
    print(f"[hist loop] {m} rows: {L['blocks']} blocks x {L['chunks']} chunks, "
          f"up to {L['tiles_per_wave']} tiles per wave", flush=True)
    assert m % 4 == 0 and L["tiles"] * 64 > m and L["tiles_per_wave"] >= 4
    Bs = np.ascontiguousarray(B[:, :m])
    bg = wdf.Background(model, torch.from_numpy(Bs).cuda())
    assert assert_histograms_equal(model.groups(), bg.histograms(), ens, Bs) == model.groups()["depth"].size
    bg.close()
