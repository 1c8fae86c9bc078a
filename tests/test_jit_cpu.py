"""CPU checks of the model-specialised kernels: the generated source compiles
for gfx950 with hipRTC (no GPU needed) for the pair and the quad gather, and
the gather reads what the layout promises."""
import os
import re

import pytest

from paper_2511_09376_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def wdf():
    from paper_2511_09376_amd import wdf as w
    if not os.path.exists(w.LIB_PATH):
        pytest.skip("libwdf.so not built")
    return w


def _edge():
    from tests.test_gpu_parity import _edge_ensemble
    return _edge_ensemble()


def _explain_body(src):
    return src[src.index("#define EXPLAIN_NAME"):]


@pytest.mark.parametrize("which", ["small", "edge"])
@pytest.mark.parametrize("quads", [False, True])
def test_specialised_source_compiles(wdf, which, quads):
    ens = synth.WORKLOADS["small"].ensemble() if which == "small" else _edge()
    kernel = wdf.KERNEL_SPECIALISED | (0 if quads else wdf.KERNEL_PAIRS)
    src = wdf.specialised_source(ens, compile=True, kernel=kernel)
    assert "wdf_hist_spec" in src and ("wdf_explain_quads" if quads else "wdf_explain_pairs") in src


def test_gather_counts_match_the_layout(wdf):
    """10 complete depth-4 trees: 8 pair groups of depth 4 per tree.  Pairs add
    one value per (group, first-occurrence position); a quad adds one per
    first-occurrence position of its two pairs, shared prefix positions once.
    Each 16-byte read returns four values of an entry: one read per pair table
    (4 values), two per quad table (5 values)."""
    ens = synth.WORKLOADS["small"].ensemble()
    pairs = _explain_body(wdf.specialised_source(ens, kernel=wdf.KERNEL_SPECIALISED | wdf.KERNEL_PAIRS))
    quads = _explain_body(wdf.specialised_source(ens, kernel=wdf.KERNEL_SPECIALISED))
    pair_adds, quad_adds = len(re.findall(r"\+= a\.", pairs)), len(re.findall(r"\+= a\.", quads))
    pair_reads, quad_reads = pairs.count("vf4 a = t["), quads.count("vf4 a = t[")
    assert pair_adds <= 10 * 8 * 4 and quad_adds <= 10 * 4 * 5
    assert quad_adds < pair_adds
    assert 0 < pair_reads <= 10 * 8 and 0 < quad_reads <= 10 * 4 * 2  # planes without a first position are skipped
    # with raw-split patterns no pattern is ever flipped in the gather
    assert "^ 1u" not in pairs and "^ 1u" not in quads
    # every feature of the model is written to phi
    for f in range(ens.n_features):
        assert f"phi[{f} * ldphi + row]" in pairs
