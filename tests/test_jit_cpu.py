"""CPU checks of the host side (no GPU needed): the generated kernels compile
for gfx950 with hipRTC for the pair and the quad gather and gather what the
layout promises; the host-built coefficient matrices equal the oracle's."""
import os
import re

import numpy as np
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
    pair_adds = len(re.findall(r"f\d+ \+= g\d+\.", pairs))
    quad_adds = len(re.findall(r"f\d+ \+= g\d+\.", quads))
    pair_reads, quad_reads = pairs.count("const vf4 g"), quads.count("const vf4 g")
    # every read's four components are consumed (added to a feature, or kept
    # by an empty asm when zero), in batches of reads issued before their adds
    for src, reads in ((pairs, pair_reads), (quads, quad_reads)):
        used = re.findall(r"f\d+ \+= g\d+\.[xyzw];|KEEP\(g\d+\.[xyzw]\);", src)
        assert len(used) == 4 * reads
        assert "__builtin_amdgcn_sched_barrier(0);" in src
    assert pair_adds <= 10 * 8 * 4 and quad_adds <= 10 * 4 * 5
    assert quad_adds < pair_adds
    assert 0 < pair_reads <= 10 * 8 and 0 < quad_reads <= 10 * 4 * 2  # planes without a first position are skipped
    # with raw-split patterns no pattern is ever flipped in the gather
    assert "^ 1u" not in pairs and "^ 1u" not in quads
    # every feature of the model is written to phi
    for f in range(ens.n_features):
        assert f"phi[{f} * ldphi + row]" in pairs


@pytest.mark.parametrize("which,bound", [("small", 1024), ("mid", 1024), ("uneven", 512)])
def test_histogram_launch_bound(wdf, which, bound):
    """The histogram kernel is compiled for 1024-thread blocks when paths have
    at most six positions and rows at most 32 rank words (95 VGPRs at the
    paper shape), else for 512; its strides come from blockDim, so any
    multiple of 64 threads up to the bound may be launched."""
    src = wdf.specialised_source(synth.WORKLOADS[which].ensemble(), kernel=wdf.KERNEL_SPECIALISED)
    assert f"__launch_bounds__({bound}) void wdf_hist_spec(" in src
    hist = src[:src.index("#define NT ")]
    assert "blockDim.x" in hist and "i += 512" not in hist and "i += 1024" not in hist


def _path_feature_sets(ens):
    """Distinct features on the path of every leaf group (a pair of sibling
    leaves, or a leaf whose sibling is an inner node)."""
    out = []
    for t in range(ens.n_trees):
        sl = ens.tree_slice(t)
        f, l, r = ens.feature[sl], ens.left[sl], ens.right[sl]
        parent = {}
        for i in range(len(f)):
            if f[i] >= 0:
                parent[int(l[i])] = i
                parent[int(r[i])] = i
        for i in range(len(f)):
            if f[i] < 0:
                continue
            for leaf_side in (int(l[i]), int(r[i])):
                if f[leaf_side] >= 0:
                    continue
                if leaf_side == int(r[i]) and f[l[i]] < 0:
                    continue  # the pair was counted with its left leaf
                feats, x = set(), i
                while True:
                    feats.add(int(f[x]))
                    if x not in parent:
                        break
                    x = parent[x]
                out.append(feats)
    return out


def test_multi_stage_kernels_compile(wdf):
    """The 100-tree depth-6 model's generated kernels compile for gfx950 with
    hipRTC: its explain kernel streams the tables through many stages (the
    small models' kernels have one or two), so every per-stage code path of
    the generator is compiled."""
    ens = synth.WORKLOADS["mid"].ensemble()
    src = wdf.specialised_source(ens, compile=True, kernel=wdf.KERNEL_SPECIALISED)
    body = _explain_body(src)
    assert body.count("__syncthreads();") >= 8
    assert body.count("STAGE_PIECE_B(") > 8


def test_explain_stage_copies_and_zero_components(wdf):
    """The explain kernel copies its table stages with buffer loads into LDS
    through a descriptor sized to the explain tables (offsets in scalar
    registers), keeps zero table components with an empty asm (no sink add,
    no sink store), and every copy piece lies inside the tables."""
    ens = synth.WORKLOADS["mid"].ensemble()
    body = _explain_body(wdf.specialised_source(ens, kernel=wdf.KERNEL_SPECIALISED))
    assert "__builtin_amdgcn_make_buffer_rsrc" in body and "STAGE_PIECE_B(" in body
    assert "STAGE_PIECE(" not in body and "global_load_lds" not in body
    assert "sink" not in body and "KEEP(" in body
    tab_bytes = int(re.search(r"#define TAB_BYTES (\d+)", body).group(1))
    nt = int(re.search(r"#define NT (\d+)", wdf.specialised_source(ens, kernel=wdf.KERNEL_SPECIALISED)).group(1))
    # thread t of a chunk reads 16 bytes at byte (stage offset + 16 (c + t)); a
    # chunk is unguarded (all NT threads) or guarded by the threads it covers
    pieces = re.findall(r"(if \(threadIdx\.x < (\d+)u\) )?STAGE_PIECE_B\((\d+)u, d_, (\d+)u\)", body)
    assert pieces
    for guard, lim, ofs, c in pieces:
        ofs, c = int(ofs), int(c)
        threads = int(lim) if guard else nt
        assert ofs % 16 == 0 and c % nt == 0 and 0 < threads <= nt
        assert ofs + 16 * (c + threads) <= tab_bytes


@pytest.mark.parametrize("which", ["small", "edge"])
def test_iv_source_matches_the_layout(wdf, which):
    """The specialised interaction kernels add one pair value per (group,
    feature i at its first occurrence, partner j), i.e. sum over groups of
    d'(d' - 1) adds, from one 16-byte read per four partners and one 4- or
    8-byte read for a last one or two; one kernel per four features; every
    output iv[i][j] is written once per row, the diagonal as 0; the pattern
    kernel stores every group's raw splits at their table slot."""
    ens = synth.WORKLOADS["small"].ensemble() if which == "small" else _edge()
    F = ens.n_features
    src = wdf.iv_source(ens)
    sets = _path_feature_sets(ens)
    assert len(re.findall(r"\ba\d+ \+= [gh]\d+", src)) == sum(len(s) * (len(s) - 1) for s in sets)
    # reads: per (group, first position) with c = d' - 1 partners, c // 4
    # 16-byte reads (one more for c % 4 == 3), and one narrow read for c % 4 in (1, 2)
    wide = sum(len(s) * ((len(s) - 1) // 4 + ((len(s) - 1) % 4 == 3)) for s in sets if len(s) > 1)
    narrow = sum(len(s) * ((len(s) - 1) % 4 in (1, 2)) for s in sets if len(s) > 1)
    assert len(re.findall(r"const vf4 g\d+_\d+ = ", src)) == wide
    assert len(re.findall(r"const (?:vf2|float) h\d+ = ", src)) == narrow
    assert len(re.findall(r"void wdf_iv_spec_\d+\(", src)) == (F + 3) // 4
    assert "void wdf_patterns_spec(" in src
    # one store per group with a path (a single-leaf tree has no pattern),
    # each at its group's 256-byte piece of the row block
    stores = [int(g) for g in re.findall(r"if \(row < ldp\) pb\[(\d+)\] = ", src)]
    assert len(stores) == len(set(stores)) == len(sets)
    assert all(s % 256 == 0 for s in stores)
    # each case stores row i of the matrix, non-temporally: from o + i F ldo,
    # one store per j, the address stepping by ldo
    writes = []
    for blk in src.split("gfp p = (gfp)o + (i64)")[1:]:
        base = int(blk[:blk.index(" ")])
        vals = re.findall(r"__builtin_nontemporal_store\((\S+), p\);", blk[:blk.index("} break;")])
        assert blk.count("p += ldo;") == len(vals) - 1
        writes += [(base + j, v) for j, v in enumerate(vals)]
    assert sorted(int(k) for k, _ in writes) == list(range(F * F))
    for k, v in writes:
        i, j = divmod(int(k), F)
        if i == j:
            assert v == "0.f"
        elif not any(i in s and j in s for s in sets):
            assert v == "0.f"
        else:
            assert v == f"a{j}"


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("values", ["shapley", "banzhaf", "shapley_iv", "banzhaf_iv"])
def test_host_coefficient_matrices_match_the_oracle(wdf, d, values):
    """The library's host-built matrices against the oracle: every pattern pair
    that Alg. 2 maps to a cube, valued by the oracle's per-cube formulas (a
    single-cube WDNF over the d distinct path features); every other pair is
    0 (a position where neither row follows the path makes the cube false)."""
    import oracle
    kind = oracle.BANZHAF if values.startswith("banzhaf") else oracle.SHAPLEY
    iv = values.endswith("_iv")
    code = {"shapley": wdf.SHAPLEY, "banzhaf": wdf.BANZHAF, "shapley_iv": wdf.SHAPLEY_IV,
            "banzhaf_iv": wdf.BANZHAF_IV}[values]
    if iv and d < 2:
        return
    M = wdf.coef_matrix(d, code)
    P = 1 << d
    pairs = [(u, v) for u in range(d) for v in range(u + 1, d)]
    expect = np.zeros((len(pairs) if iv else d, P, P))
    pc, pb, pos, neg = oracle.map_patterns_to_cube(d)
    for c, b, pm, nm in zip(pc, pb, pos, neg):
        lits = [k + 1 for k in range(d) if (pm >> k) & 1] + [-(k + 1) for k in range(d) if (nm >> k) & 1]
        if not lits:
            continue
        if iv:
            vals = oracle.wdnf_iv_values([(1.0, lits)], d, kind)
            for q, (u, v) in enumerate(pairs):
                expect[q, c, b] = vals[u, v]
        else:
            vals = oracle.wdnf_values([(1.0, lits)], d, kind)
            expect[:, c, b] = vals
    np.testing.assert_allclose(M, expect, rtol=1e-12, atol=1e-15)


def _one_tree(feature, left, right, n_features=2):
    """A one-tree ensemble from raw node arrays (node 0 is the root)."""
    n = len(feature)
    return synth.Ensemble(n_features, np.array([0, n], np.int64), np.array(feature, np.int32),
                          np.zeros(n, np.float32), np.array(left, np.int32), np.array(right, np.int32),
                          np.arange(n, dtype=np.float32), np.zeros(n, np.uint8), np.ones(n, np.float64))


def _nan_threshold():
    ens = _one_tree([0, -1, -1], [1, -1, -1], [2, -1, -1])
    ens.threshold[0] = np.nan
    return ens


def test_malformed_models_refused_on_the_host(wdf):
    """Model validation runs on the host and refuses every malformed tree with
    an error code (no GPU needed: the layout behind the generated source is
    the one a model load builds)."""
    ok = _one_tree([0, -1, -1], [1, -1, -1], [2, -1, -1])
    assert "wdf_hist_spec" in wdf.specialised_source(ok)
    cases = {
        "feature out of range": (_one_tree([2, -1, -1], [1, -1, -1], [2, -1, -1]), wdf.E_INVALID_ARG, ">= n_features"),
        "leaf with a child": (_one_tree([0, -1, -1], [1, 2, -1], [2, -1, -1]), wdf.E_INVALID_ARG, "leaf with children"),
        "NaN threshold": (_nan_threshold(), wdf.E_INVALID_ARG, "NaN threshold"),
        "child out of range": (_one_tree([0, -1, -1], [1, -1, -1], [3, -1, -1]), wdf.E_INVALID_ARG, "invalid children"),
        "root as a child": (_one_tree([0, -1, -1], [0, -1, -1], [2, -1, -1]), wdf.E_INVALID_ARG, "invalid children"),
        "same child twice": (_one_tree([0, -1, -1], [1, -1, -1], [1, -1, -1]), wdf.E_INVALID_ARG, "invalid children"),
        "node with two parents": (_one_tree([0, 1, 1, -1, -1], [1, 3, 3, -1, -1], [2, 4, 4, -1, -1]),
                                  wdf.E_INVALID_ARG, "2 parents"),
        # nodes 3 and 4 are each other's parent: one parent each, never reached from the root
        "unreachable cycle": (_one_tree([0, -1, -1, 1, 1, -1, -1], [1, -1, -1, 4, 3, -1, -1],
                                        [2, -1, -1, 5, 6, -1, -1]), wdf.E_INVALID_ARG,
                              "unreachable"),
    }

    def chain(depth):
        # inner nodes 0..depth-1 down the left; leaf `depth` ends the chain,
        # leaves depth+1.. hang off the right of each inner node
        feat = [0] * depth + [-1] * (depth + 1)
        left = list(range(1, depth + 1)) + [-1] * (depth + 1)
        right = [depth + 1 + k for k in range(depth)] + [-1] * (depth + 1)
        return _one_tree(feat, left, right)

    assert "wdf_hist_spec" in wdf.specialised_source(chain(8))  # the path limit itself (8 inner nodes)
    inf = _one_tree([0, 1, -1, -1, -1], [1, 3, -1, -1, -1], [2, 4, -1, -1, -1])
    inf.threshold[:2] = [np.inf, -np.inf]                       # infinite thresholds are valid splits
    assert "wdf_hist_spec" in wdf.specialised_source(inf)
    cases["path deeper than the limit"] = (chain(9), wdf.E_UNSUPPORTED, "more than 8 inner nodes")
    for name, (ens, code, text) in cases.items():
        with pytest.raises(wdf.WdfError) as e:
            wdf.specialised_source(ens)
        assert e.value.code == code, name
        assert text in str(e.value), (name, str(e.value))
    # arrays shorter than node_offset claims never reach the library
    short = _one_tree([0, -1, -1], [1, -1, -1], [2, -1, -1])
    short.node_offset = np.array([0, 4], np.int64)
    with pytest.raises(ValueError):
        wdf.specialised_source(short)


def test_feature_limits(wdf):
    """Models may have up to 65535 features; the specialised kernels, whose
    threshold ranks are packed for every feature, take up to 4096 and refuse
    more with UNSUPPORTED (a load with AUTO then runs the generic kernels);
    65536 features are refused at validation."""
    assert "wdf_hist_spec" in wdf.specialised_source(_one_tree([4095, -1, -1], [1, -1, -1], [2, -1, -1], 4096))
    for F, where in ((4097, "specialised kernels: 4097 features"), (65535, "specialised kernels: 65535 features"),
                     (65536, "65536 features exceeds the limit 65535")):
        with pytest.raises(wdf.WdfError) as e:
            wdf.specialised_source(_one_tree([F - 1, -1, -1], [1, -1, -1], [2, -1, -1], F))
        assert e.value.code == wdf.E_UNSUPPORTED and where in str(e.value), (F, str(e.value))


def test_explain_folds_follow_the_covers(wdf):
    """The explain tables' slot folds (entry I at I ^ (I >> a) ^ (I >> b)) are
    chosen per unit from the model's covers: a model loaded without covers
    gets the same gathers and adds with the default shifts, and with covers a
    share of the units (not all: some keep the default, which is also chosen
    on a tie) takes other shifts."""
    import dataclasses
    ens = synth.WORKLOADS["mid"].ensemble()
    with_cover = _explain_body(wdf.specialised_source(ens))
    without = _explain_body(wdf.specialised_source(dataclasses.replace(ens, cover=None)))
    for a, b in ((with_cover, without),):
        assert a.count("const vf4 g") == b.count("const vf4 g")
        assert len(re.findall(r"f\d+ \+= g\d+\.", a)) == len(re.findall(r"f\d+ \+= g\d+\.", b))
    slots = lambda src: re.findall(r"const u32 z\w+ = [^;]+;", src)
    sw, sn = slots(with_cover), slots(without)
    assert len(sw) > 0 and len(sn) > 0
    differing = len(set(sw) - set(sn))
    assert 0 < differing < len(sw)
