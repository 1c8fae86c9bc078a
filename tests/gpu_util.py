"""Helpers shared by the GPU parity tests."""
import numpy as np

import oracle


def row_scaled_error(got, ref):
    """max over rows of max_i |phi - phi_ref| / max(max_i |phi_ref|, 1e-30); arrays [F][n]."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref).max(axis=0), 1e-30)
    return float((np.abs(got - ref).max(axis=0) / scale).max()) if ref.size else 0.0


def assert_phi_close(got, ref, tol=1e-5, what="phi"):
    err = row_scaled_error(got, ref)
    assert err <= tol, f"{what}: row-scaled error {err:.3e} > {tol:.1e}"
    return err


def leaf_maps(omodel, groups):
    """Oracle leaf index of every group's left (or single) leaf and right leaf (-1)."""
    node, depth, _ = omodel.leaf_info()
    index = {int(n): i for i, n in enumerate(node)}
    left = np.array([index[int(x)] for x in groups["leaf_left"]], np.int64)
    right = np.array([index[int(x)] if x >= 0 else -1 for x in groups["leaf_right"]], np.int64)
    return left, right, depth


def expected_tables(omodel, groups, freq, off, kind):
    """Gather tables the library should hold: t[g][k][p] = s_left[k][p] + s_right[k][p ^ 1]
    from the oracle's Alg. 3 s-vectors (float64)."""
    s = oracle.woodelf_tables(omodel, freq, off, kind)
    left, right, depth = leaf_maps(omodel, groups)
    # start of each leaf's s-block
    sizes = depth.astype(np.int64) << depth.astype(np.int64)
    sstart = np.zeros(depth.size + 1, np.int64)
    sstart[1:] = np.cumsum(sizes)
    dd = groups["depth"].astype(np.int64)
    total = int(np.max(groups["table_offset"] + (dd << dd))) if dd.size else 0
    total = (total + 3) & ~3
    out = np.zeros(total, np.float64)
    for g in range(groups["depth"].size):
        d = int(groups["depth"][g])
        if d == 0:
            continue
        P = 1 << d
        to = int(groups["table_offset"][g])
        sl = s[sstart[left[g]]: sstart[left[g]] + d * P].reshape(d, P)
        t = sl.copy()
        if right[g] >= 0:
            sr = s[sstart[right[g]]: sstart[right[g]] + d * P].reshape(d, P)
            t += sr[:, np.arange(P) ^ 1]
        out[to: to + d * P] = t.ravel()
    return out


def assert_histograms_equal(groups, h, ens, B, trees=None, threads=16, cache=None):
    """Every group's histogram (uint32 counts from the library) equals the
    oracle's per-leaf counts over background B, bit for bit: the left (or
    single) leaf's bins directly, the right leaf's with the last pattern bit
    flipped.  `trees`: only the groups of these trees (the oracle then walks a
    sub-ensemble of them); None: every group.  `cache`: a dict that keeps the
    oracle's counts per (B, trees) across calls.  Returns the groups checked."""
    trees = None if trees is None else sorted(set(int(t) for t in trees))
    sub = ens if trees is None else ens.subset(trees)
    om = oracle.Model(sub)
    key = (id(B), None if trees is None else tuple(trees))
    if cache is not None and key in cache:
        href, off = cache[key]
    else:
        href, off = oracle.histograms(om, B, threads=threads)
        if cache is not None:
            cache[key] = (href, off)
    node, _, ltree = om.leaf_info()
    # the sub-ensemble's node numbers -> the full ensemble's
    src = np.arange(ens.n_trees) if trees is None else np.asarray(trees)
    shift = np.asarray(ens.node_offset)[src] - np.asarray(sub.node_offset)[:-1]
    index = {int(n) + int(shift[t]): i for i, (n, t) in enumerate(zip(node, ltree))}
    keep = set(range(ens.n_trees)) if trees is None else set(trees)
    checked = 0
    for g in range(groups["depth"].size):
        if int(groups["tree"][g]) not in keep:
            continue
        d = int(groups["depth"][g])
        ho = int(groups["hist_offset"][g])
        got = h[ho: ho + (1 << d)].astype(np.uint64)
        li = index[int(groups["leaf_left"][g])]
        np.testing.assert_array_equal(got, href[off[li]: off[li + 1]], err_msg=f"group {g} (left leaf)")
        if groups["leaf_right"][g] >= 0:
            ri = index[int(groups["leaf_right"][g])]
            np.testing.assert_array_equal(got[np.arange(1 << d) ^ 1], href[off[ri]: off[ri + 1]],
                                          err_msg=f"group {g} (right leaf)")
        checked += 1
    return checked


def chunk_trees(groups, chunk_groups):
    """The first and last tree of every histogram chunk (so that a check of
    these trees covers every chunk of the histogram kernel and its edges)."""
    trees = set()
    for c in range(len(chunk_groups) - 1):
        a, b = int(chunk_groups[c]), int(chunk_groups[c + 1])
        trees.add(int(groups["tree"][a]))
        trees.add(int(groups["tree"][b - 1]))
    return sorted(trees)
