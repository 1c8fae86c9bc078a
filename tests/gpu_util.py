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
