"""Hand-built ensembles for tests: nested tuples -> synth.Ensemble.

A node is ("leaf", value) or ("split", feature, threshold, default_left, left, right)."""
import numpy as np

from paper_2511_09376_amd.synth import Ensemble


def ensemble(trees, n_features, covers=None):
    feats, thrs, ls, rs, vals, dls, covs, offs = [], [], [], [], [], [], [], [0]
    for ti, tree in enumerate(trees):
        nodes = []

        def add(nd):
            i = len(nodes)
            nodes.append(None)
            if nd[0] == "leaf":
                nodes[i] = (-1, 0.0, 0, -1, -1, float(nd[1]))
            else:
                _, f, th, dl, l, r = nd
                li = add(l)
                ri = add(r)
                nodes[i] = (f, th, dl, li, ri, 0.0)
            return i

        add(tree)
        for (f, th, dl, li, ri, v) in nodes:
            feats.append(f); thrs.append(th); dls.append(dl); ls.append(li); rs.append(ri); vals.append(v)
        if covers is not None:
            covs.extend(covers[ti])
        else:
            covs.extend([1.0] * len(nodes))
        offs.append(offs[-1] + len(nodes))
    return Ensemble(n_features, np.array(offs, np.int64), np.array(feats, np.int32),
                    np.array(thrs, np.float32), np.array(ls, np.int32), np.array(rs, np.int32),
                    np.array(vals, np.float32), np.array(dls, np.uint8), np.array(covs, np.float64))


def colmajor(rows):
    """rows: list of per-row feature lists -> float32 [F][n]."""
    return np.ascontiguousarray(np.array(rows, np.float32).T)
