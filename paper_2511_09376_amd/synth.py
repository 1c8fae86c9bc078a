"""Seeded synthetic inputs: tree ensembles and feature matrices.

This module holds no SHAP arithmetic.  It draws the inputs that both the
GPU path and the CPU oracle consume: a decision-tree ensemble in a plain
structure-of-arrays form and column-major float32 feature matrices.  The
shapes and value distributions stand in for the paper's workload (an
XGBoost regressor of 100 depth-6 trees over 127 one-hot-expanded features,
Section 10 Experimental Results); none of the paper's datasets is used.

Ensemble layout (all numpy arrays, one entry per node, trees concatenated):
  node_offset  int64[T+1]  first node of each tree; node 0 of a tree is its root
  feature      int32[N]    split feature of an inner node, -1 for a leaf
  threshold    float32[N]  split threshold; a row goes left iff x < threshold
  left, right  int32[N]    child indices local to the tree, -1 for a leaf
  value        float32[N]  leaf output (0 for inner nodes)
  default_left uint8[N]    direction taken by a missing (NaN) value
  cover        float64[N]  rows of a seeded training-like sample reaching the node
"""
from __future__ import annotations

import concurrent.futures as _fut
import dataclasses
import os

import numpy as np

SEED_BASE = 2511093760
CHUNK_ROWS = 1 << 16


@dataclasses.dataclass
class Ensemble:
    n_features: int
    node_offset: np.ndarray
    feature: np.ndarray
    threshold: np.ndarray
    left: np.ndarray
    right: np.ndarray
    value: np.ndarray
    default_left: np.ndarray
    cover: np.ndarray

    @property
    def n_trees(self) -> int:
        return int(self.node_offset.shape[0] - 1)

    def tree_slice(self, t: int) -> slice:
        return slice(int(self.node_offset[t]), int(self.node_offset[t + 1]))

    def subset(self, trees) -> "Ensemble":
        """A new ensemble holding only the listed trees (in that order)."""
        parts = [self.tree_slice(int(t)) for t in trees]
        sizes = [s.stop - s.start for s in parts]
        off = np.zeros(len(parts) + 1, np.int64)
        off[1:] = np.cumsum(sizes)
        cat = lambda a: np.concatenate([a[s] for s in parts]) if parts else a[:0]
        return Ensemble(self.n_features, off, cat(self.feature), cat(self.threshold),
                        cat(self.left), cat(self.right), cat(self.value),
                        cat(self.default_left), cat(self.cover))


# ----------------------------------------------------------------------------
# Feature distributions
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class DataSpec:
    """Column kinds and missing-value rate of a synthetic feature matrix."""
    n_features: int
    mixed: bool          # False: all columns iid N(0,1)
    nan_rate: float

    def column_kinds(self) -> np.ndarray:
        """0 = N(0,1), 1 = LogNormal(0,1), 2 = Bernoulli(0.3), 3 = Poisson(3)."""
        k = np.zeros(self.n_features, np.int8)
        if not self.mixed:
            return k
        f = self.n_features
        # proportions of the 127-column mix: 43 normal, 42 log-normal,
        # 21 binary (one-hot-like), 21 small counts
        b1 = round(43 * f / 127)
        b2 = b1 + round(42 * f / 127)
        b3 = b2 + round(21 * f / 127)
        k[b1:b2] = 1
        k[b2:b3] = 2
        k[b3:] = 3
        return k


def _fill_block(spec: DataSpec, kinds: np.ndarray, rng: np.random.Generator,
                out: np.ndarray) -> None:
    """Fill out[F][r] (float32) with one block of rows."""
    r = out.shape[1]
    for f in range(spec.n_features):
        kind = kinds[f]
        if kind == 0:
            col = rng.standard_normal(r, dtype=np.float32)
        elif kind == 1:
            col = np.exp(rng.standard_normal(r, dtype=np.float32))
        elif kind == 2:
            col = (rng.random(r, dtype=np.float32) < 0.3).astype(np.float32)
        else:
            col = rng.poisson(3.0, r).astype(np.float32)
        out[f, :] = col
    if spec.nan_rate > 0:
        mask = rng.random((spec.n_features, r), dtype=np.float32) < spec.nan_rate
        out[mask] = np.nan


def make_matrix(spec: DataSpec, n: int, seed: np.random.SeedSequence | int,
                out: np.ndarray | None = None, threads: int | None = None) -> np.ndarray:
    """Column-major float32 matrix [F][n]; row chunks draw from child seeds, so
    any row's values depend only on (seed, row) and not on thread count."""
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    n_chunks = (n + CHUNK_ROWS - 1) // CHUNK_ROWS
    children = ss.spawn(n_chunks)
    if out is None:
        out = np.empty((spec.n_features, n), np.float32)
    kinds = spec.column_kinds()

    def work(ci: int) -> None:
        lo = ci * CHUNK_ROWS
        hi = min(n, lo + CHUNK_ROWS)
        blk = np.empty((spec.n_features, hi - lo), np.float32)
        _fill_block(spec, kinds, np.random.default_rng(children[ci]), blk)
        out[:, lo:hi] = blk

    threads = threads or min(16, os.cpu_count() or 1)
    if n_chunks <= 1 or threads <= 1:
        for ci in range(n_chunks):
            work(ci)
    else:
        with _fut.ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(n_chunks)))
    return out


def matrix_rows(spec: DataSpec, n: int, seed: np.random.SeedSequence | int,
                rows: np.ndarray) -> np.ndarray:
    """Rows `rows` of make_matrix(spec, n, seed), regenerated without the rest."""
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    n_chunks = (n + CHUNK_ROWS - 1) // CHUNK_ROWS
    children = ss.spawn(n_chunks)
    kinds = spec.column_kinds()
    rows = np.asarray(rows, np.int64)
    out = np.empty((spec.n_features, rows.size), np.float32)
    for ci in np.unique(rows // CHUNK_ROWS):
        lo = int(ci) * CHUNK_ROWS
        hi = min(n, lo + CHUNK_ROWS)
        blk = np.empty((spec.n_features, hi - lo), np.float32)
        _fill_block(spec, kinds, np.random.default_rng(children[int(ci)]), blk)
        sel = np.nonzero(rows // CHUNK_ROWS == ci)[0]
        out[:, sel] = blk[:, rows[sel] - lo]
    return out


# ----------------------------------------------------------------------------
# Ensembles
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ModelSpec:
    n_trees: int
    depth_lo: int
    depth_hi: int          # depth drawn uniformly from [depth_lo, depth_hi]
    prune_p: float         # probability that an inner node below the root becomes a leaf
    n_features: int
    feature_pool: int = 0  # >0: draw split features from the first `pool` columns only


def _tree_shape(depth: int, prune_p: float, rng: np.random.Generator):
    """BFS list of (parent, is_left, node_depth, is_leaf)."""
    nodes = [(-1, False, 0, depth == 0)]
    head = 0
    while head < len(nodes):
        parent, is_left, d, is_leaf = nodes[head]
        if not is_leaf:
            for side in (True, False):
                cd = d + 1
                leaf = cd >= depth or (prune_p > 0 and rng.random() < prune_p)
                nodes.append((head, side, cd, leaf))
        head += 1
    return nodes


def make_ensemble(mspec: ModelSpec, dspec: DataSpec, seed: np.random.SeedSequence | int,
                  sample_rows: int = 4096) -> Ensemble:
    """Random trees: features uniform over the columns, thresholds at a uniform
    quantile in [0.05, 0.95] of a seeded sample of the column's non-missing
    values, leaf values N(0,1), default directions Bernoulli(0.5) when the
    data have missing values (else left), covers counted on the sample."""
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    s_model, s_sample = ss.spawn(2)
    rng = np.random.default_rng(s_model)
    sample = make_matrix(dspec, sample_rows, s_sample)
    pool = mspec.feature_pool or mspec.n_features
    feats, thrs, lefts, rights, vals, dls, covers, offs = [], [], [], [], [], [], [], [0]
    for _ in range(mspec.n_trees):
        depth = int(rng.integers(mspec.depth_lo, mspec.depth_hi + 1))
        shape = _tree_shape(depth, mspec.prune_p, rng)
        nn = len(shape)
        f = np.full(nn, -1, np.int32)
        th = np.zeros(nn, np.float32)
        le = np.full(nn, -1, np.int32)
        ri = np.full(nn, -1, np.int32)
        va = np.zeros(nn, np.float32)
        dl = np.zeros(nn, np.uint8)
        for i, (parent, is_left, _, is_leaf) in enumerate(shape):
            if parent >= 0:
                if is_left:
                    le[parent] = i
                else:
                    ri[parent] = i
            if is_leaf:
                va[i] = np.float32(rng.standard_normal())
            else:
                fi = int(rng.integers(0, pool))
                col = sample[fi]
                col = col[~np.isnan(col)]
                q = float(rng.uniform(0.05, 0.95))
                f[i] = fi
                th[i] = np.float32(np.quantile(col.astype(np.float64), q))
                dl[i] = np.uint8(rng.random() < 0.5) if dspec.nan_rate > 0 else np.uint8(1)
        # covers: route the sample through the tree (missing -> default side)
        cov = np.zeros(nn, np.float64)
        where = np.zeros(sample_rows, np.int64)
        active = np.ones(sample_rows, bool)
        cov[0] = sample_rows
        for _ in range(depth + 1):
            idx = np.nonzero(active)[0]
            if idx.size == 0:
                break
            nodes_here = where[idx]
            inner = f[nodes_here] >= 0
            idx, nodes_here = idx[inner], nodes_here[inner]
            active[:] = False
            if idx.size == 0:
                break
            x = sample[f[nodes_here], idx]
            go_left = np.where(np.isnan(x), dl[nodes_here] == 1, x < th[nodes_here])
            child = np.where(go_left, le[nodes_here], ri[nodes_here])
            np.add.at(cov, child, 1.0)
            where[idx] = child
            active[idx] = True
        feats.append(f); thrs.append(th); lefts.append(le); rights.append(ri)
        vals.append(va); dls.append(dl); covers.append(cov)
        offs.append(offs[-1] + nn)
    return Ensemble(mspec.n_features, np.asarray(offs, np.int64),
                    np.concatenate(feats), np.concatenate(thrs), np.concatenate(lefts),
                    np.concatenate(rights), np.concatenate(vals), np.concatenate(dls),
                    np.concatenate(covers))


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    config_id: int
    model: ModelSpec
    data: DataSpec
    n_consumers: int
    n_background: int

    def seeds(self):
        """Independent seed streams: model, consumers, background, requests."""
        return np.random.SeedSequence(SEED_BASE + self.config_id).spawn(4)

    def ensemble(self) -> Ensemble:
        return make_ensemble(self.model, self.data, self.seeds()[0])

    def consumers(self, n: int | None = None, out=None) -> np.ndarray:
        return make_matrix(self.data, n or self.n_consumers, self.seeds()[1], out=out)

    def background(self, m: int | None = None, out=None) -> np.ndarray:
        return make_matrix(self.data, m or self.n_background, self.seeds()[2], out=out)

    def consumer_rows(self, rows) -> np.ndarray:
        return matrix_rows(self.data, self.n_consumers, self.seeds()[1], rows)


_F = 127
_MIX = DataSpec(_F, mixed=True, nan_rate=0.05)

WORKLOADS = {
    # 10 complete depth-4 trees on 8 iid N(0,1) features, 100 x 100 rows
    "small": Workload("small", 1, ModelSpec(10, 4, 4, 0.0, 8), DataSpec(8, False, 0.0), 100, 100),
    # 100 complete depth-6 trees on the 127-column mix, 100k x 100k rows
    "mid": Workload("mid", 2, ModelSpec(100, 6, 6, 0.0, _F), _MIX, 100_000, 100_000),
    # 500 pruned trees with depth uniform in 3..8, 1M x 1M rows
    "uneven": Workload("uneven", 3, ModelSpec(500, 3, 8, 0.15, _F), _MIX, 1_000_000, 1_000_000),
    # serving: the mid model and background, requests drawn separately
    "serve": Workload("serve", 4, ModelSpec(100, 6, 6, 0.0, _F), _MIX, 100_000, 100_000),
    # paper-scale shape: 3M consumers x 5M background rows
    "paper": Workload("paper", 5, ModelSpec(100, 6, 6, 0.0, _F), _MIX, 3_000_000, 5_000_000),
}


def request_sizes(n_req: int, seed: np.random.SeedSequence, max_rows: int = 4096) -> np.ndarray:
    """Log-uniform request sizes floor(exp(U(0, ln(max_rows+1)))) clipped to [1, max_rows]."""
    rng = np.random.default_rng(seed)
    s = np.floor(np.exp(rng.uniform(0.0, np.log(max_rows + 1), n_req))).astype(np.int64)
    return np.clip(s, 1, max_rows)
