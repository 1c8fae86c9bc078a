"""Test infrastructure only: Python access to the FP64 CPU oracle.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg import this package.  The GPU library never links, loads or calls it, and
the two share no code.  Every function here marshals numpy arrays into the C
oracle (``woodelf_oracle.c``); the arithmetic is all in C, in double precision.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "woodelf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SHAPLEY = 0
BANZHAF = 1


def build_lib() -> str:
    """Compile the oracle with gcc (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [
        ("n_trees", C.c_int32), ("n_features", C.c_int32),
        ("node_offset", C.c_void_p), ("feature", C.c_void_p), ("left", C.c_void_p),
        ("right", C.c_void_p), ("threshold", C.c_void_p), ("value", C.c_void_p),
        ("default_left", C.c_void_p), ("cover", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        L = C.CDLL(_LIB)
        P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
        L.wo_predict.argtypes = [P, P, I64, I64, P]
        L.wo_leaf_info.argtypes = [P, P, P, P]
        L.wo_leaf_info.restype = I64
        L.wo_leaf_path.argtypes = [P, I64, P, P, P]
        L.wo_patterns.argtypes = [P, P, I64, I64, P]
        L.wo_histograms.argtypes = [P, P, I64, I64, P, P, C.c_int]
        L.wo_wdnf_eval.argtypes = [C.c_int, P, P, C.c_int, P]
        L.wo_wdnf_eval.restype = C.c_double
        L.wo_wdnf_values.argtypes = [C.c_int, C.c_int, P, P, C.c_int, C.c_int, P]
        L.wo_wdnf_bruteforce.argtypes = [C.c_int, C.c_int, P, P, C.c_int, C.c_int, P]
        L.wo_wdnf_iv_values.argtypes = [C.c_int, C.c_int, P, P, C.c_int, C.c_int, P]
        L.wo_wdnf_iv_bruteforce.argtypes = [C.c_int, C.c_int, P, P, C.c_int, C.c_int, P]
        for fn in (L.wo_bg_fourrule, L.wo_bg_walk, L.wo_bg_bruteforce, L.wo_bg_iv_walk, L.wo_bg_iv_bruteforce):
            fn.argtypes = [P, P, I64, I64, P, I64, I64, C.c_int, P, I64, C.c_int]
        L.wo_map_patterns_to_cube.argtypes = [C.c_int, P, P, P, P]
        L.wo_map_patterns_to_cube.restype = I64
        L.wo_woodelf_tables.argtypes = [P, P, P, C.c_int, P]
        L.wo_pd_freq.argtypes = [P, P, P]
        L.wo_pd_bruteforce.argtypes = [P, P, I64, I64, C.c_int, P, I64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Model:
    """Keeps the ensemble arrays alive and a C view of them."""

    def __init__(self, ens):
        self.ens = ens
        self._keep = [
            np.ascontiguousarray(ens.node_offset, np.int64), np.ascontiguousarray(ens.feature, np.int32),
            np.ascontiguousarray(ens.left, np.int32), np.ascontiguousarray(ens.right, np.int32),
            np.ascontiguousarray(ens.threshold, np.float32), np.ascontiguousarray(ens.value, np.float32),
            np.ascontiguousarray(ens.default_left, np.uint8), np.ascontiguousarray(ens.cover, np.float64),
        ]
        k = self._keep
        self.c = _Model(ens.n_trees, ens.n_features, *[a.ctypes.data for a in k])
        self.n_features = ens.n_features

    @property
    def ref(self):
        return C.byref(self.c)

    def leaf_info(self):
        n = lib().wo_leaf_info(self.ref, None, None, None)
        node = np.empty(n, np.int64)
        depth = np.empty(n, np.int32)
        tree = np.empty(n, np.int32)
        lib().wo_leaf_info(self.ref, _ptr(node), _ptr(depth), _ptr(tree))
        return node, depth, tree

    def leaf_path(self, leaf_index: int):
        feats = np.empty(64, np.int32)
        dirs = np.empty(64, np.uint8)
        nodes = np.empty(64, np.int64)
        d = lib().wo_leaf_path(self.ref, int(leaf_index), _ptr(feats), _ptr(dirs), _ptr(nodes))
        return feats[:d].copy(), dirs[:d].copy(), nodes[:d].copy()

    def hist_offsets(self):
        _, depth, _ = self.leaf_info()
        off = np.zeros(depth.size + 1, np.int64)
        off[1:] = np.cumsum(np.left_shift(1, depth.astype(np.int64)))
        return off


def _colmajor(X):
    X = np.ascontiguousarray(X, np.float32)
    assert X.ndim == 2
    return X


def predict(model: Model, X) -> np.ndarray:
    X = _colmajor(X)
    n = X.shape[1]
    out = np.empty(n, np.float64)
    lib().wo_predict(model.ref, _ptr(X), n, n, _ptr(out))
    return out


def patterns(model: Model, X) -> np.ndarray:
    """[n_leaves][n] uint32 decision patterns (Def. Decision Pattern)."""
    X = _colmajor(X)
    n = X.shape[1]
    nl = lib().wo_leaf_info(model.ref, None, None, None)
    out = np.empty((nl, n), np.uint32)
    lib().wo_patterns(model.ref, _ptr(X), n, n, _ptr(out))
    return out


def histograms(model: Model, B, threads=8):
    """(hist uint64[total], offsets int64[n_leaves+1]); hist[off[l]:off[l+1]] are the
    counts of background patterns of leaf l (exact integers, the same for any
    thread count)."""
    B = _colmajor(B)
    off = model.hist_offsets()
    hist = np.empty(int(off[-1]), np.uint64)
    lib().wo_histograms(model.ref, _ptr(B), B.shape[1], B.shape[1], _ptr(hist), _ptr(off), int(threads))
    return hist, off


def _bg(fn, model, Cm, Bm, kind, threads):
    Cm, Bm = _colmajor(Cm), _colmajor(Bm)
    n, m = Cm.shape[1], Bm.shape[1]
    phi = np.zeros((model.n_features, n), np.float64)
    rc = fn(model.ref, _ptr(Cm), n, n, _ptr(Bm), m, m, kind, _ptr(phi), n, threads)
    if rc != 0:
        raise RuntimeError(f"oracle call failed ({rc})")
    return phi


def bg_fourrule(model, Cm, Bm, kind=SHAPLEY, threads=8):
    """Formula trival_bg with the four rules; phi[F][n] in float64."""
    return _bg(lib().wo_bg_fourrule, model, Cm, Bm, kind, threads)


def bg_walk(model, Cm, Bm, kind=SHAPLEY, threads=8):
    """Same values as bg_fourrule, visiting only satisfiable cubes; phi[F][n].
    With fewer rows than threads, each row's mean over the background is summed
    in contiguous background ranges that are then added in order."""
    return _bg(lib().wo_bg_walk, model, Cm, Bm, kind, threads)


def bg_bruteforce(model, Cm, Bm, kind=SHAPLEY, threads=8):
    """Coalition enumeration of the Background-SHAP game (F <= 20); phi[F][n]."""
    return _bg(lib().wo_bg_bruteforce, model, Cm, Bm, kind, threads)


def _bg_iv(fn, model, Cm, Bm, kind, threads):
    Cm, Bm = _colmajor(Cm), _colmajor(Bm)
    n, m = Cm.shape[1], Bm.shape[1]
    F = model.n_features
    iv = np.zeros((F * F, n), np.float64)
    rc = fn(model.ref, _ptr(Cm), n, n, _ptr(Bm), m, m, kind, _ptr(iv), n, threads)
    if rc != 0:
        raise RuntimeError(f"oracle call failed ({rc})")
    return iv.reshape(F, F, n)


def bg_iv_walk(model, Cm, Bm, kind=SHAPLEY, threads=8):
    """Background interaction values by the per-cube formulas (Table table_shap_iv,
    Formula banzhaf_simplified_formula_interactions) over the walk's satisfiable
    cubes; iv[i][j][n] in float64, diagonal 0."""
    return _bg_iv(lib().wo_bg_iv_walk, model, Cm, Bm, kind, threads)


def bg_iv_bruteforce(model, Cm, Bm, kind=SHAPLEY, threads=8):
    """Interaction values from their definitions on the Background-SHAP game (F <= 20)."""
    return _bg_iv(lib().wo_bg_iv_bruteforce, model, Cm, Bm, kind, threads)


def _cubes(cubes):
    """cubes: list of (weight, [signed 1-based literals])."""
    w = np.array([c[0] for c in cubes], np.float64)
    ml = max(1, max(len(c[1]) for c in cubes))
    lits = np.zeros((len(cubes), ml), np.int32)
    for k, (_, ls) in enumerate(cubes):
        lits[k, :len(ls)] = ls
    return w, lits, ml


def wdnf_eval(cubes, x) -> float:
    w, lits, ml = _cubes(cubes)
    xa = np.ascontiguousarray(x, np.uint8)
    return lib().wo_wdnf_eval(len(cubes), _ptr(w), _ptr(lits), ml, _ptr(xa))


def wdnf_values(cubes, n_vars, kind=SHAPLEY) -> np.ndarray:
    w, lits, ml = _cubes(cubes)
    out = np.empty(n_vars, np.float64)
    lib().wo_wdnf_values(n_vars, len(cubes), _ptr(w), _ptr(lits), ml, kind, _ptr(out))
    return out


def wdnf_bruteforce(cubes, n_vars, kind=SHAPLEY) -> np.ndarray:
    w, lits, ml = _cubes(cubes)
    out = np.empty(n_vars, np.float64)
    lib().wo_wdnf_bruteforce(n_vars, len(cubes), _ptr(w), _ptr(lits), ml, kind, _ptr(out))
    return out


def wdnf_iv_values(cubes, n_vars, kind=SHAPLEY) -> np.ndarray:
    """Interaction values of a WDNF by the per-cube formulas; [n_vars][n_vars]."""
    w, lits, ml = _cubes(cubes)
    out = np.empty(n_vars * n_vars, np.float64)
    lib().wo_wdnf_iv_values(n_vars, len(cubes), _ptr(w), _ptr(lits), ml, kind, _ptr(out))
    return out.reshape(n_vars, n_vars)


def wdnf_iv_bruteforce(cubes, n_vars, kind=SHAPLEY) -> np.ndarray:
    """Interaction values of a WDNF from their definitions over all assignments."""
    w, lits, ml = _cubes(cubes)
    out = np.empty(n_vars * n_vars, np.float64)
    if lib().wo_wdnf_iv_bruteforce(n_vars, len(cubes), _ptr(w), _ptr(lits), ml, kind, _ptr(out)) != 0:
        raise ValueError("wdnf_iv_bruteforce needs 2 <= n_vars <= 20")
    return out.reshape(n_vars, n_vars)


def map_patterns_to_cube(d: int):
    """Alg. 2 for a path of d distinct positions: (pc, pb, pos_mask, neg_mask) arrays."""
    n = lib().wo_map_patterns_to_cube(d, None, None, None, None)
    a = [np.empty(n, np.uint32) for _ in range(4)]
    lib().wo_map_patterns_to_cube(d, *[_ptr(x) for x in a])
    return tuple(a)


def woodelf_tables(model: Model, freq, off, kind=SHAPLEY) -> np.ndarray:
    """Alg. 3 steps 2-3: s-vectors of every leaf, position-major, concatenated."""
    _, depth, _ = model.leaf_info()
    total = int(np.sum(depth.astype(np.int64) << depth.astype(np.int64)))
    out = np.empty(total, np.float64)
    fq = np.ascontiguousarray(freq, np.float64)
    lib().wo_woodelf_tables(model.ref, _ptr(fq), _ptr(off), kind, _ptr(out))
    return out


def pd_freq(model: Model) -> tuple[np.ndarray, np.ndarray]:
    off = model.hist_offsets()
    freq = np.empty(int(off[-1]), np.float64)
    if lib().wo_pd_freq(model.ref, _ptr(off), _ptr(freq)) != 0:
        raise RuntimeError("model has no covers")
    return freq, off


def pd_bruteforce(model: Model, Cm, kind=SHAPLEY) -> np.ndarray:
    Cm = _colmajor(Cm)
    n = Cm.shape[1]
    phi = np.zeros((model.n_features, n), np.float64)
    if lib().wo_pd_bruteforce(model.ref, _ptr(Cm), n, n, kind, _ptr(phi), n) != 0:
        raise RuntimeError("oracle call failed")
    return phi


def woodelf_phi(model: Model, Cm, freq, off, kind=SHAPLEY) -> np.ndarray:
    """Alg. 3 step 4 on top of woodelf_tables: values[feature] += s[l][feature][P_c[l]]."""
    Cm = _colmajor(Cm)
    s = woodelf_tables(model, freq, off, kind)
    P = patterns(model, Cm)
    _, depth, _ = model.leaf_info()
    n = Cm.shape[1]
    phi = np.zeros((model.n_features, n), np.float64)
    sb = 0
    for l in range(depth.size):
        d = int(depth[l])
        np_ = 1 << d
        feats, _, _ = model.leaf_path(l)
        for k in range(d):
            vec = s[sb + k * np_: sb + (k + 1) * np_]
            phi[feats[k]] += vec[P[l]]
        sb += d * np_
    return phi
