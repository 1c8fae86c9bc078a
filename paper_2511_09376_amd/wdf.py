"""Python binding of the C ABI in include/wdf.h (ctypes; argument marshalling only).

Every step of the computation runs in the library's HIP kernels.  PyTorch
provides device memory and streams: matrices are torch CUDA tensors of shape
[n_features, n] (column-major per row: element (feature f, row r) is X[f, r])
and calls enqueue on torch's current stream unless another is given.
The library must be built (``python -m paper_2511_09376_amd.build``); loading
fails loudly when it is not.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwdf.so")

OK = 0
E_INVALID_ARG = -1
E_UNSUPPORTED = -2
E_OOM = -3
E_DEVICE = -4
E_BUSY = -5
E_TIMEOUT = -6
E_COMPILE = -7

SHAPLEY = 0
BANZHAF = 1
SHAPLEY_IV = 2             # interaction values (Def. shap_iv_def)
BANZHAF_IV = 3             # Def. banzhaf_iv_def

KERNEL_AUTO = 0
KERNEL_GENERIC = 1
KERNEL_SPECIALISED = 2
KERNEL_PAIRS = 16          # flag: one table per sibling pair in the specialised gather (no quads)

MAX_DEPTH = 8
SERVE_ONE_PER_LAUNCH = 1
SERVE_START_PAUSED = 2
NOALLOC_SCRATCH_BYTES = 32 << 20   # the library's scratch array (wdf_explain_iv_noalloc)


class WdfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wdf error {code}: {msg}")
        self.code = code


class _ModelDesc(C.Structure):
    _fields_ = [
        ("n_trees", C.c_int32), ("n_features", C.c_int32),
        ("node_offset", C.c_void_p), ("feature", C.c_void_p), ("left", C.c_void_p),
        ("right", C.c_void_p), ("threshold", C.c_void_p), ("value", C.c_void_p),
        ("default_left", C.c_void_p), ("cover", C.c_void_p),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
        ("batches", C.c_uint64), ("rows", C.c_uint64),
        ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double),
        ("busy_ms", C.c_double), ("copy_in_ms", C.c_double), ("explain_ms", C.c_double),
        ("copy_out_ms", C.c_double), ("pack_ms", C.c_double), ("unpack_ms", C.c_double),
        ("active_ms", C.c_double), ("slots", C.c_int), ("batch_rows", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("mem_budget", C.c_size_t), ("max_rows", C.c_int), ("batch_rows", C.c_int),
                ("queue_cap", C.c_int), ("flags", C.c_int), ("copy_threads", C.c_int)]


_lib = None
_live = []   # weak references to open handles, in creation order


def _track(obj):
    _live.append(weakref.ref(obj))


@atexit.register
def _close_all():
    """Release handles newest first while the HIP runtime is still up."""
    for ref in reversed(_live):
        obj = ref()
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass
    _live.clear()


class Tuning(C.Structure):
    _fields_ = [("quads", C.c_int), ("explain_rows", C.c_int), ("hist_rounds", C.c_int), ("hist_threads", C.c_int),
                ("explain_ms", C.c_float * (MAX_DEPTH + 1)), ("explain_rows_ms", C.c_float * 2),
                ("hist_ms", (C.c_float * 9) * 3)]


EXPORTS = [
    "wdf_last_error", "wdf_create", "wdf_destroy", "wdf_model_load", "wdf_model_destroy", "wdf_model_groups",
    "wdf_model_specialised", "wdf_bg_specialised", "wdf_background_load", "wdf_pathdep_load", "wdf_bg_destroy", "wdf_explain",
    "wdf_base_value", "wdf_explain_iv", "wdf_explain_iv_workspace", "wdf_explain_iv_noalloc", "wdf_background_refresh", "wdf_graph_create", "wdf_graph_launch", "wdf_graph_destroy",
    "wdf_debug_patterns", "wdf_debug_histograms", "wdf_debug_tables", "wdf_debug_time_contraction",
    "wdf_debug_specialised_source", "wdf_debug_iv_source", "wdf_debug_coef_matrix", "wdf_model_autotune",
    "wdf_model_set_tuning", "wdf_debug_hist_launch", "wdf_server_create",
    "wdf_server_pause", "wdf_server_submit", "wdf_server_wait", "wdf_server_stats", "wdf_server_destroy",
]


def lib():
    """Load libwdf.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_09376_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I64, I32, I = C.c_void_p, C.c_int64, C.c_int32, C.c_int
        L.wdf_last_error.restype = C.c_char_p
        L.wdf_last_error.argtypes = []
        L.wdf_create.argtypes = [I, C.POINTER(P)]
        L.wdf_destroy.argtypes = [P]
        L.wdf_model_load.argtypes = [P, P, I, C.POINTER(P)]
        L.wdf_model_destroy.argtypes = [P]
        L.wdf_model_groups.argtypes = [P, P, P, P, P, P, P]
        L.wdf_model_groups.restype = I64
        L.wdf_model_specialised.argtypes = [P]
        L.wdf_bg_specialised.argtypes = [P]
        L.wdf_background_load.argtypes = [P, P, I64, I64, I, I, P, C.POINTER(P)]
        L.wdf_pathdep_load.argtypes = [P, I, P, C.POINTER(P)]
        L.wdf_bg_destroy.argtypes = [P]
        L.wdf_explain.argtypes = [P, P, I64, I64, P, I64, P]
        L.wdf_base_value.argtypes = [P, C.POINTER(C.c_double)]
        L.wdf_explain_iv.argtypes = [P, P, I64, I64, P, I64, P, C.c_size_t, P]
        L.wdf_explain_iv_noalloc.argtypes = [P, P, I64, I64, P, I64, P]
        L.wdf_explain_iv_workspace.argtypes = [P, I64]
        L.wdf_explain_iv_workspace.restype = I64
        L.wdf_background_refresh.argtypes = [P, P, I64, P]
        L.wdf_graph_create.argtypes = [P, P, I64, P, I64, I64, P, I64, C.POINTER(P)]
        L.wdf_graph_launch.argtypes = [P, P]
        L.wdf_graph_destroy.argtypes = [P]
        L.wdf_debug_patterns.argtypes = [P, P, I64, I64, P, P]
        L.wdf_debug_histograms.argtypes = [P, P, I64]
        L.wdf_debug_histograms.restype = I64
        L.wdf_debug_time_contraction.argtypes = [P, I, P, C.POINTER(C.c_double), C.POINTER(C.c_float)]
        L.wdf_debug_tables.argtypes = [P, P, I64]
        L.wdf_debug_tables.restype = I64
        L.wdf_debug_specialised_source.argtypes = [P, I, I, P, I64]
        L.wdf_debug_specialised_source.restype = I64
        L.wdf_debug_iv_source.argtypes = [P, P, I64]
        L.wdf_debug_iv_source.restype = I64
        L.wdf_debug_coef_matrix.argtypes = [I, I, P, I64]
        L.wdf_debug_coef_matrix.restype = I64
        L.wdf_model_autotune.argtypes = [P, P, I64, I64, P, I64, I64, P, C.POINTER(Tuning)]
        L.wdf_model_set_tuning.argtypes = [P, C.POINTER(Tuning)]
        L.wdf_debug_hist_launch.argtypes = [P, I64, P, P, I64]
        L.wdf_debug_hist_launch.restype = I64
        L.wdf_server_create.argtypes = [P, C.POINTER(ServerConfig), C.POINTER(P)]
        L.wdf_server_pause.argtypes = [P, I]
        L.wdf_server_submit.argtypes = [P, P, I64, I64, P, C.POINTER(C.c_uint64)]
        L.wdf_server_wait.argtypes = [P, C.c_uint64, I]
        L.wdf_server_stats.argtypes = [P, C.POINTER(Stats)]
        L.wdf_server_destroy.argtypes = [P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise WdfError(rc, lib().wdf_last_error().decode())
    return rc


def _stream_handle(stream, device=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream)


def _on_device(X, device, what):
    if X.device.index != device:
        raise ValueError(f"{what} is on cuda:{X.device.index}, the context on cuda:{device}")


def _colmajor_tensor(X, F, what):
    import torch
    if not isinstance(X, torch.Tensor) or not X.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor of shape [n_features, n]")
    if X.dtype != torch.float32 or X.dim() != 2 or X.shape[0] != F or (X.shape[1] > 1 and X.stride(1) != 1):
        raise ValueError(f"{what}: need float32 [{F}, n] with unit stride along rows, got {tuple(X.shape)} "
                         f"{X.dtype} strides {X.stride()}")
    return X


def _model_desc(ens, with_cover=True):
    # The library reads node_offset[-1] entries of every node array: check the
    # lengths here, where they are known.
    off = np.asarray(ens.node_offset)
    if off.ndim != 1 or off.shape[0] < 2:
        raise ValueError("node_offset must be 1-D with n_trees + 1 >= 2 entries")
    n_nodes = int(off[-1])
    names = ["feature", "left", "right", "threshold", "value", "default_left"]
    if with_cover and getattr(ens, "cover", None) is not None:
        names.append("cover")
    for name in names:
        a = np.asarray(getattr(ens, name))
        if a.ndim != 1 or a.shape[0] != n_nodes:
            raise ValueError(f"{name} has shape {a.shape}, node_offset[-1] = {n_nodes} nodes")
    keep = [np.ascontiguousarray(ens.node_offset, np.int64), np.ascontiguousarray(ens.feature, np.int32),
            np.ascontiguousarray(ens.left, np.int32), np.ascontiguousarray(ens.right, np.int32),
            np.ascontiguousarray(ens.threshold, np.float32), np.ascontiguousarray(ens.value, np.float32),
            np.ascontiguousarray(ens.default_left, np.uint8)]
    cover = getattr(ens, "cover", None)
    cov = np.ascontiguousarray(cover, np.float64) if (with_cover and cover is not None) else None
    if cov is not None:
        keep.append(cov)
    desc = _ModelDesc(int(ens.node_offset.shape[0] - 1), int(ens.n_features), *[a.ctypes.data for a in keep[:7]],
                      cov.ctypes.data if cov is not None else None)
    return desc, keep


def specialised_source(ens, compile: bool = False, kernel: int = KERNEL_SPECIALISED) -> str:
    """Generated source of the model-specialised kernels (no GPU needed);
    with compile=True also compiles it for gfx950 with hipRTC."""
    desc, keep = _model_desc(ens)
    n = _check(lib().wdf_debug_specialised_source(C.byref(desc), kernel, int(compile), None, 0))
    buf = C.create_string_buffer(n + 1)
    _check(lib().wdf_debug_specialised_source(C.byref(desc), kernel, 0, buf, n + 1))
    return buf.value.decode()


def iv_source(ens) -> str:
    """Generated source of the specialised interaction-value kernel (no GPU needed)."""
    desc, keep = _model_desc(ens)
    n = _check(lib().wdf_debug_iv_source(C.byref(desc), None, 0))
    buf = C.create_string_buffer(n + 1)
    _check(lib().wdf_debug_iv_source(C.byref(desc), buf, n + 1))
    return buf.value.decode()


def coef_matrix(dprime: int, values: int = SHAPLEY) -> np.ndarray:
    """The host-built coefficient matrix [positions or position pairs][2^d'][2^d']
    (float64; no GPU needed)."""
    n = _check(lib().wdf_debug_coef_matrix(dprime, values, None, 0))
    out = np.empty(n, np.float64)
    _check(lib().wdf_debug_coef_matrix(dprime, values, out.ctypes.data_as(C.c_void_p), n))
    P = 1 << dprime
    return out.reshape(-1, P, P)


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().wdf_create(device, C.byref(h)))
        self.h = h
        self.device = device
        _track(self)

    def close(self):
        if self.h:
            lib().wdf_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: the module's globals may already be cleared
        # when the interpreter exits)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Model:
    """An ensemble (synth.Ensemble-like object) resident on the context's device."""

    def __init__(self, ctx: Context, ens, kernel: int = KERNEL_AUTO, with_cover: bool = True):
        self.ctx = ctx
        self.n_features = int(ens.n_features)
        desc, keep = _model_desc(ens, with_cover)
        h = C.c_void_p()
        _check(lib().wdf_model_load(ctx.h, C.byref(desc), kernel, C.byref(h)))
        self.h = h
        _track(self)

    @property
    def specialised(self) -> bool:
        return bool(lib().wdf_model_specialised(self.h))

    def autotune(self, B, X, stream=None) -> dict:
        """Time the specialised kernels' configurations on device tensors B
        [n_features, m] and X [n_features, n] and keep the fastest (no summary
        of this model may exist).  Returns the measurements."""
        B = _colmajor_tensor(B, self.n_features, "B")
        X = _colmajor_tensor(X, self.n_features, "X")
        t = Tuning()
        _check(lib().wdf_model_autotune(self.h, C.c_void_p(B.data_ptr()), B.shape[1], B.stride(0),
                                        C.c_void_p(X.data_ptr()), X.shape[1], X.stride(0), _stream_handle(stream),
                                        C.byref(t)))
        ex = {"pairs": float(t.explain_ms[0]), "quads": float(t.explain_ms[MAX_DEPTH])}
        ex.update({f"quads<={q}": float(t.explain_ms[q]) for q in range(1, MAX_DEPTH) if t.explain_ms[q] >= 0})
        return {"gather": "quads" if t.quads else "pairs", "quad_depth": int(t.quads),
                "explain_rows": int(t.explain_rows), "hist_rounds": int(t.hist_rounds),
                "hist_threads": int(t.hist_threads), "explain_ms": ex,
                "explain_rows_ms": {"512": float(t.explain_rows_ms[0]), "256": float(t.explain_rows_ms[1])},
                "hist_ms": {f"{nt}x{r}": float(t.hist_ms[i][r]) for i, nt in enumerate((512, 768, 1024))
                            for r in range(1, 9) if t.hist_ms[i][r] >= 0}}

    def set_tuning(self, tuning: dict):
        """Apply a configuration returned by autotune() (here or in another
        process: the dict round-trips through JSON) without measuring; its
        quad_depth (or gather), explain_rows (each kept when absent),
        hist_threads and hist_rounds are used."""
        t = Tuning()
        if "quad_depth" in tuning:
            t.quads = int(tuning["quad_depth"])
        else:
            t.quads = {"quads": MAX_DEPTH, "pairs": 0, None: -1}[tuning.get("gather")]
        t.explain_rows = int(tuning.get("explain_rows", 0))
        t.hist_threads = int(tuning["hist_threads"])
        t.hist_rounds = int(tuning["hist_rounds"])
        _check(lib().wdf_model_set_tuning(self.h, C.byref(t)))

    def hist_launch(self, m: int) -> dict:
        """Grid of the specialised histogram kernel for m background rows."""
        launch = np.zeros(6, np.int64)
        chunks = _check(lib().wdf_debug_hist_launch(self.h, int(m), launch.ctypes.data, None, 0))
        groups = np.zeros(chunks + 1, np.int64)
        _check(lib().wdf_debug_hist_launch(self.h, int(m), launch.ctypes.data, groups.ctypes.data, chunks + 1))
        keys = ["blocks", "chunks", "threads", "tiles_per_block", "tiles", "tiles_per_wave"]
        out = {k: int(v) for k, v in zip(keys, launch)}
        out["chunk_groups"] = groups
        return out

    def groups(self) -> dict:
        G = _check(lib().wdf_model_groups(self.h, None, None, None, None, None, None))
        a = dict(tree=np.empty(G, np.int32), depth=np.empty(G, np.int32), leaf_left=np.empty(G, np.int64),
                 leaf_right=np.empty(G, np.int64), hist_offset=np.empty(G, np.int64),
                 table_offset=np.empty(G, np.int64))
        _check(lib().wdf_model_groups(self.h, *[x.ctypes.data for x in a.values()]))
        return a

    def patterns(self, X, stream=None):
        """uint32 patterns [n_groups][n] as a torch CUDA tensor (debug / parity)."""
        import torch
        X = _colmajor_tensor(X, self.n_features, "X")
        n = X.shape[1]
        G = _check(lib().wdf_model_groups(self.h, None, None, None, None, None, None))
        out = torch.empty((G, n), dtype=torch.int32, device=X.device)
        _check(lib().wdf_debug_patterns(self.h, C.c_void_p(X.data_ptr()), n, X.stride(0) if n else 0,
                                        C.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().wdf_model_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: the module's globals may already be cleared
        # when the interpreter exits)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Background:
    """A background summary (histograms + tables) for one value kind."""

    def __init__(self, model: Model, B=None, values: int = SHAPLEY, stream=None, pathdep: bool = False):
        self.model = model
        h = C.c_void_p()
        if pathdep:
            _check(lib().wdf_pathdep_load(model.h, values, _stream_handle(stream), C.byref(h)))
            self.m = 0
        else:
            import torch
            if isinstance(B, torch.Tensor):
                B = _colmajor_tensor(B, model.n_features, "B")
                m = B.shape[1]
                _check(lib().wdf_background_load(model.h, C.c_void_p(B.data_ptr()), m, B.stride(0), 1, values,
                                                 _stream_handle(stream), C.byref(h)))
            else:
                Bn = np.ascontiguousarray(B, np.float32)
                if Bn.ndim != 2 or Bn.shape[0] != model.n_features:
                    raise ValueError("B must be [n_features, m]")
                m = Bn.shape[1]
                _check(lib().wdf_background_load(model.h, Bn.ctypes.data_as(C.c_void_p), m, m, 0, values,
                                                 _stream_handle(stream), C.byref(h)))
            self.m = m
        self.h = h
        _track(self)

    @property
    def specialised(self) -> bool:
        """Explained by model-specialised kernels (else the generic ones)."""
        return bool(lib().wdf_bg_specialised(self.h))

    @property
    def base_value(self) -> float:
        v = C.c_double()
        _check(lib().wdf_base_value(self.h, C.byref(v)))
        return v.value

    def explain(self, X, out=None, stream=None):
        """phi [n_features, n] float32 CUDA tensor for consumer rows X [n_features, n]."""
        import torch
        F = self.model.n_features
        X = _colmajor_tensor(X, F, "X")
        dev = self.model.ctx.device
        _on_device(X, dev, "X")
        n = X.shape[1]
        if out is None:
            out = torch.empty((F, n), dtype=torch.float32, device=X.device)
        else:
            out = _colmajor_tensor(out, F, "out")
            _on_device(out, dev, "out")
        ldx = X.stride(0) if n else 0
        ldp = out.stride(0) if n else 0
        with torch.cuda.device(dev):
            _check(lib().wdf_explain(self.h, C.c_void_p(X.data_ptr()), n, ldx, C.c_void_p(out.data_ptr()), ldp,
                                     _stream_handle(stream, dev)))
        return out

    def explain_iv(self, X, out=None, stream=None, workspace=None):
        """Interaction values [n_features, n_features, n] (float32 CUDA tensor,
        symmetric, diagonal 0) of consumer rows X [n_features, n]; the summary
        must have been loaded with SHAPLEY_IV or BANZHAF_IV.  `workspace`: a
        uint8 CUDA tensor of at least iv_workspace_bytes(n) bytes (allocated
        here when None)."""
        import torch
        F = self.model.n_features
        X = _colmajor_tensor(X, F, "X")
        dev = self.model.ctx.device
        _on_device(X, dev, "X")
        n = X.shape[1]
        if out is None:
            out = torch.empty((F, F, n), dtype=torch.float32, device=X.device)
        _on_device(out, dev, "out")
        if out.shape != (F, F, n) or out.dtype != torch.float32 or (n > 1 and out.stride(2) != 1) or \
                out.stride(1) != out.stride(0) // F:
            raise ValueError("out must be float32 [F, F, n] with rows contiguous")
        ldx = X.stride(0) if n else 0
        ldo = out.stride(1) if n else 0
        need = self.iv_workspace_bytes(n)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
        _on_device(workspace, dev, "workspace")
        with torch.cuda.device(dev):
            _check(lib().wdf_explain_iv(self.h, C.c_void_p(X.data_ptr()), n, ldx, C.c_void_p(out.data_ptr()), ldo,
                                        C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                        _stream_handle(stream, dev)))
        return out

    def explain_iv_noalloc(self, X, out, stream=None):
        """explain_iv with the patterns in the library's own scratch array
        (wdf_explain_iv_noalloc): allocates nothing, so `out` [F, F, n] must
        be given.  At most NOALLOC_SCRATCH_BYTES // groups rows per call;
        calls on one device must not overlap."""
        F = self.model.n_features
        X = _colmajor_tensor(X, F, "X")
        dev = self.model.ctx.device
        _on_device(X, dev, "X")
        _on_device(out, dev, "out")
        n = X.shape[1]
        import torch
        if out.shape != (F, F, n) or out.dtype != torch.float32 or (n > 1 and out.stride(2) != 1) or \
                out.stride(1) != out.stride(0) // F:
            raise ValueError("out must be float32 [F, F, n] with rows contiguous")
        ldx = X.stride(0) if n else 0
        ldo = out.stride(1) if n else 0
        with torch.cuda.device(dev):
            _check(lib().wdf_explain_iv_noalloc(self.h, C.c_void_p(X.data_ptr()), n, ldx, C.c_void_p(out.data_ptr()),
                                                ldo, _stream_handle(stream, dev)))
        return out

    def iv_workspace_bytes(self, n: int) -> int:
        return int(_check(lib().wdf_explain_iv_workspace(self.h, n)))

    def refresh(self, B, stream=None):
        """Recompute the summary in place from new background rows B (CUDA
        tensor [n_features, m], the same m); kernel launches only."""
        B = _colmajor_tensor(B, self.model.n_features, "B")
        if self.m and B.shape[1] != self.m:
            raise ValueError(f"refresh needs {self.m} background rows, got {B.shape[1]}")
        _check(lib().wdf_background_refresh(self.h, C.c_void_p(B.data_ptr()), B.stride(0), _stream_handle(stream)))

    def time_contraction(self, reps: int = 20, stream=None) -> tuple:
        """(ms, flops) of one MFMA contraction of this summary, averaged over reps."""
        f, t = C.c_double(), C.c_float()
        _check(lib().wdf_debug_time_contraction(self.h, reps, _stream_handle(stream), C.byref(f), C.byref(t)))
        return float(t.value), float(f.value)

    def histograms(self) -> np.ndarray:
        n = _check(lib().wdf_debug_histograms(self.h, None, 0))
        out = np.empty(n, np.uint32)
        _check(lib().wdf_debug_histograms(self.h, out.ctypes.data_as(C.c_void_p), n))
        return out

    def tables(self) -> np.ndarray:
        n = _check(lib().wdf_debug_tables(self.h, None, 0))
        out = np.empty(n, np.float32)
        _check(lib().wdf_debug_tables(self.h, out.ctypes.data_as(C.c_void_p), n))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().wdf_bg_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: the module's globals may already be cleared
        # when the interpreter exits)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A refresh of `bg` from B (optional) plus an explain of X into phi,
    recorded once into a HIP graph; launch() replays it.  The tensors are
    captured by address: keep them alive and change their contents only."""

    def __init__(self, bg: Background, X=None, phi=None, B=None):
        F = bg.model.n_features
        self.bg = bg
        self._keep = (X, phi, B)
        Bp, ldb = None, 0
        if B is not None:
            B = _colmajor_tensor(B, F, "B")
            if B.shape[1] != bg.m:
                raise ValueError(f"graph refresh needs {bg.m} background rows, got {B.shape[1]}")
            Bp, ldb = C.c_void_p(B.data_ptr()), B.stride(0)
        Xp, Pp, n, ldx, ldp = None, None, 0, 0, 0
        if X is not None:
            X = _colmajor_tensor(X, F, "X")
            phi = _colmajor_tensor(phi, F, "phi")
            n = X.shape[1]
            Xp, Pp, ldx, ldp = C.c_void_p(X.data_ptr()), C.c_void_p(phi.data_ptr()), X.stride(0), phi.stride(0)
        h = C.c_void_p()
        _check(lib().wdf_graph_create(bg.h, Bp, ldb, Xp, n, ldx, Pp, ldp, C.byref(h)))
        self.h = h
        _track(self)

    def launch(self, stream=None):
        _check(lib().wdf_graph_launch(self.h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().wdf_graph_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: the module's globals may already be cleared
        # when the interpreter exits)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching explain server over a resident background summary."""

    def __init__(self, bg: Background, mem_budget: int, max_rows: int = 4096, queue_cap: int = 1 << 16,
                 one_per_launch: bool = False, batch_rows: int = 0, copy_threads: int = 0, paused: bool = False):
        self.bg = bg
        self.n_features = bg.model.n_features
        self._inflight = {}
        cfg = ServerConfig(mem_budget, max_rows, batch_rows, queue_cap,
                           (SERVE_ONE_PER_LAUNCH if one_per_launch else 0) | (SERVE_START_PAUSED if paused else 0),
                           copy_threads)
        h = C.c_void_p()
        _check(lib().wdf_server_create(bg.h, C.byref(cfg), C.byref(h)))
        self.h = h
        _track(self)

    def pause(self, paused: bool = True):
        """Stop (or resume) admitting queued requests into batches."""
        _check(lib().wdf_server_pause(self.h, 1 if paused else 0))

    def submit(self, X: np.ndarray, phi: np.ndarray) -> int:
        """X: float32 [F, n] host array (C order); phi: float32 [F, n] C-order host array that
        receives the values; both must stay alive until wait() returns."""
        if X.dtype != np.float32 or X.ndim != 2 or X.shape[0] != self.n_features or X.strides[1] != 4:
            raise ValueError("X must be float32 [n_features, n] with unit stride along rows")
        if phi.dtype != np.float32 or phi.shape != X.shape or not phi.flags.c_contiguous:
            raise ValueError("phi must be a C-contiguous float32 array shaped like X")
        t = C.c_uint64()
        n = X.shape[1]
        _check(lib().wdf_server_submit(self.h, X.ctypes.data_as(C.c_void_p), n, X.strides[0] // 4,
                                       phi.ctypes.data_as(C.c_void_p), C.byref(t)))
        self._inflight[t.value] = (X, phi)   # the library reads X and writes phi until wait()
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> int:
        rc = lib().wdf_server_wait(self.h, ticket, timeout_ms)
        if rc != E_TIMEOUT:            # any other return releases the ticket
            self._inflight.pop(ticket, None)
        return _check(rc)

    def stats(self) -> Stats:
        s = Stats()
        _check(lib().wdf_server_stats(self.h, C.byref(s)))
        return s

    def close(self):
        if getattr(self, "h", None):
            lib().wdf_server_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: the module's globals may already be cleared
        # when the interpreter exits)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
