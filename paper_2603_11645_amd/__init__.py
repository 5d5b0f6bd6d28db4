"""Rooted spanning trees on AMD Instinct MI355X -- Python binding of librst.

A thin ctypes layer over the C ABI declared in ``include/rst.h``: it only
marshals arguments (device pointers of torch tensors, sizes, the current HIP
stream) and maps status codes to exceptions.  Every step of every method runs
in the library's HIP kernels; there is no CPU fallback, and importing a
function that needs the library fails loudly if ``librst.so`` is not built.

Names follow the C entry points without the ``rst_`` prefix.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librst.so")

RST_OK = 0
RST_E_INVAL = -1
RST_E_NOMEM = -2
RST_E_DEVICE = -3
RST_E_DISCONNECTED = -4
RST_E_RANGE = -5
RST_E_UNSUPPORTED = -6

GCONN_EULER = 0
BFS = 1
AUTO = 2
PR_RST = 3
_METHODS = {"gconn": GCONN_EULER, "gconn_euler": GCONN_EULER, "bfs": BFS, "auto": AUTO,
            "pr_rst": PR_RST, GCONN_EULER: GCONN_EULER, BFS: BFS, AUTO: AUTO, PR_RST: PR_RST}

OPT_VALIDATE = 0
OPT_BFS_LEVELS_PER_SYNC = 1
OPT_BFS_GRID = 2
OPT_RANK_ELEMS_PER_THREAD = 3
OPT_HEAVY_DEGREE = 4
OPT_SWEEP_BLOCK = 5
OPT_BFS_HEAVY_DEGREE = 6
OPT_GRAPHS = 7
OPT_RANK_STRIDE = 8
OPT_HOOK_MODE = 9
OPT_HOOK_SAMPLE = 10

PATH_CROSS_GLOBAL = 1
PATH_RANK_GLOBAL = 2
PATH_CROSS_GROUPS = 4
PATH_RANK_SPARSE = 8
PATH_HOOK_GLOBAL = 16
PATH_HOOK_GIANT = 32

STAGES = ["hook", "compress", "arcs", "succ", "rank", "parent", "bfs", "select"]

# symbols the header declares (checked by the CPU test-suite)
EXPORTS = [
    "rst_create", "rst_destroy", "rst_set_stream", "rst_set_option", "rst_spanning_tree",
    "rst_components", "rst_components_noalloc", "rst_spanning_forest", "rst_bfs",
    "rst_root_forest", "rst_list_rank",
    "rst_spanning_forest_batch", "rst_selector_load", "rst_status_string", "rst_features",
    "rst_feature_stats", "rst_mlp_forward", "rst_mlp_train_step", "rst_get_option",
    "rst_verify", "rst_autotune", "rst_tune_save", "rst_tune_load", "rst_tree_depth",
    "rst_biconnected",
]

N_FEATURES = 8
N_HIDDEN = 64
N_PARAMS = 4866
SELECTOR_MAGIC = b"RSTSEL01"


class RstError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, status_string(code), code))


class rst_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("offset_bytes", ctypes.c_int32),
                ("offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p)]


class rst_batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("vtx_off", ctypes.c_void_p),
                ("arc_off", ctypes.c_void_p), ("roots", ctypes.c_void_p)]


KERNELS = ["hook_tile", "cross", "rank_tile", "link", "rank_walk", "late_hooks", "settle",
           "parent", "rank_words", "hook_sample", "hook_global", "k11"]


class rst_tune_result(ctypes.Structure):
    _fields_ = [("num_options", ctypes.c_int32), ("options", ctypes.c_int32 * 8),
                ("values", ctypes.c_int64 * 8), ("ms_best", ctypes.c_float),
                ("ms_default", ctypes.c_float), ("candidates", ctypes.c_int32),
                ("rejected", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"options": {int(self.options[i]): int(self.values[i]) for i in range(self.num_options)},
                "ms_best": self.ms_best, "ms_default": self.ms_default,
                "candidates": self.candidates, "rejected": self.rejected}


class rst_stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_float), ("ms_stage", ctypes.c_float * 8),
                ("ms_kernel", ctypes.c_float * 12),
                ("hook_rounds", ctypes.c_int64), ("rank_rounds", ctypes.c_int64),
                ("rank_exits", ctypes.c_int64), ("cross_edges", ctypes.c_int64),
                ("bfs_levels", ctypes.c_int64), ("components", ctypes.c_int64),
                ("method_used", ctypes.c_int32), ("paths", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"ms_total": self.ms_total,
                "ms_stage": {STAGES[i]: self.ms_stage[i] for i in range(8)},
                "ms_kernel": {KERNELS[i]: self.ms_kernel[i] for i in range(11)},
                "hook_rounds": self.hook_rounds, "rank_rounds": self.rank_rounds,
                "rank_exits": self.rank_exits, "cross_edges": self.cross_edges,
                "bfs_levels": self.bfs_levels, "components": self.components,
                "method_used": self.method_used, "paths": self.paths}


_lib = None
_lib_lock = threading.Lock()


def load_library(path: Optional[str] = None):
    """Load librst.so (built by ``_build.build()``); raises if it is missing."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError("librst.so not found at %s: build it with "
                               "paper_2603_11645_amd._build.build() (hipcc, gfx950)" % p)
        lib = ctypes.CDLL(p)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        S = ctypes.c_int
        sig = {
            "rst_create": (S, [ctypes.POINTER(P), ctypes.c_int, P]),
            "rst_destroy": (None, [P]),
            "rst_set_stream": (S, [P, P]),
            "rst_set_option": (S, [P, ctypes.c_int, i64]),
            "rst_spanning_tree": (S, [P, ctypes.POINTER(rst_csr), i32, ctypes.c_int, P,
                                      ctypes.POINTER(rst_stats)]),
            "rst_components": (S, [P, ctypes.POINTER(rst_csr), P, ctypes.POINTER(i64)]),
            "rst_components_noalloc": (S, [P, ctypes.POINTER(rst_csr), P, ctypes.POINTER(i64)]),
            "rst_spanning_forest": (S, [P, ctypes.POINTER(rst_csr), P, P, P, ctypes.POINTER(i64)]),
            "rst_bfs": (S, [P, ctypes.POINTER(rst_csr), i32, P, P, ctypes.POINTER(rst_stats)]),
            "rst_root_forest": (S, [P, i64, i64, P, P, P, i32, P]),
            "rst_list_rank": (S, [P, i64, P, P]),
            "rst_spanning_forest_batch": (S, [P, ctypes.POINTER(rst_csr), ctypes.POINTER(rst_batch),
                                              P, P, P, ctypes.POINTER(rst_stats)]),
            "rst_selector_load": (S, [P, P, ctypes.c_size_t]),
            "rst_status_string": (ctypes.c_char_p, [S]),
            "rst_features": (S, [P, ctypes.POINTER(rst_csr), ctypes.POINTER(rst_batch), P]),
            "rst_feature_stats": (S, [P, P, i64, P]),
            "rst_mlp_forward": (S, [P, P, P, P, i64, P, P]),
            "rst_mlp_train_step": (S, [P, P, P, P, P, i64, ctypes.c_float, P, P, P, i64, P,
                                       ctypes.POINTER(ctypes.c_float)]),
            "rst_get_option": (S, [P, ctypes.c_int, ctypes.POINTER(i64)]),
            "rst_verify": (S, [P, ctypes.POINTER(rst_csr), i32, P, ctypes.POINTER(i64),
                               ctypes.POINTER(i64)]),
            "rst_autotune": (S, [P, ctypes.POINTER(rst_csr), i32, ctypes.c_int, i32,
                                 ctypes.POINTER(rst_tune_result)]),
            "rst_tune_save": (S, [P, ctypes.c_char_p]),
            "rst_tree_depth": (S, [P, i64, P, P, ctypes.POINTER(i64)]),
            "rst_biconnected": (S, [P, ctypes.POINTER(rst_csr), P, P, P, ctypes.POINTER(i64)]),
            "rst_tune_load": (S, [P, ctypes.c_char_p, ctypes.POINTER(rst_csr), ctypes.c_int,
                                  ctypes.POINTER(i32)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def status_string(code: int) -> str:
    try:
        return load_library().rst_status_string(code).decode()
    except Exception:  # library missing: still give a readable name
        return {0: "ok", -1: "invalid argument", -2: "out of device memory", -3: "HIP runtime error",
                -4: "graph is disconnected", -5: "out of range", -6: "unsupported"}.get(code, "?")


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_dev(t, dtype, name):
    torch = _torch()
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def make_csr(offsets, cols, n: Optional[int] = None) -> rst_csr:
    torch = _torch()
    if offsets.dtype not in (torch.int32, torch.int64):
        raise ValueError("offsets must be int32 or int64")
    _check_dev(offsets, offsets.dtype, "offsets")
    _check_dev(cols, torch.int32, "cols")
    n = offsets.shape[0] - 1 if n is None else int(n)
    return rst_csr(n, int(cols.shape[0]), 4 if offsets.dtype == torch.int32 else 8,
                   offsets.data_ptr(), cols.data_ptr())


class Context:
    """An rst_ctx bound to a device; each call runs on torch's current stream."""

    def __init__(self, device: Optional[int] = None):
        torch = _torch()
        lib = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            rc = lib.rst_create(ctypes.byref(h), self.device, ctypes.c_void_p(stream))
        if rc != RST_OK:
            raise RstError(rc, "rst_create")
        self._h = h
        self._lib = lib
        self.last_status = RST_OK

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rst_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- plumbing -------------------------------------------------------------
    def _bind(self):
        torch = _torch()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self._lib.rst_set_stream(self._h, ctypes.c_void_p(stream))

    def _call(self, name, *args, ok=(RST_OK,)):
        self._bind()
        rc = getattr(self._lib, name)(self._h, *args)
        self.last_status = rc
        if rc not in ok:
            raise RstError(rc, name)
        return rc

    def set_option(self, opt: int, value: int):
        self._call("rst_set_option", int(opt), int(value))

    def get_option(self, opt: int) -> int:
        v = ctypes.c_int64(0)
        self._call("rst_get_option", int(opt), ctypes.byref(v))
        return int(v.value)

    def verify(self, offsets, cols, root, parent):
        """(failures, first failing vertex or -1) of the device check rst_verify."""
        torch = _torch()
        g = make_csr(offsets, cols)
        _check_dev(parent, torch.int32, "parent")
        bad, first = ctypes.c_int64(0), ctypes.c_int64(0)
        self._call("rst_verify", ctypes.byref(g), int(root), ctypes.c_void_p(parent.data_ptr()),
                   ctypes.byref(bad), ctypes.byref(first))
        return int(bad.value), int(first.value)

    def autotune(self, offsets, cols, root=0, method="gconn", reps: int = 3) -> dict:
        g = make_csr(offsets, cols)
        res = rst_tune_result()
        self._call("rst_autotune", ctypes.byref(g), int(root), _METHODS[method], int(reps),
                   ctypes.byref(res))
        return res.as_dict()

    def tune_save(self, path: str):
        self._call("rst_tune_save", os.fsencode(path))

    def tune_load(self, path: str, offsets=None, cols=None, method="gconn") -> bool:
        """Merge a tuning cache file; apply the entry matching the graph if given."""
        g = make_csr(offsets, cols) if offsets is not None else None
        applied = ctypes.c_int32(0)
        self._call("rst_tune_load", os.fsencode(path), ctypes.byref(g) if g is not None else None,
                   _METHODS[method], ctypes.byref(applied))
        return bool(applied.value)

    # -- entry points ---------------------------------------------------------
    def spanning_tree(self, offsets, cols, root: int = 0, method="gconn", parent=None,
                      stats: bool = False):
        """Parent array (int32, device) of a rooted spanning tree; see rst_spanning_tree."""
        torch = _torch()
        g = make_csr(offsets, cols)
        if parent is None:
            parent = torch.empty(g.n, dtype=torch.int32, device=offsets.device)
        _check_dev(parent, torch.int32, "parent")
        st = rst_stats()
        self._call("rst_spanning_tree", ctypes.byref(g), int(root), _METHODS[method],
                   ctypes.c_void_p(parent.data_ptr()), ctypes.byref(st) if stats else None,
                   ok=(RST_OK, RST_E_DISCONNECTED))
        return (parent, st.as_dict()) if stats else parent

    def components(self, offsets, cols, label=None):
        torch = _torch()
        g = make_csr(offsets, cols)
        if label is None:
            label = torch.empty(g.n, dtype=torch.int32, device=offsets.device)
        _check_dev(label, torch.int32, "label")
        k = ctypes.c_int64(0)
        self._call("rst_components", ctypes.byref(g), ctypes.c_void_p(label.data_ptr()),
                   ctypes.byref(k))
        return label, int(k.value)

    def components_noalloc(self, offsets, cols, label=None):
        """rst_components_noalloc: the labels without device allocation by the
        library (label must be given or is allocated here, by torch)."""
        torch = _torch()
        g = make_csr(offsets, cols)
        if label is None:
            label = torch.empty(g.n, dtype=torch.int32, device=offsets.device)
        _check_dev(label, torch.int32, "label")
        k = ctypes.c_int64(0)
        self._call("rst_components_noalloc", ctypes.byref(g), ctypes.c_void_p(label.data_ptr()),
                   ctypes.byref(k))
        return label, int(k.value)

    def spanning_forest(self, offsets, cols):
        torch = _torch()
        g = make_csr(offsets, cols)
        dev = offsets.device
        label = torch.empty(g.n, dtype=torch.int32, device=dev)
        tu = torch.empty(g.n, dtype=torch.int32, device=dev)
        tv = torch.empty(g.n, dtype=torch.int32, device=dev)
        t = ctypes.c_int64(0)
        self._call("rst_spanning_forest", ctypes.byref(g), ctypes.c_void_p(label.data_ptr()),
                   ctypes.c_void_p(tu.data_ptr()), ctypes.c_void_p(tv.data_ptr()), ctypes.byref(t))
        return label, tu, tv, int(t.value)

    def bfs(self, offsets, cols, root: int = 0, stats: bool = False):
        torch = _torch()
        g = make_csr(offsets, cols)
        dev = offsets.device
        level = torch.empty(g.n, dtype=torch.int32, device=dev)
        parent = torch.empty(g.n, dtype=torch.int32, device=dev)
        st = rst_stats()
        self._call("rst_bfs", ctypes.byref(g), int(root), ctypes.c_void_p(level.data_ptr()),
                   ctypes.c_void_p(parent.data_ptr()), ctypes.byref(st) if stats else None)
        return (level, parent, st.as_dict()) if stats else (level, parent)

    def root_forest(self, n: int, eu, ev, roots, parent=None):
        torch = _torch()
        _check_dev(eu, torch.int32, "eu")
        _check_dev(ev, torch.int32, "ev")
        _check_dev(roots, torch.int32, "roots")
        t = int(eu.shape[0])
        if parent is None:
            parent = torch.empty(n, dtype=torch.int32, device=eu.device)
        self._call("rst_root_forest", int(n), t, ctypes.c_void_p(eu.data_ptr()),
                   ctypes.c_void_p(ev.data_ptr()), ctypes.c_void_p(roots.data_ptr()),
                   int(roots.shape[0]), ctypes.c_void_p(parent.data_ptr()))
        return parent

    def list_rank(self, succ, dist=None):
        torch = _torch()
        _check_dev(succ, torch.int32, "succ")
        A = int(succ.shape[0])
        if dist is None:
            dist = torch.empty(A, dtype=torch.int32, device=succ.device)
        self._call("rst_list_rank", A, ctypes.c_void_p(succ.data_ptr()),
                   ctypes.c_void_p(dist.data_ptr()))
        return dist


    def tree_depth(self, parent, depth=None):
        """(depth int32 device [n], max depth) of the rooted forest `parent`."""
        torch = _torch()
        _check_dev(parent, torch.int32, "parent")
        n = int(parent.shape[0])
        if depth is None:
            depth = torch.empty(n, dtype=torch.int32, device=parent.device)
        _check_dev(depth, torch.int32, "depth")
        mx = ctypes.c_int64(0)
        self._call("rst_tree_depth", n, ctypes.c_void_p(parent.data_ptr()),
                   ctypes.c_void_p(depth.data_ptr()), ctypes.byref(mx))
        return depth, int(mx.value)

    def biconnected(self, offsets, cols, parent):
        """rst_biconnected: (arc_label int32 device [nnz], articulation uint8
        device [n], number of components) from the rooted spanning tree
        `parent` of the graph."""
        torch = _torch()
        g = make_csr(offsets, cols)
        _check_dev(parent, torch.int32, "parent")
        label = torch.empty(max(int(g.nnz), 1), dtype=torch.int32, device=offsets.device)
        art = torch.empty(g.n, dtype=torch.uint8, device=offsets.device)
        k = ctypes.c_int64(0)
        self._call("rst_biconnected", ctypes.byref(g), ctypes.c_void_p(parent.data_ptr()),
                   ctypes.c_void_p(label.data_ptr()), ctypes.c_void_p(art.data_ptr()),
                   ctypes.byref(k))
        return label[:int(g.nnz)], art, int(k.value)

    # -- batches and the selector ---------------------------------------------
    def _batch(self, vtx_off, arc_off, roots):
        torch = _torch()
        _check_dev(vtx_off, torch.int64, "vtx_off")
        _check_dev(arc_off, torch.int64, "arc_off")
        _check_dev(roots, torch.int32, "roots")
        return rst_batch(int(roots.shape[0]), vtx_off.data_ptr(), arc_off.data_ptr(),
                         roots.data_ptr())

    def spanning_forest_batch(self, offsets, cols, vtx_off, arc_off, roots, method=None,
                              stats: bool = False, parent=None, method_out=None):
        """Parents of all packed graphs and the method used per graph (uint8)."""
        torch = _torch()
        g = make_csr(offsets, cols)
        b = self._batch(vtx_off, arc_off, roots)
        dev = offsets.device
        if parent is None:
            parent = torch.empty(g.n, dtype=torch.int32, device=dev)
        else:
            _check_dev(parent, torch.int32, "parent")
            if parent.numel() != g.n:
                raise ValueError("parent must hold n entries")
        if method_out is None:
            mout = torch.empty(b.num_graphs, dtype=torch.uint8, device=dev)
        else:
            _check_dev(method_out, torch.uint8, "method_out")
            if method_out.numel() != b.num_graphs:
                raise ValueError("method_out must hold one entry per graph")
            mout = method_out
        if method is not None:
            _check_dev(method, torch.uint8, "method")
        st = rst_stats()
        self._call("rst_spanning_forest_batch", ctypes.byref(g), ctypes.byref(b),
                   ctypes.c_void_p(_ptr(method)) if method is not None else None,
                   ctypes.c_void_p(parent.data_ptr()), ctypes.c_void_p(mout.data_ptr()),
                   ctypes.byref(st) if stats else None)
        return (parent, mout, st.as_dict()) if stats else (parent, mout)

    def features(self, offsets, cols, vtx_off, arc_off, roots):
        torch = _torch()
        g = make_csr(offsets, cols)
        b = self._batch(vtx_off, arc_off, roots)
        feat = torch.empty((b.num_graphs, N_FEATURES), dtype=torch.float32, device=offsets.device)
        self._call("rst_features", ctypes.byref(g), ctypes.byref(b),
                   ctypes.c_void_p(feat.data_ptr()))
        return feat

    def feature_stats(self, X):
        torch = _torch()
        _check_dev(X, torch.float32, "X")
        norm = torch.empty(2 * N_FEATURES, dtype=torch.float32, device=X.device)
        self._call("rst_feature_stats", ctypes.c_void_p(X.data_ptr()), int(X.shape[0]),
                   ctypes.c_void_p(norm.data_ptr()))
        return norm

    def mlp_forward(self, norm, params, X, logits: bool = True, choice: bool = True):
        torch = _torch()
        for t, nm in ((norm, "norm"), (params, "params"), (X, "X")):
            _check_dev(t, torch.float32, nm)
        B = int(X.shape[0])
        lg = torch.empty((B, 2), dtype=torch.float32, device=X.device) if logits else None
        ch = torch.empty(B, dtype=torch.uint8, device=X.device) if choice else None
        self._call("rst_mlp_forward", ctypes.c_void_p(norm.data_ptr()),
                   ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(X.data_ptr()), B,
                   ctypes.c_void_p(_ptr(lg)) if lg is not None else None,
                   ctypes.c_void_p(_ptr(ch)) if ch is not None else None)
        return lg, ch

    def mlp_train_step(self, norm, params, adam_m, adam_v, step, lr, X, y, w, grad=None):
        """One step; returns the mean weighted loss before the update."""
        torch = _torch()
        loss = ctypes.c_float(0.0)
        self._call("rst_mlp_train_step", ctypes.c_void_p(norm.data_ptr()),
                   ctypes.c_void_p(params.data_ptr()),
                   ctypes.c_void_p(_ptr(adam_m)) if adam_m is not None else None,
                   ctypes.c_void_p(_ptr(adam_v)) if adam_v is not None else None,
                   int(step), float(lr), ctypes.c_void_p(X.data_ptr()),
                   ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                   int(X.shape[0]), ctypes.c_void_p(_ptr(grad)) if grad is not None else None,
                   ctypes.byref(loss))
        return float(loss.value)

    def selector_load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._call("rst_selector_load", ctypes.cast(buf, ctypes.c_void_p), len(blob))

    def selector_load_default(self):
        """Load the selector weights shipped with the package (selector_weights.bin)."""
        with open(os.path.join(_HERE, "selector_weights.bin"), "rb") as f:
            self.selector_load(f.read())


def selector_blob(norm, params) -> bytes:
    """Serialise normalisation (16 floats) and parameters (4866 floats)."""
    import struct
    import numpy as np
    norm = np.asarray(norm, dtype="<f4").reshape(-1)
    params = np.asarray(params, dtype="<f4").reshape(-1)
    assert norm.size == 2 * N_FEATURES and params.size == N_PARAMS
    return SELECTOR_MAGIC + struct.pack("<ii", N_FEATURES, N_HIDDEN) + norm.tobytes() + \
        params.tobytes()


_default = {}


def default_context(device: Optional[int] = None) -> Context:
    torch = _torch()
    d = torch.cuda.current_device() if device is None else int(device)
    ctx = _default.get(d)
    if ctx is None:
        ctx = Context(d)
        _default[d] = ctx
    return ctx


def spanning_tree(offsets, cols, root: int = 0, method="gconn", stats: bool = False):
    return default_context(offsets.device.index).spanning_tree(offsets, cols, root, method,
                                                              stats=stats)


def components(offsets, cols):
    return default_context(offsets.device.index).components(offsets, cols)


def spanning_forest(offsets, cols):
    return default_context(offsets.device.index).spanning_forest(offsets, cols)


def bfs(offsets, cols, root: int = 0, stats: bool = False):
    return default_context(offsets.device.index).bfs(offsets, cols, root, stats=stats)


def root_forest(n, eu, ev, roots):
    return default_context(eu.device.index).root_forest(n, eu, ev, roots)


def list_rank(succ):
    return default_context(succ.device.index).list_rank(succ)
