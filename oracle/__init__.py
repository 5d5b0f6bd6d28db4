"""CPU oracle for rooted spanning trees -- TEST INFRASTRUCTURE ONLY.

Plain sequential reference implementations of what the GPU library computes
(``oracle.c``, compiled with gcc; the MLP selector's reference is ``mlp.py``
in numpy fp64).  Only the test-suite, the smoke check and the benchmark's CPU
baseline leg may import this package; the HIP library never links or calls
it, and the two share no code.

Functions follow "Beyond BFS: A Comparative Study of Rooted Spanning Tree
Algorithms on GPUs" (arXiv 2603.11645); each C function names its passage.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "_oracle.so")
_lib = None

VERIFY_CODES = {
    0: "ok",
    1: "root is not its own parent",
    2: "parent out of range",
    3: "parent edge not in graph",
    4: "cycle in parent pointers",
    5: "vertex reaches the wrong root",
    6: "invalid designated roots",
}


def build(force: bool = True) -> str:
    """Compile oracle.c into an in-tree shared object with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_bfs.restype = i64
    lib.oracle_bfs.argtypes = [i64, P, P, i32, P, P]
    lib.oracle_uf_forest.restype = i64
    lib.oracle_uf_forest.argtypes = [i64, P, P, P, P, P]
    lib.oracle_dfs_root.restype = ctypes.c_int
    lib.oracle_dfs_root.argtypes = [i64, i64, P, P, P, i32, P]
    lib.oracle_euler_root.restype = ctypes.c_int
    lib.oracle_euler_root.argtypes = [i64, i64, P, P, P, i32, P, P, P]
    lib.oracle_euler_succ.restype = ctypes.c_int
    lib.oracle_euler_succ.argtypes = [i64, i64, P, P, P, P, P, P]
    lib.oracle_list_rank.restype = i64
    lib.oracle_list_rank.argtypes = [i64, P, P]
    lib.oracle_verify_rst.restype = ctypes.c_int
    lib.oracle_verify_rst.argtypes = [i64, P, P, P, P, i32, ctypes.POINTER(i64)]
    lib.oracle_components.restype = i64
    lib.oracle_components.argtypes = [i64, P, P, P]
    lib.oracle_tree_depth.restype = i64
    lib.oracle_tree_depth.argtypes = [i64, P, P]
    lib.oracle_pr_rst.restype = i64
    lib.oracle_pr_rst.argtypes = [i64, P, P, P, i32, i64, P]
    lib.oracle_bcc.restype = i64
    lib.oracle_bcc.argtypes = [i64, P, P, P, P]
    _lib = lib
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _csr(offsets, cols):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    if c.shape[0] == 0:
        c = np.zeros(1, dtype=np.int32)
    return off, c


def _roots(roots):
    r = np.ascontiguousarray(np.atleast_1d(np.asarray(roots, dtype=np.int32)))
    if r.shape[0] == 0:
        return np.zeros(1, dtype=np.int32), 0
    return r, int(r.shape[0])


def bfs(n, offsets, cols, root):
    """Sequential FIFO BFS: (level[n] (-1 unreached), parent[n], eccentricity)."""
    off, c = _csr(offsets, cols)
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    ecc = _load().oracle_bfs(n, _p(off), _p(c), int(root), _p(level), _p(parent))
    if ecc < 0:
        raise ValueError("oracle_bfs: bad root")
    return level, parent, int(ecc)


def uf_forest(n, offsets, cols):
    """Union-find with min-id linking: (label[n], fu[t], fv[t])."""
    off, c = _csr(offsets, cols)
    label = np.empty(n, dtype=np.int32)
    fu = np.empty(max(n, 1), dtype=np.int32)
    fv = np.empty(max(n, 1), dtype=np.int32)
    t = _load().oracle_uf_forest(n, _p(off), _p(c), _p(label), _p(fu), _p(fv))
    if t < 0:
        raise ValueError("oracle_uf_forest failed (%d)" % t)
    return label, fu[:t].copy(), fv[:t].copy()


def components(n, offsets, cols):
    """(number of components, min-id labels)."""
    off, c = _csr(offsets, cols)
    label = np.empty(n, dtype=np.int32)
    k = _load().oracle_components(n, _p(off), _p(c), _p(label))
    if k < 0:
        raise MemoryError
    return int(k), label


def dfs_root(n, fu, fv, roots):
    """Root a forest (edge list) at the designated roots by DFS."""
    fu = np.ascontiguousarray(fu, dtype=np.int32)
    fv = np.ascontiguousarray(fv, dtype=np.int32)
    t = int(fu.shape[0])
    r, nr = _roots(roots)
    parent = np.empty(n, dtype=np.int32)
    rc = _load().oracle_dfs_root(n, t, _p(fu if t else np.zeros(1, np.int32)),
                                 _p(fv if t else np.zeros(1, np.int32)), _p(r), nr, _p(parent))
    if rc:
        raise ValueError("oracle_dfs_root failed (%d)" % rc)
    return parent


def euler_root(n, fu, fv, roots, return_tour: bool = False):
    """Root a forest by the Euler-tour steps (arcs, sort, succ, break, rank, parent)."""
    fu = np.ascontiguousarray(fu, dtype=np.int32)
    fv = np.ascontiguousarray(fv, dtype=np.int32)
    t = int(fu.shape[0])
    r, nr = _roots(roots)
    parent = np.empty(n, dtype=np.int32)
    succ = np.empty(max(2 * t, 1), dtype=np.int32)
    pos = np.empty(max(2 * t, 1), dtype=np.int32)
    z = np.zeros(1, np.int32)
    rc = _load().oracle_euler_root(n, t, _p(fu if t else z), _p(fv if t else z), _p(r), nr,
                                   _p(parent), _p(succ), _p(pos))
    if rc:
        raise ValueError("oracle_euler_root failed (%d)" % rc)
    if return_tour:
        return parent, succ[:2 * t].copy(), pos[:2 * t].copy()
    return parent


def euler_succ(n, src, dst, head, nxt, is_root):
    """Successor array for a given per-vertex out-arc order (twins e, e^1)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    head = np.ascontiguousarray(head, dtype=np.int32)
    nxt = np.ascontiguousarray(nxt, dtype=np.int32)
    is_root = np.ascontiguousarray(is_root, dtype=np.uint8)
    A = int(src.shape[0])
    succ = np.empty(max(A, 1), dtype=np.int32)
    rc = _load().oracle_euler_succ(n, A, _p(src), _p(dst), _p(head), _p(nxt), _p(is_root),
                                   _p(succ))
    if rc:
        raise ValueError("oracle_euler_succ failed (%d)" % rc)
    return succ[:A].copy()


def list_rank(succ):
    """Distance to the tail of every node of a set of lists: (dist, number of lists)."""
    succ = np.ascontiguousarray(succ, dtype=np.int32)
    A = int(succ.shape[0])
    dist = np.empty(max(A, 1), dtype=np.int32)
    k = _load().oracle_list_rank(A, _p(succ if A else np.zeros(1, np.int32)), _p(dist))
    if k < 0:
        raise ValueError("oracle_list_rank: not a set of simple lists (%d)" % k)
    return dist[:A].copy(), int(k)


def verify_rst(n, offsets, cols, parent, roots):
    """(code, bad vertex): code 0 iff parent is a valid RST/forest rooted as required."""
    off, c = _csr(offsets, cols)
    par = np.ascontiguousarray(parent, dtype=np.int32)
    r, nr = _roots(roots)
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_verify_rst(n, _p(off), _p(c), _p(par), _p(r), nr, ctypes.byref(bad))
    if rc == -100:
        raise MemoryError
    return int(rc), int(bad.value)


def tree_depth(parent):
    """(depth[n], max depth): parent steps from every vertex to its tree's root."""
    par = np.ascontiguousarray(parent, dtype=np.int32)
    n = int(par.shape[0])
    depth = np.empty(max(n, 1), dtype=np.int32)
    d = _load().oracle_tree_depth(n, _p(par if n else np.zeros(1, np.int32)), _p(depth))
    if d == -7:
        raise ValueError("oracle_tree_depth: parent out of range")
    if d == -8:
        raise ValueError("oracle_tree_depth: cycle in parent pointers")
    if d < 0:
        raise MemoryError
    return depth[:n].copy(), int(d)


def pr_rst(n, offsets, cols, roots, max_iters: int = -1):
    """Path-Reversal RST (Sec. III-C), sequential: (parent[n], hooking iterations).
    max_iters >= 0 stops after that many iterations (forest as it stands)."""
    off, c = _csr(offsets, cols)
    r, nr = _roots(roots)
    parent = np.empty(n, dtype=np.int32)
    it = _load().oracle_pr_rst(n, _p(off), _p(c), _p(r), nr, int(max_iters), _p(parent))
    if it == -100:
        raise MemoryError
    if it < 0:
        raise ValueError("oracle_pr_rst failed (%d)" % it)
    return parent, int(it)


def bcc(n, offsets, cols):
    """Biconnected components by Hopcroft and Tarjan's depth-first search:
    (arc_label[nnz] int32, -1 on self-loops; articulation[n] uint8; count)."""
    off, c = _csr(offsets, cols)
    nnz = int(off[n])
    label = np.empty(max(nnz, 1), dtype=np.int32)
    art = np.empty(max(n, 1), dtype=np.uint8)
    k = _load().oracle_bcc(n, _p(off), _p(c), _p(label), _p(art))
    if k < 0:
        raise MemoryError
    return label[:nnz].copy(), art[:n].copy(), int(k)


def canonical_labels(label):
    """Each entry's label replaced by the smallest index carrying the same
    label (-1 stays -1): equal partitions give equal arrays, whatever the
    label values."""
    lab = np.asarray(label)
    out = np.full(lab.shape, -1, dtype=np.int64)
    m = lab >= 0
    idx = np.nonzero(m)[0]
    if idx.size:
        _, inv = np.unique(lab[m], return_inverse=True)
        first = np.full(inv.max() + 1, np.iinfo(np.int64).max, dtype=np.int64)
        np.minimum.at(first, inv, idx)
        out[m] = first[inv]
    return out
