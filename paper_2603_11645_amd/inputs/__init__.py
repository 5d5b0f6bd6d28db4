"""Seeded synthetic input graphs for the rooted-spanning-tree library.

This module builds inputs and nothing else: edge lists from counter-based
random draws (``graphgen.c``), symmetric CSR with sorted, de-duplicated
neighbour lists, and the component restriction / re-connection steps of the
workload recipes, which use scipy's connected-components routine.  It holds
none of the arithmetic of the tree construction under test, so the HIP path
and the CPU oracle can both be fed from it.

Workloads (root 0 unless stated):

* ``C1`` 256x256 4-neighbour grid, vertex ids randomly permuted.
* ``C2`` road-like mesh: 2048x2048 grid, 15% of edges deleted, components
  re-joined by a path over their minimum ids, 0.1% local diagonals.
* ``C3`` R-MAT scale 22, edge factor 16, a=.57 b=.19 c=.19, restricted to the
  largest component, ids relabelled order-preserving.
* ``C4`` random Hamiltonian path over 2^24 vertices plus 0.5% shortcuts of
  span 2..64; 8-byte offsets.
* ``C5`` 4096 graphs, n log-uniform in [1000, 200000], alternating grids
  (10% deletions, re-joined) and R-MAT edge factor 8 (largest component),
  packed into one CSR with offset tables; root of each graph is its local 0.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "_graphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile graphgen.c into an in-tree shared object (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
    lib.gg_rng.restype = u64
    lib.gg_rng.argtypes = [u64, u64, u64]
    lib.gg_permutation.restype = None
    lib.gg_permutation.argtypes = [i64, u64, u64, P]
    lib.gg_grid_edges.restype = i64
    lib.gg_grid_edges.argtypes = [i64, i64, i64, dbl, u64, u64, P, P, P]
    lib.gg_diag_edges.restype = i64
    lib.gg_diag_edges.argtypes = [i64, i64, i64, dbl, u64, u64, P, P]
    lib.gg_rmat_edges.restype = None
    lib.gg_rmat_edges.argtypes = [i32, i64, dbl, dbl, dbl, i64, u64, u64, P, P]
    lib.gg_chain_edges.restype = i64
    lib.gg_chain_edges.argtypes = [i64, dbl, i32, u64, u64, P, P, P]
    lib.gg_build_csr.restype = i64
    lib.gg_build_csr.argtypes = [i64, i64, P, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def rng(seed: int, stream: int, idx: int) -> int:
    """The generator's counter-based 64-bit draw rng(seed, stream, idx)."""
    return int(_load().gg_rng(seed & (2**64 - 1), stream & (2**64 - 1), idx & (2**64 - 1)))


@dataclass
class Graph:
    """Symmetric CSR graph. ``offsets`` is int64 [n+1]; ``cols`` int32 [nnz]."""
    name: str
    n: int
    offsets: np.ndarray
    cols: np.ndarray
    root: int = 0
    offset_bytes: int = 4
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.cols.shape[0])

    @property
    def m(self) -> int:
        """Undirected edges (each stored twice in the CSR)."""
        return self.nnz // 2

    def offsets_typed(self) -> np.ndarray:
        """Offsets in the graph's declared width (int32 or int64)."""
        if self.offset_bytes == 4:
            assert self.nnz < 2**31
            return self.offsets.astype(np.int32)
        return self.offsets.astype(np.int64)

    def edge_list(self):
        """(u, v) arrays with u < v, one entry per undirected edge."""
        deg = np.diff(self.offsets)
        src = np.repeat(np.arange(self.n, dtype=np.int32), deg)
        keep = src < self.cols
        return src[keep], self.cols[keep]


@dataclass
class Batch:
    """G graphs packed into one CSR with global vertex ids."""
    graph: Graph                 # packed CSR (offsets int64, global ids)
    vtx_off: np.ndarray          # int64 [G+1]
    arc_off: np.ndarray          # int64 [G+1]
    roots: np.ndarray            # int32 [G] (global ids)
    kinds: List[str] = field(default_factory=list)

    @property
    def num_graphs(self) -> int:
        return int(self.roots.shape[0])


def csr_from_edges(n: int, eu: np.ndarray, ev: np.ndarray, name: str = "g",
                   root: int = 0, offset_bytes: int = 4) -> Graph:
    """Symmetric CSR: both directions, self-loops dropped, lists sorted/unique."""
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    m = int(eu.shape[0])
    assert ev.shape[0] == m
    if m:
        assert int(eu.min()) >= 0 and int(ev.min()) >= 0
        assert int(eu.max()) < n and int(ev.max()) < n
    off = np.zeros(n + 1, dtype=np.int64)
    cols = np.empty(max(2 * m, 1), dtype=np.int32)
    nnz = _load().gg_build_csr(n, m, _ptr(eu), _ptr(ev), _ptr(off), _ptr(cols))
    if nnz < 0:
        raise MemoryError("gg_build_csr")
    cols = cols[:nnz].copy()
    return Graph(name=name, n=n, offsets=off, cols=cols, root=root, offset_bytes=offset_bytes)


def _components(g: Graph):
    """scipy connected-components labels of a CSR graph (input construction only)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    data = np.ones(g.nnz, dtype=np.float64)
    indptr = g.offsets.astype(np.int32) if g.nnz < 2**31 else g.offsets
    mat = sp.csr_matrix((data, g.cols, indptr), shape=(g.n, g.n))
    # The CSR is symmetric, so its strongly connected components are exactly the
    # undirected components; scipy's strong-component routine avoids building
    # the transpose and is several times faster on large inputs.
    return connected_components(mat, directed=True, connection="strong")


def _rejoin_by_path(n: int, eu: np.ndarray, ev: np.ndarray, name: str) -> Graph:
    """Join components by a path through their minimum ids (ascending)."""
    g = csr_from_edges(n, eu, ev, name=name)
    ncomp, labels = _components(g)
    if ncomp > 1:
        _, first = np.unique(labels, return_index=True)
        mins = np.sort(first).astype(np.int32)
        eu = np.concatenate([eu, mins[:-1]])
        ev = np.concatenate([ev, mins[1:]])
        g = csr_from_edges(n, eu, ev, name=name)
        g.meta["components_rejoined"] = int(ncomp)
    else:
        g.meta["components_rejoined"] = 1
    return g


def _largest_component(n: int, eu: np.ndarray, ev: np.ndarray, name: str) -> Graph:
    """Restrict to the largest component; relabel keeping the original order."""
    g = csr_from_edges(n, eu, ev, name=name)
    ncomp, labels = _components(g)
    sizes = np.bincount(labels, minlength=ncomp)
    big = int(np.argmax(sizes))
    keep = labels == big
    newid = (np.cumsum(keep) - 1).astype(np.int32)
    emask = keep[eu] & (eu != ev)
    eu2, ev2 = newid[eu[emask]], newid[ev[emask]]
    n2 = int(keep.sum())
    del g
    g2 = csr_from_edges(n2, eu2, ev2, name=name)
    g2.meta["n_before_lcc"] = int(n)
    return g2


# ----------------------------------------------------------------------------
# workload recipes
# ----------------------------------------------------------------------------

def grid(rows: int, cols: int, p_del: float = 0.0, seed: int = 1, permute: bool = False,
         limit: Optional[int] = None, name: str = "grid") -> Graph:
    """4-neighbour grid (first ``limit`` cells, row-major); optional id permutation."""
    lib = _load()
    limit = rows * cols if limit is None else limit
    perm = None
    if permute:
        perm = np.empty(limit, dtype=np.int32)
        lib.gg_permutation(limit, seed, 7, _ptr(perm))
    eu = np.empty(2 * limit + 1, dtype=np.int32)
    ev = np.empty(2 * limit + 1, dtype=np.int32)
    m = lib.gg_grid_edges(rows, cols, limit, p_del, seed, 1, _ptr(perm), _ptr(eu), _ptr(ev))
    g = csr_from_edges(limit, eu[:m], ev[:m], name=name)
    if perm is not None:
        g.meta["perm"] = perm
    return g


def grid_permuted(side: int = 256, seed: int = 1) -> Graph:
    g = grid(side, side, 0.0, seed, permute=True, name="grid%d_perm" % side)
    return g


def road_mesh(side: int = 2048, p_del: float = 0.15, p_diag: float = 0.001,
              seed: int = 2) -> Graph:
    lib = _load()
    n = side * side
    eu = np.empty(2 * n + 1, dtype=np.int32)
    ev = np.empty(2 * n + 1, dtype=np.int32)
    m = lib.gg_grid_edges(side, side, n, p_del, seed, 1, None, _ptr(eu), _ptr(ev))
    du = np.empty(2 * n + 1, dtype=np.int32)
    dv = np.empty(2 * n + 1, dtype=np.int32)
    md = lib.gg_diag_edges(side, side, n, p_diag, seed, 2, _ptr(du), _ptr(dv))
    eu = np.concatenate([eu[:m], du[:md]])
    ev = np.concatenate([ev[:m], dv[:md]])
    del du, dv
    g = _rejoin_by_path(n, eu, ev, name="road%d" % side)
    g.meta["diagonals"] = int(md)
    return g


def rmat_lcc(scale: int = 22, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
             c: float = 0.19, seed: int = 3, n_limit: Optional[int] = None) -> Graph:
    lib = _load()
    n = (1 << scale) if n_limit is None else int(n_limit)
    ns = edge_factor * n
    eu = np.empty(ns, dtype=np.int32)
    ev = np.empty(ns, dtype=np.int32)
    lib.gg_rmat_edges(scale, ns, a, b, c, n, seed, 3, _ptr(eu), _ptr(ev))
    return _largest_component(n, eu, ev, name="rmat%d_ef%d_lcc" % (scale, edge_factor))


def long_chain(n: int = 1 << 24, p_short: float = 0.005, max_span: int = 64,
               seed: int = 4, offset_bytes: int = 8) -> Graph:
    lib = _load()
    perm = np.empty(n, dtype=np.int32)
    lib.gg_permutation(n, seed, 9, _ptr(perm))
    eu = np.empty(2 * n, dtype=np.int32)
    ev = np.empty(2 * n, dtype=np.int32)
    m = lib.gg_chain_edges(n, p_short, max_span, seed, 10, _ptr(perm), _ptr(eu), _ptr(ev))
    g = csr_from_edges(n, eu[:m], ev[:m], name="chain%d" % n, offset_bytes=offset_bytes)
    g.meta["perm"] = perm
    return g


def batch_graph_spec(g: int, seed: int = 5, nmin: int = 1000, nmax: int = 200000):
    """(kind, n, per-graph seed) of graph g of the uneven batch."""
    u = (rng(seed, 1, g) >> 11) * (1.0 / 9007199254740992.0)
    n = int(math.floor(math.exp(math.log(nmin) + u * (math.log(nmax) - math.log(nmin)))))
    n = max(nmin, min(nmax, n))
    gseed = rng(seed, 0, g)
    kind = "grid" if g % 2 == 0 else "rmat"
    return kind, n, gseed


def batch_member(g: int, seed: int = 5, nmin: int = 1000, nmax: int = 200000) -> Graph:
    kind, n, gseed = batch_graph_spec(g, seed, nmin, nmax)
    lib = _load()
    if kind == "grid":
        rows = int(math.isqrt(n))
        cols = -(-n // rows)
        eu = np.empty(2 * n + 1, dtype=np.int32)
        ev = np.empty(2 * n + 1, dtype=np.int32)
        m = lib.gg_grid_edges(rows, cols, n, 0.10, gseed, 1, None, _ptr(eu), _ptr(ev))
        return _rejoin_by_path(n, eu[:m].copy(), ev[:m].copy(), name="bgrid%d" % g)
    scale = max(1, int(math.ceil(math.log2(n))))
    ns = 8 * n
    eu = np.empty(ns, dtype=np.int32)
    ev = np.empty(ns, dtype=np.int32)
    lib.gg_rmat_edges(scale, ns, 0.57, 0.19, 0.19, n, gseed, 3, _ptr(eu), _ptr(ev))
    return _largest_component(n, eu, ev, name="brmat%d" % g)


def pack(graphs: List[Graph], kinds: Optional[List[str]] = None) -> Batch:
    """Concatenate CSRs, shifting ids by the vertex offset of each graph."""
    G = len(graphs)
    vtx_off = np.zeros(G + 1, dtype=np.int64)
    arc_off = np.zeros(G + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx_off[i + 1] = vtx_off[i] + g.n
        arc_off[i + 1] = arc_off[i] + g.nnz
    N, NNZ = int(vtx_off[-1]), int(arc_off[-1])
    assert N < 2**31
    offsets = np.empty(N + 1, dtype=np.int64)
    cols = np.empty(NNZ, dtype=np.int32)
    for i, g in enumerate(graphs):
        v0, a0 = int(vtx_off[i]), int(arc_off[i])
        offsets[v0:v0 + g.n] = g.offsets[:-1] + a0
        cols[a0:a0 + g.nnz] = g.cols + np.int32(v0)
    offsets[N] = NNZ
    roots = vtx_off[:-1].astype(np.int32) + np.array([g.root for g in graphs], dtype=np.int32)
    packed = Graph(name="batch%d" % G, n=N, offsets=offsets, cols=cols, root=0,
                   offset_bytes=8 if NNZ >= 2**31 else 4)
    return Batch(graph=packed, vtx_off=vtx_off, arc_off=arc_off, roots=roots,
                 kinds=list(kinds) if kinds else [g.name for g in graphs])


def uneven_batch(G: int = 4096, seed: int = 5, nmin: int = 1000, nmax: int = 200000,
                 workers: int = 0) -> Batch:
    """The uneven batch: G graphs built by ``batch_member`` and packed."""
    if workers and workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            graphs = list(ex.map(batch_member, range(G), [seed] * G, [nmin] * G,
                                 [nmax] * G, chunksize=16))
    else:
        graphs = [batch_member(g, seed, nmin, nmax) for g in range(G)]
    kinds = [batch_graph_spec(g, seed, nmin, nmax)[0] for g in range(G)]
    return pack(graphs, kinds)


def config(name: str) -> Graph:
    """The single-graph workloads C1..C4 at full size."""
    name = name.upper()
    if name == "C1":
        return grid_permuted(256, seed=1)
    if name == "C2":
        return road_mesh(2048, 0.15, 0.001, seed=2)
    if name == "C3":
        return rmat_lcc(22, 16, 0.57, 0.19, 0.19, seed=3)
    if name == "C4":
        return long_chain(1 << 24, 0.005, 64, seed=4, offset_bytes=8)
    raise ValueError("unknown config %r" % name)


# ----------------------------------------------------------------------------
# small shapes for tests
# ----------------------------------------------------------------------------

def path(n: int, perm: Optional[np.ndarray] = None) -> Graph:
    a = np.arange(n - 1, dtype=np.int32)
    eu, ev = a, a + 1
    if perm is not None:
        eu, ev = perm[eu], perm[ev]
    return csr_from_edges(n, eu, ev, name="path%d" % n)


def star(n: int, center: int = 0) -> Graph:
    others = np.array([v for v in range(n) if v != center], dtype=np.int32)
    return csr_from_edges(n, np.full(n - 1, center, dtype=np.int32), others, name="star%d" % n)


def random_tree(n: int, seed: int) -> Graph:
    """Random recursive tree over a seeded permutation of the ids."""
    perm = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed, 21, _ptr(perm))
    par = np.array([rng(seed, 22, i) % i for i in range(1, n)], dtype=np.int64)
    eu = perm[np.arange(1, n)]
    ev = perm[par]
    return csr_from_edges(n, eu, ev, name="tree%d" % n)


def random_graph(n: int, m: int, seed: int, connected: bool = True) -> Graph:
    """Random multigraph with m extra uniform edges; a random tree first if connected."""
    eu_l, ev_l = [], []
    if connected and n > 1:
        t = random_tree(n, seed)
        a, b = t.edge_list()
        eu_l.append(a); ev_l.append(b)
    if m:
        idx = np.arange(m, dtype=np.uint64)
        lib = _load()
        ru = np.array([lib.gg_rng(seed, 31, int(i)) % n for i in idx], dtype=np.int32)
        rv = np.array([lib.gg_rng(seed, 32, int(i)) % n for i in idx], dtype=np.int32)
        eu_l.append(ru); ev_l.append(rv)
    eu = np.concatenate(eu_l) if eu_l else np.zeros(0, np.int32)
    ev = np.concatenate(ev_l) if ev_l else np.zeros(0, np.int32)
    return csr_from_edges(n, eu, ev, name="rand%d_%d" % (n, m))
