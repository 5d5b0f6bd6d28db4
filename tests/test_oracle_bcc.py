"""CPU pins of the biconnected-components oracle (Hopcroft and Tarjan's
depth-first method; the downstream use of an RST named in Sec. I and at the
opening of Sec. IV).

The oracle is checked against what the definitions fix, not against itself:
closed forms (paths, cycles, stars, complete graphs, two triangles sharing a
vertex, a barbell), a hand-worked graph (tests/golden/bcc_example10.json),
multigraph and self-loop cases, and brute force on random small graphs: two
edges share a component exactly when they are equal or lie on a common simple
cycle (all simple cycles enumerated), and a vertex is an articulation point
exactly when two of its neighbours are connected in G but not in G - v.
Partitions are compared through canonical labels (each arc's label replaced
by the smallest arc index with the same label)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr(n, edges):
    """Symmetric CSR keeping parallel edges; a self-loop (u, u) gives one arc."""
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        if u != v:
            adj[v].append(u)
    off = np.zeros(n + 1, np.int64)
    for u in range(n):
        off[u + 1] = off[u] + len(adj[u])
    cols = np.array([w for a in adj for w in a], np.int32)
    return off, cols


def canon(label):
    return oracle.canonical_labels(label)


def arc_edges(n, off, cols):
    return [(u, int(cols[a])) for u in range(n) for a in range(off[u], off[u + 1])]


def brute_labels(n, edges):
    """Per-arc class of the edge: edges on a common simple cycle are merged."""
    idx = {}
    for u, v in edges:
        if u != v:
            idx.setdefault((min(u, v), max(u, v)), len(idx))
    parent = list(range(len(idx)))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    adj = {u: set() for u in range(n)}
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)

    def union_cycle(cyc):
        ids = [idx[(min(a, b), max(a, b))] for a, b in zip(cyc, cyc[1:] + cyc[:1])]
        r = find(ids[0])
        for e in ids[1:]:
            parent[find(e)] = r

    # simple cycles of length >= 3 whose smallest vertex is s
    for s in range(n):
        stack = [(s, [s])]
        while stack:
            x, path = stack.pop()
            for y in adj[x]:
                if y == s and len(path) >= 3:
                    union_cycle(path)
                elif y > s and y not in path:
                    stack.append((y, path + [y]))
    # parallel copies of an edge form a 2-cycle with each other: one class
    # already (same key)
    off, cols = csr(n, edges)
    lab = np.full(int(off[n]), -1, np.int64)
    for a, (u, w) in enumerate(arc_edges(n, off, cols)):
        if u != w:
            lab[a] = find(idx[(min(u, w), max(u, w))])
    return lab


def brute_art(n, edges):
    adj = {u: set() for u in range(n)}
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    art = np.zeros(n, np.uint8)
    for v in range(n):
        nb = sorted(adj[v])
        if len(nb) < 2:
            continue
        seen = {nb[0]}
        todo = [nb[0]]
        while todo:
            x = todo.pop()
            for y in adj[x]:
                if y != v and y not in seen:
                    seen.add(y)
                    todo.append(y)
        art[v] = any(w not in seen for w in nb)
    return art


def run(n, edges):
    off, cols = csr(n, edges)
    lab, art, k = oracle.bcc(n, off, cols)
    return off, cols, lab, art, k


def test_path():
    n = 9
    edges = [(i, i + 1) for i in range(n - 1)]
    off, cols, lab, art, k = run(n, edges)
    assert k == n - 1
    assert list(art) == [0] + [1] * (n - 2) + [0]
    # every edge its own component, both arcs of an edge alike
    arcs = arc_edges(n, off, cols)
    for a, (u, w) in enumerate(arcs):
        for b, (x, y) in enumerate(arcs):
            assert (lab[a] == lab[b]) == ({u, w} == {x, y})


def test_cycle_and_complete_graph():
    for n in (3, 4, 7):
        _, _, lab, art, k = run(n, [(i, (i + 1) % n) for i in range(n)])
        assert k == 1 and np.all(lab == lab[0]) and not art.any()
    n = 5
    _, _, lab, art, k = run(n, list(itertools.combinations(range(n), 2)))
    assert k == 1 and np.all(lab == lab[0]) and not art.any()


def test_star():
    n = 6
    _, _, lab, art, k = run(n, [(2, v) for v in range(n) if v != 2])
    assert k == n - 1
    assert list(art) == [0, 0, 1, 0, 0, 0]


def test_two_triangles_sharing_a_vertex():
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 2)]
    off, cols, lab, art, k = run(5, edges)
    assert k == 2
    assert list(art) == [0, 0, 1, 0, 0]
    arcs = arc_edges(5, off, cols)
    left = {a for a, (u, w) in enumerate(arcs) if max(u, w) <= 2}
    for a in range(len(arcs)):
        assert (lab[a] == lab[min(left)]) == (a in left)


def test_barbell():
    # two K4 joined by the path 3 - 8 - 4
    k4a = list(itertools.combinations([0, 1, 2, 3], 2))
    k4b = list(itertools.combinations([4, 5, 6, 7], 2))
    edges = k4a + k4b + [(3, 8), (8, 4)]
    _, _, lab, art, k = run(9, edges)
    assert k == 4
    assert list(np.nonzero(art)[0]) == [3, 4, 8]


def test_parallel_edges_and_self_loops():
    # a doubled edge 0-1 is a 2-cycle: one component with its copies; 1-2 a
    # bridge; a self-loop at 2 belongs to no component
    edges = [(0, 1), (0, 1), (1, 2), (2, 2)]
    off, cols, lab, art, k = run(3, edges)
    assert k == 2
    arcs = arc_edges(3, off, cols)
    lab_of = {}
    for a, (u, w) in enumerate(arcs):
        if u == w:
            assert lab[a] == -1
        else:
            lab_of.setdefault(frozenset((u, w)), set()).add(int(lab[a]))
    assert len(lab_of[frozenset((0, 1))]) == 1 and len(lab_of[frozenset((1, 2))]) == 1
    assert lab_of[frozenset((0, 1))] != lab_of[frozenset((1, 2))]
    assert list(art) == [0, 1, 0]


def test_disconnected_graph():
    edges = [(0, 1), (1, 2), (2, 0), (3, 4), (5, 6), (6, 7)]
    _, _, lab, art, k = run(9, edges)
    assert k == 4
    assert list(np.nonzero(art)[0]) == [6]


def test_hand_worked_graph():
    with open(os.path.join(GOLDEN, "bcc_example10.json")) as f:
        case = json.load(f)
    n, edges = case["n"], [tuple(e) for e in case["edges"]]
    off, cols, lab, art, k = run(n, edges)
    assert k == len(case["components"])
    assert sorted(np.nonzero(art)[0].tolist()) == case["articulation"]
    arcs = arc_edges(n, off, cols)
    comp_of = {}
    for ci, comp in enumerate(case["components"]):
        for u, w in comp:
            comp_of[frozenset((u, w))] = ci
    for a, (u, w) in enumerate(arcs):
        for b, (x, y) in enumerate(arcs):
            assert (lab[a] == lab[b]) == (comp_of[frozenset((u, w))] == comp_of[frozenset((x, y))])


@pytest.mark.parametrize("seed", range(60))
def test_brute_force_small_graphs(seed):
    rs = np.random.RandomState(seed)
    n = int(rs.randint(2, 8))
    pairs = list(itertools.combinations(range(n), 2))
    m = int(rs.randint(1, len(pairs) + 1))
    edges = [pairs[i] for i in rs.choice(len(pairs), m, replace=False)]
    off, cols, lab, art, k = run(n, edges)
    exp = brute_labels(n, edges)
    assert np.array_equal(canon(lab), canon(exp))
    assert np.array_equal(art, brute_art(n, edges))
    assert k == len(set(exp[exp >= 0].tolist()))
