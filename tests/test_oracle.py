"""Pins of the CPU oracle against facts outside itself (no GPU needed).

* scipy.sparse.csgraph (an independent library) for BFS distances and
  connected components;
* closed forms: paths, stars, unpermuted and permuted grids;
* brute force on tiny graphs: every parent array is enumerated and the
  verifier must accept exactly tau(G) of them, the spanning-tree count of the
  matrix-tree theorem (Kirchhoff), computed as a determinant;
* hand-worked Euler tours (tests/golden, derived from Sec. III-D);
* uniqueness of rooting a fixed tree (DFS rooting == Euler rooting == BFS
  parent on tree inputs);
* list ranking against lists whose order is known by construction.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import oracle
from paper_2603_11645_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _scipy_levels(g, root):
    mat = sp.csr_matrix((np.ones(g.nnz), g.cols, g.offsets), shape=(g.n, g.n))
    d = shortest_path(mat, method="D", unweighted=True, indices=root, directed=False)
    out = np.where(np.isinf(d), -1, d).astype(np.int64)
    return out


def _scipy_minid_labels(g):
    mat = sp.csr_matrix((np.ones(g.nnz), g.cols, g.offsets), shape=(g.n, g.n))
    k, lab = connected_components(mat, directed=False)
    first = np.full(k, g.n, dtype=np.int64)
    np.minimum.at(first, lab, np.arange(g.n))
    return k, first[lab]


def _graphs_for_crosscheck():
    out = []
    for seed in range(6):
        out.append(I.random_graph(200, 150, seed=seed, connected=False))
        out.append(I.random_graph(300, 400, seed=100 + seed, connected=True))
    out.append(I.grid(17, 23, 0.3, seed=9))
    out.append(I.rmat_lcc(10, 8, seed=11))
    return out


@pytest.mark.parametrize("gi", range(14))
def test_bfs_levels_match_scipy(gi):
    g = _graphs_for_crosscheck()[gi]
    for root in (0, g.n // 2, g.n - 1):
        level, parent, ecc = oracle.bfs(g.n, g.offsets, g.cols, root)
        ref = _scipy_levels(g, root)
        assert np.array_equal(level.astype(np.int64), ref)
        assert ecc == ref.max()
        reach = np.nonzero(level >= 0)[0]
        for v in reach:
            if v == root:
                assert parent[v] == root
                continue
            p = parent[v]
            assert level[p] == level[v] - 1
            assert p in g.cols[g.offsets[v]:g.offsets[v + 1]]


@pytest.mark.parametrize("gi", range(14))
def test_components_match_scipy(gi):
    g = _graphs_for_crosscheck()[gi]
    k_ref, lab_ref = _scipy_minid_labels(g)
    k, lab = oracle.components(g.n, g.offsets, g.cols)
    assert k == k_ref
    assert np.array_equal(lab.astype(np.int64), lab_ref)
    label, fu, fv = oracle.uf_forest(g.n, g.offsets, g.cols)
    assert len(fu) == g.n - k_ref                      # |F| = n - c
    assert np.array_equal(label.astype(np.int64), lab_ref)
    # forest edges are graph edges and join vertices of one component
    for a, b in zip(fu, fv):
        assert b in g.cols[g.offsets[a]:g.offsets[a + 1]]
        assert label[a] == label[b]


def test_closed_form_path():
    n = 37
    g = I.path(n)
    for k in (0, 5, n - 1):
        level, parent, ecc = oracle.bfs(n, g.offsets, g.cols, k)
        assert list(level) == [abs(i - k) for i in range(n)]
        exp = [i + 1 if i < k else (i - 1 if i > k else k) for i in range(n)]
        assert list(parent) == exp
        label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
        assert list(oracle.dfs_root(n, fu, fv, [k])) == exp
        assert list(oracle.euler_root(n, fu, fv, [k])) == exp
    # a path whose ids are permuted: P follows the permutation
    perm = np.random.RandomState(3).permutation(n).astype(np.int32)
    g = I.path(n, perm)
    label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
    par = oracle.euler_root(n, fu, fv, [perm[0]])
    for i in range(1, n):
        assert par[perm[i]] == perm[i - 1]


def test_closed_form_star():
    n = 9
    for c in (0, 4):
        g = I.star(n, c)
        label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
        p = oracle.euler_root(n, fu, fv, [c])
        assert all(p[v] == c for v in range(n))
        leaf = (c + 1) % n
        p = oracle.euler_root(n, fu, fv, [leaf])
        assert p[leaf] == leaf and p[c] == leaf
        assert all(p[v] == c for v in range(n) if v not in (c, leaf))


def test_closed_form_grid_levels():
    rows, cols = 13, 21
    g = I.grid(rows, cols)
    level, _, ecc = oracle.bfs(g.n, g.offsets, g.cols, 0)
    exp = np.array([(v // cols) + (v % cols) for v in range(g.n)])
    assert np.array_equal(level, exp) and ecc == rows + cols - 2
    gp = I.grid_permuted(32, seed=1)
    perm = gp.meta["perm"]
    # cell c carries vertex perm[c]; the root is vertex 0 = cell c0
    c0 = int(np.nonzero(perm == 0)[0][0])
    level, _, _ = oracle.bfs(gp.n, gp.offsets, gp.cols, 0)
    for c in range(gp.n):
        assert level[perm[c]] == abs(c // 32 - c0 // 32) + abs(c % 32 - c0 % 32)


def _matrix_tree_count(n, edges):
    """Spanning-tree count of a simple graph by Kirchhoff's matrix-tree theorem."""
    L = np.zeros((n, n))
    for a, b in edges:
        L[a, a] += 1; L[b, b] += 1; L[a, b] -= 1; L[b, a] -= 1
    if n == 1:
        return 1
    return int(round(np.linalg.det(L[1:, 1:])))


def _all_edges(n):
    return [(a, b) for a in range(n) for b in range(a + 1, n)]


def test_verifier_accepts_exactly_the_spanning_trees():
    """Every parent array of 4-vertex graphs: the verifier accepts tau(G) per root."""
    n = 4
    E = _all_edges(n)
    arrays = np.array(list(itertools.product(range(n), repeat=n)), dtype=np.int32)
    for mask in range(1, 1 << len(E)):
        edges = [E[i] for i in range(len(E)) if mask >> i & 1]
        g = I.csr_from_edges(n, np.array([a for a, _ in edges], np.int32),
                             np.array([b for _, b in edges], np.int32))
        k, _ = oracle.components(n, g.offsets, g.cols)
        if k != 1:
            continue
        tau = _matrix_tree_count(n, edges)
        for r in range(n):
            acc = sum(oracle.verify_rst(n, g.offsets, g.cols, p, [r])[0] == 0 for p in arrays)
            assert acc == tau


def test_brute_force_tiny_graphs_all_roots():
    """All graphs on 5 vertices, all roots: oracle outputs pass the verifier;
    Euler rooting equals DFS rooting of the same forest; forests match
    scipy components."""
    n = 5
    E = _all_edges(n)
    for mask in range(1 << len(E)):
        edges = [E[i] for i in range(len(E)) if mask >> i & 1]
        eu = np.array([a for a, _ in edges], np.int32)
        ev = np.array([b for _, b in edges], np.int32)
        g = I.csr_from_edges(n, eu, ev)
        k, lab = oracle.components(n, g.offsets, g.cols)
        label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
        assert len(fu) == n - k
        for r in range(n):
            p_dfs = oracle.dfs_root(n, fu, fv, [r])
            p_eul = oracle.euler_root(n, fu, fv, [r])
            assert np.array_equal(p_dfs, p_eul)
            assert oracle.verify_rst(n, g.offsets, g.cols, p_dfs, [r])[0] == 0
            level, p_bfs, _ = oracle.bfs(n, g.offsets, g.cols, r)
            if k == 1:
                assert oracle.verify_rst(n, g.offsets, g.cols, p_bfs, [r])[0] == 0


def test_sampled_six_vertex_graphs():
    n = 6
    E = _all_edges(n)
    rs = np.random.RandomState(7)
    for _ in range(600):
        mask = int(rs.randint(0, 1 << len(E)))
        edges = [E[i] for i in range(len(E)) if mask >> i & 1]
        g = I.csr_from_edges(n, np.array([a for a, _ in edges], np.int32),
                             np.array([b for _, b in edges], np.int32))
        label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
        r = int(rs.randint(n))
        p1 = oracle.dfs_root(n, fu, fv, [r])
        p2 = oracle.euler_root(n, fu, fv, [r])
        assert np.array_equal(p1, p2)
        assert oracle.verify_rst(n, g.offsets, g.cols, p1, [r])[0] == 0


@pytest.mark.parametrize("name", ["euler_tree4.json", "euler_forest6.json"])
def test_golden_euler_tours(name):
    with open(os.path.join(GOLDEN, name)) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        p, succ, pos = oracle.euler_root(gold["n"], gold["fu"], gold["fv"], case["roots"],
                                         return_tour=True)
        assert list(succ) == case["succ"]
        assert list(pos) == case["pos"]
        assert list(p) == case["parent"]
        # the list ranker agrees with the hand-derived positions (dist = len-1-pos)
        dist, k = oracle.list_rank(succ)
        assert k == len(case["roots"])


def test_tree_inputs_rooting_is_unique():
    """On trees (m = n-1) the BFS parent, DFS rooting and Euler rooting coincide."""
    for seed in range(20):
        n = 50 + 37 * seed
        g = I.random_tree(n, seed)
        assert g.m == n - 1
        label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
        r = (seed * 7919) % n
        _, p_bfs, _ = oracle.bfs(n, g.offsets, g.cols, r)
        assert np.array_equal(p_bfs, oracle.dfs_root(n, fu, fv, [r]))
        assert np.array_equal(p_bfs, oracle.euler_root(n, fu, fv, [r]))


def test_euler_root_forests_random_roots():
    rs = np.random.RandomState(5)
    for seed in range(12):
        g = I.random_graph(400, 120, seed=seed, connected=False)
        label, fu, fv = oracle.uf_forest(g.n, g.offsets, g.cols)
        comps = np.unique(label)
        chosen = []
        for c in comps[: len(comps) // 2]:
            members = np.nonzero(label == c)[0]
            chosen.append(int(members[rs.randint(len(members))]))
        p1 = oracle.dfs_root(g.n, fu, fv, chosen)
        p2, succ, pos = oracle.euler_root(g.n, fu, fv, chosen, return_tour=True)
        assert np.array_equal(p1, p2)
        assert oracle.verify_rst(g.n, g.offsets, g.cols, p1, chosen)[0] == 0
        # tour invariants: one list per non-trivial tree, length 2(size-1),
        # positions a permutation of 0..len-1, consecutive arcs chain up
        t = len(fu)
        src = np.concatenate([fu, fv]); dst = np.concatenate([fv, fu])
        dist, k = oracle.list_rank(succ)
        sizes = np.bincount(label, minlength=g.n)
        assert k == int(np.sum(sizes[comps] > 1))
        for e in range(2 * t):
            s = succ[e]
            if s >= 0:
                assert dst[e] == src[s]
                assert pos[s] == pos[e] + 1


def test_list_rank_known_lists():
    rs = np.random.RandomState(11)
    for trial in range(10):
        A = int(rs.randint(1, 5000))
        order = rs.permutation(A)
        cuts = np.sort(rs.choice(np.arange(1, A), size=min(A - 1, int(rs.randint(0, 20))),
                                 replace=False)) if A > 1 else np.array([], int)
        succ = np.full(A, -1, dtype=np.int32)
        exp = np.zeros(A, dtype=np.int32)
        pieces = np.split(order, cuts)
        for piece in pieces:
            for i in range(len(piece) - 1):
                succ[piece[i]] = piece[i + 1]
            exp[piece] = np.arange(len(piece) - 1, -1, -1)
        dist, k = oracle.list_rank(succ)
        assert k == len(pieces)
        assert np.array_equal(dist, exp)
    with pytest.raises(ValueError):
        oracle.list_rank(np.array([1, 2, 0], dtype=np.int32))   # a cycle


def test_euler_succ_any_cyclic_order():
    """Any per-vertex out-arc order gives one tour per tree of length 2(size-1)."""
    rs = np.random.RandomState(2)
    for seed in range(8):
        g = I.random_tree(300, seed)
        n = g.n
        label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
        t = len(fu)
        A = 2 * t
        src = np.empty(A, np.int32); dst = np.empty(A, np.int32)
        src[0::2], dst[0::2] = fu, fv
        src[1::2], dst[1::2] = fv, fu
        head = np.full(n, -1, np.int32); nxt = np.full(A, -1, np.int32)
        for e in rs.permutation(A):          # random insertion order
            nxt[e] = head[src[e]]; head[src[e]] = e
        root = int(rs.randint(n))
        is_root = np.zeros(n, np.uint8); is_root[root] = 1
        succ = oracle.euler_succ(n, src, dst, head, nxt, is_root)
        dist, k = oracle.list_rank(succ)
        assert k == 1
        assert dist[head[root]] == A - 1
        # parents from the rank rule equal the DFS rooting
        par = np.full(n, -1, np.int32); par[root] = root
        for x in range(t):
            e, r = 2 * x, 2 * x + 1
            if dist[e] > dist[r]:       # e earlier in the tour: descends
                par[dst[e]] = src[e]
            else:
                par[src[e]] = dst[e]
        assert np.array_equal(par, oracle.dfs_root(n, fu, fv, [root]))


def test_verifier_rejects_mutations():
    g = I.grid(9, 11, 0.0, seed=1)
    n = g.n
    label, fu, fv = oracle.uf_forest(n, g.offsets, g.cols)
    p = oracle.dfs_root(n, fu, fv, [0])
    assert oracle.verify_rst(n, g.offsets, g.cols, p, [0])[0] == 0
    q = p.copy(); q[0] = 1
    assert oracle.verify_rst(n, g.offsets, g.cols, q, [0])[0] == 1
    q = p.copy(); q[5] = n
    assert oracle.verify_rst(n, g.offsets, g.cols, q, [0])[0] == 2
    q = p.copy(); q[5] = -1
    assert oracle.verify_rst(n, g.offsets, g.cols, q, [0])[0] == 2
    q = p.copy(); q[12] = 40                      # not a neighbour
    assert oracle.verify_rst(n, g.offsets, g.cols, q, [0])[0] == 3
    q = p.copy(); a, b = 12, 13                   # 2-cycle over a real edge
    q[a], q[b] = b, a
    assert oracle.verify_rst(n, g.offsets, g.cols, q, [0])[0] == 4
    q = p.copy(); q[7] = 7                        # a second self-parent: {7,7} is no edge
    assert oracle.verify_rst(n, g.offsets, g.cols, q, [0])[0] == 3
    assert oracle.verify_rst(n, g.offsets, g.cols, p, [0, 3])[0] == 6
    # disconnected: a component without designated root must be rooted at its min id
    g2 = I.csr_from_edges(6, np.array([0, 1, 3, 4], np.int32), np.array([1, 2, 4, 5], np.int32))
    ok = np.array([0, 0, 1, 3, 3, 4], np.int32)
    assert oracle.verify_rst(6, g2.offsets, g2.cols, ok, [0])[0] == 0
    bad = np.array([0, 0, 1, 4, 4, 4], np.int32)
    assert oracle.verify_rst(6, g2.offsets, g2.cols, bad, [0])[0] == 1


def test_generated_workloads_small_versions():
    """Reduced versions of the workload recipes are connected and pass the oracle."""
    for g in (I.grid_permuted(64, seed=1), I.road_mesh(128, 0.15, 0.01, seed=2),
              I.rmat_lcc(12, 16, seed=3), I.long_chain(5000, 0.005, 64, seed=4)):
        k, _ = oracle.components(g.n, g.offsets, g.cols)
        assert k == 1
        label, fu, fv = oracle.uf_forest(g.n, g.offsets, g.cols)
        p = oracle.euler_root(g.n, fu, fv, [g.root])
        assert oracle.verify_rst(g.n, g.offsets, g.cols, p, [g.root])[0] == 0
