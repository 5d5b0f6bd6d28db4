"""Pins of the oracle's tree depth and Path-Reversal RST (no GPU).

Tree depth (Sec. IV-B, Fig. 2): closed forms on paths and stars, a
hand-worked forest (tests/golden), and on tree inputs the depth of the unique
rooted spanning tree equals the hop distance that scipy's shortest-path
routine computes from the root; malformed parent arrays are rejected.

PR-RST (Sec. III-C): a hand-worked run step by step (max round, min round with
a real path reversal, final re-rooting), every graph on 5 vertices with every
root accepted by the verifier (which is pinned by Kirchhoff enumeration in
test_oracle.py), and on tree inputs the unique answer.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_2603_11645_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_depth_closed_form_path():
    n = 57
    for k in (0, 13, n - 1):
        g = I.path(n)
        eu, ev = g.edge_list()
        par = oracle.dfs_root(n, eu, ev, [k])
        depth, mx = oracle.tree_depth(par)
        assert list(depth) == [abs(i - k) for i in range(n)]
        assert mx == max(k, n - 1 - k)


def test_depth_closed_form_star():
    n = 9
    g = I.star(n, 0)
    eu, ev = g.edge_list()
    depth, mx = oracle.tree_depth(oracle.dfs_root(n, eu, ev, [0]))
    assert list(depth) == [0] + [1] * (n - 1) and mx == 1
    depth, mx = oracle.tree_depth(oracle.dfs_root(n, eu, ev, [5]))
    assert depth[5] == 0 and depth[0] == 1 and mx == 2
    assert all(depth[v] == 2 for v in range(1, n) if v != 5)


def test_depth_golden_forest():
    with open(os.path.join(GOLDEN, "depth_forest7.json")) as f:
        case = json.load(f)
    depth, mx = oracle.tree_depth(np.array(case["parent"]))
    assert list(depth) == case["depth"] and mx == case["max_depth"]


@pytest.mark.parametrize("seed", range(4))
def test_depth_equals_scipy_hops_on_trees(seed):
    # on a tree the rooted spanning tree is unique, and the depth of a vertex
    # is its hop distance from the root
    n = 400 + 37 * seed
    g = I.random_tree(n, seed=50 + seed)
    root = (seed * 97) % n
    eu, ev = g.edge_list()
    depth, mx = oracle.tree_depth(oracle.dfs_root(n, eu, ev, [root]))
    mat = sp.csr_matrix((np.ones(g.nnz), g.cols, g.offsets), shape=(n, n))
    d = shortest_path(mat, method="D", unweighted=True, indices=root, directed=False)
    assert np.array_equal(depth.astype(np.int64), d.astype(np.int64))
    assert mx == int(d.max())


def test_depth_rejects_malformed():
    with pytest.raises(ValueError):
        oracle.tree_depth(np.array([1, 2, 0]))        # a cycle
    with pytest.raises(ValueError):
        oracle.tree_depth(np.array([0, 5, 1]))        # parent out of range
    d, mx = oracle.tree_depth(np.array([0]))
    assert list(d) == [0] and mx == 0


def test_pr_rst_golden_steps():
    with open(os.path.join(GOLDEN, "pr_rst_reversal4.json")) as f:
        case = json.load(f)
    g = I.csr_from_edges(case["n"], np.array(case["eu"]), np.array(case["ev"]))
    for k, want in case["after_iterations"].items():
        par, it = oracle.pr_rst(g.n, g.offsets, g.cols, [0], max_iters=int(k))
        assert list(par) == want and it == int(k)
    for r, want in case["rooted"].items():
        par, it = oracle.pr_rst(g.n, g.offsets, g.cols, [int(r)])
        assert list(par) == want and it == case["iterations"]


def test_pr_rst_every_graph_on_five_vertices():
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        eu = np.array([a for i, (a, b) in enumerate(pairs) if mask >> i & 1], dtype=np.int32)
        ev = np.array([b for i, (a, b) in enumerate(pairs) if mask >> i & 1], dtype=np.int32)
        g = I.csr_from_edges(n, eu, ev)
        for r in range(n):
            par, _ = oracle.pr_rst(n, g.offsets, g.cols, [r])
            code, bad = oracle.verify_rst(n, g.offsets, g.cols, par, [r])
            assert code == 0, (mask, r, oracle.VERIFY_CODES[code], bad)


@pytest.mark.parametrize("seed", range(3))
def test_pr_rst_unique_on_trees_and_valid_on_graphs(seed):
    t = I.random_tree(300, seed=70 + seed)
    eu, ev = t.edge_list()
    par, _ = oracle.pr_rst(t.n, t.offsets, t.cols, [seed])
    assert np.array_equal(par, oracle.dfs_root(t.n, eu, ev, [seed]))
    for g in (I.random_graph(500, 700, seed=80 + seed, connected=True),
              I.random_graph(400, 150, seed=90 + seed, connected=False),
              I.grid(19, 21, 0.25, seed=seed)):
        par, it = oracle.pr_rst(g.n, g.offsets, g.cols, [g.n // 3])
        code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par, [g.n // 3])
        assert code == 0, (oracle.VERIFY_CODES[code], bad)
        assert 1 <= it <= 4 * int(np.ceil(np.log2(g.n))) + 8
