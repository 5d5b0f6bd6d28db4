"""GPU parity of rst_tree_depth (tree depth by weighted Euler-tour ranking,
Sec. IV-B Fig. 2 with the tour of Sec. III-D) against the oracle's plain
walk up the parent pointers: depths are unique given the forest, so they
are compared bit for bit.  Covered: paths rooted anywhere (depth up to
2^24 - 1), stars, random trees and forests over random ids, the GConn+Euler
and BFS trees of mesh, R-MAT and chain graphs (the BFS tree's depths are also
its levels), and more trees than the ruling set holds (Wyllie fallback).
"""
import numpy as np
import pytest

import oracle
from paper_2603_11645_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11645_amd as rst
    return rst.Context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(ctx, parent):
    exp, mx = oracle.tree_depth(parent)
    got, gmx = ctx.tree_depth(dev(parent.astype(np.int32)))
    assert np.array_equal(got.cpu().numpy(), exp)
    assert gmx == mx
    return exp


def test_paths_and_stars(ctx):
    for n, k in ((1, 0), (2, 1), (1000, 0), (1000, 999), (100001, 31337)):
        g = I.path(n)
        eu, ev = g.edge_list()
        check(ctx, oracle.dfs_root(n, eu, ev, [k]))
    g = I.star(5000, 0)
    eu, ev = g.edge_list()
    check(ctx, oracle.dfs_root(5000, eu, ev, [0]))
    check(ctx, oracle.dfs_root(5000, eu, ev, [4321]))


def test_long_path_random_ids(ctx):
    n = 1 << 24
    rs = np.random.RandomState(2)
    perm = rs.permutation(n).astype(np.int32)
    parent = np.empty(n, np.int32)
    parent[perm[1:]] = perm[:-1]
    parent[perm[0]] = perm[0]
    d = check(ctx, parent)
    assert d.max() == n - 1


@pytest.mark.parametrize("seed", range(3))
def test_random_forests(ctx, seed):
    rs = np.random.RandomState(seed)
    n = 300000 + 7 * seed
    perm = rs.permutation(n).astype(np.int32)
    parent = np.empty(n, np.int32)
    roots = set(rs.choice(n, size=1 + 500 * seed, replace=False).tolist()) | {0}
    for i in range(n):
        parent[perm[i]] = perm[i] if i in roots else perm[rs.randint(0, i)]
    check(ctx, parent)


def test_gconn_and_bfs_trees(ctx):
    for g in (I.road_mesh(300, 0.15, 0.001, seed=2), I.rmat_lcc(14, 16, seed=3),
              I.long_chain(1 << 18, 0.005, 64, seed=4), I.grid_permuted(128, seed=1)):
        off, cols = dev(g.offsets_typed()), dev(g.cols)
        par = ctx.spanning_tree(off, cols, 0, "gconn").cpu().numpy()
        check(ctx, par)
        bpar = ctx.spanning_tree(off, cols, 0, "bfs").cpu().numpy()
        d = check(ctx, bpar)
        lref, _, _ = oracle.bfs(g.n, g.offsets, g.cols, 0)
        assert np.array_equal(d, lref)


def test_more_trees_than_rulers_hold(ctx):
    """1.2 million two-vertex trees over random ids: the Wyllie fallback."""
    rs = np.random.RandomState(5)
    n = 2400000
    pairs = rs.permutation(n).astype(np.int32).reshape(-1, 2)
    parent = np.arange(n, dtype=np.int32)
    parent[pairs[:, 1]] = pairs[:, 0]
    d = check(ctx, parent)
    assert d.max() == 1
