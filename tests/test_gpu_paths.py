"""GPU tests at medium sizes that drive each variant of the forest and ranking
stages, checked like the small cases: min-id labels bit-exact against the
oracle, parent arrays accepted by the oracle verifier, list ranks bit-exact.

Which variant ran is read from rst_stats.paths:
  * vertex ids without locality: every tile's cross edges hooked flat, the
    contracted tour list ranked by the one workgroup in global memory (C1
    grid) or, when longer than that workgroup takes, by multi-workgroup
    rounds (300k-vertex random graph);
  * meshes: kept cross edges of all levels merged in LDS by one workgroup
    (a few hundred on a lightly thinned mesh); when more small trees meet at
    tile borders (30% and 45% deletions), merged in LDS per group of tiles and
    then the top levels; and
    in global memory when a group meets a root outside its tiles as well
    (45% deletions plus a tile of hub vertices).
"""
import numpy as np
import pytest

import oracle
from paper_2603_11645_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rst():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11645_amd as r
    return r


@pytest.fixture(scope="module")
def ctx(rst):
    return rst.Context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mesh_plus_hub(mesh=None, seed=13):
    """A mesh (default a 512x512 road-like one, 32 tiles) and one more tile of
    8192 hub vertices, each joined to 3 random mesh vertices: the hub tile
    lists far more cross edges than vertices (hooked flat), and its hooks join
    trees of high tiles to roots in low tiles, so a group of tiles meets a root
    outside its own range.  The one-workgroup merge of all levels has no such
    limit; when the kept edges are too many for it, the group merge falls back
    to global memory."""
    mesh = mesh if mesh is not None else I.road_mesh(512, 0.15, 0.001, seed=2)
    n0 = mesh.n
    rs = np.random.RandomState(seed)
    hub = np.repeat(np.arange(n0, n0 + 8192), 3)
    far = rs.randint(0, n0, size=hub.size)
    src = np.repeat(np.arange(n0), np.diff(mesh.offsets))
    keep = src < mesh.cols
    eu = np.concatenate([src[keep], hub]).astype(np.int32)
    ev = np.concatenate([mesh.cols[keep], far]).astype(np.int32)
    return I.csr_from_edges(n0 + 8192, eu, ev, name="mesh_plus_hub")


# name: (graph builder, rst_stats.paths bits that must be set, bits that must not)
CASES = {
    # ids without locality: the tour is ranked by the sparse ruling set
    "grid_permuted_256": (lambda: I.grid_permuted(256, seed=1), 8, 7),
    # thousands of trees: the contracted tour lists may exceed the LDS ranking;
    # about 8k and 37k kept cross edges (group merges)
    "grid_1024_del30": (lambda: I.grid(1024, 1024, 0.30, seed=7), 4, 1),
    "grid_1024_del45": (lambda: I.grid(1024, 1024, 0.45, seed=7), 4, 1),
    "road_512": (lambda: I.road_mesh(512, 0.15, 0.001, seed=2), 0, 7),
    "random_300k": (lambda: I.random_graph(300000, 450000, seed=11, connected=True), 8, 2),
    "mesh_plus_hub": (mesh_plus_hub, 0, 5),
    "grid45_plus_hub": (lambda: mesh_plus_hub(I.grid(1024, 1024, 0.45, seed=7)), 5, 0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_forest_paths_verified(ctx, rst, name):
    build, must, must_not = CASES[name]
    g = build()
    off, cols = dev(g.offsets_typed()), dev(g.cols)
    k_ref, lab_ref = oracle.components(g.n, g.offsets, g.cols)
    label, k = ctx.components(off, cols)
    assert k == k_ref
    assert np.array_equal(label.cpu().numpy(), lab_ref)
    root = g.n // 2
    par, st = ctx.spanning_tree(off, cols, root, "gconn", stats=True)
    assert ctx.last_status == (0 if k_ref == 1 else rst.RST_E_DISCONNECTED)
    assert (st["paths"] & must) == must and (st["paths"] & must_not) == 0, st
    assert st["components"] == k_ref
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par.cpu().numpy(), [root])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)


def test_list_rank_paths(ctx):
    """Random lists long enough for the global one-workgroup ranking and for
    the multi-workgroup rounds."""
    rs = np.random.RandomState(21)
    for A in (100003, 600001):
        order = rs.permutation(A)
        cuts = np.sort(rs.choice(np.arange(1, A), size=5, replace=False))
        succ = np.full(A, -1, np.int32)
        for piece in np.split(order, cuts):
            succ[piece[:-1]] = piece[1:]
        exp, k = oracle.list_rank(succ)
        assert k == 6
        got = ctx.list_rank(dev(succ)).cpu().numpy()
        assert np.array_equal(got, exp)
