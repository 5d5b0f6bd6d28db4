"""GPU tests of the captured batch path of rst_spanning_forest_batch.

With fixed buffers the first call runs eagerly and the next ones replay the
captured device work (checks, method per graph, mask, GConn+Euler over the
packed forest, a fixed number of BFS steps) with one synchronisation, then
continue on the host only where needed: a BFS that outlasts the enqueued
steps, a disconnected BFS member, a ranking fallback.  Every replayed output
(parent buffer poisoned before each call) is checked by the oracle verifier
over the packed graph with one designated root per member (Sec. III-D for
every root), and members run by BFS must also form BFS trees.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def members():
    return [I.road_mesh(64, 0.15, 0.01, seed=1), I.random_graph(5000, 15000, seed=2),
            I.rmat_lcc(13, 8, seed=3), I.long_chain(3000, 0.01, 16, seed=4, offset_bytes=4),
            I.path(700), I.star(900, 3), I.random_graph(3000, 800, seed=5, connected=False),
            I.grid_permuted(120, seed=6),
            # a mesh of 1300 x 1300: wide BFS levels for thousands of levels, far
            # more than the steps enqueued in the captured graph
            I.road_mesh(1300, 0.05, 0.0, seed=7)]


_B = []


def batch():
    if not _B:
        _B.append(I.pack(members()))
    return _B[0]


def check(b, parent, method):
    g = b.graph
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, parent, b.roots)
    assert code == 0, (oracle.VERIFY_CODES[code], bad)
    for k in np.nonzero(method)[0]:
        v0, v1 = int(b.vtx_off[k]), int(b.vtx_off[k + 1])
        off = g.offsets[v0:v1 + 1] - g.offsets[v0]
        cols = g.cols[g.offsets[v0]:g.offsets[v1]] - v0
        level, _, _ = oracle.bfs(v1 - v0, off, cols, int(b.roots[k]) - v0)
        p = parent[v0:v1] - v0
        reach = np.nonzero(level > 0)[0]
        assert np.all(level[p[reach]] == level[reach] - 1), k


@pytest.mark.parametrize("mode", ["gconn", "bfs", "mixed", "mixed_big_bfs"])
def test_replays_verified(rst, mode):
    b = batch()
    G = b.num_graphs
    if mode == "gconn":
        method = np.zeros(G, np.uint8)
    elif mode == "bfs":
        method = np.ones(G, np.uint8)
    elif mode == "mixed":
        method = np.array([1, 0, 1, 0, 1, 0, 1, 0, 0], np.uint8)   # disconnected member by GConn
    else:
        method = np.array([0, 1, 0, 1, 0, 1, 1, 0, 1], np.uint8)   # disconnected + big mesh by BFS
    c = rst.Context(0)
    g = b.graph
    args = (dev(g.offsets_typed()), dev(g.cols), dev(b.vtx_off), dev(b.arc_off), dev(b.roots))
    m = dev(method)
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    mout = torch.empty(G, dtype=torch.uint8, device="cuda")
    for call in range(4):
        parent.fill_(-7)
        mout.fill_(9)
        c.spanning_forest_batch(*args, method=m, parent=parent, method_out=mout)
        assert np.array_equal(mout.cpu().numpy(), method), call
        check(b, parent.cpu().numpy(), method)


def test_replays_with_selector(rst):
    """The loaded selector chooses on the device inside the captured graph;
    every replay's choice equals the eager one and the forest is verified."""
    b = batch()
    c = rst.Context(0)
    c.selector_load_default()
    g = b.graph
    args = (dev(g.offsets_typed()), dev(g.cols), dev(b.vtx_off), dev(b.arc_off), dev(b.roots))
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    mout = torch.empty(b.num_graphs, dtype=torch.uint8, device="cuda")
    first = None
    for call in range(3):
        parent.fill_(-7)
        c.spanning_forest_batch(*args, parent=parent, method_out=mout)
        chosen = mout.cpu().numpy().copy()
        if first is None:
            first = chosen
        assert np.array_equal(chosen, first), call
        check(b, parent.cpu().numpy(), chosen)


def test_many_small_graphs(rst):
    """4096 graphs of 100 to 2000 vertices (half meshes with deletions, half
    R-MAT), mixed methods, two replays: launch count independent of G."""
    G = 4096
    graphs = [I.batch_member(k, seed=11, nmin=100, nmax=2000) for k in range(G)]
    b = I.pack(graphs)
    method = (np.arange(G) % 4 == 3).astype(np.uint8)
    c = rst.Context(0)
    g = b.graph
    args = (dev(g.offsets_typed()), dev(g.cols), dev(b.vtx_off), dev(b.arc_off), dev(b.roots))
    m = dev(method)
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    mout = torch.empty(G, dtype=torch.uint8, device="cuda")
    for call in range(3):
        parent.fill_(-7)
        c.spanning_forest_batch(*args, method=m, parent=parent, method_out=mout)
        check(b, parent.cpu().numpy(), method)


@pytest.mark.parametrize("sample", [2, 1])
def test_global_sweep_with_a_dominant_tree_per_graph(rst, sample):
    """The global sweep forced over a batch, with sampling: every packed graph
    gets its own dominant tree, whose vertices offer no arcs (sound because no
    edge joins two graphs); members of every kind, some by BFS, replays."""
    G = 600
    graphs = [I.batch_member(k, seed=13, nmin=50, nmax=6000) for k in range(G)]
    graphs[7] = I.random_graph(3000, 800, seed=5, connected=False)
    graphs[8] = I.long_chain(3000, 0.01, 16, seed=4, offset_bytes=4)
    graphs[9] = I.path(1)
    b = I.pack(graphs)
    method = (np.arange(G) % 5 == 4).astype(np.uint8)
    c = rst.Context(0)
    c.set_option(rst.OPT_HOOK_MODE, 2)
    c.set_option(rst.OPT_HOOK_SAMPLE, sample)
    g = b.graph
    args = (dev(g.offsets_typed()), dev(g.cols), dev(b.vtx_off), dev(b.arc_off), dev(b.roots))
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for m in (np.zeros(G, np.uint8), method):
        for call in range(3):
            parent.fill_(-7)
            c.spanning_forest_batch(*args, method=dev(m), parent=parent)
            check(b, parent.cpu().numpy(), m)
    _, _, st = c.spanning_forest_batch(*args, method=dev(method), stats=True)
    assert st["paths"] & rst.PATH_HOOK_GLOBAL and st["paths"] & rst.PATH_HOOK_GIANT, st["paths"]


def test_hooking_chosen_graph_by_graph(rst):
    """With the hooking variant left to the library, every GConn+Euler graph of
    a batch gets its own: the tile pass for graphs whose ids carry locality
    (meshes numbered along the mesh), the global sweep with its own dominant
    tree for the others (R-MAT, permuted grids, long chains); replays."""
    graphs = [I.road_mesh(200, 0.15, 0.01, seed=21), I.rmat_lcc(15, 8, seed=22),
              I.grid_permuted(150, seed=23), I.long_chain(30000, 0.01, 16, seed=24, offset_bytes=4),
              I.road_mesh(90, 0.1, 0.0, seed=25), I.random_graph(20000, 40000, seed=26),
              I.path(500), I.star(3000, 7)]
    b = I.pack(graphs)
    G = b.num_graphs
    c = rst.Context(0)
    g = b.graph
    args = (dev(g.offsets_typed()), dev(g.cols), dev(b.vtx_off), dev(b.arc_off), dev(b.roots))
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for m in (np.zeros(G, np.uint8), (np.arange(G) % 3 == 2).astype(np.uint8)):
        for call in range(3):
            parent.fill_(-7)
            c.spanning_forest_batch(*args, method=dev(m), parent=parent)
            check(b, parent.cpu().numpy(), m)
    _, _, st = c.spanning_forest_batch(*args, method=dev(np.zeros(G, np.uint8)), stats=True)
    assert st["paths"] & rst.PATH_HOOK_GLOBAL, st["paths"]
