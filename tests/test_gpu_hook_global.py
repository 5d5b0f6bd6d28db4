"""GPU parity of the hooking sweep in global memory (ids without locality):
sampling of each vertex's first arcs, the dominant tree found from a sample,
then the remaining arcs (Sec. III-B hooking with the edge of every union
recorded, Sec. I).

Without a dominant tree to seek, the sweep starts with a pass without finds
(every vertex hooked to the smallest of its first 16 neighbours when that is
smaller than itself); its edge cases get a graph of their own below.

Min-id component labels are unique, so they are compared bit for bit with the
oracle's union-find; spanning trees go through the oracle verifier; on tree
inputs the rooted spanning tree is unique and compared bit for bit.  Every
graph runs with the hooking forced to the tile pass and to the global sweep,
and the global sweep with every number of sampled arcs (0: each edge once
from its larger end; 1-4: sampling, then the dominant tree skipped when one
holds half the sample).  The automatic choice is checked on graphs with and
without id locality, and captured replays follow a change of the data under
the same buffers.
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


def several_components():
    """Three random graphs side by side with isolated vertices between them."""
    parts = [I.random_graph(40000, 60000, seed=3), I.random_graph(25000, 20000, seed=4),
             I.random_tree(30000, seed=5)]
    eu_l, ev_l, base = [], [], 0
    for p in parts:
        a, b = p.edge_list()
        eu_l.append(a + base)
        ev_l.append(b + base)
        base += p.n + 7          # 7 isolated vertices after each part
    eu = np.concatenate(eu_l)
    ev = np.concatenate(ev_l)
    return I.csr_from_edges(base, eu.astype(np.int32), ev.astype(np.int32), name="several")


GRAPHS = {
    "random_200k": lambda: I.random_graph(200000, 300000, seed=11),
    "rmat16": lambda: I.rmat_lcc(16, 16, seed=8),
    "grid_permuted_256": lambda: I.grid_permuted(256, seed=1),
    "chain_2_18_int64": lambda: I.long_chain(1 << 18, seed=6),
    "road_512": lambda: I.road_mesh(512, 0.15, 0.001, seed=2),
    "star_50k": lambda: I.star(50000, center=777),
    "several": several_components,
}
_CACHE = {}


def graph(name):
    if name not in _CACHE:
        _CACHE[name] = GRAPHS[name]()
    return _CACHE[name]


def run_case(ctx, rst, g, mode, sample):
    ctx.set_option(rst.OPT_HOOK_MODE, mode)
    ctx.set_option(rst.OPT_HOOK_SAMPLE, sample)
    off, cols = dev(g.offsets_typed()), dev(g.cols)
    k_ref, lab_ref = oracle.components(g.n, g.offsets, g.cols)
    label, k = ctx.components(off, cols)
    assert k == k_ref
    assert np.array_equal(label.cpu().numpy(), lab_ref)
    root = g.n // 3
    par, st = ctx.spanning_tree(off, cols, root, "gconn", stats=True)
    assert ctx.last_status == (0 if k_ref == 1 else rst.RST_E_DISCONNECTED)
    assert st["components"] == k_ref
    assert bool(st["paths"] & rst.PATH_HOOK_GLOBAL) == (mode == 2), st
    p = par.cpu().numpy()
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, p, [root])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)
    if g.m == g.n - 1 and k_ref == 1:      # a tree: the rooted spanning tree is unique
        ref = oracle.dfs_root(g.n, *g.edge_list(), [root])
        assert np.array_equal(p, ref)
    return st


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("mode,sample", [(1, -1), (2, -1), (2, 0), (2, 1), (2, 2), (2, 4)])
def test_forced_modes(ctx, rst, name, mode, sample):
    try:
        run_case(ctx, rst, graph(name), mode, sample)
    finally:
        ctx.set_option(rst.OPT_HOOK_MODE, 0)
        ctx.set_option(rst.OPT_HOOK_SAMPLE, -1)


def first_pass_cases():
    """A random graph in CSR rows of their own order: rows reversed (the
    smallest neighbour of every vertex of degree above 16 lies beyond the 16
    arcs the first pass reads), every first-pass edge of even vertices given a
    parallel copy, self-loops on every 7th vertex, and a separate path
    n-3 - n-2 - n-1, whose smallest vertex has only larger neighbours (it
    stays a root)."""
    base = I.random_graph(30000, 90000, seed=21)
    hub_u = np.full(40, 12345, np.int32)             # a vertex of degree 40+
    hub_v = np.arange(20000, 20040, dtype=np.int32)
    eu, ev = base.edge_list()
    eu = np.concatenate([eu, hub_u]).astype(np.int32)
    ev = np.concatenate([ev, hub_v]).astype(np.int32)
    n = base.n + 3                                    # a path n-3 .. n-1 apart
    eu = np.concatenate([eu, [n - 3, n - 2]]).astype(np.int32)
    ev = np.concatenate([ev, [n - 2, n - 1]]).astype(np.int32)
    g = I.csr_from_edges(n, eu, ev, name="first_pass")
    rows = []
    for v in range(n):
        r = list(g.cols[g.offsets[v]:g.offsets[v + 1]][::-1])
        if v % 2 == 0 and r:
            small = [w for w in r[:16] if w < v]
            if small:
                r.append(min(small))                  # parallel copy of the first-pass edge
        if v % 7 == 0:
            r.append(v)                               # self-loop
        rows.append(r)
    # parallel copies must be symmetric: add the reverse arc for every copy
    for v in range(0, n, 2):
        small = [w for w in list(g.cols[g.offsets[v]:g.offsets[v + 1]][::-1])[:16] if w < v]
        if small:
            rows[min(small)].append(v)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    cols = np.array([w for r in rows for w in r], dtype=np.int32)
    return I.Graph(name="first_pass", n=n, offsets=off, cols=cols)


def test_first_pass_edge_cases(ctx, rst):
    g = first_pass_cases()
    try:
        for mode, sample in [(2, 0), (2, -1), (2, 2)]:
            run_case(ctx, rst, g, mode, sample)
    finally:
        ctx.set_option(rst.OPT_HOOK_MODE, 0)
        ctx.set_option(rst.OPT_HOOK_SAMPLE, -1)


def test_dominant_tree_found_on_dense_graphs(ctx, rst):
    """R-MAT (average degree above 6): two sampled arcs per vertex join most
    vertices, so the sweep skips the dominant tree."""
    st = run_case(ctx, rst, graph("rmat16"), 2, -1)
    assert st["paths"] & rst.PATH_HOOK_GIANT, st
    ctx.set_option(rst.OPT_HOOK_MODE, 0)
    # a chain has no dominant tree after one sampled arc per vertex: each edge once
    st = run_case(ctx, rst, graph("chain_2_18_int64"), 2, 1)
    assert not st["paths"] & rst.PATH_HOOK_GIANT, st
    ctx.set_option(rst.OPT_HOOK_MODE, 0)
    ctx.set_option(rst.OPT_HOOK_SAMPLE, -1)


@pytest.mark.parametrize("name,expect_global", [("random_200k", True), ("rmat16", True),
                                                ("grid_permuted_256", True),
                                                ("chain_2_18_int64", True), ("road_512", False)])
def test_automatic_choice(ctx, rst, name, expect_global):
    assert ctx.get_option(rst.OPT_HOOK_MODE) == 0
    g = graph(name)
    off, cols = dev(g.offsets_typed()), dev(g.cols)
    par, st = ctx.spanning_tree(off, cols, 0, "gconn", stats=True)
    assert bool(st["paths"] & rst.PATH_HOOK_GLOBAL) == expect_global, st
    # ids without locality: the tour is ranked by the sparse ruling set
    if expect_global:
        assert st["paths"] & rst.PATH_RANK_SPARSE, st
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par.cpu().numpy(), [0])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)


def test_replays_follow_the_data(rst):
    """Captured replays on fixed buffers: a random-id graph (global sweep), then
    a mesh of the same size copied into the same buffers (the replay sees that
    its first arcs stay in their tiles, and the next call captures the tile
    pass), then the random graph again; every output verified.  The probe of
    an eager call picks the global sweep for the first and not the second."""
    c = rst.Context(0)
    mesh = I.road_mesh(300, 0.0, 0.0, seed=3)
    n = mesh.n
    perm = np.random.RandomState(5).permutation(n).astype(np.int32)
    a, b = mesh.edge_list()
    rnd = I.csr_from_edges(n, perm[a], perm[b], name="mesh_permuted")
    assert rnd.nnz == mesh.nnz
    off = dev(rnd.offsets.astype(np.int32))
    cols = dev(rnd.cols)
    par = torch.empty(n, dtype=torch.int32, device="cuda")
    for g in [rnd] * 4 + [mesh] * 4 + [rnd] * 4:
        off.copy_(dev(g.offsets.astype(np.int32)))
        cols.copy_(dev(g.cols))
        par.fill_(-3)
        c.spanning_tree(off, cols, 0, "gconn", parent=par)
        assert c.last_status == 0
        code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par.cpu().numpy(), [0])
        assert code == 0, (g.name, oracle.VERIFY_CODES[code], bad)
    for g, expect in ((rnd, True), (mesh, False)):
        _, st = c.spanning_tree(dev(g.offsets.astype(np.int32)), dev(g.cols), 0, "gconn",
                                stats=True)
        assert bool(st["paths"] & rst.PATH_HOOK_GLOBAL) == expect, (g.name, st)


@pytest.mark.parametrize("mode", [1, 2])
def test_alternating_graphs_share_buffers(rst, mode):
    """Labels of three different graphs of the same size, computed in turn into
    one label buffer with one context (the workspace and the output keep the
    previous graph's values): bit for bit against the oracle every time."""
    c = rst.Context(0)
    c.set_option(rst.OPT_HOOK_MODE, mode)
    n = 120000
    gs = [I.random_graph(n, 180000, seed=41), I.random_graph(n, 60000, seed=42, connected=False),
          I.path(n, perm=np.random.RandomState(43).permutation(n).astype(np.int32))]
    refs = [oracle.components(g.n, g.offsets, g.cols) for g in gs]
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    for it in range(60):
        g = gs[it % 3]
        k_ref, lab_ref = refs[it % 3]
        _, k = c.components(dev(g.offsets_typed()), dev(g.cols), label=label)
        assert k == k_ref, (it, g.name)
        assert np.array_equal(label.cpu().numpy(), lab_ref), (it, g.name)
