"""GPU tests of the captured-graph path of rst_spanning_tree (RST_OPT_GRAPHS).

Replays are checked one by one, with the program's own eager work and
synchronisations between them: every replayed parent array must pass the
oracle verifier, equal the eager result on trees (where the rooted spanning
tree is unique), and stay correct when the graph, parent buffer, root or a
setting changes (which recaptures).
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


def upload(g):
    return (torch.from_numpy(np.ascontiguousarray(g.offsets_typed())).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.cols)).cuda())


def check(g, par, root):
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par.cpu().numpy(), [root])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)


def test_replays_verified_with_eager_work_between(rst):
    c = rst.Context(0)
    assert c.get_option(rst.OPT_GRAPHS) == 1
    g = I.road_mesh(300, 0.15, 0.001, seed=5)
    off, cols = upload(g)
    par = torch.empty(g.n, dtype=torch.int32).cuda()
    other = I.rmat_lcc(12, 8, seed=6)
    ooff, ocols = upload(other)
    for i in range(6):
        par.fill_(-3)
        c.spanning_tree(off, cols, 7, "gconn", parent=par)
        check(g, par, 7)
        # eager work of the program and of the library between replays
        x = torch.arange(1000, device="cuda").sum().item()
        assert x == 499500
        if i % 2:
            lab, k = c.components(ooff, ocols)
            assert k == 1
        if i == 3:
            _, st = c.spanning_tree(off, cols, 7, "gconn", stats=True)   # eager, with events
        torch.cuda.synchronize()


def test_replay_equals_eager_on_trees(rst):
    g = I.random_tree(50000, seed=9)
    off, cols = upload(g)
    eager = rst.Context(0)
    eager.set_option(rst.OPT_GRAPHS, 0)
    ref = eager.spanning_tree(off, cols, 123, "gconn").cpu().numpy()
    c = rst.Context(0)
    par = torch.empty(g.n, dtype=torch.int32).cuda()
    for _ in range(4):
        par.fill_(-1)
        c.spanning_tree(off, cols, 123, "gconn", parent=par)
        assert np.array_equal(par.cpu().numpy(), ref)


def test_recapture_on_changes(rst):
    c = rst.Context(0)
    g1 = I.grid(200, 200, 0.2, seed=3)
    g2 = I.long_chain(30000, 0.01, 64, seed=4, offset_bytes=8)
    o1, c1 = upload(g1)
    o2, c2 = upload(g2)
    p1 = torch.empty(g1.n, dtype=torch.int32).cuda()
    p2 = torch.empty(g1.n, dtype=torch.int32).cuda()
    for root in (0, 999):
        c.spanning_tree(o1, c1, root, "gconn", parent=p1)
        check(g1, p1, root)
    c.spanning_tree(o1, c1, 5, "gconn", parent=p2)          # other parent buffer
    check(g1, p2, 5)
    c.set_option(rst.OPT_SWEEP_BLOCK, 512)                    # other setting
    c.spanning_tree(o1, c1, 5, "gconn", parent=p2)
    check(g1, p2, 5)
    c.set_option(rst.OPT_SWEEP_BLOCK, 256)
    par = c.spanning_tree(o2, c2, 11, "gconn")                # other graph (int64 offsets)
    check(g2, par, 11)
    c.spanning_tree(o1, c1, 5, "gconn", parent=p1)            # back to the first one
    check(g1, p1, 5)


def chains_linked_across_tiles(n, seed):
    """Chains of 8 consecutive ids, each chain's first vertex joined to a
    random vertex of a random earlier chain: few edges cross vertex tiles
    (ids keep their locality), yet the tour leaves its arc tile at about a
    quarter of the arcs, far more exits than one workgroup ranks."""
    rs = np.random.RandomState(seed)
    v = np.arange(n)
    inner = v[(v % 8) != 7]
    inner = inner[inner + 1 < n]
    starts = np.arange(8, n, 8)
    links = rs.randint(0, starts)
    eu = np.concatenate([inner, starts]).astype(np.int32)
    ev = np.concatenate([inner + 1, links]).astype(np.int32)
    return I.csr_from_edges(n, eu, ev, name="linked_chains")


def test_replays_with_contracted_list_fallback(rst):
    """A graph whose contracted tour list is too long for the one-workgroup
    ranking: every replay finishes with the sparse ruling set after the call's
    synchronisation, and must still give a verified tree and report one
    component (the components are counted once, in the replayed pass)."""
    c = rst.Context(0)
    g = chains_linked_across_tiles(300000, seed=11)
    off, cols = upload(g)
    par = torch.empty(g.n, dtype=torch.int32).cuda()
    p0, st = c.spanning_tree(off, cols, 11, "gconn", stats=True)
    check(g, p0, 11)
    assert 2 * st["cross_edges"] <= g.n, st          # the per-tile ranking is chosen
    assert st["paths"] & rst.PATH_RANK_SPARSE and st["components"] == 1, st
    assert not st["paths"] & rst.PATH_RANK_GLOBAL, st
    for _ in range(3):
        par.fill_(-3)
        c.spanning_tree(off, cols, 11, "gconn", parent=par)   # raises if not one component
        assert c.last_status == 0
        check(g, par, 11)


def test_replays_report_disconnected_and_counts(rst):
    """The replayed calls read their counters as the last kernel left them:
    a graph of two components reports RST_E_DISCONNECTED on every replay, and a
    connected graph on the same context afterwards (a new capture) succeeds on
    every replay, its tree verified each time."""
    c = rst.Context(0)
    a = I.road_mesh(120, 0.1, 0.01, seed=21)
    n = a.n
    # two copies of the mesh side by side: two components at least
    offs = np.concatenate([a.offsets[:-1], a.offsets + a.nnz]).astype(np.int64)
    cols = np.concatenate([a.cols, a.cols + n]).astype(np.int32)
    k_ref, _ = oracle.components(2 * n, offs, cols)
    assert k_ref >= 2
    doff = torch.from_numpy(offs.astype(np.int32)).cuda()
    dcols = torch.from_numpy(cols).cuda()
    par = torch.empty(2 * n, dtype=torch.int32).cuda()
    for _ in range(3):
        c.spanning_tree(doff, dcols, 0, "gconn", parent=par)
        assert c.last_status == rst.RST_E_DISCONNECTED
        p = par.cpu().numpy()
        roots = np.flatnonzero(p == np.arange(2 * n))   # the root and the second copy's own root
        assert len(roots) == 2 and roots[0] == 0 and n <= roots[1] < 2 * n
    off1, cols1 = upload(a)
    par1 = torch.empty(n, dtype=torch.int32).cuda()
    for _ in range(3):
        par1.fill_(-3)
        c.spanning_tree(off1, cols1, 5, "gconn", parent=par1)
        assert c.last_status == 0
        check(a, par1, 5)
