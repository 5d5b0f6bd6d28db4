"""GPU parity of rst_biconnected (Tarjan and Vishkin's biconnected components
from a rooted spanning tree; the downstream use of an RST named in Sec. I and
at the opening of Sec. IV) against the oracle's Hopcroft-Tarjan search.

The partition of the arcs into components is unique, the labels are not: both
sides are compared through canonical labels (each arc's label replaced by the
smallest arc index with the same label), bit for bit; articulation points and
the component count are unique and compared directly.  Every graph is run
with the spanning tree of GConn+Euler and with the BFS tree (different trees,
the same components), including multigraphs, self-loops, trees, cycles, a
hand-worked graph, random graphs, meshes, R-MAT graphs, long chains, and the
four full-size workloads."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_2603_11645_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11645_amd as r
    return r.Context(0)


def multigraph(n, edges):
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
    return I.Graph(name="multi", n=n, offsets=off, cols=cols, root=0, offset_bytes=4)


def check(ctx, g, methods=("gconn", "bfs")):
    off = torch.from_numpy(np.ascontiguousarray(g.offsets_typed())).cuda()
    cols = torch.from_numpy(np.ascontiguousarray(g.cols)).cuda()
    lab_ref, art_ref, k_ref = oracle.bcc(g.n, g.offsets, g.cols)
    can_ref = oracle.canonical_labels(lab_ref)
    for method in methods:
        par = ctx.spanning_tree(off, cols, g.root, method)
        lab, art, k = ctx.biconnected(off, cols, par)
        lab = lab.cpu().numpy()
        assert np.array_equal(oracle.canonical_labels(lab), can_ref), (g.name, method)
        assert np.array_equal(art.cpu().numpy(), art_ref), (g.name, method)
        assert k == k_ref, (g.name, method, k, k_ref)
        # labels are tree-edge children: vertex ids that are no root
        used = np.unique(lab[lab >= 0])
        pv = par.cpu().numpy()
        assert np.all(pv[used] != used)


def small_graphs():
    gs = [I.path(9), I.star(40, 3), I.random_tree(3000, seed=4)]
    n = 7
    gs.append(I.csr_from_edges(n, np.arange(n, dtype=np.int32),
                               ((np.arange(n) + 1) % n).astype(np.int32), name="cycle"))
    k5 = np.array(list(itertools.combinations(range(5), 2)), np.int32)
    gs.append(I.csr_from_edges(5, k5[:, 0], k5[:, 1], name="k5"))
    bow = np.array([(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 2)], np.int32)
    gs.append(I.csr_from_edges(5, bow[:, 0], bow[:, 1], name="bowtie"))
    with open(os.path.join(GOLDEN, "bcc_example10.json")) as f:
        case = json.load(f)
    e = np.array(case["edges"], np.int32)
    gs.append(I.csr_from_edges(case["n"], e[:, 0], e[:, 1], name="hand10"))
    gs.append(multigraph(4, [(0, 1), (0, 1), (1, 2), (2, 2), (2, 3), (3, 1), (3, 3)]))
    gs.append(multigraph(3, [(0, 1), (1, 2), (1, 2), (2, 0)]))
    gs.append(I.path(1))
    gs.append(I.path(2))
    for s in range(6):
        gs.append(I.random_graph(2000 + 500 * s, 2400 + 900 * s, seed=10 + s))
    gs.append(I.road_mesh(96, 0.3, 0.01, seed=3))
    gs.append(I.grid_permuted(80, seed=5))
    gs.append(I.rmat_lcc(12, 4, seed=6))
    gs.append(I.long_chain(50000, 0.01, 16, seed=7, offset_bytes=8))
    return gs


@pytest.mark.parametrize("i", range(24))
def test_small_and_medium(ctx, i):
    gs = small_graphs()
    if i >= len(gs):
        pytest.skip("no such graph")
    check(ctx, gs[i])


def test_blocks_of_the_extremum_structure(ctx):
    """Cycles of every length around one and two 64-position blocks, hung off a
    path: subtree ranges that start and end inside, at and across block
    borders."""
    for L in (62, 63, 64, 65, 127, 128, 129, 200):
        n = 300
        eu = list(range(n - 1))
        ev = list(range(1, n))
        for s in (0, 17, 63, 64, 100):
            if s + L < n:
                eu.append(s)
                ev.append(s + L)
        g = I.csr_from_edges(n, np.array(eu, np.int32), np.array(ev, np.int32), name="cyc%d" % L)
        check(ctx, g)


def test_errors(ctx):
    import paper_2603_11645_amd as r
    g = I.path(10)
    off = torch.from_numpy(g.offsets_typed()).cuda()
    cols = torch.from_numpy(g.cols).cuda()
    par = torch.arange(10, dtype=torch.int32, device="cuda")   # every vertex a root
    with pytest.raises(r.RstError) as e:
        ctx.biconnected(off, cols, par)
    assert e.value.code == r.RST_E_DISCONNECTED


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C4"])
def test_fullsize(ctx, name):
    g = I.config(name)
    check(ctx, g, methods=("gconn",))
