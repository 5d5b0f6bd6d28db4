"""GPU parity at the full workload sizes, with the library's default settings
(the launch configuration the benchmark times).

For each workload (C1 permuted grid, C2 road-like mesh, C3 R-MAT scale 22,
C4 long chain with int64 offsets): min-id component labels bit-exact against
the oracle; the GConn+Euler parent array accepted by the oracle verifier and
by the device verifier; the stage variants that ran are the expected ones.
BFS levels are compared bit for bit and BFS parents checked (one level
closer to the root, and the whole tree through the verifier on C1-C3) on all
four; C4's BFS runs about 1.3e7 levels, tens of seconds of GPU time.
"""
import numpy as np
import pytest

import oracle
from paper_2603_11645_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_GRAPHS = {}


def graph(name):
    if name not in _GRAPHS:
        _GRAPHS.clear()                     # one full-size graph in memory at a time
        _GRAPHS[name] = I.config(name)
    return _GRAPHS[name]


@pytest.fixture(scope="module")
def rst():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11645_amd as r
    return r


@pytest.fixture(scope="module")
def ctx(rst):
    return rst.Context(0)


def upload(g):
    return (torch.from_numpy(np.ascontiguousarray(g.offsets_typed())).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.cols)).cuda())


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C4"])
def test_fullsize(ctx, rst, name):
    g = graph(name)
    off, cols = upload(g)
    k_ref, lab_ref = oracle.components(g.n, g.offsets, g.cols)
    assert k_ref == 1
    label, k = ctx.components(off, cols)
    assert k == 1
    assert np.array_equal(label.cpu().numpy(), lab_ref)
    par, st = ctx.spanning_tree(off, cols, g.root, "gconn", stats=True)
    assert ctx.last_status == 0 and st["components"] == 1
    p = par.cpu().numpy()
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, p, [g.root])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)
    assert ctx.verify(off, cols, g.root, par) == (0, -1)
    if name == "C2":
        # mesh: its 10k kept cross edges merged in LDS per group of tiles and
        # then the top levels, the contracted tour ranked in one workgroup
        assert st["paths"] == 4, st
    check_tuned(rst, g, off, cols, k_ref, lab_ref)
    if name == "C4":
        return   # its BFS (1.3e7 levels) has a test of its own below
    check_bfs(ctx, g, off, cols)


def check_tuned(rst, g, off, cols, k_ref, lab_ref):
    """The launch configuration the benchmark times: the committed autotuner
    cache's setting for this graph's size class (bench.py applies it)."""
    import os
    path = os.path.join(os.path.dirname(rst.__file__), "tuned_gfx950.json")
    c = rst.Context(0)
    assert c.tune_load(path, off, cols, "gconn")
    label, k = c.components(off, cols)
    assert k == k_ref and np.array_equal(label.cpu().numpy(), lab_ref)
    par = c.spanning_tree(off, cols, g.root, "gconn")
    par = c.spanning_tree(off, cols, g.root, "gconn")   # the captured graph's replay
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par.cpu().numpy(), [g.root])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)


def check_bfs(ctx, g, off, cols):
    level, parent, st = ctx.bfs(off, cols, g.root, stats=True)
    lref, _, ecc = oracle.bfs(g.n, g.offsets, g.cols, g.root)
    assert np.array_equal(level.cpu().numpy(), lref)
    assert st["bfs_levels"] == ecc
    par = parent.cpu().numpy()
    v = np.nonzero(lref > 0)[0]
    assert np.all(lref[par[v]] == lref[v] - 1)
    assert par[g.root] == g.root
    if g.n > (1 << 23):
        return   # the verifier's pass over C4 adds nothing the level check misses
    par = ctx.spanning_tree(off, cols, g.root, "bfs").cpu().numpy()
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par, [g.root])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)
    v = np.nonzero(lref > 0)[0]
    assert np.all(lref[par[v]] == lref[v] - 1)


def test_fullsize_c4_bfs(ctx):
    """The long chain's BFS: about 1.3e7 levels, nearly all of them run by one
    workgroup many levels to a launch (tens of seconds); levels bit for bit
    against the oracle's FIFO BFS, parents one level closer to the root."""
    g = graph("C4")
    off, cols = upload(g)
    check_bfs(ctx, g, off, cols)
