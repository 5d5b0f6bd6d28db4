"""GPU parity of the Path-Reversal RST (Sec. III-C).

Which tree PR-RST returns depends on which edge wins each root's graft (any
may), so its parent arrays are checked by the oracle's verifier (the RST
definition per component, pinned by Kirchhoff enumeration); on tree inputs
the answer is unique and is compared bit for bit, the hand-worked case of
tests/golden included.  The iteration count is bounded like the oracle's.
"""
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
    import paper_2603_11645_amd as rst
    return rst.Context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(ctx, g, root):
    off, cols = dev(g.offsets_typed()), dev(g.cols)
    par, st = ctx.spanning_tree(off, cols, root, "pr_rst", stats=True)
    return par.cpu().numpy(), st


def test_golden_and_trees(ctx):
    with open(os.path.join(GOLDEN, "pr_rst_reversal4.json")) as f:
        case = json.load(f)
    g = I.csr_from_edges(case["n"], np.array(case["eu"]), np.array(case["ev"]))
    for r, want in case["rooted"].items():
        par, _ = run(ctx, g, int(r))
        assert list(par) == want
    for n, seed in ((1, 0), (2, 1), (3000, 2), (200000, 3)):
        t = I.random_tree(n, seed=seed) if n > 2 else I.path(n)
        eu, ev = t.edge_list()
        root = (seed * 7919) % n
        par, st = run(ctx, t, root)
        assert np.array_equal(par, oracle.dfs_root(n, eu, ev, [root]))
        assert st["components"] == 1


@pytest.mark.parametrize("gi", range(8))
def test_verified(ctx, gi):
    g = [I.grid(31, 37, 0.3, seed=2), I.grid_permuted(128, seed=1), I.road_mesh(200, 0.15, 0.01, seed=2),
         I.rmat_lcc(13, 16, seed=3), I.long_chain(100000, 0.005, 64, seed=4, offset_bytes=8),
         I.random_graph(20000, 30000, seed=5, connected=True),
         I.random_graph(20000, 8000, seed=6, connected=False), I.star(50001, 9)][gi]
    for root in (0, g.n // 2):
        par, st = run(ctx, g, root)
        code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par, [root])
        assert code == 0, (g.name, oracle.VERIFY_CODES[code], bad)
        k, _ = oracle.components(g.n, g.offsets, g.cols)
        assert st["components"] == k
        assert 1 <= st["hook_rounds"] <= 4 * int(np.ceil(np.log2(g.n))) + 8
