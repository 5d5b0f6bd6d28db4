"""What the trained selector gains over the method without it.

The shipped network (selector_weights.bin, trained on the GPU by the library's
own kernels on graphs of seed 1000) chooses BFS or GConn+Euler for each graph
of a third family sample (seed 3000, disjoint from training and evaluation).
Both methods are timed standalone on every graph (median of 3 after a
warm-up): the selector must save at least half of what choosing the faster
method with hindsight saves over always running GConn+Euler (the fallback),
and stay within 10% of the per-graph best.  The single-graph
entry point with RST_AUTO must follow the same choice and return verified
trees.
"""
import numpy as np
import pytest

import oracle
from paper_2603_11645_amd import selector as S

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
    c = rst.Context(0)
    c.selector_load_default()
    return c


_GRAPHS = []


def graphs():
    if not _GRAPHS:
        _GRAPHS.extend(S.family_graph(i, seed=3000) for i in range(30))
    return _GRAPHS


def test_selector_gain_over_always_gconn(ctx):
    norm, params = S.load(S.WEIGHTS_PATH)
    ds = S.build_dataset(ctx, graphs(), reps=3, log=None)
    res = S.evaluate(ctx, norm, params, ds)
    print(res)
    assert res["chose_bfs"] > 0
    # less time than the method without the selector: at least half of what
    # choosing with hindsight would save ...
    available = res["ms_always_gconn"] - res["ms_best"]
    assert available > 0, res
    assert res["gain_vs_always_gconn"] >= 0.5 * available, res
    # ... and close to choosing the faster method with hindsight
    assert res["regret_vs_best"] <= 0.1 * res["ms_best"], res


@pytest.mark.parametrize("gi", [0, 1, 2, 3, 4, 8])
def test_auto_follows_selector(ctx, rst, gi):
    g = graphs()[gi]
    off = torch.from_numpy(np.ascontiguousarray(g.offsets_typed())).cuda()
    cols = torch.from_numpy(np.ascontiguousarray(g.cols)).cuda()
    b = S.I.pack([g])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    feat = ctx.features(off, cols, dev(b.vtx_off), dev(b.arc_off), dev(np.array([0], np.int32)))
    norm, params = S.load(S.WEIGHTS_PATH)
    _, choice = ctx.mlp_forward(dev(norm), dev(params), feat, logits=False)
    par, st = ctx.spanning_tree(off, cols, 0, "auto", stats=True)
    assert st["method_used"] == int(choice.cpu().numpy()[0])
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, par.cpu().numpy(), [0])
    assert code == 0, (oracle.VERIFY_CODES[code], bad)
