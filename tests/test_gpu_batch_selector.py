"""GPU tests of batched forests and of the learned selector's kernels.

Batches: every member graph's parent array is checked by the oracle verifier
(packed graph, one designated root per member); members assigned to BFS must
also form BFS trees (parent one level closer to the root, oracle levels).
Selector: features, forward logits, the training gradient and the Adam update
are compared with the fp64 oracle (oracle/mlp.py) within the fp32 tolerances
stated in each test.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as M
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


def small_batch(G=24, seed=7):
    # the disconnected random graph sits at index 25, a BFS member in "mixed" mode
    graphs = [I.batch_member(g, seed=seed, nmin=200, nmax=6000) for g in range(G)]
    graphs += [I.path(3), I.random_graph(400, 100, seed=3, connected=False), I.path(1),
               I.star(600, 5)]
    return I.pack(graphs)


BATCH = small_batch()


def upload_batch(b):
    g = b.graph
    return (dev(g.offsets_typed()), dev(g.cols), dev(b.vtx_off), dev(b.arc_off), dev(b.roots))


def check_forest(b, parent):
    g = b.graph
    code, bad = oracle.verify_rst(g.n, g.offsets, g.cols, parent, b.roots)
    assert code == 0, (oracle.VERIFY_CODES[code], bad)


def check_bfs_members(b, parent, method):
    g = b.graph
    for k in np.nonzero(method)[0]:
        v0, v1 = int(b.vtx_off[k]), int(b.vtx_off[k + 1])
        off = g.offsets[v0:v1 + 1] - g.offsets[v0]
        cols = g.cols[g.offsets[v0]:g.offsets[v1]] - v0
        level, _, _ = oracle.bfs(v1 - v0, off, cols, int(b.roots[k]) - v0)
        p = parent[v0:v1] - v0
        reach = np.nonzero(level > 0)[0]
        assert np.all(level[p[reach]] == level[reach] - 1)


@pytest.mark.parametrize("mode", ["gconn", "bfs", "mixed"])
def test_batch_forest_verified(ctx, mode):
    b = BATCH
    G = b.num_graphs
    if mode == "gconn":
        method = np.zeros(G, np.uint8)
    elif mode == "bfs":
        method = np.ones(G, np.uint8)
    else:
        method = (np.arange(G) % 3 == 1).astype(np.uint8)
    args = upload_batch(b)
    # every entry must be written: start from a poisoned buffer
    poison = torch.full((b.graph.n,), -7, dtype=torch.int32).cuda()
    parent, mout, st = ctx.spanning_forest_batch(*args, method=dev(method), stats=True,
                                                 parent=poison)
    parent = parent.cpu().numpy()
    assert np.array_equal(mout.cpu().numpy(), method)
    check_forest(b, parent)
    check_bfs_members(b, parent, method)


def test_batch_default_method_is_gconn(ctx):
    b = BATCH
    parent, mout = ctx.spanning_forest_batch(*upload_batch(b))
    assert np.all(mout.cpu().numpy() == 0)
    check_forest(b, parent.cpu().numpy())


def test_batch_rejects_root_outside_its_graph(ctx, rst):
    b = BATCH
    roots = b.roots.copy()
    roots[3] = int(b.vtx_off[4])          # a vertex of the next graph
    g = b.graph
    with pytest.raises(rst.RstError):
        ctx.spanning_forest_batch(dev(g.offsets_typed()), dev(g.cols), dev(b.vtx_off),
                                  dev(b.arc_off), dev(roots))


def test_features_match_oracle(ctx):
    b = BATCH
    feat = ctx.features(*upload_batch(b)).cpu().numpy()
    ref = M.features(b.graph.offsets, b.graph.cols, b.vtx_off)
    # fp64 accumulation on the device, rounded to fp32 at the end
    assert np.allclose(feat, ref, rtol=1e-6, atol=1e-6)


def _params(seed):
    return np.random.RandomState(seed).randn(M.N_PARAMS).astype(np.float32) * 0.2


def test_forward_logits_match_oracle(ctx):
    rs = np.random.RandomState(1)
    X = rs.randn(300, 8).astype(np.float32) * 3 + 1
    norm = np.concatenate([X.mean(0), X.std(0)]).astype(np.float32)
    params = _params(2)
    lg, ch = ctx.mlp_forward(dev(norm), dev(params), dev(X))
    c_ref, z_ref = M.choose(params.astype(np.float64), norm.astype(np.float64), X)
    lg = lg.cpu().numpy()
    # fp32 dot products of length <= 64 against fp64
    assert np.allclose(lg, z_ref, rtol=1e-4, atol=1e-4)
    clear = np.abs(z_ref[:, 1] - z_ref[:, 0]) > 1e-3
    assert np.array_equal(ch.cpu().numpy()[clear], c_ref[clear])


def test_feature_stats(ctx):
    X = np.random.RandomState(5).randn(1000, 8).astype(np.float32) * 2 + 3
    norm = ctx.feature_stats(dev(X)).cpu().numpy()
    assert np.allclose(norm[:8], X.astype(np.float64).mean(0), rtol=1e-6, atol=1e-6)
    assert np.allclose(norm[8:], X.astype(np.float64).std(0), rtol=1e-5, atol=1e-6)


def test_gradient_and_adam_match_oracle(ctx):
    rs = np.random.RandomState(3)
    B = 257
    X = rs.randn(B, 8).astype(np.float32)
    y = rs.randint(0, 2, B).astype(np.int32)
    w = rs.uniform(0.1, 2.0, B).astype(np.float32)
    norm = np.concatenate([np.zeros(8), np.ones(8)]).astype(np.float32)
    params = _params(4)
    loss_ref, g_ref = M.loss_and_grad(params.astype(np.float64), X.astype(np.float64), y, w)
    p_dev, m_dev, v_dev = dev(params), torch.zeros(M.N_PARAMS).cuda(), torch.zeros(M.N_PARAMS).cuda()
    grad = torch.empty(M.N_PARAMS).cuda()
    loss = ctx.mlp_train_step(dev(norm), p_dev, m_dev, v_dev, 1, 1e-3, dev(X), dev(y), dev(w),
                              grad=grad)
    assert abs(loss - loss_ref) <= 1e-5 * max(1.0, abs(loss_ref))
    g = grad.cpu().numpy()
    # fp32 accumulation over fan-in 64 and a batch of 257: rel 1e-4, abs floor 1e-6
    assert np.allclose(g, g_ref, rtol=1e-4, atol=1e-6)
    p_ref, _, _ = M.adam_step(params.astype(np.float64), g.astype(np.float64),
                              np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS), 1, 1e-3)
    assert np.allclose(p_dev.cpu().numpy(), p_ref, rtol=1e-5, atol=1e-7)


def test_selector_drives_batch_choice(ctx, rst):
    b = BATCH
    args = upload_batch(b)
    feat = ctx.features(*args)
    norm = ctx.feature_stats(feat)
    params = _params(9)
    c_ref, z_ref = M.choose(params.astype(np.float64), norm.cpu().numpy().astype(np.float64),
                            feat.cpu().numpy())
    ctx.selector_load(rst.selector_blob(norm.cpu().numpy(), params))
    parent, mout = ctx.spanning_forest_batch(*args)
    mout = mout.cpu().numpy()
    clear = np.abs(z_ref[:, 1] - z_ref[:, 0]) > 1e-3
    assert np.array_equal(mout[clear], c_ref[clear])
    check_forest(b, parent.cpu().numpy())
    check_bfs_members(b, parent.cpu().numpy(), mout)
    with pytest.raises(rst.RstError):
        ctx.selector_load(b"RSTSEL01" + b"\0" * 10)
    bad = bytearray(rst.selector_blob(norm.cpu().numpy(), params))
    bad[-4:] = np.array([np.nan], np.float32).tobytes()
    with pytest.raises(rst.RstError):
        ctx.selector_load(bytes(bad))


def test_batch_cross_graph_arc_rejected(ctx, rst):
    """With validation on, an arc whose neighbour lies in another graph of the
    batch is reported (RST_E_RANGE); the same batch without it passes."""
    a, b2 = I.path(50), I.path(60)
    b = I.pack([a, b2])
    g = b.graph
    cols = g.cols.copy()
    cols[g.offsets[10]] = 55          # vertex 10 of graph 0 -> a vertex of graph 1
    off, _, vo, ao, ro = upload_batch(b)
    ctx.set_option(rst.OPT_VALIDATE, 1)
    try:
        with pytest.raises(rst.RstError) as ei:
            ctx.spanning_forest_batch(off, dev(cols), vo, ao, ro)
        assert ei.value.code == rst.RST_E_RANGE
        par, _ = ctx.spanning_forest_batch(off, dev(g.cols), vo, ao, ro)
        check_forest(b, par.cpu().numpy())
    finally:
        ctx.set_option(rst.OPT_VALIDATE, 0)
