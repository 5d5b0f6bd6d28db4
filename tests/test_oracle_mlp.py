"""Pins of the fp64 selector oracle (no GPU): splitmix64 reference outputs,
central finite differences for the gradient, closed forms for the forward
pass, the first Adam step, and graph features on shapes with known answers."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_2603_11645_amd import inputs as I


# The first five outputs of the splitmix64 generator seeded with 0 (published
# reference implementation: state += golden gamma, then the finaliser).
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                    0xF88BB8A8724C81EC, 0x1B39896A51A8749B]


def test_splitmix64_reference_sequence():
    assert M.splitmix64(0) == 16294208416658607535
    assert M.splitmix64(0x9E3779B97F4A7C15) == 7960286522194355700
    for k, want in enumerate(SPLITMIX64_SEED0):
        assert M.splitmix64((k * M.GAMMA) % 2**64) == want


def test_probe_sources_are_the_published_outputs():
    # probe s of graph g takes the (3g + s + 1)-th output: graphs 0 and 1 use
    # outputs 1..3 and 4..6
    for (g, s), want in zip([(0, 0), (0, 1), (0, 2), (1, 0), (1, 1)], SPLITMIX64_SEED0):
        for b, n in ((0, 1000), (17, 7), (5, 2**31 - 1), (123456, 200000)):
            assert M.probe_source(g, s, b, n) == b + want % n
    assert M.probe_source(3, 1, 40, 1) == 40     # a one-vertex graph probes itself


def test_normalise_non_unit_moments_and_floor():
    X = np.array([[3.0, -2.0, 0.5, 10.0, 1.0, 2.0, -1.0, 4.0]])
    mean = np.array([1.0, 0.0, 0.5, -2.0, 0.0, 1.0, 1.0, 4.0])
    std = np.array([2.0, 4.0, 0.25, 3.0, 1e-9, 0.0, 0.5, 1e-6])
    Xn = M.normalise(X, np.concatenate([mean, std]))
    # (x - mean) / std, with std floored at 1e-6
    want = [1.0, -0.5, 0.0, 4.0, 1e6, 1e6, -4.0, 0.0]
    assert np.allclose(Xn[0], want, rtol=1e-12, atol=0)


def _random_case(seed, B=37):
    rs = np.random.RandomState(seed)
    params = rs.randn(M.N_PARAMS) * 0.3
    X = rs.randn(B, M.N_IN)
    y = rs.randint(0, 2, size=B)
    w = rs.uniform(0.1, 2.0, size=B)
    return params, X, y, w


@pytest.mark.parametrize("seed", range(3))
def test_gradient_central_differences(seed):
    params, X, y, w = _random_case(seed)
    loss, grad = M.loss_and_grad(params, X, y, w)
    rs = np.random.RandomState(100 + seed)
    idx = rs.choice(M.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        p1 = params.copy(); p1[i] += h
        p0 = params.copy(); p0[i] -= h
        fd = (M.loss_and_grad(p1, X, y, w)[0] - M.loss_and_grad(p0, X, y, w)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 + 1e-5 * abs(fd)


def test_forward_closed_forms():
    W1 = np.zeros((64, 8)); b1 = np.zeros(64); W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W3 = np.zeros((2, 64)); b3 = np.array([0.25, -1.5])
    params = M.pack(W1, b1, W2, b2, W3, b3)
    X = np.random.RandomState(0).randn(5, 8)
    z, _ = M.forward(params, X)
    assert np.allclose(z, b3)
    y = np.array([0, 1, 1, 0, 1]); w = np.array([1.0, 2.0, 0.5, 1.0, 3.0])
    lse = math.log(math.exp(0.25) + math.exp(-1.5))
    exp_loss = np.mean(w * (lse - b3[y]))
    assert abs(M.loss_and_grad(params, X, y, w)[0] - exp_loss) < 1e-12
    # one active path: z1 = 3 * 2 * relu(x0) + b3[1]
    W1[0, 0] = 1.0; W2[0, 0] = 2.0; W3[1, 0] = 3.0
    params = M.pack(W1, b1, W2, b2, W3, b3)
    X = np.zeros((2, 8)); X[0, 0] = -1.0; X[1, 0] = 0.5
    z, _ = M.forward(params, X)
    assert np.allclose(z[:, 0], 0.25)
    assert np.allclose(z[:, 1], [-1.5, 3.0 * 2.0 * 0.5 - 1.5])


def test_adam_first_step_closed_form():
    rs = np.random.RandomState(4)
    p = rs.randn(M.N_PARAMS); g = rs.randn(M.N_PARAMS)
    lr = 1e-3
    p1, m, v = M.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    # bias-corrected first moments equal g and g^2 at step 1
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-8))


def test_choose_rules():
    params = np.zeros(M.N_PARAMS)
    params[-2:] = [0.0, 0.0]                 # tie -> GConn+Euler (0)
    norm = np.concatenate([np.zeros(8), np.ones(8)])
    X = np.zeros((3, 8)); X[2, 3] = np.nan   # non-finite -> GConn+Euler
    c, _ = M.choose(params, norm, X)
    assert list(c) == [0, 0, 0]
    params[-1] = 1.0
    c, _ = M.choose(params, norm, X)
    assert list(c) == [1, 1, 0]


def test_features_closed_forms():
    n = 10
    path = I.path(n)
    star = I.star(7, 0)
    batch = I.pack([path, star])
    f = M.features(batch.graph.offsets, batch.graph.cols, batch.vtx_off)
    # path: degrees 1,2,...,2,1
    assert np.isclose(f[0, 0], math.log(10)) and np.isclose(f[0, 1], math.log(1 + 9))
    assert np.isclose(f[0, 2], 1.8) and np.isclose(f[0, 3], math.log1p(0.16))
    assert np.isclose(f[0, 4], math.log1p(2))
    for s in range(3):
        src = M.probe_source(0, s, 0, n)
        assert np.isclose(f[0, 5 + s], math.log2(1 + max(src, n - 1 - src)))
    # star with centre 0: depth 1 from the centre, 2 from a leaf
    for s in range(3):
        src = M.probe_source(1, s, 10, 7) - 10
        assert np.isclose(f[1, 5 + s], math.log2(1 + (1 if src == 0 else 2)))
    assert np.isclose(f[1, 4], math.log1p(6)) and np.isclose(f[1, 2], 12 / 7)
    # a path longer than the probe cap reports the cap
    long = I.pack([I.path(500)])
    f = M.features(long.graph.offsets, long.graph.cols, long.vtx_off)
    assert np.all(f[0, 5:] == math.log2(1 + 64))


def test_probe_stops_at_the_ball_cap():
    """A broom: a hub with 1500 leaves and a 100-vertex handle.  From the hub
    the ball of radius 1 already holds 1501 >= 1024 vertices, so the probe
    stops at depth 1 although the handle is 100 hops long; from the handle's
    far end the ball first reaches 1024 vertices at radius 100 (the hub's
    leaves), past the 64-level cap."""
    hub_leaves, handle = 1500, 100
    n = 1 + hub_leaves + handle
    eu = np.concatenate([np.zeros(hub_leaves, np.int32),
                         np.arange(hub_leaves + 1, n - 1, dtype=np.int32),
                         np.array([0], np.int32)])
    ev = np.concatenate([np.arange(1, hub_leaves + 1, dtype=np.int32),
                         np.arange(hub_leaves + 2, n, dtype=np.int32),
                         np.array([hub_leaves + 1], np.int32)])
    g = I.csr_from_edges(n, eu, ev)
    level_hub, _, _ = oracle.bfs(n, g.offsets, g.cols, 0)
    assert int(level_hub.max()) == handle
    assert M.probe_depth(level_hub) == 1
    level_end, _, _ = oracle.bfs(n, g.offsets, g.cols, n - 1)
    assert M.probe_depth(level_end) == 64
    # a 40 x 40 grid from a corner: r + 1 vertices at distance r <= 39, so the
    # ball of radius 39 holds 820; then 79 - r at distance r: 859, 897, 934,
    # 970, 1005, 1039 for r = 40 .. 45, first >= 1024 at r = 45 (< 64, < 78)
    grid = I.grid(40, 40, 0.0, seed=1)
    level_c, _, _ = oracle.bfs(grid.n, grid.offsets, grid.cols, 0)
    assert int(level_c.max()) == 78
    assert M.probe_depth(level_c) == 45
