"""fp64 reference of the BFS/GConn+Euler selector -- TEST INFRASTRUCTURE ONLY.

Plain numpy (float64) versions of: the per-graph features (degree moments and
capped BFS depth probes from splitmix64-chosen sources), the 8 -> 64 -> 64 -> 2
ReLU network, its weighted softmax cross-entropy, the gradient of that loss by
the chain rule written out layer by layer, and one Adam step (Kingma & Ba,
2015, Algorithm 1).  Only the test-suite and the benchmark's CPU leg use it.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as _core

N_IN, N_H, N_OUT = 8, 64, 2
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_OUT * N_H + N_OUT
PROBES, PROBE_LEVELS, PROBE_BALL = 3, 64, 1024
_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """splitmix64 finaliser applied after one golden-ratio increment."""
    x = (x + 0x9E3779B97F4A7C15) & _M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & _M64
    return x ^ (x >> 31)


GAMMA = 0x9E3779B97F4A7C15


def probe_source(g: int, s: int, b: int, n: int) -> int:
    """Source of probe s of graph g (first vertex b, n vertices): b plus the
    (3g + s + 1)-th output of the splitmix64 generator seeded with 0, mod n.
    The k-th output of that generator is the finaliser of k * GAMMA, i.e.
    splitmix64((k - 1) * GAMMA) here."""
    k = g * PROBES + s + 1
    return b + (splitmix64(((k - 1) * GAMMA) & _M64) % n if n > 0 else 0)


def features(offsets, cols, vtx_off):
    """[G][8] float64 features of every packed graph (definition in rst.h)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int32)
    vtx_off = np.asarray(vtx_off, dtype=np.int64)
    G = len(vtx_off) - 1
    out = np.zeros((G, N_IN))
    for g in range(G):
        b, e = int(vtx_off[g]), int(vtx_off[g + 1])
        n = e - b
        deg = (offsets[b + 1:e + 1] - offsets[b:e]).astype(np.float64)
        mean = deg.mean() if n else 0.0
        var = max((deg * deg).mean() - mean * mean, 0.0) if n else 0.0
        out[g, 0] = math.log(max(n, 1))
        out[g, 1] = math.log(1.0 + deg.sum() / 2.0)
        out[g, 2] = mean
        out[g, 3] = math.log1p(var)
        out[g, 4] = math.log1p(deg.max() if n else 0.0)
        # local CSR of graph g for the probes
        loc_off = offsets[b:e + 1] - offsets[b]
        loc_cols = cols[offsets[b]:offsets[e]] - b
        for s in range(PROBES):
            src = probe_source(g, s, b, n) - b
            level, _, _ = _core.bfs(n, loc_off, loc_cols, src)
            out[g, 5 + s] = math.log2(1.0 + probe_depth(level))
    return out


def probe_depth(level):
    """Depth reached by a probe, from the BFS levels of its graph (-1 where
    unreached): the source's eccentricity, capped at PROBE_LEVELS levels and
    at the first radius whose ball (vertices within that many hops) holds at
    least PROBE_BALL vertices."""
    reach = level[level >= 0]
    ecc = int(reach.max())
    ball = np.cumsum(np.bincount(reach, minlength=ecc + 1))
    big = np.nonzero(ball >= PROBE_BALL)[0]
    first_big = int(big[0]) if big.size else ecc
    return min(ecc, PROBE_LEVELS, first_big)


def unpack(params):
    p = np.asarray(params, dtype=np.float64).reshape(-1)
    assert p.size == N_PARAMS
    o = 0
    W1 = p[o:o + N_H * N_IN].reshape(N_H, N_IN); o += N_H * N_IN
    b1 = p[o:o + N_H]; o += N_H
    W2 = p[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = p[o:o + N_H]; o += N_H
    W3 = p[o:o + N_OUT * N_H].reshape(N_OUT, N_H); o += N_OUT * N_H
    b3 = p[o:o + N_OUT]; o += N_OUT
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def normalise(X, norm):
    norm = np.asarray(norm, dtype=np.float64)
    return (np.asarray(X, dtype=np.float64) - norm[:N_IN]) / np.maximum(norm[N_IN:], 1e-6)


def forward(params, Xn):
    """Logits [B][2] and the activations needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    a1 = Xn @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (Xn, a1, h1, a2, h2)


def loss_and_grad(params, Xn, y, w):
    """Mean over samples of w * softmax cross-entropy, and its gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    z, (x, a1, h1, a2, h2) = forward(params, Xn)
    B = z.shape[0]
    zm = z - z.max(axis=1, keepdims=True)
    p = np.exp(zm) / np.exp(zm).sum(axis=1, keepdims=True)
    y = np.asarray(y, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    loss = np.mean(-w * np.log(p[np.arange(B), y]))
    onehot = np.zeros_like(p)
    onehot[np.arange(B), y] = 1.0
    dz = (w[:, None] * (p - onehot)) / B            # d loss / d z
    gW3 = dz.T @ h2
    gb3 = dz.sum(axis=0)
    dh2 = (dz @ W3) * (a2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Kingma & Ba (2015), Algorithm 1, one iteration with 1-based step."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def choose(params, norm, X):
    """1 (BFS) where its logit is strictly larger and everything is finite."""
    X = np.asarray(X, dtype=np.float64)
    z, _ = forward(params, normalise(X, norm))
    ok = np.all(np.isfinite(X), axis=1) & np.all(np.isfinite(z), axis=1)
    return ((z[:, 1] > z[:, 0]) & ok).astype(np.uint8), z
