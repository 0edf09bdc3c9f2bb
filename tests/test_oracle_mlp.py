"""Pins for the FP64 warm-start network oracle: library definitions of the
activations, central finite differences for every gradient, a closed form
for the pooling, and a textbook Adam step."""
import math

import numpy as np
import pytest

from oracle import mlp64


def test_activations_against_library_and_calculus():
    u = np.linspace(-8, 8, 2001)
    want = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in u])
    assert np.max(np.abs(mlp64.gelu(u) - want)) < 1e-15
    assert np.max(np.abs(mlp64.softplus(u) - np.log1p(np.exp(u)))) < 1e-12
    h = 1e-6
    fd = (mlp64.gelu(u + h) - mlp64.gelu(u - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp64.gelu_grad(u))) < 1e-8
    fd = (mlp64.softplus(u + h) - mlp64.softplus(u - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp64.sigmoid(u))) < 1e-8


def test_pool_closed_form():
    """A frame whose pixel values equal their 2x2-block index, one masked
    pixel per block and one block fully masked: each pooled value is the block
    index over the masked mean."""
    ny = nx = 64
    t = np.zeros((ny, nx))
    m = np.ones((ny, nx))
    for i in range(32):
        for j in range(32):
            t[2 * i:2 * i + 2, 2 * j:2 * j + 2] = i * 32 + j + 1
            m[2 * i, 2 * j] = 0
    m[0:2, 2:4] = 0  # block (0, 1) fully masked
    t[0, 0] = 1e9    # masked pixels are ignored
    X, s = mlp64.pool(t.reshape(1, -1), m.reshape(1, -1), ny, nx)
    on = m > 0
    smean = t[on].mean()
    assert abs(s[0] - smean) < 1e-9 * smean
    want = (np.arange(1024) + 1.0) / smean
    want[1] = 0.0
    assert np.max(np.abs(X[0] - want)) < 1e-12


def test_pool_pads_ragged_frames():
    ny, nx = 200, 200   # blocks of 7 x 7 over a 224 x 224 padded frame
    g = np.random.default_rng(0)
    t = g.uniform(1, 2, (2, ny * nx))
    m = (g.random((2, ny * nx)) > 0.3).astype(float)
    X, s = mlp64.pool(t, m, ny, nx)
    tt = t[0].reshape(ny, nx)
    mm = m[0].reshape(ny, nx)
    blk = (slice(28 * 7, 200), slice(0, 7))  # last block row is only 4 px tall
    v = tt[blk][mm[blk] > 0].mean() / s[0]
    assert abs(X[0, 28 * 32 + 0] - v) < 1e-12
    assert np.all(X[:, 29 * 32:] == 0)  # rows beyond the frame are padding


@pytest.fixture(scope="module")
def net():
    g = np.random.default_rng(1)
    k, F = 7, 5
    p = mlp64.init_params(g, k, d_in=24, d_h=16)
    X = g.normal(0, 1, (F, 24))
    s = g.uniform(0.5, 2.0, F)
    H = g.gamma(1.0, 1.0, (k, 40))
    G = H @ H.T
    wstar = g.gamma(2.0, 1.0, (F, k))
    return p, X, s, wstar, G


def test_every_gradient_matches_central_differences(net):
    p, X, s, wstar, G = net
    _, grads = mlp64.loss_and_grads(p, X, s, wstar, G)
    h = 1e-6
    for name, val in p.items():
        flat = val.reshape(-1)
        idx = np.random.default_rng(2).choice(flat.size, min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = mlp64.loss_and_grads(p, X, s, wstar, G)[0]
            flat[i] = old - h
            lm = mlp64.loss_and_grads(p, X, s, wstar, G)[0]
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, an)


def test_loss_zero_at_target_and_scale_free(net):
    p, X, s, wstar, G = net
    assert mlp64.loss(wstar, wstar, G) == 0.0
    w = wstar * 1.1
    assert abs(mlp64.loss(w, wstar, G) - 0.01) < 1e-12
    assert abs(mlp64.loss(3 * w, 3 * wstar, G) - mlp64.loss(w, wstar, G)) < 1e-14


def test_adam_first_step_is_signed_learning_rate():
    """With bias correction the first Adam step moves every parameter by
    lr * sign(g) (up to eps)."""
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -1e-3, 2.0])}
    st = {"m": {}, "v": {}}
    out = mlp64.adam_step({k: v.copy() for k, v in p.items()}, g, st, 1, lr=0.01, eps=0.0)
    assert np.allclose(out["a"], p["a"] - 0.01 * np.sign(g["a"]), rtol=0, atol=1e-15)
