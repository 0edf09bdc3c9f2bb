"""GPU parity of the learned warm start (pooling, network forward, gradients,
Adam) against the FP64 oracle, through the C ABI.  The network's parameters
are drawn on the host by the oracle and uploaded.

Bars: split-precision products (bf16x3, FP32 accumulation): forward 1e-5,
gradients 1e-4 (relative, per parameter block); bf16 operands: forward
2e-2, gradients 5e-2 (measured errors printed).
"""
import numpy as np
import pytest

from oracle import mlp64
from paper_2309_04623_amd import nmf, synth
from tests.helpers import dev, host, say

pytestmark = pytest.mark.gpu


def _frames(F, ny, nx, seed):
    g = np.random.default_rng(seed)
    H = synth.components_speckle(g, 12, ny, nx)
    T = g.gamma(2.0, 1.0, (F, 12)) @ H
    T = g.poisson(T * 1e4 / T.max()) / 1e4 * T.max()
    MT = (g.random(T.shape) > 0.05) * synth.mask_wedge(ny, nx, 6.0)[None, :]
    return T.astype(np.float32), MT.astype(np.float32), H


@pytest.mark.parametrize("ny,nx", [(200, 200), (224, 288), (64, 64)])
def test_pool_parity(ny, nx):
    T, MT, _ = _frames(5, ny, nx, seed=ny + nx)
    say("ws pool", ny, nx)
    X, s = nmf.ws_pool(dev(T), dev(MT), ny, nx)
    Xo, so = mlp64.pool(T, MT, ny, nx)
    assert np.max(np.abs(host(s) - so) / so) < 1e-6
    assert np.max(np.abs(host(X) - Xo)) < 1e-5 * np.abs(Xo).max()


@pytest.fixture(scope="module")
def batch():
    g = np.random.default_rng(3)
    k, b = 40, 96
    p = mlp64.init_params(g, k)
    X = g.normal(0, 1, (b, 1024)).astype(np.float32)
    s = g.uniform(0.5, 2.0, b).astype(np.float32)
    H = g.gamma(1.0, 1.0, (k, 300))
    G = (H @ H.T).astype(np.float32)
    cstar = g.gamma(2.0, 1.0, (b, k)).astype(np.float32)
    return k, p, X, s, G, cstar


@pytest.mark.parametrize("precision,tol_f,tol_g", [("fp32", 1e-5, 1e-4), ("bf16", 2e-2, 5e-2)])
def test_forward_and_gradients(batch, precision, tol_f, tol_g):
    k, p, X, s, G, cstar = batch
    say("ws grads", precision)
    st = nmf.ws_state_from_params(p, k)
    C = host(nmf.ws_infer(st, dev(X), dev(s), k, precision))
    Co, _ = mlp64.forward(p, X.astype(np.float64), s.astype(np.float64))
    ef = np.max(np.abs(C - Co)) / np.abs(Co).max()
    loss, grads = nmf.ws_step(st, dev(X), dev(s), dev(cstar), dev(G), k, precision, want_grads=True)
    lo, go = mlp64.loss_and_grads(p, X.astype(np.float64), s.astype(np.float64),
                                  cstar.astype(np.float64), G.astype(np.float64))
    gg = nmf.ws_unpack(grads, k)
    eg = {n: np.linalg.norm(gg[n] - go[n]) / np.linalg.norm(go[n]) for n in nmf.WS_NAMES}
    print(f"  forward {ef:.2e} loss {abs(loss - lo) / lo:.2e} grads "
          + " ".join(f"{n}={v:.1e}" for n, v in eg.items()), flush=True)
    assert ef <= tol_f
    assert abs(loss - lo) / lo <= tol_g
    assert max(eg.values()) <= tol_g


def test_adam_step_matches_oracle(batch):
    k, p, X, s, G, cstar = batch
    say("ws adam")
    st = nmf.ws_state_from_params(p, k)
    nmf.ws_step(st, dev(X), dev(s), dev(cstar), dev(G), k, "fp32", lr=1e-3, step=1)
    pg = nmf.ws_unpack(st[: nmf.ws_param_count(k)], k)
    _, go = mlp64.loss_and_grads(p, X.astype(np.float64), s.astype(np.float64),
                                 cstar.astype(np.float64), G.astype(np.float64))
    po = mlp64.adam_step({n: v.copy() for n, v in p.items()}, go, {"m": {}, "v": {}}, 1, lr=1e-3)
    for n in nmf.WS_NAMES:
        d = np.abs(pg[n] - po[n])
        # the first Adam step is lr * sign(g): entries whose gradient is at
        # rounding level may take either sign
        assert np.mean(d < 1e-6) > 0.995, n


def test_training_lowers_the_loss():
    """A few epochs on projection targets of a small synthetic set lower the
    warm-start loss (the network learns the map frame -> coefficients)."""
    g = np.random.default_rng(5)
    ny = nx = 64
    k, F = 10, 512
    H = synth.components_speckle(g, k, ny, nx)
    W = g.gamma(2.0, 1.0, (F, k))
    T = (W @ H).astype(np.float32)
    MT = np.ones_like(T)
    say("ws train")
    X, s = nmf.ws_pool(dev(T), dev(MT), ny, nx)
    G = dev(H @ H.T)
    st = nmf.ws_init(k, seed=1)
    l0 = nmf.ws_step(st, X[:256], s[:256], dev(W[:256]), G, k)
    hist = nmf.ws_train(st, X, s, dev(W), G, k, epochs=20, batch=64, lr=1e-3, seed=2)
    l1 = nmf.ws_step(st, X[:256], s[:256], dev(W[:256]), G, k)
    print(f"  loss {l0:.3e} -> {l1:.3e}; epochs {hist[0]:.3e} .. {hist[-1]:.3e}", flush=True)
    assert np.all(np.isfinite(hist))
    assert l1 < 0.2 * l0
