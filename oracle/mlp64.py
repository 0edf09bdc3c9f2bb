"""FP64 reference of the learned warm start for target modelling (oracle).

Not in the paper: a small network predicts a frame's projection
coefficients so that the Eq. 3 W-rule iteration (Sec. 4.1, target
modelling) starts near its limit; the iteration itself is unchanged and
cold start stays the fallback.

Definitions (all float64):
  pooling   s = masked mean of t over pixels with m > 0 (1 if none);
            the ny x nx frame is padded with weight 0 to 32*by x 32*bx,
            by = ceil(ny/32), bx = ceil(nx/32), and each by x bx block is
            averaged over its pixels with m > 0 (0 if none); x = pooled / s
  network   a1 = x W1 + b1,  h1 = gelu(a1)          (1024 -> 512)
            a2 = h1 W2 + b2, h2 = gelu(a2)          (512 -> 512)
            z  = h2 W3 + b3                          (512 -> K)
            w  = max(s * softplus(z), 1e-6 s)
  gelu(u)   = u/2 (1 + erf(u / sqrt 2)),  softplus(u) = log(1 + e^u)
  loss      L = mean_f (w_f - w*_f) G (w_f - w*_f)^T / (w*_f G w*_f^T),
            G = H H^T (K x K), the model-space error relative to the target
  Adam      m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
            p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
from __future__ import annotations

import math

import numpy as np

SQRT_HALF = 1.0 / math.sqrt(2.0)
FLOOR_REL = 1e-6
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def _erf(x):
    from scipy.special import erf
    return erf(x)


def gelu(u):
    return 0.5 * u * (1.0 + _erf(u * SQRT_HALF))


def gelu_grad(u):
    return 0.5 * (1.0 + _erf(u * SQRT_HALF)) + u * INV_SQRT_2PI * np.exp(-0.5 * u * u)


def softplus(u):
    return np.logaddexp(0.0, u)


def sigmoid(u):
    return 0.5 * (1.0 + np.tanh(0.5 * u))


def pool(T, MT, ny, nx, grid=32):
    """Masked-mean pooling of F frames (F x ny*nx) to F x grid*grid, and the
    per-frame masked mean s."""
    T = np.asarray(T, np.float64)
    MT = np.asarray(MT, np.float64)
    F = T.shape[0]
    by, bx = -(-ny // grid), -(-nx // grid)
    on = MT > 0
    tv = np.where(on, T, 0.0)
    cnt = on.sum(axis=1)
    s = np.where(cnt > 0, tv.sum(axis=1) / np.maximum(cnt, 1), 1.0)
    s = np.where(s > 0, s, 1.0)
    X = np.zeros((F, grid, grid))
    tv = tv.reshape(F, ny, nx)
    on = on.reshape(F, ny, nx)
    pt = np.zeros((F, grid * by, grid * bx))
    po = np.zeros((F, grid * by, grid * bx))
    pt[:, :ny, :nx] = tv
    po[:, :ny, :nx] = on
    bs = pt.reshape(F, grid, by, grid, bx).sum(axis=(2, 4))
    bc = po.reshape(F, grid, by, grid, bx).sum(axis=(2, 4))
    X = np.where(bc > 0, bs / np.maximum(bc, 1), 0.0)
    return X.reshape(F, grid * grid) / s[:, None], s


def init_params(rng: np.random.Generator, k, d_in=1024, d_h=512):
    """He-style normal init (weights), zero biases."""
    W1 = rng.normal(0, math.sqrt(2.0 / d_in), (d_in, d_h))
    W2 = rng.normal(0, math.sqrt(2.0 / d_h), (d_h, d_h))
    W3 = rng.normal(0, math.sqrt(1.0 / d_h), (d_h, k))
    return {"W1": W1, "b1": np.zeros(d_h), "W2": W2, "b2": np.zeros(d_h), "W3": W3,
            "b3": np.zeros(k)}


def forward(p, X, s):
    a1 = X @ p["W1"] + p["b1"]
    h1 = gelu(a1)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(a2)
    z = h2 @ p["W3"] + p["b3"]
    raw = s[:, None] * softplus(z)
    floor = FLOOR_REL * s[:, None]
    w = np.maximum(raw, floor)
    cache = {"X": X, "s": s, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "z": z,
             "live": raw > floor}
    return w, cache


def loss(w, wstar, G):
    d = w - wstar
    num = np.einsum("fk,kl,fl->f", d, G, d)
    den = np.einsum("fk,kl,fl->f", wstar, G, wstar)
    return float(np.mean(num / den))


def loss_grad(w, wstar, G):
    d = w - wstar
    den = np.einsum("fk,kl,fl->f", wstar, G, wstar)
    return 2.0 * (d @ G) / den[:, None] / w.shape[0]


def backward(p, cache, dw):
    """Gradients of the loss w.r.t. every parameter given dL/dw."""
    s = cache["s"]
    dz = dw * s[:, None] * sigmoid(cache["z"]) * cache["live"]
    g = {"W3": cache["h2"].T @ dz, "b3": dz.sum(axis=0)}
    dh2 = dz @ p["W3"].T
    da2 = dh2 * gelu_grad(cache["a2"])
    g["W2"] = cache["h1"].T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"].T
    da1 = dh1 * gelu_grad(cache["a1"])
    g["W1"] = cache["X"].T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def loss_and_grads(p, X, s, wstar, G):
    w, cache = forward(p, X, s)
    return loss(w, wstar, G), backward(p, cache, loss_grad(w, wstar, G))


def adam_step(p, g, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); state holds 'm' and 'v' dicts."""
    for name in p:
        m = state["m"].setdefault(name, np.zeros_like(p[name]))
        v = state["v"].setdefault(name, np.zeros_like(p[name]))
        m[...] = b1 * m + (1 - b1) * g[name]
        v[...] = b2 * v + (1 - b2) * g[name] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)
    return p
