"""FP64 reference of the steps around the factorisation (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``frame_distances`` / ``closest_frames`` -- reference selection (Sec. 4.1:
  a percentage of the library frames closest to the target, by the Euclidean
  norm, the cost NMF itself minimises; Sec. 5.3: the largest SNR gain).
* ``best_factor`` -- the per-frame scale of the model PSF applied before
  subtraction ("best factor finding", Sec. 2 and Sec. 4.1, after Ren et al.
  2018).  The paper does not define it; the reading here is the scale that
  minimises the standard deviation of the residual t - s (c H) over the
  frame's valid pixels inside an optional region (the region keeps the
  circumstellar signal out of the fit), clamped to a caller range.
* ``build_basis_sequential`` -- component-by-component construction (the
  variant of the basis build the paper's package uses, Sec. 2): stage j
  starts from the j - 1 components of stage j - 1 plus one new random
  component and runs the Eq. 3 iteration.

Readings of points the paper leaves open (each applies on the GPU too):

* Distance: the squared Euclidean norm of t - v over the pixels valid in
  both frames (weight > 0 in the target and in the reference); data under
  zero weight are ignored whatever their value.
* Selection: per target, the ``n_sel`` references of smallest distance,
  ordered by distance, equal distances by reference index.
* Best factor: s = cov(t, m) / var(m) over the pixels used (the exact
  minimiser of the residual variance, a quadratic in s), then clamped to
  [s_lo, s_hi]; s = 1 when fewer than two pixels are used or the model is
  constant over them (var(m) <= 1e-12 mean(m^2)).
* Sequential build: the new component of stage j takes W column j - 1 from
  the seeded U(0,1) stream of matrix id 3 and H row j - 1 from matrix id 4,
  both at the indices they would have in an n x K / K x p matrix, so that a
  stage's start depends only on the seed and the previous stage.
"""
from __future__ import annotations

import numpy as np

from oracle import nmf64, prng

MAT_SEQ_W = 3
MAT_SEQ_H = 4


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# Reference selection (Sec. 4.1)
# --------------------------------------------------------------------------

def frame_distances(T, MT, V, M):
    """d[f, n] = sum_p [MT_fp > 0][M_np > 0] (T_fp - V_np)^2, in FP64, by a
    plain loop over target frames."""
    T, MT, V, M = _f64(T), _f64(MT), _f64(V), _f64(M)
    vv = M > 0
    Vh = np.where(vv, V, 0.0)
    d = np.zeros((T.shape[0], V.shape[0]))
    for f in range(T.shape[0]):
        tv = MT[f] > 0
        th = np.where(tv, T[f], 0.0)
        both = vv & tv[None, :]
        diff = np.where(both, th[None, :] - Vh, 0.0)
        d[f] = np.sum(diff * diff, axis=1)
    return d


def closest_frames(T, MT, V, M, n_sel):
    """Indices (f x n_sel) of the n_sel references closest to each target,
    by increasing distance, ties by increasing reference index."""
    d = frame_distances(T, MT, V, M)
    idx = np.empty((d.shape[0], n_sel), np.int64)
    for f in range(d.shape[0]):
        order = sorted(range(d.shape[1]), key=lambda n: (d[f, n], n))
        idx[f] = order[:n_sel]
    return idx, d


# --------------------------------------------------------------------------
# Best factor (Sec. 2 / Sec. 4.1)
# --------------------------------------------------------------------------

def best_factor(T, MT, H, C, region=None, s_lo=0.0, s_hi=np.inf):
    """Per frame, s minimising the variance of t - s (c H) over the pixels
    with weight > 0 (and region > 0 when a region is given), clamped to
    [s_lo, s_hi]."""
    T, MT = _f64(T), _f64(MT)
    model = _f64(C) @ _f64(H)
    s = np.ones(T.shape[0])
    for f in range(T.shape[0]):
        use = MT[f] > 0
        if region is not None:
            use &= _f64(region) > 0
        t = T[f][use]
        m = model[f][use]
        if t.size < 2:
            continue
        tc = t - t.mean()
        mc = m - m.mean()
        var_m = np.mean(mc * mc)
        # a model that is constant over the pixels (up to rounding) has no
        # scale to fit
        if not var_m > 1e-12 * np.mean(m * m):
            continue
        s[f] = min(max(np.mean(tc * mc) / var_m, s_lo), s_hi)
    return s


# --------------------------------------------------------------------------
# Component-by-component basis construction (Sec. 2)
# --------------------------------------------------------------------------

def sequential_start(W_prev, H_prev, seed, n, p, K):
    """Start of stage j = W_prev.shape[1] + 1: the previous components plus
    one new seeded U(0,1) component (column j - 1 of matrix 3, row j - 1 of
    matrix 4, read as n x K and K x p matrices)."""
    j = 1 if W_prev is None else W_prev.shape[1] + 1
    wcol = prng.init_matrix(seed, MAT_SEQ_W, n, K)[:, j - 1]
    hrow = prng.init_matrix(seed, MAT_SEQ_H, K, p)[j - 1]
    if W_prev is None:
        return wcol[:, None].copy(), hrow[None, :].copy()
    return np.hstack([_f64(W_prev), wcol[:, None]]), np.vstack([_f64(H_prev), hrow[None, :]])


def build_basis_sequential(V, M, K, iters, seed, eps=nmf64.EPS_FLOOR):
    """Stages j = 1..K, each ``iters`` iterations of Eq. 3 from the previous
    stage's components plus a new random one.  Returns (W, H, J_stages)
    with J_stages[j - 1] the Eq. 2 cost at the end of stage j."""
    n, p = np.shape(V)
    W = H = None
    J_st = []
    for _ in range(K):
        W0, H0 = sequential_start(W, H, seed, n, p, K)
        W, H, J = nmf64.build_basis(V, M, W0, H0, iters, eps)
        J_st.append(J[-1])
    return W, H, np.array(J_st)
