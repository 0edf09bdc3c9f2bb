"""FP64 reference of the weighted multiplicative-update NMF (oracle).

Notation.  The paper writes the data as X, the weights as V (Eq. 1-2).  Here
the data matrix is V (N images x P pixels, one image per row), the per-pixel
weights are M (N x P, 0 = missing), W is N x K and H is K x P, so that
V ~ W H.  Everything is float64; inputs may be float32 and are widened.

Readings of points the paper leaves open (each applies on the GPU too):

* Objective (Eq. 2): J = sum M * (V - W H)^2 -- the weight enters linearly,
  because ||M^(1/2) o R||_F^2 = sum M R^2.
* Update order (Eq. 3 lists H first): each iteration updates H from the
  current W, then W from the *new* H.
* Zero denominator: where a denominator is exactly 0 (a pixel masked in every
  image, or an image masked everywhere) the factor is kept (ratio := 1).
* Non-negativity floor: after each update x := max(x, eps), eps = 1e-30.
* Masked pixels are missing data and ignored (Sec. 4.1): where M == 0 the
  data value is replaced by 0 before anything else, so NaN or garbage there
  cannot reach the result.
* Target modelling (Sec. 4.1): a science frame t with weights m is modelled
  with the basis fixed, by iterating the W-rule of Eq. 3 on its 1 x K
  coefficient row.
* Subtraction (Sec. 1, Sec. 4.1): residual = t - s * (c H) with s = 1 unless
  a scale is given; masked pixels of the residual are NaN.
"""
from __future__ import annotations

import numpy as np

EPS_FLOOR = 1e-30


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# Staging
# --------------------------------------------------------------------------

def prep(V, M):
    """Mask-aware staging of data and weights (Sec. 2, weights carry the
    missing data; Sec. 4.1, masked pixels ignored).

    Returns (Vhat, M, status) where Vhat = V where M > 0 else 0, and status is
    0 if the data are usable, or one of 'negative_weight', 'nonfinite',
    'negative' describing the first problem found under positive weight."""
    V = _f64(V)
    M = _f64(M)
    if np.any(~np.isfinite(M)) or np.any(M < 0):
        status = "negative_weight"
    else:
        status = 0
    pos = M > 0
    Vh = np.where(pos, V, 0.0)
    if status == 0:
        if np.any(~np.isfinite(Vh)):
            status = "nonfinite"
        elif np.any(Vh < 0):
            status = "negative"
    return Vh, M, status


# --------------------------------------------------------------------------
# Objective and update rules
# --------------------------------------------------------------------------

def objective(Vh, M, W, H):
    """Weighted Frobenius cost of Eq. 2: sum M * (Vhat - W H)^2."""
    R = _f64(Vh) - _f64(W) @ _f64(H)
    return float(np.sum(_f64(M) * R * R))


def ratio(num, den):
    """num / den elementwise, 1 where den == 0 (kept factor)."""
    num = _f64(num)
    den = _f64(den)
    out = np.ones_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


def update_H(Vh, M, W, H, eps=EPS_FLOOR):
    """H-rule of Eq. 3: H <- H o W^T (M o V) / W^T [M o (W H)], floored."""
    Vh, M, W, H = _f64(Vh), _f64(M), _f64(W), _f64(H)
    Y = W @ H
    num = W.T @ (M * Vh)
    den = W.T @ (M * Y)
    return np.maximum(H * ratio(num, den), eps)


def update_W(Vh, M, W, H, eps=EPS_FLOOR):
    """W-rule of Eq. 3: W <- W o (M o V) H^T / [M o (W H)] H^T, floored."""
    Vh, M, W, H = _f64(Vh), _f64(M), _f64(W), _f64(H)
    Y = W @ H
    num = (M * Vh) @ H.T
    den = (M * Y) @ H.T
    return np.maximum(W * ratio(num, den), eps)


def build_basis(V, M, W0, H0, iters, eps=EPS_FLOOR, normalize=False, history=True):
    """Basis construction by the Eq. 3 iteration from (W0, H0).

    Returns (W, H, J) with J[t] the Eq. 2 objective before iteration t and
    J[iters] after the last one (J is None when ``history`` is False)."""
    Vh, Mw, status = prep(V, M)
    if status:
        raise ValueError(f"unusable data: {status}")
    W = _f64(W0).copy()
    H = _f64(H0).copy()
    J = [] if history else None
    for _ in range(iters):
        if history:
            J.append(objective(Vh, Mw, W, H))
        H = update_H(Vh, Mw, W, H, eps)
        W = update_W(Vh, Mw, W, H, eps)
    if history:
        J.append(objective(Vh, Mw, W, H))
        J = np.array(J)
    if normalize:
        W, H = normalize_components(W, H)
    return W, H, J


def stop_test(J, t, check_every, tol):
    """Stopping rule (Sec. 2, after Eq. 3: iterate until the change reaches a
    set value or the iteration cap).  The quantity is not defined in the
    paper; the reading here is the relative decrease of the Eq. 2 cost over
    the last ``check_every`` iterations, tested when t is a positive multiple
    of ``check_every``:  (J[t - c] - J[t]) / J[t - c] < tol."""
    c = int(check_every)
    if c <= 0 or t < c or t % c:
        return False
    j0 = J[t - c]
    return bool(j0 > 0 and (j0 - J[t]) / j0 < tol)


def build_basis_tol(V, M, W0, H0, max_iter, check_every, tol, eps=EPS_FLOOR):
    """Basis construction with the stopping rule of ``stop_test``.  J[t] is
    the cost of the iterate entering iteration t; iteration t is carried out
    in full (H-rule, then W-rule) and, if the rule passes at t, it is the
    last one.  Returns (W, H, J, iterations run) with J[0..run]."""
    Vh, Mw, status = prep(V, M)
    if status:
        raise ValueError(f"unusable data: {status}")
    W = _f64(W0).copy()
    H = _f64(H0).copy()
    J = []
    run = 0
    for t in range(max_iter):
        J.append(objective(Vh, Mw, W, H))
        H = update_H(Vh, Mw, W, H, eps)
        W = update_W(Vh, Mw, W, H, eps)
        run = t + 1
        if stop_test(J, t, check_every, tol):
            break
    J.append(objective(Vh, Mw, W, H))
    return W, H, np.array(J), run


def normalize_components(W, H):
    """Rescale each component to unit L2 norm, moving the scale into W, so
    W H is unchanged (the paper is silent; optional post-processing)."""
    W, H = _f64(W), _f64(H)
    d = np.sqrt(np.sum(H * H, axis=1))
    d = np.where(d > 0, d, 1.0)
    return W * d[None, :], H / d[:, None]


# --------------------------------------------------------------------------
# Target modelling and subtraction
# --------------------------------------------------------------------------

def project(T, MT, H, C0, iters, eps=EPS_FLOOR):
    """Model each science frame with the basis H fixed (Sec. 4.1): iterate
    the W-rule of Eq. 3 on the frame's coefficient row, direct form
    den = [m o (c H)] H^T."""
    Th, MTw, status = prep(T, MT)
    if status:
        raise ValueError(f"unusable data: {status}")
    H = _f64(H)
    C = _f64(C0).copy()
    num = (MTw * Th) @ H.T
    for _ in range(iters):
        den = (MTw * (C @ H)) @ H.T
        C = np.maximum(C * ratio(num, den), eps)
    return C


def project_gram(T, MT, H, C0, iters, eps=EPS_FLOOR):
    """The same iteration re-associated through each frame's masked Gram
    matrix G_f = H diag(m_f) H^T, den_f = c_f G_f (identical in exact
    arithmetic to ``project``)."""
    Th, MTw, status = prep(T, MT)
    if status:
        raise ValueError(f"unusable data: {status}")
    H = _f64(H)
    C = _f64(C0).copy()
    num = (MTw * Th) @ H.T
    for f in range(C.shape[0]):
        G = (H * MTw[f][None, :]) @ H.T
        c = C[f]
        for _ in range(iters):
            c = np.maximum(c * ratio(num[f], c @ G), eps)
        C[f] = c
    return C


def frame_objective(T, MT, H, C):
    """Per-frame Eq. 2 cost of the model C H against frames T."""
    Th, MTw, _ = prep(T, MT)
    R = Th - _f64(C) @ _f64(H)
    return np.sum(MTw * R * R, axis=1)


def subtract(T, MT, H, C, scale=None):
    """Model PSF and residual: model = C H (every pixel), residual =
    T - s * model with NaN where the frame's weight is 0."""
    T, MT = _f64(T), _f64(MT)
    model = _f64(C) @ _f64(H)
    s = np.ones(T.shape[0]) if scale is None else _f64(scale)
    resid = T - s[:, None] * model
    resid[MT == 0] = np.nan
    return model, resid


def ragged_to_dense(offsets, pix, val, wt, p):
    f = len(offsets) - 1
    T = np.zeros((f, p))
    MT = np.zeros((f, p))
    for i in range(f):
        s, e = int(offsets[i]), int(offsets[i + 1])
        T[i, pix[s:e]] = val[s:e]
        MT[i, pix[s:e]] = wt[s:e]
    return T, MT


def project_ragged(offsets, pix, val, wt, H, C0, iters, eps=EPS_FLOOR):
    """Projection of frames given as CSR rows (pixels absent from a frame
    carry weight 0)."""
    H = _f64(H)
    C = _f64(C0).copy()
    for i in range(len(offsets) - 1):
        s, e = int(offsets[i]), int(offsets[i + 1])
        Hs = H[:, pix[s:e]]
        t = _f64(val[s:e])
        m = _f64(wt[s:e])
        t = np.where(m > 0, t, 0.0)
        num = Hs @ (m * t)
        c = C[i]
        for _ in range(iters):
            den = Hs @ (m * (c @ Hs))
            c = np.maximum(c * ratio(num, den), eps)
        C[i] = c
    return C


def project_gram_tol(T, MT, H, C0, max_iter, check_every, tol, eps=EPS_FLOOR, C_cold=None):
    """Projection (Gram form) with a per-frame stop rule.  Every
    ``check_every`` iterations (t = c, 2c, ..., before iteration t + 1) the
    relative change of the frame's model since the previous check (or the
    start, at t = c) is tested,
        (c_t - c_prev) G (c_t - c_prev)^T  <=  tol^2  c_t G c_t^T,
    G = H diag(m) H^T (the weighted squared norm of the model change against
    that of the model); when it passes the frame stops after t iterations.
    The paper leaves the criterion open (Sec. 2: until the change reaches a
    set value or the cap); this reading measures the change in model space.

    With ``C_cold`` given, C0 is a warm start: per frame it is raised to the
    floor, kept only if its Eq. 2 cost is not above that of the cold start
    C_cold[f], and a kept warm start that has not met the rule by the cap
    restarts from C_cold[f] with the same cap.
    Returns (C, iterations run per frame, fallback per frame: 0 warm kept,
    1 cold from the start, 2 restarted cold; all 0 without C_cold)."""
    Th, MTw, status = prep(T, MT)
    if status:
        raise ValueError(f"unusable data: {status}")
    H = _f64(H)
    C = _f64(C0).copy()
    F = C.shape[0]
    warm = C_cold is not None
    if warm:
        C = np.maximum(C, eps)
        Cc = _f64(C_cold)
    num = (MTw * Th) @ H.T
    its = np.zeros(F, np.int64)
    fb = np.zeros(F, np.int64)
    ce = int(check_every)

    def run(c, G, b):
        cp = c.copy()
        t = 0
        while t < max_iter:
            if ce > 0 and t > 0 and t % ce == 0:
                d = c - cp
                if d @ G @ d <= tol * tol * (c @ G @ c):
                    return c, t, True
                cp = c.copy()
            c = np.maximum(c * ratio(b, c @ G), eps)
            t += 1
        return c, t, False

    for f in range(F):
        G = (H * MTw[f][None, :]) @ H.T
        c = C[f]
        if warm:
            Jw = np.sum(MTw[f] * (Th[f] - c @ H) ** 2)
            Jc = np.sum(MTw[f] * (Th[f] - Cc[f] @ H) ** 2)
            if not Jw <= Jc:
                c, fb[f] = Cc[f].copy(), 1
        c, t, met = run(c, G, num[f])
        if warm and fb[f] == 0 and ce > 0 and not met:
            c, t2, _ = run(Cc[f].copy(), G, num[f])
            t, fb[f] = t + t2, 2
        C[f] = c
        its[f] = t
    return C, its, fb
