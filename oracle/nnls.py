"""Exact weighted non-negative least squares (oracle).

Projecting a frame t with weights m onto a fixed basis H (Sec. 4.1, target
modelling) is the convex problem

    w* = argmin_{w >= 0}  sum_p m_p (t_p - (w H)_p)^2
       = argmin_{w >= 0}  w G w^T - 2 b w^T + const,
    G = H diag(m) H^T,   b = H (m o t).

The multiplicative iteration of Eq. 3 (W-rule, H fixed) converges to w*, so
w* is the plain definition the projection must reach.  Two independent
routes compute it: brute force over all 2^K supports (K <= 4) and scipy's
active-set NNLS on the square-root-weighted system.
"""
from __future__ import annotations

import itertools

import numpy as np


def normal_equations(H, t, m):
    H = np.asarray(H, np.float64)
    t = np.asarray(t, np.float64)
    m = np.asarray(m, np.float64)
    t = np.where(m > 0, t, 0.0)
    G = (H * m[None, :]) @ H.T
    b = H @ (m * t)
    c = float(np.sum(m * t * t))
    return G, b, c


def cost(G, b, c, w):
    return float(w @ G @ w - 2.0 * b @ w + c)


def nnls_bruteforce(G, b, c=0.0):
    """Minimise w G w - 2 b w + c over w >= 0 by trying every support S:
    solve G_SS w_S = b_S, keep feasible solutions, return the cheapest."""
    K = G.shape[0]
    best_w, best_j = np.zeros(K), c
    for r in range(1, K + 1):
        for S in itertools.combinations(range(K), r):
            S = list(S)
            try:
                wS = np.linalg.solve(G[np.ix_(S, S)], b[S])
            except np.linalg.LinAlgError:
                continue
            if np.any(wS < 0):
                continue
            w = np.zeros(K)
            w[S] = wS
            j = cost(G, b, c, w)
            if j < best_j:
                best_w, best_j = w, j
    return best_w, best_j


def nnls_scipy(H, t, m):
    """scipy.optimize.nnls on (sqrt(m) o H)^T w = sqrt(m) o t."""
    from scipy.optimize import nnls
    H = np.asarray(H, np.float64)
    m = np.asarray(m, np.float64)
    t = np.where(m > 0, np.asarray(t, np.float64), 0.0)
    sq = np.sqrt(m)
    w, _ = nnls((H * sq[None, :]).T, sq * t, maxiter=50 * H.shape[0])
    return w


def nnls_gram(G, b):
    """NNLS from the normal equations via a Cholesky factor G = L L^T:
    minimise ||L^T w - L^-1 b||^2 over w >= 0 (same minimiser)."""
    from scipy.optimize import nnls
    L = np.linalg.cholesky(G)
    rhs = np.linalg.solve(L, b)
    w, _ = nnls(L.T, rhs, maxiter=50 * G.shape[0])
    return w


def kkt_residual(G, b, w):
    """Largest violation of the KKT conditions of the NNLS problem:
    gradient g = G w - b must be >= 0 where w == 0 and == 0 where w > 0."""
    g = G @ w - b
    scale = max(np.abs(b).max(), 1e-300)
    act = w <= 0
    v1 = np.max(np.maximum(-g[act], 0.0), initial=0.0)
    v2 = np.max(np.abs(g[~act]), initial=0.0)
    return max(v1, v2) / scale
