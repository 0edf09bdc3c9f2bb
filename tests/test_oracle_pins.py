"""Pins for the FP64 oracle: facts fixed by the paper and by mathematics,
independent of the oracle's own formulas.

Each test names the passage of arXiv:2309.04623 it checks and the kind of
pin (worked value, closed form, invariant, library routine, brute force).
"""
import json
import os

import numpy as np
import pytest

from oracle import nmf64, nnls, prng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _tiny(seed, n=5, p=9, k=3, mask_frac=0.2):
    g = np.random.default_rng(seed)
    V = g.gamma(2.0, 1.0, (n, p))
    M = g.uniform(0.2, 3.0, (n, p)) * (g.random((n, p)) >= mask_frac)
    W = g.uniform(0.05, 1.0, (n, k))
    H = g.uniform(0.05, 1.0, (k, p))
    return V, M, W, H


# ---------------------------------------------------------------- init (a2)

def test_splitmix64_published_vectors():
    """Counter-mode generator reproduces SplitMix64's published outputs."""
    gold = _golden("splitmix64.json")
    for vec in gold["vectors"]:
        if "outputs_hex" in vec:
            want = [int(x, 16) for x in vec["outputs_hex"]]
        else:
            want = vec["outputs"]
        assert prng.splitmix64_outputs(vec["seed"], len(want)) == want


def test_uniform_open_interval_exact_float32():
    u = prng.uniform(7, prng.MAT_H, 200000)
    assert u.min() > 0.0 and u.max() < 1.0
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert abs(u.mean() - 0.5) < 3e-3
    # element i of a longer draw equals element i of a shorter one (counter mode)
    assert np.array_equal(prng.uniform(7, prng.MAT_H, 10), u[:10])
    assert not np.array_equal(prng.uniform(7, prng.MAT_W, 10), u[:10])


# ---------------------------------------------------------- objective (a3)

def test_objective_hand_worked_value():
    """Eq. 2 weights the squared residual by V (here M) linearly."""
    g = _golden("objective_2x2.json")
    J = nmf64.objective(np.array(g["V"]), np.array(g["M"]), np.array(g["W"]), np.array(g["H"]))
    assert J == g["J"]


# -------------------------------------------------------- updates (a4, a5)

@pytest.mark.parametrize("seed", range(100))
def test_monotone_each_half_step(seed):
    """Eq. 3's rules never increase the Eq. 2 cost (auxiliary-function
    argument for weighted multiplicative updates), H-step and W-step alike."""
    V, M, W, H = _tiny(seed)
    Vh, Mw, _ = nmf64.prep(V, M)
    J = nmf64.objective(Vh, Mw, W, H)
    for _ in range(20):
        H = nmf64.update_H(Vh, Mw, W, H)
        J1 = nmf64.objective(Vh, Mw, W, H)
        assert J1 <= J * (1 + 1e-13) + 1e-300
        W = nmf64.update_W(Vh, Mw, W, H)
        J2 = nmf64.objective(Vh, Mw, W, H)
        assert J2 <= J1 * (1 + 1e-13) + 1e-300
        J = J2
        assert W.min() >= nmf64.EPS_FLOOR and H.min() >= nmf64.EPS_FLOOR


@pytest.mark.parametrize("seed", [0, 1, 3])
def test_planted_exact_low_rank_recovered(seed):
    """V = W0 H0 exactly with K = K0: the iteration drives the relative cost
    below 1e-10 (seed 2 of this family stalls in a local minimum; the method
    is non-convex, Sec. 2)."""
    g = np.random.default_rng(seed)
    N, P, K = 6, 12, 2
    W0 = g.uniform(0.5, 2.0, (N, K))
    H0 = g.uniform(0.5, 2.0, (K, P))
    H0[0, : P // 2] *= 0.1
    H0[1, P // 2:] *= 0.1
    V = W0 @ H0
    M = np.ones_like(V)
    M[g.random(V.shape) < 0.1] = 0
    W = g.uniform(0.1, 1, (N, K))
    H = g.uniform(0.1, 1, (K, P))
    W, H, J = nmf64.build_basis(V, M, W, H, 3000)
    Vh, Mw, _ = nmf64.prep(V, M)
    assert J[-1] / np.sum(Mw * Vh ** 2) < 1e-10


def test_planted_fixed_point():
    """If W H reproduces the data, numerator equals denominator and one
    iteration leaves (W, H) unchanged up to rounding."""
    g = np.random.default_rng(11)
    W0 = g.uniform(0.5, 2, (7, 3))
    H0 = g.uniform(0.5, 2, (3, 10))
    V = W0 @ H0
    M = g.uniform(0.5, 2, V.shape)
    W, H, _ = nmf64.build_basis(V, M, W0, H0, 1)
    assert np.max(np.abs(W / W0 - 1)) < 1e-14
    assert np.max(np.abs(H / H0 - 1)) < 1e-14


def test_rank1_unweighted_reaches_svd():
    """M = 1, K = 1: the optimum is the leading singular triple, which is
    non-negative for a positive matrix (Perron); J* = ||V||^2 - s1^2."""
    g = np.random.default_rng(5)
    V = g.uniform(0.5, 2.0, (8, 11))
    M = np.ones_like(V)
    W, H, J = nmf64.build_basis(V, M, np.full((8, 1), 0.5), np.full((1, 11), 0.5), 500)
    s = np.linalg.svd(V, compute_uv=False)
    Jstar = np.sum(V ** 2) - s[0] ** 2
    assert abs(J[-1] - Jstar) <= 1e-10 * np.sum(V ** 2)
    U, S, Vt = np.linalg.svd(V)
    best = S[0] * np.outer(np.abs(U[:, 0]), np.abs(Vt[0]))
    assert np.max(np.abs(W @ H - best)) < 1e-6


def test_eckart_young_lower_bound():
    """M = 1: no rank-K product beats the truncated SVD, so every iterate's
    cost is at least the sum of the discarded squared singular values."""
    g = np.random.default_rng(6)
    V = g.gamma(2.0, 1.0, (9, 14))
    K = 3
    s = np.linalg.svd(V, compute_uv=False)
    bound = np.sum(s[K:] ** 2)
    _, _, J = nmf64.build_basis(V, np.ones_like(V), g.uniform(0.1, 1, (9, K)),
                                g.uniform(0.1, 1, (K, 14)), 300)
    assert np.all(J >= bound * (1 - 1e-12))
    assert J[-1] < J[0]


def test_unweighted_lee_seung_association():
    """With M = 1, W^T (W H) = (W^T W) H, so the H-rule equals the classic
    unweighted form H o (W^T V) / (W^T W H) computed another way."""
    V, _, W, H = _tiny(21)
    M = np.ones_like(V)
    h1 = nmf64.update_H(V, M, W, H)
    h2 = H * (W.T @ V) / ((W.T @ W) @ H)
    assert np.max(np.abs(h1 / h2 - 1)) < 1e-13
    w1 = nmf64.update_W(V, M, W, h1)
    w2 = W * (V @ h1.T) / (W @ (h1 @ h1.T))
    assert np.max(np.abs(w1 / w2 - 1)) < 1e-13


@pytest.mark.parametrize("seed", range(6))
def test_H_rule_alone_reaches_columnwise_nnls(seed):
    """With W fixed, the H-rule on column p is the projection iteration of
    that column; its limit is the weighted NNLS minimiser, found here by
    brute force over supports (K <= 4)."""
    V, M, W, H = _tiny(100 + seed, n=7, p=5, k=3, mask_frac=0.15)
    Vh, Mw, _ = nmf64.prep(V, M)
    for _ in range(40000):
        H = nmf64.update_H(Vh, Mw, W, H, eps=0.0)
    for p in range(V.shape[1]):
        G, b, c = nnls.normal_equations(W.T, Vh[:, p], Mw[:, p])
        w_star, j_star = nnls.nnls_bruteforce(G, b, c)
        j = nnls.cost(G, b, c, H[:, p])
        assert j - j_star <= 1e-9 * max(j_star, 1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_W_rule_alone_reaches_rowwise_nnls(seed):
    V, M, W, H = _tiny(200 + seed, n=5, p=8, k=3, mask_frac=0.15)
    Vh, Mw, _ = nmf64.prep(V, M)
    for _ in range(40000):
        W = nmf64.update_W(Vh, Mw, W, H, eps=0.0)
    for n in range(V.shape[0]):
        G, b, c = nnls.normal_equations(H, Vh[n], Mw[n])
        _, j_star = nnls.nnls_bruteforce(G, b, c)
        assert nnls.cost(G, b, c, W[n]) - j_star <= 1e-9 * max(j_star, 1e-12)


# ---------------------------------------------------------- invariances (a1)

def test_weight_scaling_is_bitwise_invariant():
    V, M, W, H = _tiny(31)
    a = nmf64.build_basis(V, M, W, H, 30)
    b = nmf64.build_basis(V, M * 8.0, W, H, 30)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_data_scaling_moves_into_H_bitwise():
    V, M, W, H = _tiny(32)
    a = nmf64.build_basis(V, M, W, H, 30)
    b = nmf64.build_basis(V * 16.0, M, W, H * 16.0, 30)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1] * 16.0, b[1])


def test_masked_garbage_is_ignored():
    """Masked pixels are missing data (Sec. 4.1): NaN, Inf or negative values
    under zero weight leave every iterate bitwise unchanged."""
    V, M, W, H = _tiny(33)
    Vg = V.copy()
    holes = M == 0
    vals = np.array([np.nan, np.inf, -5.0, 1e30])
    Vg[holes] = vals[np.arange(holes.sum()) % 4]
    a = nmf64.build_basis(V, M, W, H, 25)
    b = nmf64.build_basis(Vg, M, W, H, 25)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_prep_flags_bad_data_under_weight():
    V, M, _, _ = _tiny(34)
    M[0, 0] = 1.0
    bad = V.copy()
    bad[0, 0] = np.nan
    assert nmf64.prep(bad, M)[2] == "nonfinite"
    bad[0, 0] = -1.0
    assert nmf64.prep(bad, M)[2] == "negative"
    M2 = M.copy()
    M2[1, 1] = -0.5
    assert nmf64.prep(V, M2)[2] == "negative_weight"
    assert nmf64.prep(V, M)[2] == 0


def test_fully_masked_row_and_column_keep_factors():
    """A pixel masked in every image (den = 0) keeps its H column; an image
    masked everywhere keeps its W row."""
    V, M, W, H = _tiny(35)
    M[:, 2] = 0
    M[3, :] = 0
    W1, H1, J = nmf64.build_basis(V, M, W, H, 10)
    assert np.array_equal(H1[:, 2], H[:, 2])
    assert np.array_equal(W1[3], W[3])
    assert np.all(np.diff(J) <= 1e-12 * J[0])


# ------------------------------------------------------- projection (a8)

def test_projection_k1_one_step_closed_form():
    """K = 1: one update from any c > 0 lands on sum m t h / sum m h^2."""
    g = np.random.default_rng(41)
    H = g.uniform(0.2, 2, (1, 30))
    t = g.uniform(0, 3, (1, 30))
    m = g.uniform(0, 2, (1, 30)) * (g.random((1, 30)) > 0.2)
    c = nmf64.project(t, m, H, np.array([[0.37]]), 1)
    want = np.sum(m * t * H) / np.sum(m * H * H)
    assert abs(c[0, 0] / want - 1) < 1e-14


@pytest.mark.parametrize("seed", range(10))
def test_projection_limit_is_bruteforce_nnls(seed):
    g = np.random.default_rng(300 + seed)
    K, P = int(g.integers(1, 5)), 40
    H = g.uniform(0.0, 1.0, (K, P)) ** 2
    t = g.uniform(0.0, 1.0, (1, P)) + (g.uniform(0, 1, K) @ H)
    m = g.uniform(0.1, 2.0, (1, P)) * (g.random((1, P)) > 0.1)
    c = nmf64.project(t, m, H, np.full((1, K), 0.5), 60000, eps=0.0)
    G, b, cc = nnls.normal_equations(H, t[0], m[0])
    w_star, j_star = nnls.nnls_bruteforce(G, b, cc)
    j = nnls.cost(G, b, cc, c[0])
    assert j - j_star <= 1e-9 * j_star
    if np.all(w_star > 1e-3 * w_star.max()):
        assert np.linalg.norm(c[0] - w_star) <= 1e-6 * np.linalg.norm(w_star)


def test_projection_limit_matches_scipy_nnls_k8():
    g = np.random.default_rng(51)
    K, P = 8, 120
    H = g.gamma(1.0, 1.0, (K, P))
    t = g.uniform(0, 0.2, (1, P)) + g.gamma(2, 1, K) @ H
    m = 1.0 / (t + 0.01)
    c = nmf64.project(t, m, H, np.full((1, K), 0.5), 20000)
    w = nnls.nnls_scipy(H, t[0], m[0])
    G, b, cc = nnls.normal_equations(H, t[0], m[0])
    assert nnls.kkt_residual(G, b, w) < 1e-8
    assert abs(nnls.cost(G, b, cc, c[0]) - nnls.cost(G, b, cc, w)) <= 1e-8 * nnls.cost(G, b, cc, w)
    assert np.allclose(nnls.nnls_gram(G, b), w, rtol=1e-7, atol=1e-9)


def test_gram_form_matches_direct_form():
    g = np.random.default_rng(61)
    K, P, F = 6, 200, 4
    H = g.gamma(1.0, 1.0, (K, P))
    T = g.gamma(2, 1, (F, K)) @ H + g.uniform(0, 0.1, (F, P))
    MT = (1.0 / (T + 0.01)) * (g.random((F, P)) > 0.05)
    C0 = prng.init_matrix(3, prng.MAT_C, F, K)
    a = nmf64.project(T, MT, H, C0, 300)
    b = nmf64.project_gram(T, MT, H, C0, 300)
    assert np.max(np.abs(a / b - 1)) < 1e-12


def test_ragged_projection_equals_dense_with_zero_weights():
    g = np.random.default_rng(62)
    K, P = 5, 64
    H = g.gamma(1.0, 1.0, (K, P))
    sizes = [10, 64, 33]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    pix = np.concatenate([np.sort(g.choice(P, s, replace=False)) for s in sizes]).astype(np.int32)
    val = g.uniform(0, 3, offs[-1])
    wt = g.uniform(0.5, 2, offs[-1])
    C0 = prng.init_matrix(4, prng.MAT_C, 3, K)
    T, MT = nmf64.ragged_to_dense(offs, pix, val, wt, P)
    a = nmf64.project(T, MT, H, C0, 50)
    b = nmf64.project_ragged(offs, pix, val, wt, H, C0, 50)
    assert np.max(np.abs(a / b - 1)) < 1e-12


# ------------------------------------------------------ subtraction (a9)

def test_subtract_definition():
    g = np.random.default_rng(71)
    H = g.uniform(0, 1, (3, 20))
    C = g.uniform(0, 1, (2, 3))
    T = g.uniform(0, 2, (2, 20))
    MT = (g.random((2, 20)) > 0.3).astype(float)
    model, resid = nmf64.subtract(T, MT, H, C, scale=np.array([1.0, 0.5]))
    assert np.allclose(model, np.einsum("fk,kp->fp", C, H), rtol=1e-15)
    ok = MT > 0
    assert np.all(np.isnan(resid[~ok]))
    s = np.array([1.0, 0.5])[:, None] * np.ones_like(T)
    assert np.allclose((resid + s * model)[ok], T[ok], rtol=1e-14)


def test_normalisation_keeps_product():
    V, M, W, H = _tiny(81)
    W2, H2 = nmf64.normalize_components(W, H)
    assert np.allclose(W2 @ H2, W @ H, rtol=1e-14)
    assert np.allclose(np.linalg.norm(H2, axis=1), 1.0, rtol=1e-14)


# -------------------------------------------- per-frame objective (a8)

def _golden_frames(name):
    g = _golden(name)
    arr = lambda x: np.array([[np.nan if v == "nan" else v for v in row] for row in x], float)
    return g, arr


def test_frame_objective_hand_worked():
    """Per-frame Eq. 2 cost of a model c H (Sec. 4.1): worked by hand, with a
    masked NaN pixel that must be ignored and a non-unit weight that must
    enter linearly."""
    g, arr = _golden_frames("frame_objective_2x3.json")
    J = nmf64.frame_objective(arr(g["T"]), arr(g["MT"]), arr(g["H"]), arr(g["C"]))
    assert np.array_equal(J, np.array(g["J"]))


def test_frame_objective_equals_nnls_cost():
    """The per-frame objective equals the quadratic form of the normal
    equations, c G c^T - 2 b c^T + t^T diag(m) t (an independent route)."""
    g = np.random.default_rng(91)
    K, P, F = 4, 50, 3
    H = g.uniform(0, 1, (K, P))
    C = g.uniform(0, 2, (F, K))
    T = g.uniform(0, 3, (F, P))
    MT = g.uniform(0.1, 2, (F, P)) * (g.random((F, P)) > 0.2)
    J = nmf64.frame_objective(T, MT, H, C)
    for f in range(F):
        G, b, c = nnls.normal_equations(H, T[f], MT[f])
        assert abs(J[f] - nnls.cost(G, b, c, C[f])) <= 1e-12 * J[f]


# ------------------------------------------------------ subtraction (a9)

def test_subtract_hand_worked():
    """Model and residual worked by hand, including the NaN pattern at the
    zero-weight pixel and the per-frame scale."""
    g, arr = _golden_frames("subtract_2x3.json")
    model, resid = nmf64.subtract(arr(g["T"]), arr(g["MT"]), arr(g["H"]), arr(g["C"]),
                                  scale=np.array(g["scale"]))
    assert np.array_equal(model, arr(g["model"]))
    want = arr(g["resid"])
    assert np.array_equal(np.isnan(resid), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.array_equal(resid[ok], want[ok])


# ------------------------------------------------------ exact NNLS (a8)

@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_nnls_matches_scipy(seed):
    """The two exact NNLS routes (brute force over supports, scipy's
    active-set solver) agree on random K <= 4 problems with and without
    active constraints."""
    g = np.random.default_rng(500 + seed)
    K, P = 1 + seed % 4, 30
    H = g.uniform(0, 1, (K, P)) ** 2
    w_true = g.uniform(-0.5, 1.5, K)
    t = np.maximum(w_true @ H + g.normal(0, 0.05, P), 0)
    m = g.uniform(0.2, 2.0, P) * (g.random(P) > 0.1)
    G, b, c = nnls.normal_equations(H, t, m)
    wb, jb = nnls.nnls_bruteforce(G, b, c)
    ws = nnls.nnls_scipy(H, t, m)
    assert abs(nnls.cost(G, b, c, ws) - jb) <= 1e-10 * max(jb, 1e-12)
    assert np.allclose(wb, ws, atol=1e-8 * max(1.0, np.abs(wb).max()))
    assert nnls.kkt_residual(G, b, wb) < 1e-9


# ------------------------------------------------- stopping rule (a6, f4)

def test_stop_test_hand_worked():
    """The relative-decrease rule on a hand-made history: with c = 2 and
    tol = 0.1 the decreases over two iterations are 100->60 (0.4) at t = 2,
    60->50 (0.167) at t = 4 and 50->47 (0.06) at t = 6, so it first passes
    at t = 6; odd t are never tested."""
    J = [100.0, 80.0, 60.0, 55.0, 50.0, 49.9, 47.0, 46.0]
    passes = [t for t in range(len(J)) if nmf64.stop_test(J, t, 2, 0.1)]
    assert passes == [6]
    assert not nmf64.stop_test(J, 5, 2, 0.1)
    assert not nmf64.stop_test(J, 6, 0, 0.1)


def test_build_basis_tol_stops_at_the_rule():
    """With the rule off the tolerant build equals the fixed-count build
    bitwise; with it on it stops after the first iteration at which the rule
    passes, and its history is the fixed-count history cut there."""
    V, M, W, H = _tiny(92, n=8, p=12, k=2)
    Wf, Hf, Jf = nmf64.build_basis(V, M, W, H, 200)
    Wt, Ht, Jt, run = nmf64.build_basis_tol(V, M, W, H, 200, 0, 0.0)
    assert run == 200 and np.array_equal(Wt, Wf) and np.array_equal(Jt, Jf)
    Wt, Ht, Jt, run = nmf64.build_basis_tol(V, M, W, H, 200, 5, 1e-3)
    first = next(t for t in range(5, 200, 5) if (Jf[t - 5] - Jf[t]) / Jf[t - 5] < 1e-3)
    assert run == first + 1
    Wr, Hr, Jr = nmf64.build_basis(V, M, W, H, run)
    assert np.array_equal(Wt, Wr) and np.array_equal(Jt, Jr)


def test_projection_stop_rule_by_hand_and_limits():
    """Per-frame stop rule of the projection: hand-checked decision on a K = 1
    frame (one step lands on the optimum, so the change at the next check
    is 0), no stop with tol = 0 unless the start is a fixed point, and the
    stopped iterate matches the fixed-count run at the same count."""
    H = np.array([[1.0, 2.0, 3.0]])
    T = np.array([[2.0, 4.0, 6.0]])       # t = 2 h exactly: w* = 2
    MT = np.ones_like(T)
    C, its, _ = nmf64.project_gram_tol(T, MT, H, np.array([[0.5]]), 50, 2, 1e-12)
    # iteration 1: w = 0.5 * (b / (w G)) = 0.5 * 28 / 7 = 2; iteration 2
    # keeps 2; the check at t = 2 sees w_2 - w_0 = 1.5 (no stop), the one at
    # t = 4 sees 0 (stop)
    assert its[0] == 4 and C[0, 0] == 2.0
    g = np.random.default_rng(3)
    Hr = g.gamma(1, 1, (4, 60))
    Tr = g.gamma(2, 1, (3, 4)) @ Hr + np.abs(g.normal(0, 0.1, (3, 60)))
    Mr = (g.random(Tr.shape) > 0.1).astype(float)
    C0 = g.uniform(0.1, 1, (3, 4))
    C1, its1, _ = nmf64.project_gram_tol(Tr, Mr, Hr, C0, 200, 10, 0.0)
    assert np.all(its1 == 200)
    assert np.allclose(C1, nmf64.project_gram(Tr, Mr, Hr, C0, 200), rtol=1e-12, atol=0)
    C2, its2, _ = nmf64.project_gram_tol(Tr, Mr, Hr, C0, 5000, 10, 1e-3)
    assert np.all(its2 % 10 == 0) and np.all(its2 < 5000)
    for f in range(3):
        ref = nmf64.project_gram(Tr[f:f + 1], Mr[f:f + 1], Hr, C0[f:f + 1], int(its2[f]))
        assert np.allclose(C2[f], ref[0], rtol=1e-12, atol=0)


def test_projection_stop_rule_warm_restart():
    """Warm start under the stop rule: the exact optimum as warm start stops
    at the first check with the start kept; a warm start worse than the cold
    one is replaced by it from the start (the run equals the cold run); a
    kept warm start that misses the rule by the cap is followed by a full
    cold run (iterations add up, the result is the cold run's)."""
    H = np.array([[1.0, 2.0, 3.0]])
    T = np.array([[2.0, 4.0, 6.0]])
    MT = np.ones_like(T)
    cold = np.array([[0.5]])
    C, its, fb = nmf64.project_gram_tol(T, MT, H, np.array([[2.0]]), 50, 3, 1e-12, C_cold=cold)
    assert its[0] == 3 and fb[0] == 0 and C[0, 0] == 2.0
    g = np.random.default_rng(5)
    Hr = g.gamma(1, 1, (5, 80))
    Tr = g.gamma(2, 1, (4, 5)) @ Hr + np.abs(g.normal(0, 0.1, (4, 80)))
    Mr = (g.random(Tr.shape) > 0.1).astype(float)
    Cc = g.uniform(0.1, 1, (4, 5))
    bad = 1e3 * np.ones((4, 5))
    C, its, fb = nmf64.project_gram_tol(Tr, Mr, Hr, bad, 40, 5, 1e-3, C_cold=Cc)
    Cr, itsr, _ = nmf64.project_gram_tol(Tr, Mr, Hr, Cc, 40, 5, 1e-3)
    assert np.all(fb == 1) and np.array_equal(its, itsr) and np.array_equal(C, Cr)
    # near the solution but the rule is unreachable within the cap
    near = nmf64.project_gram(Tr, Mr, Hr, Cc, 30)
    C, its, fb = nmf64.project_gram_tol(Tr, Mr, Hr, near, 20, 5, 1e-14, C_cold=Cc)
    assert np.all(fb == 2) and np.all(its == 40)
    assert np.allclose(C, nmf64.project_gram(Tr, Mr, Hr, Cc, 20), rtol=1e-12, atol=0)


def test_stored_nnls_solutions_of_the_projection_set():
    """The stored exact NNLS solutions used to judge projections to the 1e-4
    tolerance are what the generator's frames give: same input bytes, and on
    a few re-solved frames the same minimiser, optimal by its KKT
    conditions and by the active-set route on the square-root-weighted
    system (an independent solve)."""
    import hashlib
    import os
    from paper_2309_04623_amd import synth
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "oracle_nnls_proj_k100.npz"))
    n_s = int(z["n_sample"])
    ps = synth.make_projection_set(int(z["n_frames"]))
    sha = lambda x: hashlib.sha256(np.ascontiguousarray(x, np.float32).tobytes()).hexdigest()
    assert sha(ps.H) == str(z["h_sha"])
    assert sha(ps.T[:n_s]) == str(z["t_sha"]) and sha(ps.MT[:n_s]) == str(z["m_sha"])
    assert np.max(z["kkt"]) < 1e-10
    for f in (0, 101, n_s - 1):
        G, b, c = nnls.normal_equations(ps.H, ps.T[f], ps.MT[f])
        w = z["w_star"][f]
        assert nnls.kkt_residual(G, b, w) < 1e-10
        ws = nnls.nnls_scipy(ps.H, ps.T[f], ps.MT[f])
        assert nnls.cost(G, b, c, ws) >= nnls.cost(G, b, c, w) * (1 - 1e-9)
        dm = np.sqrt((ws - w) @ G @ (ws - w) / (w @ G @ w))
        assert dm < 1e-6, dm
