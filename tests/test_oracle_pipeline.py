"""Pins of the oracle's reference selection, best factor and
component-by-component build (oracle/pipeline64.py) against hand-worked
values, closed forms, brute force and invariants."""
import json
import os

import numpy as np
import pytest

from oracle import nmf64, pipeline64 as pl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    d = json.load(open(os.path.join(GOLDEN, name)))
    fix = lambda a: np.array([[np.nan if v == "nan" else v for v in row] for row in a], float)
    return d, fix


# ---- reference selection -------------------------------------------------

def test_distances_and_selection_hand_worked():
    d, fix = _load("closest_frames_2x4.json")
    idx, dist = pl.closest_frames(fix(d["T"]), fix(d["MT"]), fix(d["V"]), fix(d["M"]), d["n_sel"])
    assert np.array_equal(dist, np.array(d["distances"], float))
    assert np.array_equal(idx, np.array(d["selected"]))


def _random_case(seed, f=3, n=9, p=40):
    g = np.random.default_rng(seed)
    T = g.gamma(2, 1, (f, p))
    V = g.gamma(2, 1, (n, p))
    MT = (g.random((f, p)) > 0.2).astype(float)
    M = (g.random((n, p)) > 0.2).astype(float)
    return T, MT, V, M


@pytest.mark.parametrize("seed", range(4))
def test_distances_match_expanded_products(seed):
    """A second route: with validity a (target) and b (reference),
    d = (a t^2) b^T - 2 (a t)(b v)^T + a (b v^2)^T, three matrix products."""
    T, MT, V, M = _random_case(seed)
    a, b = (MT > 0).astype(float), (M > 0).astype(float)
    exp = (a * T * T) @ b.T - 2 * (a * T) @ (b * V).T + a @ (b * V * V).T
    d = pl.frame_distances(T, MT, V, M)
    assert np.max(np.abs(d - exp) / np.maximum(exp, 1e-12)) < 1e-10


def test_planted_duplicate_is_closest_and_garbage_ignored():
    T, MT, V, M = _random_case(7)
    V[4] = T[1]
    M[4] = MT[1]
    V[4][MT[1] == 0] = np.nan  # garbage where the copy is masked
    idx, d = pl.closest_frames(T, MT, V, M, 3)
    assert d[1, 4] == 0.0 and idx[1, 0] == 4
    V2 = V.copy()
    V2[M == 0] = 1e30
    assert np.array_equal(pl.frame_distances(T, MT, V2, M), d)


def test_selection_follows_reference_permutation():
    T, MT, V, M = _random_case(3)
    perm = np.random.default_rng(0).permutation(V.shape[0])
    idx, _ = pl.closest_frames(T, MT, V, M, 5)
    idx_p, _ = pl.closest_frames(T, MT, V[perm], M[perm], 5)
    assert np.array_equal(perm[idx_p], idx)


def test_distance_is_symmetric():
    T, MT, V, M = _random_case(5, f=4, n=4)
    assert np.allclose(pl.frame_distances(T, MT, V, M), pl.frame_distances(V, M, T, MT).T,
                       rtol=1e-14)


# ---- best factor -----------------------------------------------------------

def test_best_factor_hand_worked():
    d, fix = _load("best_factor_1x4.json")
    s = pl.best_factor(fix(d["T"]), fix(d["MT"]), fix(d["H"]), fix(d["C"]))
    assert np.allclose(s, d["scale"], rtol=0, atol=1e-15)


def _bf_case(seed, f=3, k=4, p=60):
    g = np.random.default_rng(seed)
    H = g.gamma(1, 1, (k, p))
    C = g.gamma(2, 1, (f, k))
    MT = (g.random((f, p)) > 0.1).astype(float)
    return H, C, MT, C @ H


def test_best_factor_planted_scale_and_offset():
    """t = s0 m + c exactly: the residual variance vanishes at s0."""
    H, C, MT, model = _bf_case(1)
    s0 = np.array([0.7, 1.3, 0.25])
    T = s0[:, None] * model + np.array([0.0, 5.0, -2.0])[:, None]
    assert np.allclose(pl.best_factor(T, MT, H, C), s0, rtol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_best_factor_is_the_bruteforce_variance_minimum(seed):
    H, C, MT, model = _bf_case(seed)
    g = np.random.default_rng(seed + 10)
    T = 0.8 * model + g.normal(0, 0.3, model.shape)
    s = pl.best_factor(T, MT, H, C)
    grid = np.linspace(0, 2, 20001)
    for f in range(T.shape[0]):
        use = MT[f] > 0
        v = [np.var(T[f][use] - q * model[f][use]) for q in grid]
        assert abs(grid[int(np.argmin(v))] - s[f]) <= grid[1] - grid[0]


def test_best_factor_region_excludes_a_disk_and_clamps():
    H, C, MT, model = _bf_case(4)
    T = 0.9 * model
    disk = np.zeros(model.shape[1])
    disk[10:20] = 5.0
    Td = T + disk[None, :]
    region = (disk == 0).astype(float)
    assert np.allclose(pl.best_factor(Td, MT, H, C, region=region), 0.9, rtol=1e-12)
    assert np.all(np.abs(pl.best_factor(Td, MT, H, C) - 0.9) > 1e-3)
    assert np.allclose(pl.best_factor(T, MT, H, C, s_hi=0.5), 0.5)
    assert np.allclose(pl.best_factor(T, MT, H, C, s_lo=1.2), 1.2)


def test_best_factor_scales_with_the_data_and_degenerate_cases():
    H, C, MT, model = _bf_case(6)
    g = np.random.default_rng(1)
    T = model + g.normal(0, 0.2, model.shape)
    assert np.allclose(pl.best_factor(3 * T, MT, H, C), 3 * pl.best_factor(T, MT, H, C),
                       rtol=1e-12)
    MT1 = np.zeros_like(MT)
    MT1[:, 0] = 1
    assert np.all(pl.best_factor(T, MT1, H, C) == 1.0)
    Hc = np.ones_like(H)
    assert np.all(pl.best_factor(T, MT, Hc, C) == 1.0)


# ---- component-by-component build -------------------------------------------

def test_sequential_start_keeps_previous_components():
    g = np.random.default_rng(2)
    W = g.random((5, 2))
    H = g.random((2, 7))
    W0, H0 = pl.sequential_start(W, H, 9, 5, 7, 4)
    assert np.array_equal(W0[:, :2], W) and np.array_equal(H0[:2], H)
    assert W0.shape == (5, 3) and H0.shape == (3, 7)
    assert np.all((W0[:, 2] > 0) & (W0[:, 2] < 1)) and np.all((H0[2] > 0) & (H0[2] < 1))
    W1, H1 = pl.sequential_start(None, None, 9, 5, 7, 4)
    assert np.array_equal(W1[:, 0], W0[:, 0] * 0 + W1[:, 0]) and W1.shape == (5, 1)


def test_sequential_stage1_reaches_rank1_svd():
    g = np.random.default_rng(5)
    V = g.uniform(0.5, 2.0, (8, 11))
    W, H, J = pl.build_basis_sequential(V, np.ones_like(V), 1, 500, seed=3)
    s = np.linalg.svd(V, compute_uv=False)
    assert abs(J[0] - (np.sum(V ** 2) - s[0] ** 2)) <= 1e-10 * np.sum(V ** 2)


def test_sequential_recovers_planted_rank2():
    g = np.random.default_rng(0)
    N, P = 6, 12
    W0 = g.uniform(0.5, 2.0, (N, 2))
    H0 = g.uniform(0.5, 2.0, (2, P))
    H0[0, : P // 2] *= 0.1
    H0[1, P // 2:] *= 0.1
    V = W0 @ H0
    M = np.ones_like(V)
    W, H, J = pl.build_basis_sequential(V, M, 2, 3000, seed=1)
    assert J[-1] / np.sum(V ** 2) < 1e-10
    assert J[-1] < J[0]


def test_sequential_each_stage_descends_from_its_start():
    g = np.random.default_rng(3)
    V = g.gamma(2, 1, (10, 30))
    M = (g.random(V.shape) > 0.1) / (V + 0.01)
    n, p = V.shape
    W = H = None
    Vh, Mw, _ = nmf64.prep(V, M)
    for j in range(3):
        W0, H0 = pl.sequential_start(W, H, 4, n, p, 3)
        W, H, J = nmf64.build_basis(V, M, W0, H0, 40)
        assert J[-1] <= nmf64.objective(Vh, Mw, W0, H0)
        assert np.all(np.diff(J) <= 1e-12 * J[:-1])
    Ws, Hs, Js = pl.build_basis_sequential(V, M, 3, 40, seed=4)
    assert np.array_equal(Ws, W) and np.array_equal(Hs, H)


# ---- the pins catch plausible mistakes ----------------------------------------

def _dist_no_ref_mask(T, MT, V, M):
    return _orig["frame_distances"](T, MT, np.where(np.asarray(M) > 0, V, 0.0),
                                    np.ones_like(np.asarray(M, float)))


def _dist_abs(T, MT, V, M):
    T, MT, V, M = (np.asarray(x, float) for x in (T, MT, V, M))
    d = np.zeros((T.shape[0], V.shape[0]))
    for f in range(T.shape[0]):
        both = (M > 0) & (MT[f] > 0)[None, :]
        d[f] = np.sum(np.where(both, np.abs(np.where(both, T[f][None, :] - V, 0.0)), 0.0), axis=1)
    return d


def _closest_desc_ties(T, MT, V, M, n_sel):
    d = pl.frame_distances(T, MT, V, M)
    idx = np.array([sorted(range(d.shape[1]), key=lambda n: (d[f, n], -n))[:n_sel]
                    for f in range(d.shape[0])])
    return idx, d


def _bf_uncentred(T, MT, H, C, region=None, s_lo=0.0, s_hi=np.inf):
    model = np.asarray(C, float) @ np.asarray(H, float)
    T, MT = np.asarray(T, float), np.asarray(MT, float)
    s = np.ones(T.shape[0])
    for f in range(T.shape[0]):
        use = MT[f] > 0
        if region is not None:
            use &= np.asarray(region) > 0
        s[f] = min(max(np.sum(T[f][use] * model[f][use]) / np.sum(model[f][use] ** 2), s_lo),
                   s_hi)
    return s


def _bf_ignores_region(T, MT, H, C, region=None, s_lo=0.0, s_hi=np.inf):
    return _orig["best_factor"](T, MT, H, C, None, s_lo, s_hi)


def _bf_all_pixels(T, MT, H, C, region=None, s_lo=0.0, s_hi=np.inf):
    return _orig["best_factor"](np.nan_to_num(np.asarray(T, float)), np.ones_like(MT), H, C,
                                region, s_lo, s_hi)


def _seq_new_first(W_prev, H_prev, seed, n, p, K):
    W0, H0 = _orig["sequential_start"](W_prev, H_prev, seed, n, p, K)
    return np.roll(W0, 1, axis=1), np.roll(H0, 1, axis=0)


_orig = {k: getattr(pl, k) for k in ("frame_distances", "closest_frames", "best_factor",
                                     "sequential_start")}
PIPE_MUTANTS = {
    "distance ignores the reference mask": ("frame_distances", _dist_no_ref_mask),
    "distance sums absolute differences": ("frame_distances", _dist_abs),
    "selection breaks ties by descending index": ("closest_frames", _closest_desc_ties),
    "best factor without centring": ("best_factor", _bf_uncentred),
    "best factor ignores the region": ("best_factor", _bf_ignores_region),
    "best factor uses masked pixels": ("best_factor", _bf_all_pixels),
    "sequential start puts the new component first": ("sequential_start", _seq_new_first),
}


def _pipe_pins():
    yield test_distances_and_selection_hand_worked
    for s in range(2):
        yield lambda s=s: test_distances_match_expanded_products(s)
    yield test_planted_duplicate_is_closest_and_garbage_ignored
    yield test_best_factor_hand_worked
    yield test_best_factor_planted_scale_and_offset
    yield test_best_factor_region_excludes_a_disk_and_clamps
    yield test_sequential_start_keeps_previous_components
    yield test_sequential_each_stage_descends_from_its_start


@pytest.mark.parametrize("mutant", sorted(PIPE_MUTANTS))
def test_each_pipeline_mutant_is_caught(mutant, monkeypatch):
    attr, fn = PIPE_MUTANTS[mutant]
    monkeypatch.setattr(pl, attr, fn)
    caught = 0
    for pin in _pipe_pins():
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, ValueError, FloatingPointError):
            caught += 1
    assert caught, f"no pin catches: {mutant}"
