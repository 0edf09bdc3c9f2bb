"""GPU parity of reference selection, best factor and the
component-by-component basis build against the FP64 oracle
(oracle/pipeline64.py), through the C ABI.

Bars: distances within 1e-6 relative (FP32 differences, FP64 across
chunks); the selected index sets equal wherever the oracle's distances
separate them by more than that, and every selection valid (no unselected
reference strictly closer beyond the tolerance); best factor within 1e-9
relative (the model is formed in FP64 from the same FP32 inputs); the
sequential build's objective after every stage within 1e-5 relative and the
final model within 1e-4 (the basis-build bars).
"""
import numpy as np
import pytest

from oracle import nmf64, pipeline64 as pl
from paper_2309_04623_amd import nmf, synth
from tests.helpers import dev, host, objective64, rel_model_err, say

pytestmark = pytest.mark.gpu

DIST_TOL = 1e-6


def _check_selection(idx_g, d_o, n_sel):
    """GPU indices against the oracle's distances: valid selections, equal to
    the oracle's wherever the distances are separated."""
    for f in range(d_o.shape[0]):
        order = sorted(range(d_o.shape[1]), key=lambda n: (d_o[f, n], n))
        kth = d_o[f, order[n_sel - 1]]
        sel = set(int(i) for i in idx_g[f])
        assert len(sel) == n_sel
        # every selected reference is within tolerance of the n_sel-th distance
        assert max(d_o[f, i] for i in sel) <= kth * (1 + 4 * DIST_TOL) + 1e-300
        # every reference clearly closer than the n_sel-th one is selected
        clear = {n for n in range(d_o.shape[1]) if d_o[f, n] < kth * (1 - 4 * DIST_TOL)}
        assert clear <= sel
        # ordered by distance
        ds = [d_o[f, int(i)] for i in idx_g[f]]
        assert all(ds[i] <= ds[i + 1] * (1 + 4 * DIST_TOL) for i in range(len(ds) - 1))


@pytest.mark.parametrize("f,n,p,n_sel", [(5, 300, 3000, 30), (9, 70, 1111, 70), (1, 1, 64, 1),
                                         (17, 130, 257, 13)])
def test_closest_frames_random(f, n, p, n_sel):
    g = np.random.default_rng(f * 1000 + n)
    V = g.gamma(2, 1, (n, p)).astype(np.float32)
    T = g.gamma(2, 1, (f, p)).astype(np.float32)
    M = (g.random((n, p)) > 0.05).astype(np.float32)
    MT = (g.random((f, p)) > 0.05).astype(np.float32)
    V[M == 0] = np.nan  # masked data is never read
    say("closest frames", f, n, p, n_sel)
    idx, dist = nmf.closest_frames(dev(V), dev(M), dev(T), dev(MT), n_sel, want_dist=True)
    idx_o, d_o = pl.closest_frames(T, MT, V, M, n_sel)
    dg = dist.cpu().numpy()
    assert np.max(np.abs(dg - d_o) / np.maximum(d_o, 1e-30)) < DIST_TOL
    _check_selection(idx.cpu().numpy(), d_o, n_sel)


def test_closest_frames_stis_library_with_planted_duplicates():
    """STIS-shaped library (500 images of 200x200 px, occulting wedge) and 8
    of its science frames; two library frames are replaced by copies of
    targets, which must come first at distance 0."""
    lib = synth.make_cfg2(frames=8)
    V, M = lib.V.copy(), lib.M.copy()
    V[123] = lib.T[2]
    M[123] = lib.MT[2]
    V[7] = lib.T[5]
    M[7] = lib.MT[5]
    say("closest frames STIS")
    idx, dist = nmf.closest_frames(dev(V), dev(M), dev(lib.T), dev(lib.MT), 50, want_dist=True)
    idx_g = idx.cpu().numpy()
    assert idx_g[2, 0] == 123 and idx_g[5, 0] == 7
    dg = dist.cpu().numpy()
    assert dg[2, 123] == 0.0 and dg[5, 7] == 0.0
    d_o = pl.frame_distances(lib.T, lib.MT, V, M)
    assert np.max(np.abs(dg - d_o) / np.maximum(d_o, 1e-30)) < DIST_TOL
    _check_selection(idx_g, d_o, 50)


def test_closest_frames_rejects_nonfinite_data_under_weight():
    V = np.ones((4, 100), np.float32)
    V[2, 5] = np.inf
    say("closest frames nonfinite")
    with pytest.raises(nmf.NmfError) as e:
        nmf.closest_frames(dev(V), dev(np.ones_like(V)), dev(np.ones((1, 100))),
                           dev(np.ones((1, 100))), 2)
    assert e.value.status == nmf.NMF_ERR_NONFINITE


@pytest.mark.parametrize("f,k,p", [(4, 8, 4096), (50, 30, 40000), (3, 100, 777)])
def test_best_factor_and_scaled_subtraction(f, k, p):
    g = np.random.default_rng(k)
    H = g.gamma(1, 1, (k, p)).astype(np.float32)
    C = g.gamma(2, 1, (f, k)).astype(np.float32)
    model = C.astype(np.float64) @ H
    s0 = g.uniform(0.6, 1.1, f)
    T = (s0[:, None] * model + g.normal(0, 0.05 * model.std(), model.shape)).astype(np.float32)
    MT = (g.random((f, p)) > 0.1).astype(np.float32)
    region = (g.random(p) > 0.3).astype(np.float32)
    say("best factor", f, k, p)
    for reg, lo, hi in ((None, 0.0, np.inf), (region, 0.0, np.inf), (None, 0.8, 0.9)):
        s = host(nmf.best_factor(dev(H), dev(C), dev(T), dev(MT),
                                 None if reg is None else dev(reg), lo, hi))
        s_o = pl.best_factor(T, MT, H, C, reg, lo, hi)
        assert np.max(np.abs(s - s_o) / np.abs(s_o)) < 1e-6  # FP32 result of an FP64 value
    s_t = nmf.best_factor(dev(H), dev(C), dev(T), dev(MT))
    _, resid = nmf.subtract(dev(H), dev(C), dev(T), dev(MT), scale=s_t)
    _, r_o = nmf64.subtract(T, MT, H, C, scale=host(s_t))
    rg = resid.cpu().numpy()
    assert np.array_equal(np.isnan(rg), np.isnan(r_o))
    ok = ~np.isnan(r_o)
    assert np.max(np.abs(rg[ok] - r_o[ok])) <= 1e-6 * np.max(np.abs(T))


def test_best_factor_degenerate_frames():
    H = np.ones((2, 50), np.float32)
    C = np.array([[1.0, 2.0], [0.5, 0.5]], np.float32)
    T = np.random.default_rng(0).random((2, 50)).astype(np.float32)
    MT = np.ones((2, 50), np.float32)
    MT[1, 1:] = 0
    say("best factor degenerate")
    s = host(nmf.best_factor(dev(H), dev(C), dev(T), dev(MT)))
    assert np.array_equal(s, [1.0, 1.0])


@pytest.mark.parametrize("n,p,k,iters", [(40, 300, 5, 30), (80, 700, 34, 6)])
def test_sequential_build_matches_oracle(n, p, k, iters):
    g = np.random.default_rng(n + k)
    W0 = g.gamma(2, 1, (n, k + 2))
    H0 = g.gamma(1, 1, (k + 2, p))
    V = (W0 @ H0 + np.abs(g.normal(0, 0.05, (n, p)))).astype(np.float32)
    M = ((g.random((n, p)) > 0.1) / (V + 0.01)).astype(np.float32)
    say("sequential build", n, p, k, iters)
    W, H, stages, rep = nmf.build_basis_sequential(dev(V), dev(M), k, iters, seed=6)
    Wo, Ho, Jo = pl.build_basis_sequential(V, M, k, iters, seed=6)
    assert rep["iters_run"] == k * iters
    rel = np.abs(stages - Jo) / Jo
    print(f"  stage objectives max rel {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-5
    Wg, Hg = host(W), host(H)
    assert rel_model_err(M, Wg @ Hg, Wo @ Ho) <= 1e-4
    J64 = objective64(V, M, Wg, Hg)
    assert abs(J64 - Jo[-1]) / Jo[-1] <= 1e-5
