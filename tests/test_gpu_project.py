"""GPU parity of target modelling (projection with the basis fixed) and of
model-PSF subtraction against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import nmf64, nnls, prng
from paper_2309_04623_amd import nmf, synth
from tests.helpers import dev, host, rel_model_err, say

pytestmark = pytest.mark.gpu


def _basis(k, p, seed=0):
    g = np.random.default_rng(seed)
    return (g.gamma(1.0, 1.0, (k, p)) * g.uniform(0.2, 1.0, (k, 1))).astype(np.float32)


def _frames(H, f, seed=1, mask_frac=0.1, peak=None, noise=0.05):
    """Frames t = c H + noise: Poisson-like at ``peak`` counts (paper-like
    photon noise) or |N(0, noise)| when ``peak`` is None (near noiseless)."""
    g = np.random.default_rng(seed)
    k, p = H.shape
    clean = g.gamma(2.0, 1.0, (f, k)) @ H
    if peak is None:
        T = clean + np.abs(g.normal(0, noise, (f, p)))
    else:
        gain = peak / clean.max(axis=1, keepdims=True)
        T = g.poisson(gain * clean) / gain
    MT = (g.random((f, p)) >= mask_frac) / (T + 0.01)
    return T.astype(np.float32), MT.astype(np.float32)


def _projection_case(f, k, p, iters, precision, peak):
    H = _basis(k, p, seed=k)
    T, MT = _frames(H, f, seed=f + k, peak=peak)
    C0 = prng.init_matrix(5, prng.MAT_C, f, k)
    say("project", f, k, p, iters, precision, peak)
    C, obj, _ = nmf.project(dev(H), dev(T), dev(MT), iters, precision=precision, seed=5,
                            want_objective=True)
    Cg = host(C)
    Co = nmf64.project(T, MT, H, C0, iters)
    Jo = nmf64.frame_objective(T, MT, H, Co)
    Jg = nmf64.frame_objective(T, MT, H, Cg)
    relJ = np.abs(Jg - Jo) / Jo
    model = np.array([rel_model_err(MT[i:i + 1], Cg[i:i + 1] @ H, Co[i:i + 1] @ H) for i in range(f)])
    # signal-to-residual ratio ||m o model|| / ||m o (t - model)|| per frame
    Th = np.where(MT > 0, T, 0.0)
    mod = Co @ H
    snr = np.linalg.norm(MT * mod, axis=1) / np.linalg.norm(MT * (Th - mod), axis=1)
    print(f"  relJ={relJ.max():.3e} model={model.max():.3e} snr={snr.max():.1f}", flush=True)
    assert np.all(Cg >= 0)
    # the device objective matches the FP64 cost of the returned coefficients
    assert np.max(np.abs(host(obj) - Jg) / Jg) < 1e-6
    return relJ, model, snr


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("f,k,p,iters", [(1, 8, 4096, 200), (50, 30, 6400, 300), (37, 5, 1000, 100),
                                         (3, 100, 3000, 80), (70, 33, 777, 120)])
def test_projection_parity(f, k, p, iters, precision):
    """Photon-noise frames (peak 1e4 counts): relative objective <= 1e-5 and
    model error <= 1e-4 in both precision forms."""
    relJ, model, _ = _projection_case(f, k, p, iters, precision, peak=1e4)
    assert relJ.max() <= 1e-5 and model.max() <= 1e-4


@pytest.mark.parametrize("f,k,p,iters", [(50, 30, 6400, 300), (70, 33, 777, 120)])
def test_projection_parity_near_noiseless(f, k, p, iters):
    """Near-noiseless frames: the residual is ~1/snr of the model, so any
    relative change d of the FP32 model moves J by ~2 d snr.  The objective
    bar is derived from a model error of 16 FP32 ulps (1e-6):
    relJ <= max(1e-5, 2 * 1e-6 * snr); the model bar stays 1e-4."""
    relJ, model, snr = _projection_case(f, k, p, iters, "fp32", peak=None)
    assert np.all(relJ <= np.maximum(1e-5, 2e-6 * snr))
    assert model.max() <= 1e-4


def test_projection_converges_to_nnls():
    """Run long enough and the projection reaches the exact weighted NNLS
    minimiser (brute force over supports, K = 4)."""
    H = _basis(4, 500, seed=3)
    T, MT = _frames(H, 6, seed=4)
    say("project->nnls")
    C, _ = nmf.project(dev(H), dev(T), dev(MT), 20000, seed=2)
    C = host(C)
    for i in range(6):
        G, b, c = nnls.normal_equations(H, T[i], MT[i])
        w, j = nnls.nnls_bruteforce(G, b, c)
        assert nnls.cost(G, b, c, C[i]) - j <= 1e-5 * j


def test_cfg2_projection_full_size():
    """50 STIS-shaped science frames (200x200 px, disks at 1e-3) projected on a
    30-component basis for 1000 iterations."""
    lib = synth.make_cfg2(n=60, frames=50)
    H = np.abs(lib.H0[:30]).astype(np.float32)
    say("cfg2 projection 50 frames")
    C, _ = nmf.project(dev(H), dev(lib.T), dev(lib.MT), 1000, seed=8)
    Cg = host(C)
    C0 = prng.init_matrix(8, prng.MAT_C, 50, 30)
    sel = [0, 17, 49]
    Co = nmf64.project(lib.T[sel], lib.MT[sel], H, C0[sel], 1000)
    for j, i in enumerate(sel):
        assert rel_model_err(lib.MT[i:i + 1], Cg[i:i + 1] @ H, Co[j:j + 1] @ H) <= 1e-4


@pytest.mark.parametrize("f,k,p", [(1, 8, 4096), (50, 30, 40000), (7, 100, 1001)])
def test_subtract_parity(f, k, p):
    g = np.random.default_rng(f + k)
    H = g.gamma(1.0, 1.0, (k, p)).astype(np.float32)
    C = g.gamma(2.0, 1.0, (f, k)).astype(np.float32)
    T = (C.astype(np.float64) @ H + g.normal(0, 0.1, (f, p))).astype(np.float32)
    MT = (g.random((f, p)) > 0.1).astype(np.float32)
    T[MT == 0] = np.nan  # masked pixels may hold anything
    scale = g.uniform(0.5, 1.5, f).astype(np.float32)
    say("subtract", f, k, p)
    model, resid = nmf.subtract(dev(H), dev(C), dev(T), dev(MT), scale=dev(scale))
    mo, ro = nmf64.subtract(T, MT, H, C, scale=scale)
    mg, rg = host(model), host(resid)
    assert np.max(np.abs(mg - mo) / np.abs(mo)) < 1e-7
    assert np.array_equal(np.isnan(rg), np.isnan(ro))
    ok = ~np.isnan(ro)
    assert np.max(np.abs(rg[ok] - ro[ok]) / (np.abs(mo[ok]) + np.abs(T[ok]))) < 1e-7


def test_stis_timing_workload_meets_nnls_tolerance():
    """The STIS-shaped timing workload (500 x 40000 library, K = 30 built
    with 1000 iterations, 50 science frames projected in the masked-Gram
    form, the same seeds): with 100000 iterations every frame's model PSF is
    within 1e-4 of the exact weighted-NNLS model (FP64, Cholesky-reduced
    normal equations), so such a run counts as frames reaching that
    tolerance.  Multiplicative updates approach the NNLS minimiser slowly
    (cond(G) ~ 4e3 here); shorter runs are reported for information."""
    lib = synth.make_cfg2()
    say("stis workload: basis build")
    _, H, _, _ = nmf.build_basis(dev(lib.V), dev(lib.M), 30, 1000, seed=1)
    Hh = host(H)
    ref = []
    for i in range(lib.T.shape[0]):
        G, b, _ = nnls.normal_equations(Hh, lib.T[i], lib.MT[i])
        ref.append(nnls.nnls_gram(G, b) @ Hh)
    for iters in (1000, 10000, STIS_TOL_ITERS):
        say("stis workload: projection", iters)
        C, _ = nmf.project(H, dev(lib.T), dev(lib.MT), iters, seed=2, gram=True)
        Cg = host(C)
        errs = np.array([rel_model_err(lib.MT[i:i + 1], Cg[i:i + 1] @ Hh, ref[i][None])
                         for i in range(lib.T.shape[0])])
        print(f"  {iters} iterations: model error max {errs.max():.2e} median "
              f"{np.median(errs):.2e}; met {np.mean(errs <= 1e-4):.2f}", flush=True)
    assert errs.max() <= 1e-4


# iterations at which every frame of the STIS-shaped timing workload meets the
# 1e-4 model tolerance (the projection count the benchmark times)
STIS_TOL_ITERS = 100000


def test_frame_objective_follows_weight_flags():
    """The per-frame objective of a projection uses the weights as the
    projection staged them: with NMF_F_BINARY_WEIGHTS every positive weight
    counts as 1, with NMF_F_CLIP_NEGATIVE negative data is masked."""
    H = _basis(6, 900, seed=9)
    T, MT = _frames(H, 5, seed=10, peak=1e4)
    MT = MT * np.random.default_rng(11).uniform(0.5, 3.0, MT.shape).astype(np.float32)
    T[0, :7] = -1.0
    say("frame objective flags")
    for flags in (nmf.F_BINARY_WEIGHTS | nmf.F_CLIP_NEGATIVE, nmf.F_CLIP_NEGATIVE):
        for gram in (False, True):
            C, obj, _ = nmf.project(dev(H), dev(T), dev(MT), 50, seed=1, flags=flags,
                                    gram=gram, want_objective=True)
            Mo = (MT > 0).astype(np.float64) if flags & nmf.F_BINARY_WEIGHTS else MT.astype(np.float64)
            Mo = np.where(T < 0, 0.0, Mo)
            Jo = nmf64.frame_objective(T, Mo, H, host(C))
            assert np.max(np.abs(host(obj) - Jo) / Jo) < 1e-6
