"""GPU parity of the basis construction (Eq. 3 iterated) against the FP64
oracle, through the C ABI.

Bar (stated per case): after a fixed iteration count from identical
initialisation,
  * relative objective |J(W_gpu, H_gpu) - J_oracle| / J_oracle <= 1e-5 (FP32)
    with J evaluated in FP64 on the GPU's factors;
  * relative model error ||M o (W_gpu H_gpu - W_o H_o)|| / ||M o W_o H_o||
    <= 1e-4 (FP32);
  * the GPU's own FP64-accumulated J history within 1e-5 of the oracle's.
The split-precision path (bf16x3) is held to the same bars; its measured
errors are printed.
"""
import numpy as np
import pytest

from oracle import nmf64, prng
from paper_2309_04623_amd import nmf, synth
from tests.helpers import dev, host, objective64, random_problem, rel_model_err, say

pytestmark = pytest.mark.gpu

TOL = {"fp32": (1e-5, 1e-4), "bf16x3": (1e-5, 1e-4)}


def _check_run(V, M, k, iters, precision, seed=7, tag="", flags=0):
    n, p = V.shape
    W0 = prng.init_matrix(seed, prng.MAT_W, n, k)
    H0 = prng.init_matrix(seed, prng.MAT_H, k, p)
    say(tag, f"n={n} p={p} k={k} iters={iters} prec={precision}")
    Wg, Hg, Jg, rep = nmf.build_basis(dev(V), dev(M), k, iters, precision=precision, seed=seed,
                                      flags=flags)
    Wg, Hg = host(Wg), host(Hg)
    Wo, Ho, Jo = nmf64.build_basis(V, M, W0, H0, iters)
    Jgpu64 = objective64(V, M, Wg, Hg)
    relJ = abs(Jgpu64 - Jo[-1]) / Jo[-1]
    Vh = np.where(M > 0, V, 0.0)
    model = rel_model_err(M, Wg @ Hg, Wo @ Ho)
    hist = np.max(np.abs(Jg - Jo) / Jo)
    self_j = abs(Jg[-1] - Jgpu64) / Jgpu64
    print(f"  relJ={relJ:.3e} model={model:.3e} hist={hist:.3e} selfJ={self_j:.3e} "
          f"relobj={rep['objective_rel']:.3e}", flush=True)
    tj, tm = TOL[precision]
    assert np.all(Wg >= 0) and np.all(Hg >= 0)
    assert relJ <= tj
    assert model <= tm
    assert hist <= tj
    assert self_j <= (1e-6 if precision == "fp32" else 1e-4)
    assert rep["iters_run"] == iters
    assert abs(rep["objective_rel"] - Jg[-1] / np.sum(M.astype(np.float64) * Vh ** 2)) < 1e-9
    return Wg, Hg, Jg


def test_init_uniform_bitwise():
    for seed, mid, r, c in [(0, 0, 64, 8), (12345, 1, 8, 4096), (2 ** 63 + 5, 2, 3, 1001)]:
        say("init", seed, mid, r, c)
        got = host(nmf.init_uniform(seed, mid, r, c))
        assert np.array_equal(got, prng.init_matrix(seed, mid, r, c))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_objective_matches_fp64(precision):
    V, M = random_problem(1, 70, 333, 6)
    g = np.random.default_rng(2)
    W = g.uniform(0, 1, (70, 6)).astype(np.float32)
    H = g.uniform(0, 1, (6, 333)).astype(np.float32)
    say("objective", precision)
    J = nmf.objective(dev(V), dev(M), dev(W), dev(H), precision=precision)
    J64 = objective64(V, M, W, H)
    assert abs(J - J64) / J64 < (1e-6 if precision == "fp32" else 2e-4)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_cfg1_parity(precision):
    """64 images of 64x64 px, K = 8, 200 iterations (the small configuration)."""
    lib = synth.make_cfg1()
    _check_run(lib.V, lib.M, 8, 200, precision, tag="cfg1")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,p,k,iters", [(37, 1000, 5, 60), (70, 333, 30, 40), (33, 2050, 33, 30),
                                         (150, 900, 90, 20), (130, 700, 100, 20),
                                         (200, 1057, 64, 25), (230, 1100, 150, 12),
                                         (210, 700, 180, 10), (260, 800, 200, 10)])
def test_ragged_shapes_parity(n, p, k, iters, precision):
    """Shapes that span several tiles with ragged tails in both directions and
    every padded component count (32 ... 224); from 96 on the wide-basis
    kernel runs, with column groups whose last waves have no tile."""
    V, M = random_problem(n * 7 + p, n, p, k)
    _check_run(V, M, k, iters, precision, tag="ragged")


def test_cfg2_reduced_parity():
    """STIS-like structure (speckle PSF, diagonal wedge, Poisson noise) at
    reduced size: 120 images of 80x80 px, K = 30, 150 iterations."""
    lib = synth.make_cfg2(n=120, ny=80, nx=80, k0=40, frames=2)
    _check_run(lib.V, lib.M, 30, 150, "fp32", tag="cfg2-reduced")


def test_binary_weights_parity():
    lib = synth.make_cfg3(n=96, ny=40, nx=48, k0=20, frames=1)
    _check_run(lib.V, lib.M, 16, 60, "fp32", tag="cfg3-reduced")
    _check_run(lib.V, lib.M, 16, 60, "bf16x3", tag="cfg3-reduced")
    _check_run(lib.V, lib.M, 16, 60, "fp32", tag="cfg3-reduced bitmask",
               flags=nmf.F_BINARY_WEIGHTS)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_binary_weights_wide_basis_parity(precision):
    """MIRI-like binary-weight library with a wide basis (K = 100, the
    precision-study component count) from bitmask weights."""
    lib = synth.make_cfg3(n=160, ny=56, nx=72, k0=120, frames=1)
    _check_run(lib.V, lib.M, 100, 25, precision, tag="cfg3-reduced wide bitmask",
               flags=nmf.F_BINARY_WEIGHTS)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,ny,nx,k", [(96, 40, 48, 16), (120, 25, 40, 100), (40, 9, 37, 40)])
def test_binary_weight_bitmask_bitwise(precision, n, ny, nx, k):
    """Binary weights stored as bitmasks (4 B + 1 bit per element instead of
    8 B) give bit-identical factors and objective history to the same 0/1
    weights stored as floats; any positive weight counts as 1."""
    lib = synth.make_cfg3(n=n, ny=ny, nx=nx, k0=min(k + 4, n), frames=1)
    V, M = lib.V, lib.M
    say("bitmask", precision, n, ny * nx, k)
    # a fresh handle and the bitmask build first, so that no captured graph of
    # the float-weight build can stand in for the bitmask kernels
    h = nmf.Handle(0)
    W2, H2, J2, r2 = nmf.build_basis(dev(V), dev(M), k, 25, precision=precision, seed=4,
                                     flags=nmf.F_BINARY_WEIGHTS, handle=h)
    W1, H1, J1, r1 = nmf.build_basis(dev(V), dev(M), k, 25, precision=precision, seed=4, handle=h)
    assert np.array_equal(host(W1), host(W2)) and np.array_equal(host(H1), host(H2))
    assert np.array_equal(J1, J2)
    M3 = M * np.random.default_rng(1).uniform(0.5, 3.0, M.shape).astype(np.float32)
    W3, H3, J3, _ = nmf.build_basis(dev(V), dev(M3), k, 25, precision=precision, seed=4,
                                    flags=nmf.F_BINARY_WEIGHTS, handle=h)
    assert np.array_equal(host(W1), host(W3)) and np.array_equal(host(H1), host(H3))
    h.close()


def test_weight_storage_change_on_one_handle():
    """Builds of one shape on one handle that switch between bitmask and float
    weight storage each meet the oracle (the captured iteration graphs are
    keyed by the weight storage)."""
    lib = synth.make_cfg3(n=64, ny=30, nx=40, k0=12, frames=1)
    n, p = lib.V.shape
    g = np.random.default_rng(3)
    Mf = (lib.M * g.uniform(0.5, 3.0, lib.M.shape)).astype(np.float32)
    h = nmf.Handle(0)
    say("storage switch: bitmask, then float weights, then bitmask")
    runs = [(lib.M, nmf.F_BINARY_WEIGHTS), (Mf, 0), (lib.M, nmf.F_BINARY_WEIGHTS), (Mf, 0)]
    W0 = prng.init_matrix(6, prng.MAT_W, n, 8)
    H0 = prng.init_matrix(6, prng.MAT_H, 8, p)
    for M, flags in runs:
        W, H, J, _ = nmf.build_basis(dev(lib.V), dev(M), 8, 40, seed=6, flags=flags, handle=h)
        Mo = (M > 0).astype(np.float64) if flags else M
        Wo, Ho, Jo = nmf64.build_basis(lib.V, Mo, W0, H0, 40)
        relJ = abs(objective64(lib.V, Mo, host(W), host(H)) - Jo[-1]) / Jo[-1]
        print(f"  flags={flags} relJ={relJ:.2e}", flush=True)
        assert relJ <= 1e-5
        assert np.max(np.abs(J - Jo) / Jo) <= 1e-5
    h.close()


def test_binary_weight_bitmask_projection_bitwise():
    lib = synth.make_cfg3(n=64, ny=40, nx=50, k0=12, frames=37)
    H = np.abs(lib.H0[:10]).astype(np.float32)
    say("bitmask projection")
    C1, _ = nmf.project(dev(H), dev(lib.T), dev(lib.MT), 200, seed=5)
    C2, _ = nmf.project(dev(H), dev(lib.T), dev(lib.MT), 200, seed=5, flags=nmf.F_BINARY_WEIGHTS)
    assert np.array_equal(host(C1), host(C2))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_masked_garbage_and_weight_scaling_bitwise(precision):
    V, M = random_problem(5, 50, 700, 7, mask_frac=0.2)
    say("invariance", precision)
    W1, H1, J1, _ = nmf.build_basis(dev(V), dev(M), 7, 30, precision=precision, seed=3)
    Vg = V.copy()
    holes = M == 0
    vals = np.array([np.nan, np.inf, -7.0, 3e38], np.float32)
    Vg[holes] = vals[np.arange(holes.sum()) % 4]
    W2, H2, _, _ = nmf.build_basis(dev(Vg), dev(M), 7, 30, precision=precision, seed=3)
    assert np.array_equal(host(W1), host(W2)) and np.array_equal(host(H1), host(H2))
    W3, H3, J3, _ = nmf.build_basis(dev(V), dev(M * 8), 7, 30, precision=precision, seed=3)
    assert np.array_equal(host(W1), host(W3)) and np.array_equal(host(H1), host(H3))


def test_deterministic_and_resumable():
    """Fixed-order reductions: repeated runs are bitwise equal, and T
    iterations equal T/2, then T/2 more from the saved factors."""
    V, M = random_problem(6, 90, 900, 12)
    say("determinism")
    a = nmf.build_basis(dev(V), dev(M), 12, 40, seed=9)
    b = nmf.build_basis(dev(V), dev(M), 12, 40, seed=9)
    assert np.array_equal(host(a[0]), host(b[0])) and np.array_equal(host(a[1]), host(b[1]))
    assert np.array_equal(a[2], b[2])
    h1 = nmf.build_basis(dev(V), dev(M), 12, 20, seed=9)
    h2 = nmf.build_basis(dev(V), dev(M), 12, 20, W_init=h1[0], H_init=h1[1])
    assert np.array_equal(host(a[0]), host(h2[0])) and np.array_equal(host(a[1]), host(h2[1]))


def test_data_errors_and_guards():
    V, M = random_problem(8, 40, 300, 4)
    say("validation")
    bad = V.copy()
    bad[3, 5] = np.nan
    M2 = M.copy()
    M2[3, 5] = 1.0
    with pytest.raises(nmf.NmfError) as e:
        nmf.build_basis(dev(bad), dev(M2), 4, 5, flags=nmf.F_VALIDATE_DATA)
    assert e.value.status == nmf.NMF_ERR_NONFINITE
    bad[3, 5] = -2.0
    with pytest.raises(nmf.NmfError) as e:
        nmf.build_basis(dev(bad), dev(M2), 4, 5, flags=nmf.F_VALIDATE_DATA)
    assert e.value.status == nmf.NMF_ERR_NEGATIVE
    # clipping treats the negative pixel as masked
    W, H, J, _ = nmf.build_basis(dev(bad), dev(M2), 4, 5, flags=nmf.F_VALIDATE_DATA | nmf.F_CLIP_NEGATIVE)
    M3 = M2.copy()
    M3[3, 5] = 0
    W3, H3, J3, _ = nmf.build_basis(dev(bad), dev(M3), 4, 5)
    assert np.array_equal(host(W), host(W3))
    negw = M.copy()
    negw[0, 0] = -1.0
    with pytest.raises(nmf.NmfError) as e:
        nmf.build_basis(dev(V), dev(negw), 4, 5)
    assert e.value.status == nmf.NMF_ERR_NEGATIVE
    # a pixel masked in every image and an image masked everywhere keep their factors
    Mz = M.copy()
    Mz[:, 17] = 0
    Mz[11, :] = 0
    W0 = nmf.init_uniform(4, 0, 40, 4)
    H0 = nmf.init_uniform(4, 1, 4, 300)
    W, H, J, _ = nmf.build_basis(dev(V), dev(Mz), 4, 10, W_init=W0, H_init=H0)
    assert np.array_equal(host(H)[:, 17], host(H0)[:, 17])
    assert np.array_equal(host(W)[11], host(W0)[11])


@pytest.mark.parametrize("c,tol", [(10, 1e-4), (7, 3e-4), (25, 3e-5)])
def test_tolerance_stop_matches_oracle_rule(c, tol):
    """The on-device stop rule (relative decrease of J over c iterations,
    tested at multiples of c; the iteration at which it passes is the last)
    stops at the iteration the oracle's rule picks from its own history, and
    the histories agree."""
    lib = synth.make_cfg1(n=48, ny=40, nx=40, k0=6)
    n, p = lib.V.shape
    T = 3000
    say("tol-stop", c, tol)
    W, H, J, rep = nmf.build_basis(dev(lib.V), dev(lib.M), 6, T, tol=tol, check_every=c, seed=3)
    W0 = prng.init_matrix(3, prng.MAT_W, n, 6)
    H0 = prng.init_matrix(3, prng.MAT_H, 6, p)
    Wo, Ho, Jo, run = nmf64.build_basis_tol(lib.V, lib.M, W0, H0, T, c, tol)
    print(f"  device stopped after {rep['iters_run']}, oracle after {run}", flush=True)
    assert run < T
    # the decisive relative decrease is not within rounding of tol, so both
    # sides must take the same decision
    t = run - 1
    margin = abs((Jo[t - c] - Jo[t]) / Jo[t - c] - tol) / tol
    assert margin > 1e-3
    assert rep["iters_run"] == run
    assert rep["status"] == 0
    assert len(J) == run + 1
    assert np.max(np.abs(J - Jo) / Jo) <= 1e-5
    J64 = objective64(lib.V, lib.M, host(W), host(H))
    assert abs(J64 - Jo[-1]) / Jo[-1] <= 1e-5


def test_tolerance_not_met_warns_maxiter():
    lib = synth.make_cfg1(n=48, ny=40, nx=40, k0=6)
    say("tol-stop maxiter")
    W, H, J, rep = nmf.build_basis(dev(lib.V), dev(lib.M), 6, 40, tol=1e-12, check_every=10)
    assert rep["iters_run"] == 40 and rep["status"] == nmf.NMF_WARN_MAXITER


def test_normalisation_matches_oracle():
    """NMF_F_NORMALIZE_H equals the oracle's unit-L2 component normalisation
    applied to the same build's unnormalised factors."""
    lib = synth.make_cfg1(n=48, ny=40, nx=40, k0=6)
    say("normalisation")
    Wn, Hn, Jn, _ = nmf.build_basis(dev(lib.V), dev(lib.M), 6, 50, flags=nmf.F_NORMALIZE_H)
    Wp, Hp, Jp, _ = nmf.build_basis(dev(lib.V), dev(lib.M), 6, 50)
    Wo, Ho = nmf64.normalize_components(host(Wp), host(Hp))
    assert np.max(np.abs(host(Hn) - Ho) / np.abs(Ho).max(axis=1, keepdims=True)) < 2e-7
    assert np.max(np.abs(host(Wn) - Wo) / np.abs(Wo).max(axis=0, keepdims=True)) < 2e-7
    assert np.array_equal(Jn, Jp)


def test_cfg2_full_size_one_iteration():
    """STIS-shaped library at full size (500 x 200x200 px, K = 30): one
    iteration from the seeded start matches the oracle's iterate."""
    lib = synth.make_cfg2(frames=1)
    V, M = lib.V, lib.M
    say("cfg2-full one iteration")
    Wg, Hg, Jg, _ = nmf.build_basis(dev(V), dev(M), 30, 1, seed=11)
    W0 = prng.init_matrix(11, 0, 500, 30)
    H0 = prng.init_matrix(11, 1, 30, 40000)
    Wo, Ho, Jo = nmf64.build_basis(V, M, W0, H0, 1)
    for g, o in ((host(Wg), Wo), (host(Hg), Ho)):
        assert np.linalg.norm(g - o) / np.linalg.norm(o) < 1e-5
    assert np.max(np.abs(Jg - Jo) / Jo) < 1e-6


def test_cfg2_full_size_trajectory_properties():
    """The benchmarked configuration (500 x 40000, K = 30, 1000 FP32
    iterations): objective non-increasing up to FP32 rounding, factors
    non-negative, the reported J equals the FP64 cost of the returned
    factors."""
    lib = synth.make_cfg2(frames=1)
    say("cfg2-full 1000 iterations")
    W, H, J, rep = nmf.build_basis(dev(lib.V), dev(lib.M), 30, 1000, seed=1)
    assert rep["status"] == 0
    assert np.all(np.diff(J) <= 1e-6 * J[:-1])
    W, H = host(W), host(H)
    assert W.min() >= 0 and H.min() >= 0
    J64 = objective64(lib.V, lib.M, W, H)
    assert abs(J[-1] - J64) / J64 < 1e-6


def test_graph_replay_matches_eager_launches():
    """Iterations replayed from captured graphs give the same bits as eager
    launches (timing on disables graphs), over several calls with other
    device work in between; 150 iterations span three graph chunks."""
    import torch
    V, M = random_problem(12, 70, 1500, 9)
    say("graph vs eager")
    h = nmf.Handle(0)
    nmf.profile_enable(h, True)
    We, He, Je, _ = nmf.build_basis(dev(V), dev(M), 9, 150, seed=5, handle=h)
    nmf.profile_enable(h, False)
    for _ in range(3):
        Wg, Hg, Jg, _ = nmf.build_basis(dev(V), dev(M), 9, 150, seed=5, handle=h)
        torch.cuda.synchronize()
        assert torch.equal(Wg, We) and torch.equal(Hg, He)
        assert np.array_equal(Jg, Je)
        _ = torch.randn(4096, device="cuda").sum().item()
    h.close()


def test_autotuned_shapes_give_oracle_parity():
    """With NMF_F_AUTOTUNE the launch shapes are timed on first use and
    cached; results still meet the FP32 bars."""
    lib = synth.make_cfg2(n=96, ny=64, nx=64, k0=20, frames=1)
    say("autotune")
    h = nmf.Handle(0)
    n, p = lib.V.shape
    W, H, J, rep = nmf.build_basis(dev(lib.V), dev(lib.M), 16, 80, seed=2, flags=nmf.F_AUTOTUNE,
                                   handle=h)
    report = nmf.autotune_report(h)
    print(report, flush=True)
    assert report.count("\n") == 2
    Wo, Ho, Jo = nmf64.build_basis(lib.V, lib.M, prng.init_matrix(2, 0, n, 16),
                                   prng.init_matrix(2, 1, 16, p), 80)
    J64 = objective64(lib.V, lib.M, host(W), host(H))
    assert abs(J64 - Jo[-1]) / Jo[-1] <= 1e-5
    h.close()
