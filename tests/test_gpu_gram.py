"""GPU parity of the masked-Gram projection (dense frames and CSR frames in
one persistent launch) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import nmf64, nnls, prng
from paper_2309_04623_amd import nmf, synth
from tests.helpers import dev, host, rel_model_err, say

pytestmark = pytest.mark.gpu


def _basis(k, p, seed=0):
    g = np.random.default_rng(seed)
    return (g.gamma(1.0, 1.0, (k, p)) * g.uniform(0.2, 1.0, (k, 1))).astype(np.float32)


def _photon_frames(H, f, seed, peak=1e4, mask_frac=0.1):
    g = np.random.default_rng(seed)
    clean = g.gamma(2.0, 1.0, (f, H.shape[0])) @ H
    gain = peak / clean.max(axis=1, keepdims=True)
    T = g.poisson(gain * clean) / gain
    MT = (g.random(T.shape) >= mask_frac) / (T + 0.01)
    return T.astype(np.float32), MT.astype(np.float32)


# Relative model error of one product: 16 FP32 ulps for FP32, and for the
# bf16 x 3 split form the terms it drops (lo*lo and the two residuals of the
# split, each up to 2^-18 of the product), 3 * 2^-18 ~ 1.1e-5.
MODEL_ULP = {"fp32": 1e-6, "bf16x3": 1.1e-5}


def _compare(T, MT, H, Cg, Co, tol_j=1e-5, tol_m=1e-4, derived=False, precision="fp32"):
    """Objective and model bars.  With ``derived`` the objective bar is
    max(tol_j, 2 d snr): a relative change d of the model (MODEL_ULP of the
    precision form) moves J by about 2 d times the model-to-residual ratio
    snr."""
    Jo = nmf64.frame_objective(T, MT, H, Co)
    Jg = nmf64.frame_objective(T, MT, H, Cg)
    # frames the basis fits exactly (fewer pixels than components) have J ~ 0:
    # only their model error is compared
    base = np.sum(MT * np.where(MT > 0, T, 0.0) ** 2, axis=1)
    fit = Jo > 1e-9 * base
    relJ = np.where(fit, np.abs(Jg - Jo) / np.where(fit, Jo, 1.0), 0.0)
    model = max(rel_model_err(MT[i:i + 1], Cg[i:i + 1] @ H, Co[i:i + 1] @ H) for i in range(len(T)))
    Th = np.where(MT > 0, T, 0.0)
    mod = Co @ H
    snr = np.linalg.norm(MT * mod, axis=1) / np.maximum(np.linalg.norm(MT * (Th - mod), axis=1), 1e-300)
    bar = np.maximum(tol_j, 2 * MODEL_ULP[precision] * snr) if derived else tol_j
    print(f"  relJ={relJ.max():.3e} model={model:.3e} snr={snr.max():.1f}", flush=True)
    assert np.all(relJ <= bar) and model <= tol_m
    assert np.all(Cg >= 0)


@pytest.mark.parametrize("f,k,p,iters", [(1, 8, 4096, 200), (50, 30, 6400, 300), (37, 5, 1000, 100),
                                         (3, 100, 3000, 80), (9, 33, 777, 120), (4, 200, 2500, 60),
                                         (5, 130, 1100, 50)])
def test_gram_dense_parity(f, k, p, iters):
    """Dense frames through the Gram form: the oracle's direct-form iterate
    (same value in exact arithmetic) within 1e-5 objective / 1e-4 model."""
    H = _basis(k, p, seed=k)
    T, MT = _photon_frames(H, f, seed=f + k)
    C0 = prng.init_matrix(5, prng.MAT_C, f, k)
    say("gram dense", f, k, p, iters)
    C, obj, _ = nmf.project(dev(H), dev(T), dev(MT), iters, seed=5, gram=True, want_objective=True)
    Co = nmf64.project(T, MT, H, C0, iters)
    _compare(T, MT, H, host(C), Co)
    Jg = nmf64.frame_objective(T, MT, H, host(C))
    assert np.max(np.abs(host(obj) - Jg) / Jg) < 1e-6


def _ragged(H, sizes, seed, binary=False):
    g = np.random.default_rng(seed)
    k, p = H.shape
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pix = np.concatenate([np.sort(g.choice(p, s, replace=False)) for s in sizes]).astype(np.int32)
    w = g.gamma(2.0, 1.0, (len(sizes), k))
    val = np.empty(offs[-1], np.float32)
    for i in range(len(sizes)):
        if sizes[i] == 0:
            continue
        clean = w[i] @ H[:, pix[offs[i]:offs[i + 1]]]
        gain = 1e4 / max(clean.max(), 1e-30)
        val[offs[i]:offs[i + 1]] = g.poisson(gain * clean) / gain
    wt = np.ones_like(val) if binary else (1.0 / (val + 0.01)).astype(np.float32)
    return offs, pix, val, wt


@pytest.mark.parametrize("k,p,sizes,binary", [
    (8, 4096, [4096, 100, 1, 2000, 33], False),
    (30, 6400, [6400, 0, 3000, 31, 32, 33, 5000], True),
    (100, 3000, [2999, 1500, 64, 700], False),
    (200, 2500, [2500, 1200, 300], True),
])
def test_ragged_parity(k, p, sizes, binary):
    """CSR frames of uneven size (including an empty frame and sizes around
    the 32-pixel chunk) match the oracle frame by frame."""
    H = _basis(k, p, seed=k + 1)
    offs, pix, val, wt = _ragged(H, sizes, seed=k, binary=binary)
    f = len(sizes)
    iters = 100
    C0 = prng.init_matrix(9, prng.MAT_C, f, k)
    say("ragged", k, p, sizes)
    C, ticks, rep = nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val),
                                       None if binary else dev(wt), iters, seed=9, want_ticks=True)
    Cg = host(C)
    Co = nmf64.project_ragged(offs, pix, val, wt, H, C0, iters)
    T, MT = nmf64.ragged_to_dense(offs, pix, val, wt, p)
    nonempty = [i for i in range(f) if sizes[i] > 0]
    _compare(T[nonempty], MT[nonempty], H, Cg[nonempty], Co[nonempty], derived=True,
             precision="bf16x3")
    for i in range(f):
        if sizes[i] == 0:  # no data: den = 0 keeps the start values
            assert np.array_equal(Cg[i], C0[i].astype(np.float32))
    t = host(ticks).astype(np.int64).reshape(f, 2)
    assert np.all(t[:, 1] >= t[:, 0]) and np.all(t[:, 0] > 0)


def dev_i64(x):
    import torch
    return torch.as_tensor(np.asarray(x, np.int64)).cuda()


def dev_i32(x):
    import torch
    return torch.as_tensor(np.asarray(x, np.int32)).cuda()


def test_ragged_bad_entries_rejected():
    H = _basis(4, 100, seed=1)
    offs = np.array([0, 3, 6], np.int64)
    pix = np.array([1, 2, 3, 4, 5, 100], np.int32)  # 100 is out of range
    val = np.ones(6, np.float32)
    say("ragged bad pixel")
    with pytest.raises(nmf.NmfError) as e:
        nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val), None, 5)
    assert e.value.status == nmf.NMF_ERR_ARG
    offs = np.array([0, 3, 9], np.int64)  # past nnz
    pix[5] = 5
    with pytest.raises(nmf.NmfError) as e:
        nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val), None, 5)
    assert e.value.status == nmf.NMF_ERR_ARG


def test_ragged_graph_replay_matches_eager():
    """The captured graph replays to the same bits as an eager (timed) run,
    several replays in a row with other work in between."""
    H = _basis(30, 2000, seed=2)
    offs, pix, val, wt = _ragged(H, [2000, 50, 1234, 700] * 8, seed=3)
    args = (dev(H), dev_i64(offs), dev_i32(pix), dev(val), dev(wt))
    say("ragged graph replay")
    h = nmf.Handle(0)
    nmf.profile_enable(h, True)
    ref, _ = nmf.project_ragged(*args, 50, seed=4, handle=h)
    nmf.profile_enable(h, False)
    import torch
    C0 = nmf.init_uniform(4, nmf.MAT_C, len(offs) - 1, 30)
    for i in range(4):
        C, _ = nmf.project_ragged(*args, 50, seed=4, C_init=C0, handle=h)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
        _ = torch.randn(1000, device="cuda").sum().item()
    h.close()


def test_gram_projection_reaches_nnls():
    H = _basis(4, 600, seed=7)
    T, MT = _photon_frames(H, 5, seed=8)
    say("gram -> nnls")
    C, _ = nmf.project(dev(H), dev(T), dev(MT), 30000, seed=1, gram=True)
    C = host(C)
    for i in range(5):
        G, b, c = nnls.normal_equations(H, T[i], MT[i])
        w, j = nnls.nnls_bruteforce(G, b, c)
        assert nnls.cost(G, b, c, C[i]) - j <= 1e-5 * j


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["bf16x3", "fp32"])
def test_cfg4_batch_256_sampled_frames(precision):
    """The batched workload at full size: 4096 MIRI-shaped CSR frames
    (224 x 288 px, keeping P_f ~ U{10000..64512} pixels nearest the star
    outside the cross), K = 200, 300 iterations, one persistent launch.
    256 frames drawn at random (seeded) match the oracle (Gram form, equal
    to the direct form in exact arithmetic) frame by frame."""
    k, ny, nx, iters = 200, 224, 288, 300
    g = np.random.default_rng(0)
    H = synth.components_speckle(g, k, ny, nx).astype(np.float32)
    rf = synth.make_ragged(H.astype(np.float64), ny, nx, 4096, 10000, 64512)
    say("cfg4 4096 frames", precision)
    C, ticks, _ = nmf.project_ragged(dev(H), dev_i64(rf.offsets), dev_i32(rf.pix), dev(rf.val),
                                     None, iters, seed=2, precision=precision, want_ticks=True)
    Cg = host(C)
    C0 = prng.init_matrix(2, prng.MAT_C, rf.f, k)
    sel = np.sort(np.random.default_rng(1).choice(rf.f, 256, replace=False))
    o = rf.offsets
    worst_j = worst_m = 0.0
    for i in sel:
        sub_off = np.array([0, o[i + 1] - o[i]])
        sl = slice(o[i], o[i + 1])
        T, MT = nmf64.ragged_to_dense(sub_off, rf.pix[sl], rf.val[sl], rf.wt[sl], ny * nx)
        co = nmf64.project_gram(T, MT, H, C0[i:i + 1], iters)
        Jo = nmf64.frame_objective(T, MT, H, co)[0]
        Jg = nmf64.frame_objective(T, MT, H, Cg[i:i + 1])[0]
        Th = np.where(MT > 0, T, 0.0)
        mod = co @ H
        snr = np.linalg.norm(MT * mod) / np.linalg.norm(MT * (Th - mod))
        relj = abs(Jg - Jo) / Jo
        model = rel_model_err(MT, Cg[i:i + 1] @ H, mod)
        worst_j, worst_m = max(worst_j, relj), max(worst_m, model)
        bar = max(1e-5, 2 * MODEL_ULP[precision] * snr)
        assert relj <= bar and model <= 1e-4, (i, relj, model, snr)
    print(f"  256 sampled frames: max relJ={worst_j:.3e} max model={worst_m:.3e}", flush=True)
    t = host(ticks).astype(np.int64).reshape(rf.f, 2)
    assert np.all(t[:, 0] > 0) and np.all(t[:, 1] >= t[:, 0])


@pytest.mark.parametrize("k,p,sizes,binary", [(30, 6400, [6400, 0, 3000, 31, 32, 33, 5000], True),
                                              (100, 3000, [2999, 1500, 64, 700], True),
                                              (200, 2500, [2500, 1200, 300], True),
                                              (64, 2100, [2100, 1000, 65], False),
                                              (80, 2000, [2000, 900, 81, 40], False),
                                              (100, 3000, [2999, 1500, 64, 700], False),
                                              (150, 2000, [1999, 1000, 151], True),
                                              (180, 2200, [2200, 700, 5], False),
                                              (197, 2500, [2500, 1200, 300], False)])
def test_ragged_bf16x3_parity(k, p, sizes, binary):
    """Split-precision Gram products on CSR frames, every operand-block
    grouping of the staged (H o sqrt m) array and both launch forms, 0/1 and
    inverse-variance weights: model within 1e-4, the objective within the
    bar derived from the split form's product error (frames of about K
    pixels are fitted almost exactly, so their objective is a small
    difference that a model change moves a lot)."""
    H = _basis(k, p, seed=k + 1)
    offs, pix, val, wt = _ragged(H, sizes, seed=k, binary=binary)
    f = len(sizes)
    C0 = prng.init_matrix(9, prng.MAT_C, f, k)
    say("ragged bf16x3", k, p, sizes, binary)
    C, _ = nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val),
                              None if binary else dev(wt), 100, seed=9, precision="bf16x3")
    Cg = host(C)
    Co = nmf64.project_ragged(offs, pix, val, wt, H, C0, 100)
    T, MT = nmf64.ragged_to_dense(offs, pix, val, wt, p)
    nonempty = [i for i in range(f) if sizes[i] > 0]
    _compare(T[nonempty], MT[nonempty], H, Cg[nonempty], Co[nonempty], derived=True,
             precision="bf16x3")


def test_ragged_many_frames_longest_first_order_is_a_permutation():
    """More frames than the in-LDS sort takes (9000 > 8192): the longest-first
    order comes from the radix sort; every frame is processed exactly once
    (a frame skipped or processed twice would leave or clobber its
    coefficients), so every frame matches the oracle."""
    k, p = 4, 300
    H = _basis(k, p, seed=3)
    g = np.random.default_rng(4)
    sizes = g.integers(1, p + 1, 9000)
    offs, pix, val, wt = _ragged(H, sizes, seed=5, binary=True)
    f = len(sizes)
    iters = 30
    C0 = prng.init_matrix(11, prng.MAT_C, f, k)
    say("ragged 9000 frames")
    C, ticks, _ = nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val), None, iters,
                                     seed=11, want_ticks=True)
    Cg = host(C)
    Co = nmf64.project_ragged(offs, pix, val, wt, H, C0, iters)
    scale = np.maximum(np.abs(Co).max(axis=1, keepdims=True), 1e-30)
    assert np.max(np.abs(Cg - Co) / scale) < 1e-4
    t = host(ticks).astype(np.int64).reshape(f, 2)
    assert np.all(t[:, 0] > 0) and np.all(t[:, 1] >= t[:, 0])
    # the queue handed out every frame exactly once
    v = nmf.frame_visits()
    assert v is not None and v.shape == (f,) and np.all(v == 1)


@pytest.mark.parametrize("k,f", [(60, 700), (100, 1500), (200, 300)])
def test_queue_visits_each_frame_once(k, f):
    """Dense frames (one or two-phase launch by K) and CSR frames: the
    persistent launch takes every frame from its queue exactly once, also on
    a graph replay of the same call."""
    p = 900
    H = _basis(k, p, seed=k)
    T, MT = _photon_frames(H, f, seed=k + 1)
    for rep in range(2):
        say("queue visits dense", k, f, rep)
        nmf.project(dev(H), dev(T), dev(MT), 5, seed=1, gram=True)
        v = nmf.frame_visits()
        assert v.shape == (f,) and np.all(v == 1)
    g = np.random.default_rng(k)
    sizes = g.integers(0, p + 1, f)
    offs, pix, val, wt = _ragged(H, sizes, seed=k + 2, binary=True)
    say("queue visits ragged", k, f)
    nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val), None, 5, seed=1)
    v = nmf.frame_visits()
    assert v.shape == (f,) and np.all(v == 1)


def _check_ratio(T, MT, H, C0, t, ce):
    """sqrt(d G d^T / c G c^T) of the oracle's iterate at check t (d: change
    since the check at t - ce)."""
    c = nmf64.project_gram(T, MT, H, C0, t)[0]
    cp = nmf64.project_gram(T, MT, H, C0, t - ce)[0]
    G = (H.astype(np.float64) * np.where(MT[0] > 0, MT[0], 0.0)[None, :]) @ H.T.astype(np.float64)
    d = c - cp
    return np.sqrt(max(d @ G @ d, 0.0) / (c @ G @ c))


@pytest.mark.parametrize("k,ce,tol,precision", [(20, 10, 1e-4, "fp32"), (150, 25, 3e-4, "fp32"),
                                                (60, 10, 1e-4, "bf16x3")])
def test_stop_rule_matches_oracle(k, ce, tol, precision):
    """Per-frame stop rule: each frame stops at the oracle's count or one
    check period away (the FP32 iterate and its model change differ from
    the FP64 ones in the last digits, which can move a test that sits at the
    threshold), the stop is legitimate for the oracle's iterate (its ratio
    at that check within 20% of tol, the previous check's not below tol/1.2),
    and the coefficients match the oracle's fixed-count iterate at the
    frame's own count."""
    f, p, cap = 24, 2000, 3000
    H = _basis(k, p, seed=k + 1)
    T, MT = _photon_frames(H, f, seed=k + 2)
    C0 = prng.init_matrix(7, prng.MAT_C, f, k)
    say("stop rule", k, ce, tol, precision)
    C, rep = nmf.project(dev(H), dev(T), dev(MT), cap, seed=7, gram=True, precision=precision,
                         tol=tol, check_every=ce)
    its = nmf.frame_iters()
    assert its is not None and len(its) == f
    Cg = host(C)
    _, its_o, _ = nmf64.project_gram_tol(T, MT, H, C0, cap, ce, tol)
    print(f"  iterations gpu {its.min()}..{its.max()}, oracle {its_o.min()}..{its_o.max()}, "
          f"equal {np.sum(its == its_o)}/{f}", flush=True)
    assert rep["iters_run"] == its.max()
    assert np.all(its % ce == 0) and np.all(its < cap)
    assert np.all(np.abs(its - its_o) <= ce) and np.sum(its == its_o) >= 0.75 * f
    for i in range(f):
        sl = slice(i, i + 1)
        assert _check_ratio(T[sl], MT[sl], H, C0[sl], int(its[i]), ce) <= 1.2 * tol
        if its[i] > ce:
            assert _check_ratio(T[sl], MT[sl], H, C0[sl], int(its[i]) - ce, ce) >= tol / 1.2
        Co = nmf64.project_gram(T[sl], MT[sl], H, C0[sl], int(its[i]))
        _compare(T[sl], MT[sl], H, Cg[sl], Co, derived=True, precision=precision)


def test_stop_rule_warm_start_restart_and_fallback():
    """Warm starts under the stop rule: a start worse than the cold one is
    replaced from the start; a kept start that misses the rule by the cap
    restarts cold with the same cap (iterations add up, flagged as fallen
    back, the call warns that the rule was not met); a kept start at the
    solution stops at the first check.  Against the oracle's warm rule."""
    k, p, f, cap, ce = 12, 1500, 12, 30, 5
    H = _basis(k, p, seed=21)
    T, MT = _photon_frames(H, f, seed=22)
    Cc = prng.init_matrix(3, prng.MAT_C, f, k)
    Cw = np.empty((f, k), np.float32)
    Cw[:4] = 1e3                                            # rejected
    Cw[4:8] = nmf64.project_gram(T[4:8], MT[4:8], H, Cc[4:8], 20)   # kept, misses tol by cap
    Cw[8:] = nmf64.project_gram(T[8:], MT[8:], H, Cc[8:], 30000)     # kept, at the solution
    say("stop rule warm")
    tol = 1e-6
    C, rep = nmf.project(dev(H), dev(T), dev(MT), cap, seed=3, gram=True, C_init=dev(Cw),
                         warm=True, tol=tol, check_every=ce)
    its = nmf.frame_iters()
    Co, its_o, fb_o = nmf64.project_gram_tol(T, MT, H, Cw, cap, ce, tol, C_cold=Cc)
    print(f"  gpu its {its.tolist()}\n  oracle its {its_o.tolist()} fallback {fb_o.tolist()}",
          flush=True)
    assert list(fb_o[:8]) == [1] * 4 + [2] * 4
    assert np.array_equal(its[:8], its_o[:8])
    assert nmf.warm_fallbacks() == int(np.sum(fb_o != 0))
    assert rep["status_flags"] & (1 << nmf.NMF_WARN_MAXITER)  # frames 0..7 never met it
    assert np.all(its[8:] <= 2 * ce)
    _compare(T[:8], MT[:8], H, host(C)[:8], Co[:8])


@pytest.mark.parametrize("k,precision", [(100, "bf16x3"), (30, "fp32"), (200, "bf16x3"), (170, "fp32")])
def test_autotuned_gather_depth_gives_the_same_bits(k, precision):
    """With NMF_F_AUTOTUNE the gather depth of the persistent launch is timed
    on the call's own inputs and cached per shape; it changes no arithmetic,
    so dense and CSR results equal the default launch's bit for bit (first
    call: tuning runs, second call: cached choice)."""
    p, f = 1500, 40
    H = _basis(k, p, seed=k)
    T, MT = _photon_frames(H, f, seed=k + 1)
    g = np.random.default_rng(k)
    offs, pix, val, wt = _ragged(H, g.integers(0, p + 1, f), seed=k + 2, binary=False)
    h = nmf.Handle(0)
    say("autotune gram dense", k, precision)
    Cd, _ = nmf.project(dev(H), dev(T), dev(MT), 40, seed=3, gram=True, precision=precision)
    Cr, _ = nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val), dev(wt), 40, seed=3,
                               precision=precision)
    for rep in range(2):
        say("autotune gram", k, precision, rep)
        Ct, _ = nmf.project(dev(H), dev(T), dev(MT), 40, seed=3, gram=True, precision=precision,
                            flags=nmf.F_AUTOTUNE, handle=h)
        assert np.array_equal(host(Ct), host(Cd))
        Ct, _ = nmf.project_ragged(dev(H), dev_i64(offs), dev_i32(pix), dev(val), dev(wt), 40,
                                   seed=3, precision=precision, flags=nmf.F_AUTOTUNE, handle=h)
        assert np.array_equal(host(Ct), host(Cr))
    report = nmf.autotune_report(h)
    print(report, flush=True)
    lines = [l for l in report.splitlines() if l.startswith("gram.")]
    assert len(lines) == 2 and all("pipeline=1" in l or "pipeline=2" in l for l in lines)
    h.close()
