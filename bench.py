#!/usr/bin/env python3
"""Benchmark of the weighted multiplicative-update NMF hot path on one MI355X.

Headline workload (MIRI-shaped precision study, synthetic): a reference
library of N = 2000 images of 224 x 288 px (P = 64512) with a 4QPM-like cross
mask and 2% bad pixels per image, binary weights stored as bitmasks; a
K = 100 basis is built with 500 iterations of Eq. 3 in split-precision
(bf16x3) products, then the library's science frames are projected onto it
(masked-Gram form, one persistent launch, 500 iterations) and the model PSF
is subtracted.  One step = all of that; ``value`` = basis iterations per
second of the whole step (500 / step time), timed on the production path
(iterations replayed from captured hipGraphs, no per-launch timing).

The same JSON line carries:
  * ``precision_forms``: the step in both precision forms (FP32 and bf16x3),
    each with its kernel times and a roofline for its dominant kernel;
  * ``roofline``: the dominant kernel of the headline form; its duration is
    the average over the launches of a separate instrumented step (HIP events
    around every launch on the library's stream, which also turns graph
    replay off), and ``traffic`` comes from stored hardware counters when
    they were taken on the current kernel source;
  * ``batched``: 4096 CSR frames with P_f ~ U{10000..64512} valid pixels
    projected onto a K = 200 basis (built by the library from the same
    library) for 300 iterations each in one persistent launch: frames/s and
    per-frame p50/p99 latency from device timestamps;
  * ``to_tolerance``: projected frames/s to the 1e-4 model tolerance.  STIS-
    shaped frames (200 x 200 px) are modelled on a seeded K = 100 basis; a
    frame meets the tolerance when ||m o (c H - w* H)|| <= 1e-4 ||m o w* H||
    with w* its exact weighted NNLS solution, stored by the oracle for the
    first 256 frames (tests/golden/oracle_nnls_proj_k100.npz).  Plain FP32
    multiplicative updates (direct form, cold start) run until at least 99%
    of the sample meets it; the batched masked-Gram launch runs cold and
    warm-started (network trained here on frames the method projected)
    with a per-frame stop rule whose threshold is the loosest that brings
    99% of the sample within the tolerance;
  * ``cpu_baseline``: the FP64 oracle, untuned, on this host's cores, on a
    bounded sample of basis iterations of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NMF iterations/s and GEMM TFLOP/s (% MFMA roofline); projected frames/s to 1e-4 residual"
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
PEAKS = {"fp32": PEAK_FP32_TFLOPS, "bf16x3": PEAK_BF16_TFLOPS / 3.0}

K_HRULE, K_WRULE, K_WFINISH, K_OBJ, K_PROJECT, K_SUBTRACT, K_OTHER = range(7)
K_NAMES = ["hrule", "wrule", "wfinish", "objective", "project", "subtract", "other"]

WORKLOADS = {
    "miri": dict(make="make_cfg3", k=100, iters=500, frames=8, proj_iters=500, binary=True,
                 shape=[224, 288],
                 name="MIRI-shaped basis build (2000 images of 224x288 px, K=100, 500 iterations, "
                      "binary weights as bitmasks) + projection and subtraction of 8 frames"),
    "stis": dict(make="make_cfg2", k=30, iters=1000, frames=50, proj_iters=1000, binary=False,
                 shape=[200, 200],
                 name="STIS-shaped basis build (500 images of 200x200 px, K=30, 1000 iterations, "
                      "weights mask/(V+0.01)) + projection and subtraction of 50 frames"),
}
# hardware counters stored for the dominant kernel (see profiles/)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_wide_miri_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2309_04623_amd", "csrc", "k_wide.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(lib, k, seconds):
    """The FP64 oracle, untuned, on this host's cores: basis iterations of the
    same workload until ``seconds`` have elapsed (at least one)."""
    from oracle import nmf64, prng
    try:
        from threadpoolctl import threadpool_info
        cores = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        cores = os.cpu_count() or 1
    n, p = lib.V.shape
    Vh, Mw, _ = nmf64.prep(lib.V, lib.M)
    W = prng.init_matrix(1, prng.MAT_W, n, k)
    H = prng.init_matrix(1, prng.MAT_H, k, p)
    t0 = time.perf_counter()
    it = 0
    while True:
        H = nmf64.update_H(Vh, Mw, W, H)
        W = nmf64.update_W(Vh, Mw, W, H)
        it += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": it / el, "unit": "iterations/s", "cores": int(cores), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{it} FP64 basis iterations (Eq. 3, H then W) of the same N={n} P={p} "
                      f"K={k} library from the seeded start ({el:.1f} s)"}


def stored_traffic():
    """HBM bytes per launch from stored counters, if they were taken on the
    current source of the dominant kernel."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="miri", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3"])
    ap.add_argument("--iters", type=int, default=None, help="basis iterations per step")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-frame batched leg")
    ap.add_argument("--batched-frames", type=int, default=4096)
    ap.add_argument("--no-tolerance", action="store_true",
                    help="skip the projection-to-tolerance leg")
    ap.add_argument("--train-frames", type=int, default=4096,
                    help="frames the warm-start network is trained on")
    ap.add_argument("--single-precision", action="store_true",
                    help="time only --precision (by default both precision forms are timed)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain elementwise copy of MIB MiB (reads and writes "
                         "MIB MiB), the reference dispatch for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (pixels of "
              "the basis build and frames of the projection would shard across GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_04623_amd import nmf, synth

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    nmf.lib()  # fails loudly if the HIP library was not built

    W_ = WORKLOADS[args.workload]
    K = W_["k"]
    iters = args.iters or W_["iters"]
    flags = nmf.F_BINARY_WEIGHTS if W_["binary"] else 0
    log(f"generating the {args.workload} workload ...")
    lib = getattr(synth, W_["make"])(frames=W_["frames"])
    n, p = lib.V.shape
    f = lib.T.shape[0]
    dev = torch.device("cuda:0")
    V = torch.from_numpy(lib.V).to(dev)
    M = torch.from_numpy(lib.M).to(dev)
    T = torch.from_numpy(lib.T).to(dev)
    MT = torch.from_numpy(lib.MT).to(dev)
    h = nmf.Handle(0)
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(nel, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log(f"calibration copy of {args.copy_calibration} MiB done")

    def step(prec):
        W, H, J, rep = nmf.build_basis(V, M, K, iters, precision=prec, seed=1, flags=flags,
                                       handle=h)
        C, _ = nmf.project(H, T, MT, W_["proj_iters"], seed=2, gram=True, flags=flags,
                           precision=prec, handle=h)
        model, resid = nmf.subtract(H, C, T, MT, handle=h)
        return J, rep

    def measure(prec):
        """Warm-up, then exactly ``steps`` timed steps bracketed by device
        synchronisation (graph replay, no per-launch timing); then one
        instrumented step for per-kernel device times."""
        for i in range(args.warmup):
            log(f"[{prec}] warmup step {i + 1}/{args.warmup}")
            step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            J, rep = step(prec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        log(f"[{prec}] timed {args.steps} steps: {el:.3f} s; final J {J[-1]:.6e} "
            f"rel {rep['objective_rel']:.3e}")
        nmf.profile_enable(h, True)
        step(prec)
        torch.cuda.synchronize()
        prof = {K_NAMES[c]: nmf.profile_get(h, c) for c in range(7)}
        nmf.profile_enable(h, False)
        return el, prof, J

    def summarize(prec, el, prof, J):
        flops = 6.0 * n * K * p  # per half-step launch: Y, num, den (N x K x P each)
        # algorithmic HBM bytes per launch: the data once (4 B/px) and the
        # weights (1/8 B/px as bitmask, 4 B/px as FP32), plus the factors
        wbytes = 0.125 if W_["binary"] else 4.0
        bytes_ = (4.0 + wbytes) * n * p + 4.0 * 3 * K * (n + p)
        dom = max(("hrule", "wrule"), key=lambda c: prof[c][1])
        cnt, tot = prof[dom]
        avg_s = tot * 1e-3 / cnt
        peak = PEAKS[prec]
        t_mfma = flops / (peak * 1e12)
        t_hbm = bytes_ / (PEAK_HBM_GBS * 1e9)
        if t_mfma >= t_hbm:
            roof = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": peak,
                    "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": bytes_ / avg_s / 1e9, "peak": PEAK_HBM_GBS,
                    "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = None
        roof["kernel"] = (f"k_wide ({dom} half-step, {prec}), avg {avg_s * 1e6:.2f} us over "
                          f"{cnt} launches of the instrumented step")
        roof["algorithmic_flops_per_launch"] = flops
        roof["algorithmic_bytes_per_launch"] = bytes_
        roof["hbm_GBs_algorithmic"] = bytes_ / avg_s / 1e9
        roof["mfma_TFLOPs_algorithmic"] = flops / avg_s / 1e12
        if prec == "bf16x3":
            roof["peak_note"] = "dense bf16 2500 TFLOP/s / 3 products per split-precision product"
        gemm_ms = prof["hrule"][1] + prof["wrule"][1]
        basis_ms = sum(prof[c][1] for c in ("hrule", "wrule", "wfinish", "objective"))
        return {
            "iterations_per_s": iters * args.steps / el,
            "ms_per_step": el * 1e3 / args.steps,
            "gemm_tflops": 12.0 * n * K * p * iters / (gemm_ms * 1e-3) / 1e12,
            "basis_iters_per_s_device": iters / (basis_ms * 1e-3),
            "final_objective": float(J[-1]),
            "kernel_ms_per_step": {c: prof[c][1] for c in K_NAMES},
            "kernel_launches_per_step": {c: prof[c][0] for c in K_NAMES},
            "roofline": roof,
        }

    forms = {}
    order = [args.precision] + ([] if args.single_precision else
                                [q for q in ("fp32", "bf16x3") if q != args.precision])
    for prec in order:
        forms[prec] = summarize(prec, *measure(prec))
    main_sum = forms[args.precision]
    traffic = stored_traffic()
    if traffic and traffic.get("precision") == args.precision:
        main_sum["roofline"]["traffic"] = traffic["hbm_bytes_per_launch"]
        main_sum["roofline"]["traffic_source"] = traffic.get("source")

    batched = None
    if not args.no_batched and args.workload == "miri":
        batched = batched_leg(args, nmf, synth, lib, V, M, h, torch)

    tolerance = None
    if not args.no_tolerance:
        tolerance = tolerance_leg(args, nmf, synth, h, torch)

    out = {
        "metric": METRIC,
        "value": main_sum["iterations_per_s"],
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_sum["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if args.precision == "bf16x3" else "f32",
        "data": "synthetic",
        "config": {"workload": W_["name"], "images": n, "pixels": p,
                   "image_shape": W_["shape"], "k": K, "basis_iters": iters, "frames": f,
                   "proj_iters": W_["proj_iters"], "weights": "binary bitmask" if W_["binary"]
                   else "FP32", "projection": "masked-Gram", "precision": args.precision},
    }
    for key in ("gemm_tflops", "basis_iters_per_s_device", "kernel_ms_per_step",
                "kernel_launches_per_step", "roofline"):
        out[key] = main_sum[key]
    out["precision_forms"] = {q: {k: v for k, v in s.items() if k != "kernel_launches_per_step"}
                              for q, s in forms.items()}
    if batched:
        out["batched"] = batched
    if tolerance:
        out["to_tolerance"] = tolerance
    if not args.no_cpu_baseline:
        log(f"timing the FP64 oracle on host cores for ~{args.cpu_seconds:.0f} s ...")
        out["cpu_baseline"] = cpu_baseline(lib, K, args.cpu_seconds)
    h.close()
    print(json.dumps(out), flush=True)


def batched_leg(args, nmf, synth, lib, V, M, h, torch):
    """4096 ragged frames (P_f ~ U{10000..64512} valid pixels near the star,
    outside the cross) projected onto a K = 200 basis, 300 iterations each,
    in one persistent launch."""
    K2, ITERS = 200, 300
    log("building the K = 200 basis for the batched leg ...")
    _, Hb, _, _ = nmf.build_basis(V, M, K2, 30, precision="bf16x3", seed=3,
                                  flags=nmf.F_BINARY_WEIGHTS, handle=h)
    log(f"generating {args.batched_frames} ragged frames ...")
    rag = synth.make_ragged(lib.H0, 224, 288, args.batched_frames, 10000, 64512)
    dev = V.device
    off = torch.from_numpy(rag.offsets).to(dev)
    pix = torch.from_numpy(rag.pix).to(dev)
    val = torch.from_numpy(rag.val).to(dev)
    kw = dict(seed=4, flags=nmf.F_BINARY_WEIGHTS, want_ticks=True, handle=h, precision="bf16x3")
    nmf.project_ragged(Hb, off, pix, val, None, ITERS, **kw)  # warm-up (captures the graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C, ticks, _ = nmf.project_ragged(Hb, off, pix, val, None, ITERS, **kw)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    tk = ticks.cpu().numpy().reshape(-1, 2)
    khz = nmf.device_clock_khz(h)
    lat_us = (tk[:, 1] - tk[:, 0]) / khz * 1e3
    F = rag.f
    nnz = int(rag.offsets[-1])
    sizes = np.diff(rag.offsets)
    flops = float(np.sum(2.0 * K2 * K2 * sizes + 2.0 * K2 * sizes) + F * ITERS * 2.0 * K2 * K2)
    log(f"batched: {F} frames in {el * 1e3:.2f} ms")
    return {"frames": F, "k": K2, "iters": ITERS, "nnz": nnz,
            "pixels_per_frame": [int(sizes.min()), int(sizes.max())],
            "form": "masked-Gram, CSR frames, one persistent launch (hipGraph), bf16x3 Gram "
                    "products, FP32 storage",
            "ms_per_batch": el * 1e3, "frames_per_s": F / el,
            "latency_us_p50": float(np.percentile(lat_us, 50)),
            "latency_us_p99": float(np.percentile(lat_us, 99)),
            "algorithmic_tflops": flops / el / 1e12,
            "mfma_roofline_frac": flops / el / 1e12 / (2500.0 / 3),
            "roofline_note": "flops counted as the full Gram products 2 K^2 P_f (+ b and the "
                             "iterations) against the bf16x3 peak (dense bf16 2500 TFLOP/s / 3); "
                             "the kernel forms the 32-blocked upper triangle of G only"}


def tolerance_leg(args, nmf, synth, h, torch):
    """Frames/s to the 1e-4 model tolerance: plain FP32 direct-form updates
    against the batched masked-Gram launch, cold and warm-started."""
    TOL = 1e-4
    path = os.path.join(ROOT, "tests", "golden", "oracle_nnls_proj_k100.npz")
    fx = np.load(path)
    n_s, F = int(fx["n_sample"]), int(fx["n_frames"])
    log(f"generating {F} STIS-shaped frames on the K = 100 basis ...")
    ps = synth.make_projection_set(F)
    sha = lambda x: hashlib.sha256(np.ascontiguousarray(x, np.float32).tobytes()).hexdigest()
    if (sha(ps.H) != str(fx["h_sha"]) or sha(ps.T[:n_s]) != str(fx["t_sha"])
            or sha(ps.MT[:n_s]) != str(fx["m_sha"])):
        raise RuntimeError("the generator no longer draws the frames the stored solutions are for")
    K, P = ps.H.shape
    dev = torch.device("cuda:0")
    Hd = torch.from_numpy(ps.H).to(dev)
    Td = torch.from_numpy(ps.T).to(dev)
    Md = torch.from_numpy(ps.MT).to(dev)
    H64 = ps.H.astype(np.float64)
    Ms = ps.MT[:n_s].astype(np.float64)
    ref = fx["w_star"] @ H64
    refn = np.linalg.norm(Ms * ref, axis=1)

    def errors(C):
        Cn = C[:n_s].detach().cpu().double().numpy()
        return np.linalg.norm(Ms * (Cn @ H64 - ref), axis=1) / refn

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # plain FP32: direct-form updates from the cold start, in chunks (the
    # iteration is memoryless, so the chunks continue one run); the sample is
    # checked between chunks, outside the timed calls
    CHUNK, CAP = 10000, 400000
    Tp, Mp = Td[:n_s], Md[:n_s]
    C, el, it, met = None, 0.0, 0, 0.0
    while it < CAP:
        (C, _), dt = timed(lambda: nmf.project(Hd, Tp, Mp, CHUNK, C_init=C, seed=7, handle=h))
        el += dt
        it += CHUNK
        err = errors(C)
        met = float(np.mean(err <= TOL))
        log(f"plain FP32: {it} iterations, {el:.2f} s, met {met:.3f}, median error "
            f"{np.median(err):.2e}")
        if met >= 0.99:
            break
    plain = {"form": "plain multiplicative updates (direct form, Eq. 3 W-rule per frame), FP32, "
                     "cold start, fixed count", "frames": n_s, "iterations": it,
             "met_fraction": met, "seconds": el, "frames_per_s": n_s / el,
             "median_error": float(np.median(err)), "max_error": float(err.max())}

    CE, ITERS = 500, 400000
    TAUS = (1e-5, 5e-6, 2e-6, 1e-6, 7e-7, 5e-7, 3.5e-7, 2.5e-7, 2e-7, 1.5e-7, 1e-7, 7e-8,
            5e-8, 3e-8, 2e-8, 1e-8)

    def gram_run(tau, C0=None, pre=None):
        def go():
            c0 = C0
            if pre is not None:
                c0 = pre()
            return nmf.project(Hd, Td, Md, ITERS, gram=True, precision="bf16x3", seed=7,
                               C_init=c0, warm=c0 is not None, tol=tau, check_every=CE, handle=h)
        (C, rep), dt = timed(go)
        its = nmf.frame_iters(h)
        err = errors(C)
        return {"tol": tau, "check_every": CE, "cap": ITERS, "frames": F,
                "met_fraction": float(np.mean(err <= TOL)), "seconds": dt, "frames_per_s": F / dt,
                "iterations_mean": float(its.mean()), "iterations_p50": float(np.median(its)),
                "iterations_p99": float(np.percentile(its, 99)),
                "median_error": float(np.median(err)), "max_error": float(err.max()),
                "fallbacks": int(nmf.warm_fallbacks(h)) if C0 is not None or pre else 0}

    def scan(label, **kw):
        r = None
        for tau in TAUS:
            r = gram_run(tau, **kw)
            log(f"{label}: tol {tau:.1e}: met {r['met_fraction']:.3f}, {r['seconds']:.3f} s, "
                f"mean iterations {r['iterations_mean']:.0f}")
            if r["met_fraction"] >= 0.99:
                break
        return r

    nmf.project(Hd, Td, Md, 10, gram=True, precision="bf16x3", seed=7, tol=1e-5, check_every=5,
                handle=h)  # warm-up
    cold = scan("batched cold")
    cold["form"] = ("masked-Gram, one persistent launch, bf16x3 Gram products, cold start, "
                    "per-frame stop rule (model change over check_every iterations)")

    # warm start: the method projects a training set to stationarity, the
    # network is trained on those pairs by the library's kernels
    log(f"warm start: {args.train_frames} training frames ...")
    tr = synth.make_projection_set(args.train_frames, sub=1)
    Ttr, Mtr = torch.from_numpy(tr.T).to(dev), torch.from_numpy(tr.MT).to(dev)
    (Ctr, _), t_tgt = timed(lambda: nmf.project(Hd, Ttr, Mtr, ITERS, gram=True, precision="fp32",
                                                seed=9, tol=1e-8, check_every=CE, handle=h))
    Xtr, str_ = nmf.ws_pool(Ttr, Mtr, ps.ny, ps.nx, handle=h)
    # training metric G = I: the loss measures coefficient error.  With the
    # model-space metric (G = H H^T) the network reaches a 2% model error on
    # these strongly correlated components but leaves ~30% of each frame's
    # support coefficients near zero, which multiplicative updates are slow
    # to grow back
    Gm = torch.eye(K, dtype=torch.float32, device=dev)
    st = nmf.ws_init(K, seed=11, handle=h)
    EPOCHS = 40
    hist, t_train = timed(lambda: nmf.ws_train(st, Xtr, str_, Ctr, Gm, K, epochs=EPOCHS, batch=64,
                                               lr=1e-3, seed=12, handle=h))
    del Ttr, Mtr, Xtr, tr
    log(f"warm start: targets {t_tgt:.1f} s, training {t_train:.1f} s, loss {hist[0]:.3e} -> "
        f"{hist[-1]:.3e}")

    def infer():
        X, s = nmf.ws_pool(Td, Md, ps.ny, ps.nx, handle=h)
        return nmf.ws_infer(st, X, s, K, handle=h)

    C0 = infer()
    warm_err0 = errors(C0)
    c0 = C0[:n_s].detach().cpu().double().numpy()
    sup = fx["w_star"] > 1e-2 * fx["w_star"].mean(axis=1, keepdims=True)
    ratio = c0[sup] / fx["w_star"][sup]
    warm = scan("batched warm", pre=infer)
    warm["form"] = ("masked-Gram, one persistent launch, bf16x3 Gram products, warm start from "
                    "the network (pooling and inference inside the timed region), per-frame "
                    "stop rule, cold restart of a frame that misses it by the cap")
    warm["network_start_median_error"] = float(np.median(warm_err0))
    warm["network_start_coefficients"] = {
        "median_relative_error_on_support": float(np.median(np.abs(ratio - 1.0))),
        "fraction_of_support_below_a_tenth": float(np.mean(ratio < 0.1))}
    warm["training"] = {"frames": args.train_frames, "targets": "the library's masked-Gram "
                        "projection to tol 1e-8", "loss": "relative coefficient error (metric G = I)",
                        "epochs": EPOCHS, "batch": 64, "lr": 1e-3,
                        "loss_first_last": [float(hist[0]), float(hist[-1])],
                        "seconds_targets": t_tgt, "seconds_training": t_train}
    return {
        "workload": f"{F} STIS-shaped frames (200x200 px, 12 px wedge, 1% bad pixels, weights "
                    "mask/(T+0.01), ring disks at 1e-3 on half) modelled on a seeded K=100 basis",
        "tolerance": TOL,
        "criterion": f"||m o (c H - w* H)|| / ||m o w* H|| <= {TOL} against the exact FP64 "
                     f"weighted NNLS solution w* (stored oracle solutions, first {n_s} frames)",
        "plain_fp32": plain, "batched_cold": cold, "batched_warm": warm,
        "speedup_batched_cold_vs_plain": cold["frames_per_s"] / plain["frames_per_s"],
        "speedup_batched_warm_vs_plain": warm["frames_per_s"] / plain["frames_per_s"],
        "speedup_warm_vs_cold": warm["frames_per_s"] / cold["frames_per_s"],
    }


if __name__ == "__main__":
    main()
