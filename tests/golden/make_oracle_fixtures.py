#!/usr/bin/env python3
"""Write the FP64 oracle's expected values for the full-size basis-build
parity tests (tests/test_gpu_fullsize.py).

Calls only ``oracle/`` (and the input generators of
``paper_2309_04623_amd.synth``, which hold none of the method's arithmetic).
The full-size libraries are too large for the oracle to run inside a GPU
test, so it runs here once and the expected values are stored:

* ``J``        : the Eq. 2 objective before every iteration and after the last
                 one (T + 1 values, FP64), from the seeded init of the library's
                 counter-based generator (W: matrix 0, H: matrix 1);
* ``ck_iters`` : checkpoint iteration counts;
* ``W_ck``     : the oracle's W rows ``rows`` at each checkpoint (float32);
* ``H_ck``     : the oracle's H columns ``cols`` at each checkpoint (float32),
                 so that the model W H is known on the rows x cols block;
* ``v_sha``, ``m_sha`` : SHA-256 of the float32 inputs, so a test can tell
                 that it generated the same library.

For the projection-to-tolerance measurement it stores the exact weighted
NNLS coefficients (``oracle.nnls``) of a sample of frames:

* ``w_star``   : the NNLS minimiser of the first ``n_sample`` frames of the
                 1024-frame projection set (K = 100, FP64, from the normal
                 equations by a Cholesky-reduced active-set solve);
* ``kkt``      : each solution's KKT residual (a check that it is optimal);
* ``h_sha``, ``t_sha``, ``m_sha`` : SHA-256 of the float32 basis and of the
                 sample's frames and weights.

Usage:  python tests/golden/make_oracle_fixtures.py {stis|miri|proj} [out.npz]
  stis: 500 images of 200 x 200 px, K = 30, 1000 iterations, weights
        mask / (V + 0.01) (seed 1)
  miri: 2000 images of 224 x 288 px, K = 100, 500 iterations, binary
        weights (seed 1)
  proj: the first 256 of 1024 STIS-shaped frames on the seeded K = 100 basis
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import nmf64, nnls, prng  # noqa: E402
from paper_2309_04623_amd import synth  # noqa: E402

CASES = {
    "stis": dict(make=lambda: synth.make_cfg2(frames=1), k=30, iters=1000, ck=(100, 500, 1000),
                 seed=1),
    "miri": dict(make=lambda: synth.make_cfg3(frames=1), k=100, iters=500, ck=(100, 250, 500),
                 seed=1),
}
N_ROWS, N_COLS = 96, 1536


def sha(x: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(x, np.float32).tobytes()).hexdigest()


PROJ_FRAMES, PROJ_SAMPLE = 1024, 256


def main_proj(out):
    ps = synth.make_projection_set(PROJ_FRAMES)
    H = ps.H.astype(np.float64)
    W, kkt = [], []
    t0 = time.time()
    for f in range(PROJ_SAMPLE):
        G, b, _ = nnls.normal_equations(H, ps.T[f], ps.MT[f])
        w = nnls.nnls_gram(G, b)
        W.append(w)
        kkt.append(nnls.kkt_residual(G, b, w))
        if f % 32 == 31:
            print(f"proj: {f + 1}/{PROJ_SAMPLE} frames, max KKT residual {max(kkt):.1e} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(out, w_star=np.array(W), kkt=np.array(kkt), n_sample=PROJ_SAMPLE,
                        n_frames=PROJ_FRAMES, h_sha=sha(ps.H), t_sha=sha(ps.T[:PROJ_SAMPLE]),
                        m_sha=sha(ps.MT[:PROJ_SAMPLE]))
    print(f"wrote {out}", flush=True)


def main():
    name = sys.argv[1]
    if name == "proj":
        main_proj(sys.argv[2] if len(sys.argv) > 2 else os.path.join(
            os.path.dirname(os.path.abspath(__file__)), "oracle_nnls_proj_k100.npz"))
        return
    out = sys.argv[2] if len(sys.argv) > 2 else os.path.join(
        os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}_fullsize.npz")
    c = CASES[name]
    lib = c["make"]()
    n, p = lib.V.shape
    k, T = c["k"], c["iters"]
    g = np.random.default_rng(20230904)
    rows = np.sort(g.choice(n, N_ROWS, replace=False))
    cols = np.sort(g.choice(p, N_COLS, replace=False))
    W = prng.init_matrix(c["seed"], prng.MAT_W, n, k)
    H = prng.init_matrix(c["seed"], prng.MAT_H, k, p)
    J = []
    W_ck, H_ck = [], []
    t = 0
    t0 = time.time()
    for ck in c["ck"]:
        # the iteration is memoryless, so chunks continue it exactly
        W, H, Jc = nmf64.build_basis(lib.V, lib.M, W, H, ck - t)
        J.extend(Jc[:-1])
        t = ck
        W_ck.append(W[rows].astype(np.float32))
        H_ck.append(H[:, cols].astype(np.float32))
        print(f"{name}: {t}/{T} iterations, J = {Jc[-1]:.10e} ({time.time() - t0:.0f} s)",
              flush=True)
    J.append(Jc[-1])
    assert t == T and len(J) == T + 1
    np.savez_compressed(out, J=np.array(J), ck_iters=np.array(c["ck"]), rows=rows, cols=cols,
                        W_ck=np.stack(W_ck), H_ck=np.stack(H_ck), k=k, iters=T, seed=c["seed"],
                        v_sha=sha(lib.V), m_sha=sha(lib.M))
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
