"""Shared helpers for the GPU parity tests (test-side only)."""
import sys

import numpy as np


def say(*msg):
    """Name the case before a GPU step, flushed, so a lost run still shows it."""
    print("[case]", *msg, flush=True)
    sys.stdout.flush()


def dev(x, device="cuda:0"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).to(device)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def objective64(V, M, W, H):
    """Eq. 2 cost of a (W, H) pair in FP64 (used to score GPU factors)."""
    V = np.asarray(V, np.float64)
    M = np.asarray(M, np.float64)
    Vh = np.where(M > 0, V, 0.0)
    R = Vh - np.asarray(W, np.float64) @ np.asarray(H, np.float64)
    return float(np.sum(M * R * R))


def rel_model_err(M, A, B):
    """||M o (A - B)||_2 / ||M o B||_2 for two model images A, B."""
    M = np.asarray(M, np.float64)
    return float(np.linalg.norm(M * (A - B)) / np.linalg.norm(M * B))


def random_problem(seed, n, p, k, mask_frac=0.1, binary=False):
    g = np.random.default_rng(seed)
    W0 = g.gamma(2.0, 1.0, (n, k + 2))
    H0 = g.gamma(1.0, 1.0, (k + 2, p))
    V = W0 @ H0 + np.abs(g.normal(0, 0.05, (n, p)))
    keep = g.random((n, p)) >= mask_frac
    M = keep.astype(np.float64) if binary else keep / (V + 0.01)
    return V.astype(np.float32), M.astype(np.float32)
