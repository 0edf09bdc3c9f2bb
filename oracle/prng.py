"""Counter-based SplitMix64 uniform generator (oracle side).

The paper only says W and H start from random values (Sec. 2, the text after
Eq. 3).  This build fixes that reading: every initial element is U(0,1) on the
open interval, drawn from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter mode:

    mix(z)    = SplitMix64 output finaliser of the 64-bit word z
    out(s, i) = mix(s + (i + 1) * GAMMA)            (the i-th output of a
                                                     generator seeded with s)
    key       = out(seed, matrix_id)                (one stream per matrix)
    u64       = out(key, element_index)
    value     = ((u64 >> 41) + 0.5) * 2^-23         (exact in float32 and in
                                                     float64, inside (0, 1))

Written independently of the GPU generator; the two must agree bitwise.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1

MAT_W, MAT_H, MAT_C = 0, 1, 2


def mix_int(z: int) -> int:
    """SplitMix64 finaliser on a Python int (reference scalar form)."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * MUL1) & _MASK
    z = ((z ^ (z >> 27)) * MUL2) & _MASK
    return z ^ (z >> 31)


def splitmix64_outputs(seed: int, count: int) -> list[int]:
    """The first ``count`` outputs of SplitMix64 seeded with ``seed``."""
    return [mix_int(seed + (i + 1) * GAMMA) for i in range(count)]


def _mix_vec(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(MUL1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(MUL2)
    z ^= z >> np.uint64(31)
    return z


def uniform(seed: int, matrix_id: int, count: int) -> np.ndarray:
    """``count`` open-interval U(0,1) values (float64, each exactly a float32)."""
    key = mix_int(seed + (matrix_id + 1) * GAMMA)
    idx = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + idx * np.uint64(GAMMA)
        u = _mix_vec(z)
    top = (u >> np.uint64(41)).astype(np.float64)
    return (top + 0.5) * 2.0 ** -23


def init_matrix(seed: int, matrix_id: int, rows: int, cols: int) -> np.ndarray:
    """Row-major ``rows x cols`` init matrix, element index = r * cols + c."""
    return uniform(seed, matrix_id, rows * cols).reshape(rows, cols)
