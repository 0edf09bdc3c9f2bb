"""Seeded synthetic coronagraphy workloads.

This module only draws inputs: reference libraries V, weights M, science
frames T and their weights M_T, with the shapes and structure of the STIS-
and MIRI-like workloads (a centrally peaked stellar PSF with speckle
structure, an occulter mask, bad pixels, Poisson-like noise and a faint
circumstellar disk).  It contains none of the factorisation arithmetic, so
the FP64 oracle and the GPU library can both be fed from it without sharing
any of the method's code.

The paper's own data (HST-STIS WedgeA1.0 and JWST-MIRI 4QPM frames, Sec. 3)
are archival; seeded synthetic frames of the same kind stand in for them.

Every generator is driven by ``numpy.random.Generator(PCG64(SeedSequence(
[ROOT_SEED, cfg, stream])))`` with streams 0 = library, 1 = masks,
2 = noise, 3 = init, 4 = science frames, 5 = disks.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOT_SEED = 230904623
S_LIBRARY, S_MASK, S_NOISE, S_INIT, S_SCIENCE, S_DISK = range(6)


def rng(cfg: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, cfg, stream, sub])))


def radius_grid(ny: int, nx: int):
    """Distance of each pixel from the frame centre ((ny-1)/2, (nx-1)/2)."""
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    cy, cx = (ny - 1) / 2.0, (nx - 1) / 2.0
    return yy - cy, xx - cx, np.hypot(yy - cy, xx - cx)


# --------------------------------------------------------------------------
# PSF components
# --------------------------------------------------------------------------

def components_radial_gamma(g: np.random.Generator, k0: int, ny: int, nx: int) -> np.ndarray:
    """Gamma(1,1) pixel fields under a 1/r^2 envelope (capped at r < 1)."""
    _, _, r = radius_grid(ny, nx)
    env = 1.0 / np.maximum(r * r, 1.0)
    return g.gamma(1.0, 1.0, size=(k0, ny * nx)) * env.reshape(1, -1)


def _gauss_smooth(img: np.ndarray, sigma: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(img, sigma, mode="reflect")


def components_speckle(g: np.random.Generator, k0: int, ny: int, nx: int,
                       core: float = 3.0, smooth: float = 1.5) -> np.ndarray:
    """Speckle fields (Gamma(1,1) noise smoothed to ~2 px speckles) under a
    Moffat-like stellar halo e(r) = (1 + (r/core)^2)^-1.5."""
    _, _, r = radius_grid(ny, nx)
    env = (1.0 + (r / core) ** 2) ** -1.5
    out = np.empty((k0, ny * nx))
    for k in range(k0):
        s = _gauss_smooth(g.gamma(1.0, 1.0, size=(ny, nx)), smooth)
        out[k] = (env * s).reshape(-1)
    return out


# --------------------------------------------------------------------------
# Masks (1 = use, 0 = masked / missing)
# --------------------------------------------------------------------------

def mask_disc(ny: int, nx: int, radius: float) -> np.ndarray:
    _, _, r = radius_grid(ny, nx)
    return (r > radius).reshape(-1)


def mask_wedge(ny: int, nx: int, half_width: float) -> np.ndarray:
    """Diagonal occulting wedge: pixels within ``half_width`` of the 45-degree
    line through the centre are masked (a 2*half_width wide bar)."""
    dy, dx, _ = radius_grid(ny, nx)
    dist = np.abs(dy - dx) / math.sqrt(2.0)
    return (dist > half_width).reshape(-1)


def mask_cross(ny: int, nx: int, disc: float, arm_half: float) -> np.ndarray:
    """4QPM-like mask: a central disc plus horizontal and vertical arms."""
    dy, dx, r = radius_grid(ny, nx)
    bad = (r <= disc) | (np.abs(dx) <= arm_half) | (np.abs(dy) <= arm_half)
    return (~bad).reshape(-1)


def bad_pixels(g: np.random.Generator, rows: int, p: int, frac: float) -> np.ndarray:
    return g.random((rows, p)) >= frac


# --------------------------------------------------------------------------
# Disk model
# --------------------------------------------------------------------------

def disk_ring(ny: int, nx: int, a: float, sigma: float, inc_deg: float, pa_deg: float) -> np.ndarray:
    """Unit-flux inclined Gaussian ring of semi-major axis ``a`` pixels."""
    dy, dx, _ = radius_grid(ny, nx)
    pa = math.radians(pa_deg)
    u = dx * math.cos(pa) + dy * math.sin(pa)
    v = -dx * math.sin(pa) + dy * math.cos(pa)
    v = v / max(math.cos(math.radians(inc_deg)), 1e-3)
    img = np.exp(-0.5 * ((np.hypot(u, v) - a) / sigma) ** 2)
    return (img / img.sum()).reshape(-1)


# --------------------------------------------------------------------------
# Workload containers
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Library:
    """A reference library and its science frames, all float32, row-major
    with the pixel index fastest."""
    name: str
    ny: int
    nx: int
    V: np.ndarray          # N x P data
    M: np.ndarray          # N x P weights (0 = missing)
    T: np.ndarray          # F x P science frames
    MT: np.ndarray         # F x P science weights
    W0: np.ndarray         # planted coefficients (float64, for reference only)
    H0: np.ndarray         # planted components (float64)
    binary: bool = False

    @property
    def n(self):
        return self.V.shape[0]

    @property
    def p(self):
        return self.V.shape[1]


def make_cfg1(n: int = 64, ny: int = 64, nx: int = 64, k0: int = 8, frames: int = 1,
              cfg: int = 1) -> Library:
    """64x64 px library: Gamma(2,1) coefficients on Gamma(1,1) fields under a
    1/r^2 envelope plus |N(0, 0.01)| noise; a central r <= 6 occulter and 1%
    bad pixels per image; weights 1/(V + 0.01) on unmasked pixels."""
    p = ny * nx
    g = rng(cfg, S_LIBRARY)
    H0 = components_radial_gamma(g, k0, ny, nx)
    W0 = g.gamma(2.0, 1.0, size=(n, k0))
    gn = rng(cfg, S_NOISE)
    V = W0 @ H0 + np.abs(gn.normal(0.0, 0.01, size=(n, p)))
    gm = rng(cfg, S_MASK)
    mask = mask_disc(ny, nx, 6.0)[None, :] & bad_pixels(gm, n, p, 0.01)
    M = np.where(mask, 1.0 / (V + 0.01), 0.0)
    gs = rng(cfg, S_SCIENCE)
    ws = gs.gamma(2.0, 1.0, size=(frames, k0))
    T = ws @ H0 + np.abs(gs.normal(0.0, 0.01, size=(frames, p)))
    mt = mask_disc(ny, nx, 6.0)[None, :] & bad_pixels(gs, frames, p, 0.01)
    MT = np.where(mt, 1.0 / (T + 0.01), 0.0)
    return Library("cfg1", ny, nx, V.astype(np.float32), M.astype(np.float32),
                   T.astype(np.float32), MT.astype(np.float32), W0, H0)


def _poisson_library(g: np.random.Generator, W0: np.ndarray, H0: np.ndarray, peak: float = 1e6):
    clean = W0 @ H0
    gain = peak / clean.max()
    return g.poisson(gain * clean) / gain


def _science_with_disks(cfg: int, H0: np.ndarray, ny: int, nx: int, frames: int,
                        disk_rel_flux: float, disk_a: float, disk_sigma: float,
                        peak: float = 1e6):
    gs = rng(cfg, S_SCIENCE)
    gd = rng(cfg, S_DISK)
    k0 = H0.shape[0]
    ws = gs.gamma(2.0, 1.0, size=(frames, k0))
    star = ws @ H0
    T = np.empty_like(star)
    for f in range(frames):
        inc = gd.uniform(30.0, 80.0)
        pa = gd.uniform(0.0, 180.0)
        disk = disk_ring(ny, nx, disk_a, disk_sigma, inc, pa) * (disk_rel_flux * star[f].sum())
        clean = star[f] + disk
        gain = peak / clean.max()
        T[f] = gs.poisson(gain * clean) / gain
    return T


def make_cfg2(n: int = 500, ny: int = 200, nx: int = 200, k0: int = 40, frames: int = 50,
              cfg: int = 2, wedge_half_width: float = 6.0, disk_a: float = 50.0) -> Library:
    """STIS-like library: speckle components under a Moffat-like halo,
    Gamma(2,1) coefficients, Poisson-like noise (peak 1e6 counts), a 12 px
    wide diagonal occulting wedge, weights 1/(V + 0.01).  Science frames
    carry an inclined ring disk at 1e-3 of the stellar flux."""
    p = ny * nx
    g = rng(cfg, S_LIBRARY)
    H0 = components_speckle(g, k0, ny, nx)
    W0 = g.gamma(2.0, 1.0, size=(n, k0))
    V = _poisson_library(rng(cfg, S_NOISE), W0, H0)
    wedge = mask_wedge(ny, nx, wedge_half_width)[None, :]
    M = np.where(wedge, 1.0 / (V + 0.01), 0.0)
    T = _science_with_disks(cfg, H0, ny, nx, frames, 1e-3, disk_a * min(ny, nx) / 200.0, 3.0)
    MT = np.where(wedge, 1.0 / (T + 0.01), 0.0)
    return Library("cfg2", ny, nx, V.astype(np.float32), M.astype(np.float32),
                   T.astype(np.float32), MT.astype(np.float32), W0, H0)


def make_cfg3(n: int = 2000, ny: int = 224, nx: int = 288, k0: int = 120, frames: int = 4,
              cfg: int = 3) -> Library:
    """MIRI-like library: the cfg2 PSF and noise model on a 224 x 288 frame
    with a 4QPM-like cross (r <= 8 disc, arms 5 px wide) and 2% bad pixels
    per image; binary weights."""
    p = ny * nx
    g = rng(cfg, S_LIBRARY)
    H0 = components_speckle(g, k0, ny, nx)
    W0 = g.gamma(2.0, 1.0, size=(n, k0))
    V = _poisson_library(rng(cfg, S_NOISE), W0, H0)
    cross = mask_cross(ny, nx, 8.0, 2.0)[None, :]
    M = (cross & bad_pixels(rng(cfg, S_MASK), n, p, 0.02)).astype(np.float64)
    T = _science_with_disks(cfg, H0, ny, nx, frames, 1e-3, 50.0, 3.0)
    MT = (cross & bad_pixels(rng(cfg, S_MASK, 1), frames, p, 0.02)).astype(np.float64)
    return Library("cfg3", ny, nx, V.astype(np.float32), M.astype(np.float32),
                   T.astype(np.float32), MT.astype(np.float32), W0, H0, binary=True)


# --------------------------------------------------------------------------
# Projection set: frames modelled on a fixed seeded basis
# --------------------------------------------------------------------------

@dataclasses.dataclass
class ProjectionSet:
    """Science frames (float32, F x P) and their weights for projection onto
    the fixed basis H (float32, K x P)."""
    ny: int
    nx: int
    H: np.ndarray
    T: np.ndarray
    MT: np.ndarray


def projection_basis(k: int = 100, k0: int = 120, ny: int = 200, nx: int = 200,
                     cfg: int = 5) -> np.ndarray:
    """The k0 speckle components of the projection set (float64); the first
    k are the basis the frames are modelled with."""
    return components_speckle(rng(cfg, S_LIBRARY), k0, ny, nx)


def make_projection_set(frames: int, k: int = 100, k0: int = 120, ny: int = 200, nx: int = 200,
                        cfg: int = 5, sub: int = 0, comps: np.ndarray | None = None,
                        chunk: int = 512) -> ProjectionSet:
    """STIS-shaped frames to be modelled on a fixed K-component basis: each
    frame is a Poisson-like realisation (1e6 counts at its peak) of a
    Gamma(2,1) mixture of k0 >= k speckle components, the basis and k0 - k
    more (so frames lie near, not in, the span of the basis); every other
    frame carries an inclined ring disk at 1e-3 of its stellar flux.  The
    weights are mask / (T + 0.01) with the 12 px diagonal wedge and 1% bad
    pixels per frame.  ``sub`` selects independent frame streams over the
    same components."""
    comps = projection_basis(k, k0, ny, nx, cfg) if comps is None else comps
    p = ny * nx
    gs, gd, gm = rng(cfg, S_SCIENCE, sub), rng(cfg, S_DISK, sub), rng(cfg, S_MASK, sub)
    wedge = mask_wedge(ny, nx, 6.0)
    dy, dx, _ = radius_grid(ny, nx)
    T = np.empty((frames, p), np.float32)
    MT = np.empty((frames, p), np.float32)
    for c0 in range(0, frames, chunk):
        n = min(chunk, frames - c0)
        clean = gs.gamma(2.0, 1.0, size=(n, k0)) @ comps
        for i in range(c0 % 2 == 0, n, 2):  # odd frames carry a disk
            inc, pa = math.radians(gd.uniform(30.0, 80.0)), math.radians(gd.uniform(0.0, 180.0))
            u = dx * math.cos(pa) + dy * math.sin(pa)
            v = (-dx * math.sin(pa) + dy * math.cos(pa)) / max(math.cos(inc), 1e-3)
            ring = np.exp(-0.5 * ((np.hypot(u, v) - 50.0) / 3.0) ** 2).reshape(-1)
            clean[i] += ring * (1e-3 * clean[i].sum() / ring.sum())
        gain = 1e6 / clean.max(axis=1, keepdims=True)
        t = gs.poisson(gain * clean) / gain
        T[c0:c0 + n] = t
        keep = wedge[None, :] & (gm.random((n, p)) >= 0.01)
        MT[c0:c0 + n] = np.where(keep, 1.0 / (t + 0.01), 0.0)
    return ProjectionSet(ny, nx, comps[:k].astype(np.float32), T, MT)


# --------------------------------------------------------------------------
# Ragged frames (batched projection)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class RaggedFrames:
    """Frames stored as CSR rows: frame f owns entries offsets[f]:offsets[f+1]
    of ``pix`` (int32 pixel index), ``val`` (float32 data) and ``wt``
    (float32 weight)."""
    offsets: np.ndarray
    pix: np.ndarray
    val: np.ndarray
    wt: np.ndarray
    p: int

    @property
    def f(self):
        return self.offsets.shape[0] - 1

    def dense(self):
        T = np.zeros((self.f, self.p), np.float32)
        MT = np.zeros((self.f, self.p), np.float32)
        for i in range(self.f):
            s, e = self.offsets[i], self.offsets[i + 1]
            T[i, self.pix[s:e]] = self.val[s:e]
            MT[i, self.pix[s:e]] = self.wt[s:e]
        return T, MT


def make_ragged(H0: np.ndarray, ny: int, nx: int, frames: int, pmin: int, pmax: int,
                cfg: int = 4, binary: bool = True, peak: float = 1e6) -> RaggedFrames:
    """Frames that keep a compact region of P_f ~ U{pmin..pmax} pixels
    nearest the star outside the 4QPM-like cross (ties by flat index), drawn
    as Poisson-like realisations of random non-negative mixtures of H0.
    Pixels of a frame are stored in increasing index order."""
    p = ny * nx
    cross = mask_cross(ny, nx, 8.0, 2.0)
    _, _, r = radius_grid(ny, nx)
    order = np.lexsort((np.arange(p), r.reshape(-1)))
    order = order[cross[order]]
    pmax = min(pmax, order.size)
    pmin = min(pmin, pmax)
    # rank of every valid pixel in the distance order, listed by pixel index:
    # frame f keeps exactly the valid pixels of rank < P_f
    valid = np.sort(order)
    rank = np.empty(p, np.int64)
    rank[order] = np.arange(order.size)
    vrank = rank[valid]
    g = rng(cfg, S_SCIENCE)
    sizes = g.integers(pmin, pmax + 1, size=frames)
    k0 = H0.shape[0]
    ws = g.gamma(2.0, 1.0, size=(frames, k0))
    offsets = np.zeros(frames + 1, np.int64)
    offsets[1:] = np.cumsum(sizes)
    nnz = int(offsets[-1])
    pix = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float32)
    wt = np.empty(nnz, np.float32)
    Hv = np.ascontiguousarray(H0[:, valid])
    chunk = 256
    for c0 in range(0, frames, chunk):
        clean_rows = ws[c0:c0 + chunk] @ Hv
        for i, row in enumerate(clean_rows):
            f = c0 + i
            keep = vrank < sizes[f]
            clean = row[keep]
            gain = peak / clean.max()
            v = g.poisson(gain * clean) / gain
            s, e = offsets[f], offsets[f + 1]
            pix[s:e] = valid[keep]
            val[s:e] = v
            wt[s:e] = 1.0 if binary else 1.0 / (v + 0.01)
    return RaggedFrames(offsets, pix, val, wt, p)


def uniform_init(cfg: int, rows: int, cols: int, sub: int = 0) -> np.ndarray:
    """A seeded U(0,1) float32 matrix for callers that bring their own init."""
    g = rng(cfg, S_INIT, sub)
    return (g.random((rows, cols)) * (1 - 2 ** -23) + 2 ** -24).astype(np.float32)
