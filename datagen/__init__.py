"""Seeded synthetic inputs for the altGDmin reconstruction.

This module produces *inputs only*: ground-truth image sequences Z*, coil
sensitivity maps, k-space sampling masks and unit-variance complex noise
draws.  It contains none of the reconstruction's arithmetic (no Fourier
transform, no measurement operator, no least squares).  The measurements
y = A(Z*) + noise are formed by whichever side consumes these inputs, with its
own operator: the FP64 oracle in the tests, the GPU library in the benchmark.

Conventions shared by every consumer:

* an image is an ``ny x nx`` array flattened row-major, pixel p = x + nx*y,
  x (readout) fastest; Z* is ``n x q`` with one vectorised frame per column;
* k-space locations use the same flattening, index = ky*nx + kx, in natural
  FFT order (DC at index 0, no fftshift);
* a 1D Cartesian mask is, per frame, a sorted list of sampled phase-encode
  lines ky (every line fully sampled along kx); a general mask is, per frame,
  a sorted list of flat k-space indices;
* coil maps are ``nc x n`` and are normalised so that sum_c |s_c(p)|^2 = 1.

Workloads follow the shapes of the paper's datasets (Sec. V and App. A:
cardiac cine / perfusion, 1D Cartesian variable density and golden-angle
pseudo-radial undersampling); the real datasets are not available, so these
phantoms stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GOLDEN_ANGLE_DEG = 180.0 * (np.sqrt(5.0) - 1.0) / 2.0  # 111.246...


# ---------------------------------------------------------------------------
# coordinates and coil maps
# ---------------------------------------------------------------------------
def grid(nx: int, ny: int):
    """Normalised coordinates in [-1, 1), returned as (X, Y) arrays ny x nx."""
    xs = -1.0 + 2.0 * np.arange(nx) / nx
    ys = -1.0 + 2.0 * np.arange(ny) / ny
    return np.meshgrid(xs, ys, indexing="xy")


def coil_maps(nx: int, ny: int, nc: int, layout: str = "ring") -> np.ndarray:
    """Smooth Gaussian-bump coil sensitivities, normalised to sum |s_c|^2 = 1.

    Each coil carries a constant phase 2*pi*c/nc so that a missing complex
    conjugate anywhere downstream changes results.  ``layout='corners'`` puts
    the bump centres at the four corners (sigma 1.0); ``'ring'`` puts them on
    a ring of radius 1.2 (sigma 0.8).
    """
    X, Y = grid(nx, ny)
    if layout == "corners":
        corners = [(-1.0, -1.0), (1.0, -1.0), (1.0, 1.0), (-1.0, 1.0)]
        centres = [corners[c % 4] for c in range(nc)]
        sigma = 1.0
    elif layout == "ring":
        ang = 2.0 * np.pi * np.arange(nc) / max(nc, 1)
        centres = [(1.2 * np.cos(a), 1.2 * np.sin(a)) for a in ang]
        sigma = 0.8
    elif layout == "flat":
        centres = [(0.0, 0.0)] * nc
        sigma = np.inf
    else:
        raise ValueError(layout)
    maps = np.empty((nc, ny * nx), dtype=np.complex128)
    for c, (cx, cy) in enumerate(centres):
        if np.isinf(sigma):
            mag = np.ones_like(X)
        else:
            mag = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sigma ** 2))
        maps[c] = (mag * np.exp(1j * 2.0 * np.pi * c / nc)).ravel()
    norm = np.sqrt(np.sum(np.abs(maps) ** 2, axis=0))
    return maps / norm[None, :]


def random_phase_coils(nx: int, ny: int, nc: int, rng) -> np.ndarray:
    """Coil maps with random magnitudes and phases per pixel (not normalised).

    Used by operator tests where smoothness is irrelevant and any structure
    would hide indexing mistakes.
    """
    mag = 0.5 + rng.random((nc, ny * nx))
    ph = rng.random((nc, ny * nx)) * 2.0 * np.pi
    return mag * np.exp(1j * ph)


# ---------------------------------------------------------------------------
# masks
# ---------------------------------------------------------------------------
def uniform_lines(ny: int, q: int, n_centre: int, n_other: int, rng):
    """Per frame: the n_centre lines around DC plus n_other uniform draws."""
    freqs = np.arange(-ny // 2, ny // 2)
    centre = freqs[(freqs >= -n_centre // 2) & (freqs < n_centre - n_centre // 2)]
    others = np.setdiff1d(freqs, centre)
    out = []
    for _ in range(q):
        pick = rng.choice(others, size=n_other, replace=False)
        f = np.concatenate([centre, pick])
        out.append(np.sort(np.mod(f, ny)).astype(np.int32))
    return out


def variable_density_lines(ny: int, q: int, n_lines: int, n_centre: int, rng):
    """1D Cartesian variable-density mask, redrawn per frame.

    n_centre lines around DC are always taken; the remaining lines are drawn
    without replacement with weight (1 - 2|f|/ny)^3 + 0.05 over frequency f.
    """
    freqs = np.arange(-ny // 2, ny // 2)
    centre = freqs[(freqs >= -n_centre // 2) & (freqs < n_centre - n_centre // 2)]
    others = np.setdiff1d(freqs, centre)
    w = (1.0 - 2.0 * np.abs(others) / ny) ** 3 + 0.05
    w = w / w.sum()
    out = []
    for _ in range(q):
        pick = rng.choice(others, size=n_lines - len(centre), replace=False, p=w)
        f = np.concatenate([centre, pick])
        out.append(np.sort(np.mod(f, ny)).astype(np.int32))
    return out


def golden_angle_radial(nx: int, ny: int, q: int, spokes: int, continuing: bool = True):
    """Pseudo-radial mask: radial spokes rounded onto the Cartesian grid.

    Spoke g of the whole acquisition sits at angle g * golden angle when
    ``continuing`` (one golden-angle sequence across frames); otherwise each
    frame has ``spokes`` evenly spaced spokes rotated by k * golden angle.
    Each frame's mask is the de-duplicated, sorted set of flat indices.
    """
    out = []
    t = np.arange(-max(nx, ny) // 2, max(nx, ny) // 2, dtype=np.float64)
    for k in range(q):
        idx = []
        for s in range(spokes):
            if continuing:
                theta = np.deg2rad((k * spokes + s) * GOLDEN_ANGLE_DEG)
            else:
                theta = np.deg2rad(k * GOLDEN_ANGLE_DEG) + np.pi * s / spokes
            kx = np.floor(t * np.cos(theta) + 0.5).astype(np.int64) % nx
            ky = np.floor(t * np.sin(theta) + 0.5).astype(np.int64) % ny
            idx.append(ky * nx + kx)
        out.append(np.unique(np.concatenate(idx)).astype(np.int32))
    return out


def random_locations(n: int, q: int, m: int, rng):
    """m distinct k-space locations per frame, uniform at random."""
    return [np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32) for _ in range(q)]


# ---------------------------------------------------------------------------
# phantoms
# ---------------------------------------------------------------------------
def crandn(rng, *shape) -> np.ndarray:
    """i.i.d. circular complex Gaussian CN(0, 1)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def lowrank_gaussian(n: int, q: int, r: int, rng):
    """Z* = U* B*, U* orthonormalised CN(0,1), B* i.i.d. CN(0,1)."""
    g = crandn(rng, n, r)
    ustar, _ = np.linalg.qr(g)
    bstar = crandn(rng, r, q)
    return ustar @ bstar, ustar


def _ellipse(X, Y, cx, cy, ax, ay, width=0.02):
    rho = np.sqrt(((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2)
    return 1.0 / (1.0 + np.exp(np.clip(-(1.0 - rho) / width, -700.0, 700.0)))


def motion_ellipse(nx: int, ny: int, q: int, rng, period: float = 20.0,
                   sparse_frac: float = 0.01, sparse_amp: float = 0.05,
                   jitter: bool = False) -> np.ndarray:
    """Cardiac-cine-like sequence: static body and organs plus a 'heart'
    ellipse whose radius and intensity move periodically, a smooth phase and
    a sparse per-frame residual (a fraction of pixels at a small amplitude)."""
    X, Y = grid(nx, ny)
    body = dict(c=(0.0, 0.0), a=(0.75, 0.6), v=0.6)
    org1 = dict(c=(-0.35, 0.2), a=(0.15, 0.25), v=0.8)
    org2 = dict(c=(0.35, -0.25), a=(0.2, 0.12), v=0.4)
    heart = dict(c=(0.1, 0.05), a=(0.22, 0.18), v=1.0)
    phase0 = 0.0
    if jitter:
        for e in (body, org1, org2, heart):
            e["c"] = (e["c"][0] + rng.uniform(-0.1, 0.1), e["c"][1] + rng.uniform(-0.1, 0.1))
            e["a"] = (e["a"][0] * rng.uniform(0.8, 1.2), e["a"][1] * rng.uniform(0.8, 1.2))
            e["v"] = e["v"] * rng.uniform(0.8, 1.2)
        phase0 = rng.uniform(0.0, 2.0 * np.pi)
    static = sum(e["v"] * _ellipse(X, Y, *e["c"], *e["a"]) for e in (body, org1, org2))
    smooth_phase = np.exp(1j * np.pi * 0.25 * (X + Y))
    n = nx * ny
    Z = np.empty((n, q), dtype=np.complex128)
    for k in range(q):
        s = 1.0 + 0.2 * np.sin(2.0 * np.pi * k / period + phase0)
        v = heart["v"] * (1.0 + 0.15 * np.cos(2.0 * np.pi * k / period + phase0))
        img = static + v * _ellipse(X, Y, *heart["c"], heart["a"][0] * s, heart["a"][1] * s)
        img = (img * smooth_phase).ravel()
        npx = int(round(sparse_frac * n))
        if npx > 0:
            pos = rng.choice(n, size=npx, replace=False)
            img = img.copy()
            img[pos] += sparse_amp * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, npx))
        Z[:, k] = img
    return Z


def perfusion(nx: int, ny: int, q: int, rng, n_regions: int = 6) -> np.ndarray:
    """Perfusion-like sequence: tissue regions with gamma-variate uptake
    curves (region-specific onset and peak) over a static baseline, smooth
    phase, scaled to unit peak magnitude."""
    X, Y = grid(nx, ny)
    base = 0.2 * _ellipse(X, Y, 0.0, 0.0, 0.8, 0.7)
    t = np.arange(q, dtype=np.float64)
    regions = []
    for _ in range(n_regions):
        ang = rng.uniform(0.0, 2.0 * np.pi)
        rad = rng.uniform(0.0, 0.45)
        c = (rad * np.cos(ang), rad * np.sin(ang))
        a = (rng.uniform(0.08, 0.25), rng.uniform(0.08, 0.25))
        t0 = rng.uniform(5.0, 30.0)
        alpha = rng.uniform(1.5, 3.0)
        tau = rng.uniform(3.0, 10.0)
        amp = rng.uniform(0.3, 1.0)
        tt = np.clip(t - t0, 0.0, None) / tau
        curve = amp * tt ** alpha * np.exp(-tt)
        curve = curve / max(curve.max(), 1e-30) * amp
        regions.append((_ellipse(X, Y, *c, *a), curve))
    smooth_phase = np.exp(1j * np.pi * 0.25 * (X - Y))
    n = nx * ny
    Z = np.empty((n, q), dtype=np.complex128)
    for k in range(q):
        img = base.copy()
        for shape, curve in regions:
            img = img + curve[k] * shape
        Z[:, k] = (img * smooth_phase).ravel()
    return Z / np.abs(Z).max()


# ---------------------------------------------------------------------------
# a problem instance
# ---------------------------------------------------------------------------
@dataclass
class Problem:
    """One synthetic reconstruction problem (inputs only)."""
    name: str
    nx: int
    ny: int
    nc: int
    q: int
    r: int
    kind: str                    # 'lines' or 'index'
    masks: list                  # per frame: int32 lines (kind 'lines') or flat indices
    coils: np.ndarray            # nc x n complex128
    zstar: np.ndarray            # n x q complex128
    snr_db: Optional[float]      # None: noise-free
    noise: np.ndarray            # q x nc x m_max complex128, unit variance (unused if noise-free)
    t_iters: int = 70
    ustar: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def m_k(self) -> np.ndarray:
        """Samples per coil in each frame."""
        if self.kind == "lines":
            return np.array([len(l) * self.nx for l in self.masks], dtype=np.int32)
        return np.array([len(l) for l in self.masks], dtype=np.int32)

    @property
    def m_max(self) -> int:
        return int(self.m_k().max())

    def mask_array(self) -> np.ndarray:
        """Masks padded with -1: q x L_max (lines) or q x m_max (index)."""
        width = max(len(l) for l in self.masks)
        out = -np.ones((self.q, width), dtype=np.int32)
        for k, l in enumerate(self.masks):
            out[k, : len(l)] = l
        return out


def add_noise(y_clean: np.ndarray, w: np.ndarray, m_k: np.ndarray, snr_db) -> np.ndarray:
    """y = y_clean + sigma * w on the sampled entries only.

    sigma^2 = ||y_clean||^2 / (N * 10^(snr/10)) with N the number of sampled
    entries over the whole dataset; padding entries stay zero.  y_clean and w
    are q x nc x m_max.
    """
    if snr_db is None:
        return y_clean.copy()
    valid = np.arange(y_clean.shape[2])[None, None, :] < m_k[:, None, None]
    n_samp = int(np.broadcast_to(valid, y_clean.shape).sum())
    sigma = np.sqrt(np.sum(np.abs(y_clean) ** 2) / (n_samp * 10.0 ** (snr_db / 10.0)))
    return np.where(valid, y_clean + sigma * w, 0.0)


def _noise(rng, q, nc, m_max):
    return crandn(rng, q, nc, m_max)


# ---------------------------------------------------------------------------
# the workload presets
# ---------------------------------------------------------------------------
PRESETS = {
    # 64x64, 4 coils at the corners, 16 frames, rank 4, exact low rank, noise-free
    "gauss64": dict(nx=64, ny=64, nc=4, q=16, r=4, t=20),
    # 256x256 cine-like, 12 ring coils, 40 frames, rank 8, VD R=8, 30 dB
    "cine256": dict(nx=256, ny=256, nc=12, q=40, r=8, t=70),
    # 128x128 perfusion-like, 8 coils, 100 frames, rank 10, 16 golden-angle spokes, 25 dB
    "radial128": dict(nx=128, ny=128, nc=8, q=100, r=10, t=50),
    # 256x256 cine-like, 16 coils, 64 frames, rank 16, VD R=12, 30 dB
    "cine256r16": dict(nx=256, ny=256, nc=16, q=64, r=16, t=70),
    # 128x128 cine-like, 8 coils, 48 frames, rank 6, VD R=8, 30 dB
    "cine128": dict(nx=128, ny=128, nc=8, q=48, r=6, t=70),
}


def make(name: str, seed: int, jitter: bool = False) -> Problem:
    """Build a preset workload with a fixed seed."""
    rng = np.random.default_rng(seed)
    if name == "gauss64":
        nx = ny = 64
        nc, q, r = 4, 16, 4
        masks = uniform_lines(ny, q, 4, 12, rng)
        zstar, ustar = lowrank_gaussian(nx * ny, q, r, rng)
        coils = coil_maps(nx, ny, nc, "corners")
        snr, t = None, 20
        kind = "lines"
    elif name in ("cine256", "cine256r16", "cine128"):
        p = PRESETS[name]
        nx, ny, nc, q, r, t = p["nx"], p["ny"], p["nc"], p["q"], p["r"], p["t"]
        accel = {"cine256": 8, "cine256r16": 12, "cine128": 8}[name]
        n_lines = int(round(ny / accel))
        masks = variable_density_lines(ny, q, n_lines, 8, rng)
        zstar = motion_ellipse(nx, ny, q, rng, jitter=jitter)
        ustar = None
        coils = coil_maps(nx, ny, nc, "ring")
        snr = 30.0
        kind = "lines"
    elif name == "radial128":
        nx = ny = 128
        nc, q, r, t = 8, 100, 10, 50
        masks = golden_angle_radial(nx, ny, q, 16)
        zstar = perfusion(nx, ny, q, rng)
        ustar = None
        coils = coil_maps(nx, ny, nc, "ring")
        snr = 25.0
        kind = "index"
    else:
        raise KeyError(name)
    m_k = (np.array([len(l) * nx for l in masks]) if kind == "lines"
           else np.array([len(l) for l in masks]))
    noise = _noise(rng, q, nc, int(m_k.max())) if snr is not None else np.zeros((q, nc, int(m_k.max())), np.complex128)
    return Problem(name=name, nx=nx, ny=ny, nc=nc, q=q, r=r, kind=kind, masks=masks,
                   coils=coils, zstar=zstar, snr_db=snr, noise=noise, t_iters=t, ustar=ustar)


def make_small(nx: int, ny: int, nc: int, q: int, r: int, seed: int, kind: str = "lines",
               n_lines: Optional[int] = None, m: Optional[int] = None,
               lowrank: bool = True, snr_db: Optional[float] = None,
               coils: str = "ring", variable_m: bool = False) -> Problem:
    """A small random problem for tests (any grid, either mask kind)."""
    rng = np.random.default_rng(seed)
    if kind == "lines":
        L = n_lines if n_lines is not None else max(2, ny // 4)
        if variable_m:
            masks = [np.sort(rng.choice(ny, size=int(rng.integers(max(1, L // 2), L + 1)),
                                        replace=False)).astype(np.int32) for _ in range(q)]
        else:
            masks = [np.sort(rng.choice(ny, size=L, replace=False)).astype(np.int32)
                     for _ in range(q)]
    elif kind == "index":
        mm = m if m is not None else max(4, nx * ny // 4)
        if variable_m:
            masks = [np.sort(rng.choice(nx * ny, size=int(rng.integers(max(1, mm // 2), mm + 1)),
                                        replace=False)).astype(np.int32) for _ in range(q)]
        else:
            masks = random_locations(nx * ny, q, mm, rng)
    else:
        raise ValueError(kind)
    if lowrank:
        zstar, ustar = lowrank_gaussian(nx * ny, q, r, rng)
    else:
        zstar, ustar = crandn(rng, nx * ny, q), None
    if coils == "random":
        cm = random_phase_coils(nx, ny, nc, rng)
    else:
        cm = coil_maps(nx, ny, nc, coils)
    m_k = (np.array([len(l) * nx for l in masks]) if kind == "lines"
           else np.array([len(l) for l in masks]))
    noise = crandn(rng, q, nc, int(m_k.max()))
    return Problem(name=f"small{nx}x{ny}", nx=nx, ny=ny, nc=nc, q=q, r=r, kind=kind,
                   masks=masks, coils=cm, zstar=zstar, snr_db=snr_db, noise=noise,
                   ustar=ustar, t_iters=20)
