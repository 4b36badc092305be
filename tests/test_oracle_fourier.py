"""Pins for the oracle's DFT (Sec. II-A: F is the 2D DFT as a matrix).

The dense backend is checked against a pure-Python evaluation of the DFT sum
and against closed forms (plane waves, deltas); the FFT backend is checked
against the dense one on tiny grids, including non-square ones.
"""
import cmath
import math

import numpy as np
import pytest

from oracle.operators import DFT2, dft_matrix_2d


def brute_dft2(img):
    """sum_{y,x} img[y,x] exp(-2 pi i (ky y/ny + kx x/nx)) / sqrt(n), by loops."""
    ny, nx = img.shape
    out = np.zeros((ny, nx), dtype=np.complex128)
    for ky in range(ny):
        for kx in range(nx):
            s = 0j
            for y in range(ny):
                for x in range(nx):
                    s += img[y, x] * cmath.exp(-2j * math.pi * (ky * y / ny + kx * x / nx))
            out[ky, kx] = s / math.sqrt(nx * ny)
    return out


@pytest.mark.parametrize("nx,ny", [(4, 4), (4, 2), (2, 4), (8, 4)])
def test_dense_matches_brute_force(nx, ny):
    rng = np.random.default_rng(nx * 10 + ny)
    img = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    ref = brute_dft2(img).ravel()
    F = dft_matrix_2d(nx, ny)
    assert np.allclose(F @ img.ravel(), ref, atol=1e-12, rtol=0)


@pytest.mark.parametrize("nx,ny", [(4, 4), (8, 8), (16, 16), (8, 16), (16, 8)])
def test_fft_backend_matches_dense(nx, ny):
    rng = np.random.default_rng(7)
    v = rng.standard_normal((3, nx * ny)) + 1j * rng.standard_normal((3, nx * ny))
    fd, ff = DFT2(nx, ny, "dense"), DFT2(nx, ny, "fft")
    a, b = fd.fwd(v), ff.fwd(v)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
    a, b = fd.adj(v), ff.adj(v)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


@pytest.mark.parametrize("backend", ["dense", "fft"])
def test_plane_wave_lands_on_its_frequency(backend):
    # exp(+2 pi i (a x / nx + b y / ny)) has all its energy at kx = a, ky = b:
    # pins the sign of the exponent and which axis is x (fastest).
    nx, ny, a, b = 8, 4, 3, 1
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    img = np.exp(2j * np.pi * (a * x / nx + b * y / ny))
    out = DFT2(nx, ny, backend).fwd(img.ravel())
    expect = np.zeros(nx * ny, dtype=np.complex128)
    expect[b * nx + a] = math.sqrt(nx * ny)
    assert np.allclose(out, expect, atol=1e-12)


@pytest.mark.parametrize("backend", ["dense", "fft"])
def test_delta_gives_phase_ramp_and_unitarity(backend):
    nx, ny, x0, y0 = 8, 8, 2, 5
    v = np.zeros(nx * ny, dtype=np.complex128)
    v[y0 * nx + x0] = 1.0
    F = DFT2(nx, ny, backend)
    out = F.fwd(v)
    ky, kx = np.divmod(np.arange(nx * ny), nx)
    expect = np.exp(-2j * np.pi * (kx * x0 / nx + ky * y0 / ny)) / math.sqrt(nx * ny)
    assert np.allclose(out, expect, atol=1e-12)
    assert np.allclose(F.adj(out), v, atol=1e-12)
