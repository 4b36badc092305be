"""Pins for the oracle's measurement operator (Sec. II-A, eq. Ymat)."""
import numpy as np
import pytest

import datagen
from oracle import operators as O


def _random_op(nx, ny, nc, q, kind, backend, seed, variable_m=True):
    rng = np.random.default_rng(seed)
    coils = datagen.random_phase_coils(nx, ny, nc, rng)
    if kind == "lines":
        masks = [np.sort(rng.choice(ny, size=int(rng.integers(1, ny + 1)), replace=False))
                 for _ in range(q)]
    else:
        masks = [np.sort(rng.choice(nx * ny, size=int(rng.integers(1, nx * ny + 1)), replace=False))
                 for _ in range(q)]
    return O.Operator(nx, ny, coils, O.omegas(kind, masks, nx), backend), rng


@pytest.mark.parametrize("kind", ["lines", "index"])
@pytest.mark.parametrize("backend,nx,ny", [("dense", 4, 4), ("dense", 8, 4), ("fft", 8, 16), ("fft", 16, 16)])
def test_adjoint_identity(kind, backend, nx, ny):
    """<A(X), Y> = <X, A^H(Y)> for random X, Y, random-phase coils and masks."""
    op, rng = _random_op(nx, ny, 3, 5, kind, backend, seed=nx + ny)
    X = datagen.crandn(rng, nx * ny, op.q)
    Y = datagen.crandn(rng, op.q, op.nc, op.m_max)
    valid = np.arange(op.m_max)[None, None, :] < op.m_k[:, None, None]
    Y = np.where(valid, Y, 0)
    lhs = np.vdot(op.apply_A(X), Y)
    rhs = np.vdot(X, op.apply_AH(Y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_apply_A_pads_with_zeros_and_AH_ignores_padding():
    op, rng = _random_op(8, 8, 2, 6, "index", "fft", seed=3)
    X = datagen.crandn(rng, 64, op.q)
    Y = op.apply_A(X)
    for k in range(op.q):
        assert np.all(Y[k, :, op.m_k[k]:] == 0)
    Yj = Y + 0.0
    for k in range(op.q):
        Yj[k, :, op.m_k[k]:] = 123.0
    assert np.allclose(op.apply_AH(Yj), op.apply_AH(Y), atol=0, rtol=0)


@pytest.mark.parametrize("backend", ["dense", "fft"])
def test_full_sampling_is_parseval(backend):
    """All n locations sampled and sum_c |s_c|^2 = 1 give A_k^H A_k = I."""
    nx, ny, nc = 8, 4, 3
    coils = datagen.coil_maps(nx, ny, nc, "ring")
    op = O.Operator(nx, ny, coils, [np.arange(nx * ny)] * 2, backend)
    rng = np.random.default_rng(0)
    x = datagen.crandn(rng, nx * ny)
    y = op.A(0, x)
    assert np.allclose(op.AH(0, y), x, atol=1e-12)
    assert abs(np.vdot(y, y).real - np.vdot(x, x).real) < 1e-12 * np.vdot(x, x).real


def test_single_coil_is_subsampled_fft2():
    """nc = 1 with s = 1 reduces A_k to H_k F (Sec. II-A); compare with
    numpy's own 2D FFT, an independent library routine."""
    nx, ny = 16, 8
    rng = np.random.default_rng(1)
    om = np.sort(rng.choice(nx * ny, size=37, replace=False))
    op = O.Operator(nx, ny, np.ones((1, nx * ny)), [om], "fft")
    x = datagen.crandn(rng, nx * ny)
    ref = np.fft.fft2(x.reshape(ny, nx), norm="ortho").ravel()[om]
    assert np.allclose(op.A(0, x)[0], ref, atol=1e-12)


def test_lines_mask_is_full_readout_rows():
    nx, ny = 8, 8
    om = O.omegas_from_lines([np.array([0, 3])], nx)[0]
    assert list(om) == [0, 1, 2, 3, 4, 5, 6, 7, 24, 25, 26, 27, 28, 29, 30, 31]
