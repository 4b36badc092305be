"""Planted mistakes in the oracle must trip its pins.

Each test swaps one oracle routine for a plausible wrong version (on the
CPU, inside the test only) and checks that the corresponding pin check
reports a large error, so a mistake of that kind could not pass unnoticed.
"""
import numpy as np

from oracle import altgdmin as AG
from oracle import operators as O

from oracle_checks import adjoint_error, fd_gradient_error, inv_error, small_problem


def test_missing_coil_conjugate_breaks_adjoint(monkeypatch):
    def bad_AH(self, k, v):
        grid = np.zeros((self.nc, self.n), dtype=np.complex128)
        grid[:, self.omegas[k]] = v
        return np.sum(self.coils * self.F.adj(grid), axis=0)   # conj dropped
    _, op, _, _, rng = small_problem("index")
    monkeypatch.setattr(O.Operator, "AH", bad_AH)
    assert adjoint_error(op, rng) > 1e-3


def test_forward_transform_in_adjoint_breaks_adjoint(monkeypatch):
    def bad_AH(self, k, v):
        grid = np.zeros((self.nc, self.n), dtype=np.complex128)
        grid[:, self.omegas[k]] = v
        return np.sum(np.conj(self.coils) * self.F.fwd(grid), axis=0)  # F instead of F^H
    _, op, _, _, rng = small_problem("lines")
    monkeypatch.setattr(O.Operator, "AH", bad_AH)
    assert adjoint_error(op, rng) > 1e-3


def _bad_gradient(kind):
    def grad(op, U, B, Y, FU=None):
        G = np.zeros_like(U)
        for k in range(op.q):
            M = op.AU(k, U)
            res = (M @ B[:, k] - op.frame_vec(Y, k)).reshape(op.nc, op.m_k[k])
            if kind == "no_conj_b":
                G += np.outer(op.AH(k, res), B[:, k])
            elif kind == "sign":
                G -= np.outer(op.AH(k, res), np.conj(B[:, k]))
            elif kind == "drop_y":
                res = (M @ B[:, k]).reshape(op.nc, op.m_k[k])
                G += np.outer(op.AH(k, res), np.conj(B[:, k]))
        return G
    return grad


def test_gradient_mistakes_fail_finite_difference():
    for kind in ("no_conj_b", "sign", "drop_y"):
        _, op, Y, U, rng = small_problem("index", seed=3)
        assert fd_gradient_error(op, Y, U, rng, grad_fn=_bad_gradient(kind)) > 1e-2, kind


def test_gradient_mistakes_break_orthogonality():
    for kind in ("drop_y",):
        _, op, Y, U, _ = small_problem("lines", seed=5)
        assert inv_error(op, Y, U, grad_fn=_bad_gradient(kind)) > 1e-3, kind


def test_mean_instead_of_max_m_fails_truncation_example(monkeypatch):
    real = AG.truncation

    def bad(op, Y, c):
        class Shim:
            pass
        s = Shim()
        s.m_max = float(np.mean(op.m_k))
        s.q, s.m_k = op.q, op.m_k
        return real(s, Y, c)
    om = [np.arange(10), np.arange(20)]
    op = O.Operator(5, 4, np.ones((2, 20)), om, "fft")
    Y = np.zeros((2, 2, 20), dtype=np.complex128)
    Y[0, 0, :10] = 1.0
    Y[1, 0, :19] = 1j
    Y[1, 0, 19] = 20.0
    Ytr, gamma, _ = bad(op, Y, 36.0)
    assert Ytr[1, 0, 19] != 0        # the hand example's expectation is violated


def test_wrong_dft_sign_fails_plane_wave():
    nx, ny, a, b = 8, 4, 3, 1
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    img = np.exp(2j * np.pi * (a * x / nx + b * y / ny))
    F = O.DFT2(nx, ny, "fft")
    out = F.adj(img.ravel())      # the opposite sign convention
    assert abs(out[b * nx + a]) < 1e-9
