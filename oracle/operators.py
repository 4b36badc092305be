"""Multi-coil Cartesian measurement operator (oracle, test infrastructure).

Sec. II-A of the paper: for frame k, coil c,

    y_{k,c} = H_k F D_c z_k,

with F the n x n 2D DFT, D_c = diag(s_c) the coil sensitivity and H_k the
0/1 row selector of the sampled k-space locations Omega_k.  The frame's
operator stacks the coils, A_k = [H_k F D_1; ...; H_k F D_nc].  The padded
forms (eq. Ymat) stack frames column-wise with zeros beyond m_k.

Readings (the paper leaves these open):
* F is unitary (1/sqrt(n)); the footnote on the DFT normalisation in
  Sec. III-B says the constant depends on the normalisation, and the
  iterates of U do not depend on it (a scale alpha on F scales y and A_k
  alike, leaves b_k, U_0 and the U-trajectory unchanged).
* natural FFT index order, DC at index 0, no fftshift.
* pixel p = x + nx*y and k-space index ky*nx + kx.
* "transpose" is the conjugate transpose throughout (Sec. II-A notation).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

# threads for the FFT backend: the OpenMP thread budget if one is set, else
# the CPUs this process may run on
WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0)) or 1


# ---------------------------------------------------------------------------
# DFT backends
# ---------------------------------------------------------------------------
def dft_matrix_2d(nx: int, ny: int) -> np.ndarray:
    """The unitary 2D DFT matrix from its definition (dense backend).

    F[(ky,kx), (y,x)] = exp(-2 pi i (ky y / ny + kx x / nx)) / sqrt(nx ny),
    rows and columns flattened as ky*nx + kx and y*nx + x.
    """
    n = nx * ny
    p = np.arange(n)
    x, y = p % nx, p // nx
    kx, ky = x, y  # same flattening for the frequency index
    phase = np.outer(ky, y) / ny + np.outer(kx, x) / nx
    return np.exp(-2j * np.pi * phase) / np.sqrt(n)


class DFT2:
    """Unitary 2D DFT on flattened images; backend 'fft' or 'dense'."""

    def __init__(self, nx: int, ny: int, backend: str = "fft"):
        self.nx, self.ny, self.n = nx, ny, nx * ny
        self.backend = backend
        if backend == "dense":
            if self.n > 256:
                raise ValueError("dense backend is for grids up to 16x16")
            self.F = dft_matrix_2d(nx, ny)
        elif backend != "fft":
            raise ValueError(backend)

    def fwd(self, v: np.ndarray) -> np.ndarray:
        """F v for v of shape (..., n)."""
        if self.backend == "dense":
            return v @ self.F.T
        img = v.reshape(v.shape[:-1] + (self.ny, self.nx))
        return sfft.fft2(img, norm="ortho", workers=WORKERS).reshape(v.shape)

    def adj(self, v: np.ndarray) -> np.ndarray:
        """F^H v for v of shape (..., n)."""
        if self.backend == "dense":
            return v @ self.F.conj()
        img = v.reshape(v.shape[:-1] + (self.ny, self.nx))
        return sfft.ifft2(img, norm="ortho", workers=WORKERS).reshape(v.shape)


# ---------------------------------------------------------------------------
# masks
# ---------------------------------------------------------------------------
def omegas_from_lines(lines, nx: int):
    """Flat k-space indices of fully sampled phase-encode lines, in the order
    [line l][kx] used for y (a 1D Cartesian H_k, Sec. II-A / Sec. V)."""
    out = []
    for l in lines:
        l = np.asarray(l, dtype=np.int64)
        out.append((l[:, None] * nx + np.arange(nx)[None, :]).ravel())
    return out


def omegas(kind: str, masks, nx: int):
    if kind == "lines":
        return omegas_from_lines(masks, nx)
    if kind == "index":
        return [np.asarray(m, dtype=np.int64) for m in masks]
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# the operator
# ---------------------------------------------------------------------------
class Operator:
    """A_k = [H_k F D_c]_{c=1..nc} for every frame k (Sec. II-A)."""

    def __init__(self, nx: int, ny: int, coils: np.ndarray, omega_list, backend: str = "fft"):
        self.nx, self.ny, self.n = nx, ny, nx * ny
        self.coils = np.asarray(coils, dtype=np.complex128)
        self.nc = self.coils.shape[0]
        self.omegas = [np.asarray(o, dtype=np.int64) for o in omega_list]
        self.q = len(self.omegas)
        self.m_k = np.array([len(o) for o in self.omegas], dtype=np.int64)
        self.m_max = int(self.m_k.max())
        self.F = DFT2(nx, ny, backend)

    # --- single frame ------------------------------------------------------
    def A(self, k: int, x: np.ndarray) -> np.ndarray:
        """y_k = A_k x as an (nc, m_k) array: y_{k,c} = (F (s_c o x))[Omega_k]."""
        full = self.F.fwd(self.coils * x[None, :])
        return full[:, self.omegas[k]]

    def AH(self, k: int, v: np.ndarray) -> np.ndarray:
        """A_k^H v = sum_c conj(s_c) o F^H (scatter of v_c onto Omega_k)."""
        grid = np.zeros((self.nc, self.n), dtype=np.complex128)
        grid[:, self.omegas[k]] = v
        return np.sum(np.conj(self.coils) * self.F.adj(grid), axis=0)

    def AU(self, k: int, U: np.ndarray, FU=None) -> np.ndarray:
        """The (nc m_k) x r matrix A_k U, rows ordered [c][i].

        FU, if given, holds F(s_c o u_j) as (nc, r, n): the transform of each
        coil-weighted basis vector does not depend on k, only the selection
        H_k does, so a caller may compute it once.
        """
        if FU is None:
            FU = self.transform_basis(U)
        sel = FU[:, :, self.omegas[k]]            # (nc, r, m_k)
        return np.transpose(sel, (0, 2, 1)).reshape(self.nc * self.m_k[k], -1)

    def transform_basis(self, U: np.ndarray) -> np.ndarray:
        """F(s_c o u_j) for all c, j as (nc, r, n)."""
        r = U.shape[1]
        out = np.empty((self.nc, r, self.n), dtype=np.complex128)
        for j in range(r):
            out[:, j, :] = self.F.fwd(self.coils * U[:, j][None, :])
        return out

    # --- padded stacking (eq. Ymat) ----------------------------------------
    def apply_A(self, X: np.ndarray) -> np.ndarray:
        """Y = A(X) as (q, nc, m_max), zero beyond m_k."""
        Y = np.zeros((self.q, self.nc, self.m_max), dtype=np.complex128)
        for k in range(self.q):
            Y[k, :, : self.m_k[k]] = self.A(k, X[:, k])
        return Y

    def apply_AH(self, Y: np.ndarray) -> np.ndarray:
        """X = A^H(Y) as n x q; entries beyond m_k are ignored."""
        X = np.empty((self.n, self.q), dtype=np.complex128)
        for k in range(self.q):
            X[:, k] = self.AH(k, Y[k, :, : self.m_k[k]])
        return X

    def frame_vec(self, Y: np.ndarray, k: int) -> np.ndarray:
        """y_k as one vector of length nc*m_k, ordered [c][i]."""
        return Y[k, :, : self.m_k[k]].reshape(-1)


def from_problem(prob, backend: str = "fft") -> Operator:
    """Operator for a datagen.Problem."""
    return Operator(prob.nx, prob.ny, prob.coils, omegas(prob.kind, prob.masks, prob.nx), backend)


class MatrixOperator:
    """Single-coil A_k given as explicit m x n matrices (e.g. the i.i.d.
    Gaussian A_k of the paper's guarantee, Sec. III-B).  Same interface as
    Operator, with nc = 1."""

    def __init__(self, mats):
        self.mats = [np.asarray(a, dtype=np.complex128) for a in mats]
        self.q = len(self.mats)
        self.n = self.mats[0].shape[1]
        self.nc = 1
        self.m_k = np.array([a.shape[0] for a in self.mats], dtype=np.int64)
        self.m_max = int(self.m_k.max())

    def A(self, k, x):
        return (self.mats[k] @ x)[None, :]

    def AH(self, k, v):
        return self.mats[k].conj().T @ np.asarray(v).reshape(-1)

    def transform_basis(self, U):
        return U

    def AU(self, k, U, FU=None):
        return self.mats[k] @ U

    def apply_A(self, X):
        Y = np.zeros((self.q, 1, self.m_max), dtype=np.complex128)
        for k in range(self.q):
            Y[k, 0, : self.m_k[k]] = self.mats[k] @ X[:, k]
        return Y

    def apply_AH(self, Y):
        X = np.empty((self.n, self.q), dtype=np.complex128)
        for k in range(self.q):
            X[:, k] = self.AH(k, Y[k, 0, : self.m_k[k]])
        return X

    def frame_vec(self, Y, k):
        return Y[k, :, : self.m_k[k]].reshape(-1)
