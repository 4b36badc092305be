"""FP64 restatements of the algebra a fast implementation uses (oracle).

Each function here computes, by a different route, a quantity that
``altgdmin`` computes literally; the tests check the two against each other
so that the GPU library can be compared with either.

* Hybrid (ky, x) form for fully sampled readout lines.  With every sampled
  phase-encode line complete along kx, H_k F = (S_{L_k} F_y) (x) F_x, and
  I (x) F_x is unitary on each line, so an inverse DFT along kx of the data
  (y'_k) turns every norm ||y_k - A_k U b||, and hence the LS step, the cost
  and the gradient, into the same quantities for A'_k = [(S_{L_k} F_y) D_c]_c,
  which acts on each image column x separately.
* Gram + Cholesky LS: b_k = G_k^{-1} h_k with G_k = (A_k U)^H (A_k U) and
  h_k = (A_k U)^H y_k, the definition M^dagger = (M^H M)^{-1} M^H of Sec. II-A.
* Folded gradient: the sum over frames of Algorithm 2's gradient moved
  before the inverse transform.  Per coil,
      K_c = sum_k scatter_{Omega_k}(A_{k,c} U b_k - y_{k,c}) b_k^H,
  which per k-space location i is W_c(i,:) S_i - Y_c(i,:) with
  S_i = sum_{k: i in Omega_k} b_k b_k^H and
  Y_c(i,:) = sum_{k: i in Omega_k} y_{k,c}(i) b_k^H; then
      grad = sum_c conj(s_c) o F^H K_c.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .operators import Operator, WORKERS


# ---------------------------------------------------------------------------
# hybrid (ky, x) form, 1D Cartesian masks
# ---------------------------------------------------------------------------
def hybrid_data(Y: np.ndarray, lines, nx: int) -> np.ndarray:
    """y'_{k,c}(l, x): unitary inverse DFT along kx of every sampled line.

    Y is (q, nc, m_max) with each frame ordered [c][l][kx]; the result has
    the same shape ordered [c][l][x] (padding stays zero)."""
    q, nc, m_max = Y.shape
    out = np.zeros_like(Y)
    for k in range(q):
        L = len(lines[k])
        blk = Y[k, :, : L * nx].reshape(nc, L, nx)
        out[k, :, : L * nx] = sfft.ifft(blk, axis=-1, norm="ortho", workers=WORKERS).reshape(nc, L * nx)
    return out


def hybrid_basis(U: np.ndarray, coils: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """W_{c,j}(ky, x) = F_y(s_c o u_j): unitary DFT along y only, (nc, r, ny, nx)."""
    nc, r = coils.shape[0], U.shape[1]
    imgs = (coils[:, None, :] * U.T[None, :, :]).reshape(nc, r, ny, nx)
    return sfft.fft(imgs, axis=2, norm="ortho", workers=WORKERS)


def hybrid_gram_rhs(W: np.ndarray, Yh: np.ndarray, lines, nx: int):
    """G_k = sum_{c, l, x} W_c(ky_l, x, :)^H W_c(ky_l, x, :) and
    h_k = sum_{c, l, x} conj(W_c(ky_l, x, :)) y'_{k,c}(l, x).  Returns
    G (q, r, r) and h (q, r)."""
    nc, r, ny, _ = W.shape
    q = len(lines)
    G = np.empty((q, r, r), dtype=np.complex128)
    h = np.empty((q, r), dtype=np.complex128)
    for k in range(q):
        L = len(lines[k])
        Wk = W[:, :, lines[k], :]                        # (nc, r, L, nx)
        M = np.transpose(Wk, (0, 2, 3, 1)).reshape(-1, r)  # rows [c][l][x]
        G[k] = M.conj().T @ M
        h[k] = M.conj().T @ Yh[k, :, : L * nx].reshape(-1)
    return G, h


def hybrid_gradient(W: np.ndarray, Yh: np.ndarray, B: np.ndarray, coils: np.ndarray,
                    lines, nx: int, ny: int) -> np.ndarray:
    """grad = sum_c conj(s_c) o F_y^H K_c, with K_c folded over frames per
    phase-encode line: K_c(ky, x, :) = W_c(ky, x, :) S_ky - Y_c(ky, x, :)."""
    nc, r = W.shape[0], W.shape[1]
    q = len(lines)
    S = np.zeros((ny, r, r), dtype=np.complex128)
    Yc = np.zeros((nc, ny, nx, r), dtype=np.complex128)
    for k in range(q):
        bb = np.outer(B[:, k], np.conj(B[:, k]))
        L = len(lines[k])
        yk = Yh[k, :, : L * nx].reshape(nc, L, nx)
        for l, ky in enumerate(lines[k]):
            S[ky] += bb
            Yc[:, ky, :, :] += yk[:, l, :, None] * np.conj(B[:, k])[None, None, :]
    Wt = np.transpose(W, (0, 2, 3, 1))                    # (nc, ny, nx, r)
    K = np.einsum("cyxi,yij->cyxj", Wt, S) - Yc           # (nc, ny, nx, r)
    img = sfft.ifft(K, axis=1, norm="ortho", workers=WORKERS)  # along ky -> y
    G = np.sum(np.conj(coils).reshape(nc, ny, nx)[:, :, :, None] * img, axis=0)
    return G.reshape(ny * nx, r)


# ---------------------------------------------------------------------------
# Gram + Cholesky LS (any mask)
# ---------------------------------------------------------------------------
def gram_rhs(op: Operator, U: np.ndarray, Y: np.ndarray, FU=None):
    """G_k = (A_k U)^H (A_k U), h_k = (A_k U)^H y_k for every frame."""
    if FU is None:
        FU = op.transform_basis(U)
    r = U.shape[1]
    G = np.empty((op.q, r, r), dtype=np.complex128)
    h = np.empty((op.q, r), dtype=np.complex128)
    for k in range(op.q):
        M = op.AU(k, U, FU)
        G[k] = M.conj().T @ M
        h[k] = M.conj().T @ op.frame_vec(Y, k)
    return G, h


def cholesky_solve(G: np.ndarray, h: np.ndarray) -> np.ndarray:
    """b_k = G_k^{-1} h_k via G_k = L L^H; returns B as r x q."""
    q, r, _ = G.shape
    B = np.empty((r, q), dtype=np.complex128)
    for k in range(q):
        L = np.linalg.cholesky(G[k])
        z = np.linalg.solve(L, h[k])
        B[:, k] = np.linalg.solve(L.conj().T, z)
    return B


def min_cost(op: Operator, U: np.ndarray, Y: np.ndarray) -> float:
    """f(U) = min_B f(U, B) = sum_k (||y_k||^2 - h_k^H G_k^{-1} h_k)."""
    G, h = gram_rhs(op, U, Y)
    B = cholesky_solve(G, h)
    ysq = float(np.sum(np.abs(Y) ** 2))
    return ysq - float(np.sum(np.einsum("kr,rk->k", h.conj(), B)).real)


# ---------------------------------------------------------------------------
# folded gradient (any mask)
# ---------------------------------------------------------------------------
def folded_gradient(op: Operator, U: np.ndarray, B: np.ndarray, Y: np.ndarray, FU=None) -> np.ndarray:
    """grad = sum_c conj(s_c) o F^H K_c with K_c(i,:) = W_c(i,:) S_i - Y_c(i,:),
    where W_c = F(s_c o U) per column; nc*r inverse transforms in total."""
    if FU is None:
        FU = op.transform_basis(U)                          # (nc, r, n)
    r = U.shape[1]
    S = np.zeros((op.n, r, r), dtype=np.complex128)
    Yc = np.zeros((op.nc, op.n, r), dtype=np.complex128)
    for k in range(op.q):
        om = op.omegas[k]
        S[om] += np.outer(B[:, k], np.conj(B[:, k]))[None, :, :]
        yk = Y[k, :, : op.m_k[k]]                           # (nc, m_k)
        Yc[:, om, :] += yk[:, :, None] * np.conj(B[:, k])[None, None, :]
    Wt = np.transpose(FU, (0, 2, 1))                        # (nc, n, r)
    K = np.einsum("cni,nij->cnj", Wt, S) - Yc               # (nc, n, r)
    grad = np.zeros((op.n, r), dtype=np.complex128)
    for j in range(r):
        grad[:, j] = np.sum(np.conj(op.coils) * op.F.adj(K[:, :, j]), axis=0)
    return grad


# ---------------------------------------------------------------------------
# closed forms for the QR step
# ---------------------------------------------------------------------------
def qr_closed_form(U: np.ndarray, grad: np.ndarray, eta: float):
    """With U^H U = I and U^H grad = 0: Uhat^H Uhat = I + eta^2 grad^H grad,
    R = chol(I + eta^2 grad^H grad) (upper), U+ = Uhat R^{-1}, and
    SD(U, U+)^2 = sum_i eta^2 s_i^2 / (1 + eta^2 s_i^2), s_i = sv(grad)."""
    r = U.shape[1]
    Gm = np.eye(r) + eta ** 2 * (grad.conj().T @ grad)
    R = np.linalg.cholesky(Gm).conj().T
    Uplus = np.linalg.solve(R.T, (U - eta * grad).T).T
    s = np.linalg.svd(grad, compute_uv=False)
    sd2 = float(np.sum(eta ** 2 * s ** 2 / (1.0 + eta ** 2 * s ** 2)))
    return Uplus, R, sd2
