"""auto-altGDmin with a fixed rank (oracle, test infrastructure).

Follows Algorithm 2 of the paper (auto-altGDmin) and Sec. III-B, with the
rank r given (the automatic-rank rule is not used), fed the measurements
directly (y~_k = y_k, the setting of the paper's guarantee in Sec. III-B).
Steps, in the paper's order:

1. truncation threshold gamma and the truncated measurements;
2. scaled back-projection X_0 = [A_k^H y_{k,trnc} / sqrt(m_k mbar)]_k;
3. U_0 = top-r left singular vectors of X_0;
4. loop: b_k = (A_k U)^dagger y_k, x_k = U b_k,
   grad = sum_k A_k^H (A_k U b_k - y_k) b_k^H, eta at t = 1,
   U^+ = U - eta grad, QR, exit rule.

Everything is complex128 and literal: the LS step calls lstsq per frame, the
gradient is summed frame by frame with nc inverse transforms per frame, and
the QR is LAPACK's.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .operators import Operator
from . import metrics


@dataclass
class Params:
    """Algorithm 2's constants (the ones printed in blue in the paper)."""
    r: int
    t_max: int = 70
    trunc_c: float = 36.0      # gamma = trunc_c * sum |y|^2 / (m q); <= 0 disables truncation
    eta_c: float = 0.14        # eta = eta_c / ||grad_0||
    eta_cap_c: float = 0.0     # > 0: cap eta by eta_cap_c * n / (mbar ||B_0||^2)
    eps_exit: float = 0.0      # > 0: exit when SD(U, U+)/sqrt(r) < eps_exit (paper: 0.01)
    exit_consec: int = 1       # exit after this many consecutive small steps (Sec. VI variant: > 1)


@dataclass
class Result:
    U: np.ndarray               # U_T
    U_prev: np.ndarray          # U_{T-1}
    B: np.ndarray               # B_T, computed from U_{T-1}
    eta: float
    iters: int
    U0: np.ndarray
    gamma: float
    trunc_frac: float
    history: dict = field(default_factory=dict)

    @property
    def X(self) -> np.ndarray:
        """X_T = U_{T-1} B_T (the output after the loop, Algorithm 2)."""
        return self.U_prev @ self.B


# ---------------------------------------------------------------------------
# initialisation
# ---------------------------------------------------------------------------
def truncation(op: Operator, Y: np.ndarray, trunc_c: float):
    """gamma = trunc_c * sum_{i,k} |y_ik|^2 / (m q) and y o 1{|y| <= sqrt(gamma)}.

    Algorithm 2, initialisation; m = max_k m_k (Sec. II-A, the padded Y).
    Reading: the sum runs over every coil and sample of every frame while m
    counts samples per coil, as written; the test is inclusive and on the
    complex modulus.  trunc_c <= 0 disables truncation.
    Returns (y_trnc, gamma, fraction of valid samples removed).
    """
    if trunc_c <= 0:
        return Y.copy(), np.inf, 0.0
    total = float(np.sum(np.abs(Y) ** 2))
    gamma = trunc_c * total / (op.m_max * op.q)
    keep = np.abs(Y) <= np.sqrt(gamma)
    valid = np.arange(Y.shape[2])[None, None, :] < op.m_k[:, None, None]
    valid = np.broadcast_to(valid, Y.shape)
    removed = np.count_nonzero(valid & ~keep) / max(np.count_nonzero(valid), 1)
    return np.where(keep, Y, 0.0), gamma, removed


def truncation_count(op: Operator, Y: np.ndarray, trunc_c: float) -> int:
    """The number of valid samples (every frame and coil) that the
    truncation of Algorithm 2 zeroes."""
    if trunc_c <= 0:
        return 0
    _, gamma, _ = truncation(op, Y, trunc_c)
    valid = np.arange(Y.shape[2])[None, None, :] < op.m_k[:, None, None]
    return int(np.count_nonzero(np.broadcast_to(valid, Y.shape) & (np.abs(Y) > np.sqrt(gamma))))


def backprojection(op: Operator, Ytrnc: np.ndarray) -> np.ndarray:
    """X_0 = [A_k^H y_{k,trnc} / sqrt(m_k mbar)]_k with mbar = sum_k m_k / q.

    Algorithm 2, initialisation, and the remark in Sec. III-B that replaces
    1/m by 1/sqrt(m_k mbar) for time-varying m_k.
    """
    mbar = float(np.sum(op.m_k)) / op.q
    X0 = op.apply_AH(Ytrnc)
    return X0 / np.sqrt(op.m_k.astype(np.float64) * mbar)[None, :]


def spectral_init(X0: np.ndarray, r: int) -> np.ndarray:
    """U_0 = the top-r left singular vectors of X_0 (Algorithm 2)."""
    u, _, _ = np.linalg.svd(X0, full_matrices=False)
    return u[:, :r].copy()


# ---------------------------------------------------------------------------
# one iteration's pieces
# ---------------------------------------------------------------------------
def ls_step(op: Operator, U: np.ndarray, Y: np.ndarray, FU=None) -> np.ndarray:
    """b_k = (A_k U)^dagger y_k for every frame (Algorithm 2; M^dagger of
    Sec. II-A), by lstsq.  Returns B as r x q."""
    if FU is None:
        FU = op.transform_basis(U)
    r = U.shape[1]
    B = np.empty((r, op.q), dtype=np.complex128)
    for k in range(op.q):
        M = op.AU(k, U, FU)
        B[:, k] = np.linalg.lstsq(M, op.frame_vec(Y, k), rcond=None)[0]
    return B


def cost(op: Operator, U: np.ndarray, B: np.ndarray, Y: np.ndarray, FU=None) -> float:
    """f(U, B) = sum_k ||y_k - A_k U b_k||^2 (Sec. III-B)."""
    if FU is None:
        FU = op.transform_basis(U)
    f = 0.0
    for k in range(op.q):
        res = op.frame_vec(Y, k) - op.AU(k, U, FU) @ B[:, k]
        f += float(np.vdot(res, res).real)
    return f


def gradient(op: Operator, U: np.ndarray, B: np.ndarray, Y: np.ndarray, FU=None) -> np.ndarray:
    """grad_U f = sum_k A_k^H (A_k U b_k - y_k) b_k^H (Algorithm 2).

    Literal: each frame's residual goes through its own adjoint (nc inverse
    transforms per frame).  This is the Wirtinger derivative df/d(conj U):
    d/de f(U + e D) at e = 0 equals 2 Re tr(grad^H D).
    """
    if FU is None:
        FU = op.transform_basis(U)
    G = np.zeros_like(U)
    for k in range(op.q):
        M = op.AU(k, U, FU)
        res = (M @ B[:, k] - op.frame_vec(Y, k)).reshape(op.nc, op.m_k[k])
        G += np.outer(op.AH(k, res), np.conj(B[:, k]))
    return G


def step_size(grad0: np.ndarray, eta_c: float) -> float:
    """eta = eta_c / ||grad_U f(U_0, B_0)|| (Algorithm 2, Sec. III-B).

    The paper's norm without subscript is the induced l2 (spectral) norm.
    """
    return eta_c / np.linalg.norm(grad0, 2)


def step_size_cap(op, B0: np.ndarray, cap_c: float) -> float:
    """The conservative step size eta = c / (m ||U_0 B_0||^2) of Sec. III-B
    (parameter setting), used only as an upper bound on Algorithm 2's eta.

    Reading: with a unitary F and sum_c |s_c|^2 = 1, E[A_k^H A_k] = (m_k/n) I,
    so the paper's m (for unnormalised Gaussian A_k) becomes mbar/n here;
    ||U_0 B_0||_2 = ||B_0||_2 for an orthonormal U_0 (spectral norm).
    """
    mbar = float(np.sum(op.m_k)) / op.q
    return cap_c * op.n / (mbar * float(np.linalg.norm(B0, 2)) ** 2)


def qr_project(Uhat: np.ndarray) -> np.ndarray:
    """U^+ = Q of the QR decomposition of U-hat (Algorithm 2)."""
    q_, _ = np.linalg.qr(Uhat)
    return q_


# ---------------------------------------------------------------------------
# the whole algorithm
# ---------------------------------------------------------------------------
def run(op: Operator, Y: np.ndarray, params: Params, U0: Optional[np.ndarray] = None,
        Zstar: Optional[np.ndarray] = None, Ustar: Optional[np.ndarray] = None,
        t_fixed: Optional[int] = None, eta: Optional[float] = None,
        record: bool = True) -> Result:
    """auto-altGDmin with fixed rank r (Algorithm 2).

    U0: a given initial basis (warm start); otherwise the truncated spectral
    initialisation.  t_fixed: run exactly this many iterations (the exit rule
    is still evaluated and its firing iteration recorded).  eta: a given step
    size (resume); otherwise set at t = 1.

    Guard (reading; the paper does not say what happens when grad_0 = 0):
    if ||grad_0|| <= 1e-12 * sum_k ||y_k||^2 the starting point is already
    stationary; no step is taken and iters = 0.
    """
    r = params.r
    hist = {k: [] for k in ("f", "sd", "grad_norm", "nmse", "nsmse", "sd_star")}
    Ytr, gamma, frac = truncation(op, Y, params.trunc_c)
    if U0 is None:
        X0 = backprojection(op, Ytr)
        U0 = spectral_init(X0, r)
    U = U0.copy()
    U_prev = U.copy()
    B = None
    T = params.t_max if t_fixed is None else t_fixed
    ysq = float(np.sum(np.abs(Y) ** 2))
    iters = 0
    run_small = 0
    hist["exit_at"] = None
    for t in range(1, T + 1):
        FU = op.transform_basis(U)
        B = ls_step(op, U, Y, FU)
        U_prev = U
        G = gradient(op, U, B, Y, FU)
        gnorm = float(np.linalg.norm(G, 2))
        if eta is None:
            if gnorm <= 1e-12 * ysq:
                hist["converged_at_start"] = True
                iters = 0
                break
            eta = step_size(G, params.eta_c)
            if params.eta_cap_c > 0:
                cap = step_size_cap(op, B, params.eta_cap_c)
                hist["eta_capped"] = bool(cap < eta)
                eta = min(eta, cap)
        Uplus = qr_project(U - eta * G)
        sd = metrics.subspace_distance(U, Uplus)
        if record:
            hist["f"].append(cost(op, U, B, Y, FU))
            hist["sd"].append(sd)
            hist["grad_norm"].append(gnorm)
            if Zstar is not None:
                X = U @ B
                hist["nmse"].append(metrics.nmse(X, Zstar))
                hist["nsmse"].append(metrics.nsmse(X, Zstar))
            if Ustar is not None:
                hist["sd_star"].append(metrics.subspace_distance(Ustar, Uplus))
        iters = t
        U = Uplus
        # exit rule (Algorithm 2); with exit_consec > 1 the variant of Sec. VI
        # that asks for several consecutive small steps
        run_small = run_small + 1 if (params.eps_exit > 0 and sd / np.sqrt(r) < params.eps_exit) else 0
        if params.eps_exit > 0 and run_small >= max(1, params.exit_consec):
            if hist["exit_at"] is None:
                hist["exit_at"] = t
            if t_fixed is None:
                break
    if B is None:
        B = ls_step(op, U, Y)
    return Result(U=U, U_prev=U_prev, B=B, eta=(eta if eta is not None else 0.0),
                  iters=iters, U0=U0, gamma=gamma, trunc_frac=frac, history=hist)
