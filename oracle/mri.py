"""altGDmin-MRI around the altGDmin loop (oracle, test infrastructure).

The paper's full method (Algorithm 1, Sec. III-A) wraps auto-altGDmin
(Algorithm 2) in a mean-image step before it and a modelling-error
correction (MEC, Sec. III-C, Algorithm 3) after it, and Sec. IV runs the
whole thing over mini-batches (Algorithm 4) or frame by frame (Algorithm 5).
Everything here is complex128 and literal, frame by frame; the linear
operators are the oracle's own A_k (``operators.Operator``).

* ``cgls``        -- conjugate gradients for least squares (the textbook
                     residual form), with a relative stopping rule on the
                     normal-equation residual;
* ``mean_image``  -- Algorithm 1, step 1: zbar = argmin sum_k ||y_k - A_k z||^2
                     by CGLS (tolerance 1e-3, at most 10 iterations);
* ``residual``    -- y_k - A_k (zbar + x_k) (Algorithm 1, steps 2a and 3a);
* ``auto_rank``   -- Algorithm 2's rank rule (b = 85 % of the energy of the
                     first min(n, q, nc min_k m_k)/10 singular values of X_0);
* ``mec1``        -- Algorithm 3, model 1: 3 CGLS iterations per frame from 0;
* ``mec2``        -- Algorithm 3, model 2: ISTA with a complex soft threshold
                     on the temporal DFT of the error;
* ``altgdmin_mri`` -- Algorithm 1 end to end;
* ``minibatch_st`` / ``online_st`` -- Algorithms 4 and 5.

Readings where the paper is silent or garbled are stated at each function.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import altgdmin as AG
from .operators import Operator


def _inner(a: np.ndarray, b: np.ndarray) -> float:
    """Re <a, b> over all entries."""
    return float(np.vdot(a, b).real)


# ---------------------------------------------------------------------------
# CGLS
# ---------------------------------------------------------------------------
def cgls(A: Callable, AH: Callable, y: np.ndarray, x0: np.ndarray, tol: float, maxit: int):
    """min_x ||y - A x||^2 by conjugate gradients in the residual form
    (CGLS: CG applied to A^H A x = A^H y without forming A^H A).

    From x_0: r = y - A x, s = A^H r, p = s, gamma = ||s||^2; each
    iteration takes q = A p, alpha = gamma / ||q||^2, x += alpha p,
    r -= alpha q, s = A^H r, gamma' = ||s||^2, p = s + (gamma'/gamma) p.
    Stopping rule (the paper gives only "tolerance" and a maximum count;
    reading): stop after the iteration at which ||s|| <= tol ||s_0||, or
    after maxit iterations, or when A p = 0 (exact solution reached).
    Returns (x, iterations done)."""
    x = x0.copy()
    r = y - A(x)
    s = AH(r)
    p = s.copy()
    gamma = _inner(s, s)
    norm_s0 = np.sqrt(gamma)
    done = 0
    for _ in range(maxit):
        if gamma == 0.0:
            break
        q = A(p)
        delta = _inner(q, q)
        if delta == 0.0:
            break
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        s = AH(r)
        gamma_new = _inner(s, s)
        done += 1
        if np.sqrt(gamma_new) <= tol * norm_s0:
            break
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
    return x, done


# ---------------------------------------------------------------------------
# Algorithm 1, steps 1 and 2a / 3a
# ---------------------------------------------------------------------------
def mean_image(op: Operator, Y: np.ndarray, tol: float = 1e-3, maxit: int = 10):
    """zbar = argmin_z sum_k ||y_k - A_k z||^2 by CGLS from z = 0
    (Algorithm 1, step 1: tolerance 1e-3, at most 10 iterations).
    The operator stacks every frame's A_k on the one image z:
    z -> [A_1 z; ...; A_q z] (the padded measurement array), and its
    adjoint v -> sum_k A_k^H v_k.  Returns (zbar, iterations)."""
    def A(z):
        return op.apply_A(np.repeat(z[:, None], op.q, axis=1))

    def AH(v):
        return op.apply_AH(v).sum(axis=1)

    return cgls(A, AH, Y, np.zeros(op.n, dtype=np.complex128), tol, maxit)


def residual(op: Operator, Y: np.ndarray, zbar: Optional[np.ndarray] = None,
             X: Optional[np.ndarray] = None) -> np.ndarray:
    """y_k - A_k (zbar + x_k) for every frame, in the padded form
    (Algorithm 1: step 2a with X = 0, step 3a with X the altGDmin output)."""
    Z = np.zeros((op.n, op.q), dtype=np.complex128)
    if zbar is not None:
        Z += zbar[:, None]
    if X is not None:
        Z += X
    return Y - op.apply_A(Z)


# ---------------------------------------------------------------------------
# Algorithm 2's parameter setting: the rank
# ---------------------------------------------------------------------------
def rank_cap(op: Operator) -> int:
    """floor(min(n, q, nc min_k m_k) / 10), at least 1.  Reading: the
    paper's "mc min_k m_k" is the number of measurements of the smallest
    frame over all coils; the bound is rounded down."""
    return max(1, int(min(op.n, op.q, op.nc * int(np.min(op.m_k))) // 10))


def auto_rank(X0: np.ndarray, r_cap: int, b: float = 85.0) -> int:
    """The smallest r with sum_{j<=r} sigma_j^2 >= (b/100) sum_{j<=r_cap}
    sigma_j^2, sigma_j the singular values of X_0 (Algorithm 2; the
    garbled upper limit of the left sum is read as r)."""
    s2 = np.linalg.svd(X0, compute_uv=False)[:r_cap] ** 2
    target = (b / 100.0) * float(np.sum(s2))
    acc = 0.0
    for j, v in enumerate(s2):
        acc += float(v)
        if acc >= target:
            return j + 1
    return r_cap


# ---------------------------------------------------------------------------
# Algorithm 3: modelling-error correction
# ---------------------------------------------------------------------------
def mec1(op: Operator, Yres: np.ndarray, iters: int = 3, tol: float = 1e-36) -> np.ndarray:
    """Model 1 (no structure on E): for each frame, `iters` CGLS iterations
    from e = 0 on min_e ||yres_k - A_k e||^2 (Algorithm 3; Sec. III-C:
    tolerance 1e-36, 3 iterations).  Returns E (n x q)."""
    E = np.zeros((op.n, op.q), dtype=np.complex128)
    for k in range(op.q):
        yk = Yres[k, :, : op.m_k[k]]
        e, _ = cgls(lambda v, k=k: op.A(k, v), lambda w, k=k: op.AH(k, w), yk,
                    np.zeros(op.n, dtype=np.complex128), tol, iters)
        E[:, k] = e
    return E


def temporal_dft(E: np.ndarray) -> np.ndarray:
    """The unitary 1D DFT of every row of an n x q matrix (along the frames).
    Reading: the normalisation of this DFT cannot change the MEC-2 output,
    because the threshold is set relative to the largest coefficient."""
    q = E.shape[1]
    k = np.arange(q)
    F = np.exp(-2j * np.pi * np.outer(k, k) / q) / np.sqrt(q)
    return E @ F.T


def temporal_idft(S: np.ndarray) -> np.ndarray:
    q = S.shape[1]
    k = np.arange(q)
    F = np.exp(-2j * np.pi * np.outer(k, k) / q) / np.sqrt(q)
    return S @ F.conj()


def soft_threshold(S: np.ndarray, omega: float) -> np.ndarray:
    """Complex soft threshold: s/|s| (|s| - omega) where |s| > omega, else 0
    (Sec. III-C; sign(s) read as s/|s| for complex entries)."""
    mag = np.abs(S)
    out = np.zeros_like(S)
    big = mag > omega
    out[big] = S[big] / mag[big] * (mag[big] - omega)
    return out


@dataclass
class IstaResult:
    E: np.ndarray
    iters: int                  # threshold updates done
    omega: float
    changes: list = field(default_factory=list)  # ||M_t - M_{t-1}|| / ||M_{t-1}||


def mec2(op: Operator, Yres: np.ndarray, max_iter: int = 10, omega_frac: float = 1e-3,
         tol: float = 0.0025) -> IstaResult:
    """Model 2 (E sparse along time in the Fourier domain): ISTA
    (Algorithm 3).  From E_0 = 0, for t = 0, 1, ...:
        M_t     = F_t(E_t + A^H(Yres - A(E_t)))      (F_t: DFT along frames)
        omega   = omega_frac * max |M_0|               (t = 0 only)
        E_{t+1} = F_t^{-1}(SThr_omega(M_t)).
    Reading of the garbled loop: each update uses the M just computed; the
    loop ends after max_iter updates, or after the update that follows an M_t
    (t >= 1) with ||M_t - M_{t-1}||_F / ||M_{t-1}||_F < tol."""
    E = np.zeros((op.n, op.q), dtype=np.complex128)
    M_prev = None
    omega = 0.0
    res = IstaResult(E=E, iters=0, omega=0.0)
    for t in range(max_iter):
        V = E + op.apply_AH(Yres - op.apply_A(E))
        M = temporal_dft(V)
        if t == 0:
            omega = omega_frac * float(np.max(np.abs(M)))
        stop = False
        if M_prev is not None:
            ch = float(np.linalg.norm(M - M_prev) / np.linalg.norm(M_prev))
            res.changes.append(ch)
            stop = ch < tol
        E = temporal_idft(soft_threshold(M, omega))
        res.iters = t + 1
        M_prev = M
        if stop:
            break
    res.E, res.omega = E, omega
    return res


# ---------------------------------------------------------------------------
# Algorithm 1 end to end
# ---------------------------------------------------------------------------
@dataclass
class MriResult:
    Z: np.ndarray            # zbar 1^T + X + E
    zbar: np.ndarray
    X: np.ndarray
    E: np.ndarray
    U: np.ndarray            # the final basis of the altGDmin step
    r: int
    mean_iters: int
    gd: AG.Result
    mec_iters: int = 0


def altgdmin_mri(op: Operator, Y: np.ndarray, params: AG.Params, mec: Optional[int] = 1,
                 auto: bool = False, U0: Optional[np.ndarray] = None, t_fixed: Optional[int] = None,
                 Zstar: Optional[np.ndarray] = None) -> MriResult:
    """Algorithm 1: zbar by CGLS; ytilde_k = y_k - A_k zbar; auto-altGDmin on
    ytilde (rank params.r, or the automatic rank when auto); the second
    residual; MEC model 1 or 2 (mec = None: no correction).  U0 replaces
    the initialisation (Algorithm 4's warm start)."""
    zbar, mit = mean_image(op, Y)
    Yt = residual(op, Y, zbar)
    prm = params
    if auto and U0 is None:
        Ytr, _, _ = AG.truncation(op, Yt, params.trunc_c)
        r = auto_rank(AG.backprojection(op, Ytr), rank_cap(op))
        prm = AG.Params(**{**params.__dict__, "r": r})
    gd = AG.run(op, Yt, prm, U0=U0, t_fixed=t_fixed,
                Zstar=None if Zstar is None else Zstar - zbar[:, None], record=Zstar is not None)
    X = gd.X
    E = np.zeros_like(X)
    mec_iters = 0
    if mec is not None:
        Ytt = residual(op, Yt, X=X)
        if mec == 1:
            E = mec1(op, Ytt)
            mec_iters = 3
        else:
            ir = mec2(op, Ytt)
            E, mec_iters = ir.E, ir.iters
    return MriResult(Z=zbar[:, None] + X + E, zbar=zbar, X=X, E=E, U=gd.U, r=prm.r, mean_iters=mit, gd=gd,
                     mec_iters=mec_iters)


# ---------------------------------------------------------------------------
# Sec. IV: subspace tracking
# ---------------------------------------------------------------------------
def sub_operator(op: Operator, frames) -> Operator:
    """The operator of a subset of the frames (same coils and grid)."""
    return Operator(op.nx, op.ny, op.coils, [op.omegas[k] for k in frames],
                    "dense" if op.F.backend == "dense" else "fft")


def minibatch_st(op: Operator, Y: np.ndarray, params: AG.Params, alpha: int, mec: int = 1,
                 t_first: int = 70, t_next: int = 5) -> np.ndarray:
    """Algorithm 4: Algorithm 1 on consecutive mini-batches of alpha frames;
    the first with its own initialisation and T_max = 70, every later one
    starting from the previous batch's final basis (U_0 <- U^(j-1), which
    replaces Algorithm 2's initialisation) with T_max = 5.  The batches run
    their iterations to T_max (the exit rule, if enabled in params, still
    ends a batch early).  Returns Z (n x q)."""
    Z = np.zeros((op.n, op.q), dtype=np.complex128)
    U = None
    for j0 in range(0, op.q, alpha):
        frames = list(range(j0, min(op.q, j0 + alpha)))
        sop = sub_operator(op, frames)
        Yj = Y[frames][:, :, : sop.m_max]
        T = t_first if U is None else t_next
        prm = AG.Params(**{**params.__dict__, "t_max": T})
        res = altgdmin_mri(sop, Yj, prm, mec=mec, U0=U)
        Z[:, frames] = res.Z
        U = res.U
    return Z


def online_st(op: Operator, Y: np.ndarray, params: AG.Params, alpha: int) -> np.ndarray:
    """Algorithm 5: Algorithm 1 (MEC model 1) on the first alpha frames; for
    every later frame k (the garbled "k > alpha + 1" read as k > alpha), with
    the first batch's zbar and U fixed: ytilde_k = y_k - A_k zbar,
    b_k = (A_k U)^dagger ytilde_k, the second residual, e_k by 3 CGLS
    iterations, x_k = zbar + U b_k + e_k."""
    first = list(range(min(alpha, op.q)))
    sop = sub_operator(op, first)
    res = altgdmin_mri(sop, Y[first][:, :, : sop.m_max], params, mec=1)
    Z = np.zeros((op.n, op.q), dtype=np.complex128)
    Z[:, first] = res.Z
    zbar, U = res.zbar, res.U
    FU = op.transform_basis(U)
    for k in range(len(first), op.q):
        yk = Y[k, :, : op.m_k[k]].reshape(-1)
        ytk = yk - op.A(k, zbar).reshape(-1)
        M = op.AU(k, U, FU)
        b = np.linalg.lstsq(M, ytk, rcond=None)[0]
        ytt = (ytk - M @ b).reshape(op.nc, op.m_k[k])
        e, _ = cgls(lambda v, k=k: op.A(k, v), lambda w, k=k: op.AH(k, w), ytt,
                    np.zeros(op.n, dtype=np.complex128), 1e-36, 3)
        Z[:, k] = zbar + U @ b + e
    return Z
