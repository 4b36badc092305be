"""altGDmin-MRI end to end on the device: the method's full pipeline
(Algorithm 1: mean image, residual, auto-altGDmin, second residual, MEC) and
the subspace-tracking drivers of Sec. IV (Algorithm 4: mini-batches with a
warm-started basis; Algorithm 5: frame-by-frame online reconstruction).

These functions only sequence calls of the C ABI (include/altgdmin.h): every
arithmetic step runs in the library's kernels; PyTorch only holds the device
buffers.  Images are (q, n) complex64 tensors (frame k is row k, pixel
p = x + nx*y); measurements use the library's padded layout (q, nc, m_max).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from ._lib import AltGDmin, MASK_LINES, FP32


@dataclass
class MriOutput:
    Z: torch.Tensor          # (q, n): zbar + U b_k + e_k
    zbar: torch.Tensor       # (n,)
    U: torch.Tensor          # (r, n): the final basis U_T
    U_prev: torch.Tensor     # (r, n): U_{T-1}, with which X_T = U_{T-1} B_T
    B: torch.Tensor          # (q, r)
    E: Optional[torch.Tensor]
    r: int
    mean_iters: int
    mec_iters: int


def _bind(ctx: AltGDmin, coils, mask, m_k, y):
    ws = ctx._keep[4] if ctx._keep else None
    ctx.set_problem(coils, mask, m_k, y, workspace=ws)


def altgdmin_mri(coils, mask, m_k, y, nx, ny, r, mask_kind=MASK_LINES, precision=FP32, mec: Optional[int] = 1,
                 auto_rank: bool = False, T: Optional[int] = None, U0=None, trunc_c=36.0, eps_exit=0.0,
                 exit_consec=1, mean_tol=1e-3, mean_maxit=10, b_percent=85.0) -> MriOutput:
    """Algorithm 1 on one sequence.

    mean image zbar by CG on the normal equations (tolerance mean_tol, at most
    mean_maxit iterations); ytilde = y - A(zbar 1^T); auto-altGDmin on ytilde
    (rank r, or Algorithm 2's automatic rank when auto_rank; the spectral
    initialisation, or the warm start U0 of Algorithm 4); the second residual
    ytilde - A(X); MEC model 1 (3 CGLS iterations per frame) or 2 (ISTA), or
    none (mec = None); Z = zbar 1^T + X + E.  T: iterations (default t_max =
    70, with Algorithm 2's exit rule when eps_exit > 0)."""
    q, nc, m_max = y.shape
    t_max = 70 if T is None else T
    ctx = AltGDmin(nx, ny, nc, q, r, m_max, mask_kind, precision, trunc_c=trunc_c, eps_exit=eps_exit,
                   t_max=t_max, exit_consec=exit_consec)
    _bind(ctx, coils, mask, m_k, y)
    zbar, mean_iters = ctx.mean(mean_tol, mean_maxit, sync=True)
    yt = ctx.residual(zbar=zbar)
    _bind(ctx, coils, mask, m_k, yt)
    if auto_rank and U0 is None:
        rr, _ = ctx.auto_rank(b_percent)
        if rr != r:
            r = rr
            ctx = AltGDmin(nx, ny, nc, q, r, m_max, mask_kind, precision, trunc_c=trunc_c, eps_exit=eps_exit,
                           t_max=t_max, exit_consec=exit_consec)
            _bind(ctx, coils, mask, m_k, yt)
    if U0 is None:
        U = ctx.init()
    else:
        U = ctx.init_from(U0.contiguous().clone())
    Up = torch.empty_like(U)
    B = ctx.iterate(t_max, U, U_prev=Up)
    E = None
    mec_iters = 0
    if mec is not None:
        X = ctx.expand(Up, B)
        ytt = ctx.residual(X=X)          # ytilde - A(X): ytilde is what ctx holds
        if mec == 1:
            E = ctx.mec_cgls(ytt, 3, 1e-36)
            mec_iters = 3
        else:
            E, mec_iters = ctx.mec_ista(ytt, 10, 1e-3, 0.0025, sync=True)
    Z = ctx.expand(Up, B, zbar, E)
    return MriOutput(Z=Z, zbar=zbar, U=U, U_prev=Up, B=B, E=E, r=r, mean_iters=mean_iters, mec_iters=mec_iters)


def _frames(mask, m_k, y, k0, k1):
    return mask[k0:k1].contiguous(), m_k[k0:k1].contiguous(), y[k0:k1].contiguous()


def minibatch_st(coils, mask, m_k, y, nx, ny, r, alpha, mask_kind=MASK_LINES, mec=1, t_first=70, t_next=5,
                 **kw) -> torch.Tensor:
    """Algorithm 4: Algorithm 1 on consecutive mini-batches of alpha frames;
    the first with its own initialisation and T = t_first, each later one
    from the previous batch's final basis with T = t_next.  Returns Z (q, n)."""
    q = y.shape[0]
    n = nx * ny
    Z = torch.empty(q, n, dtype=torch.complex64, device=y.device)
    U = None
    for k0 in range(0, q, alpha):
        k1 = min(q, k0 + alpha)
        mk, mkk, yk = _frames(mask, m_k, y, k0, k1)
        T = t_first if U is None else t_next
        out = altgdmin_mri(coils, mk, mkk, yk, nx, ny, r, mask_kind=mask_kind, mec=mec, T=T, U0=U, **kw)
        Z[k0:k1] = out.Z
        U = out.U
    return Z


def online_st(coils, mask, m_k, y, nx, ny, r, alpha, mask_kind=MASK_LINES, **kw) -> torch.Tensor:
    """Algorithm 5: Algorithm 1 with MEC model 1 on the first alpha frames;
    then, frame by frame with the first batch's zbar and U fixed:
    ytilde_k = y_k - A_k zbar, b_k = (A_k U)^dagger ytilde_k, the residual
    ytilde_k - A_k U b_k, e_k by 3 CGLS iterations, z_k = zbar + U b_k + e_k.
    Each later frame runs on a one-frame context (rank r > q = 1 is allowed
    for the LS step).  Returns Z (q, n)."""
    q, nc, m_max = y.shape
    n = nx * ny
    first = altgdmin_mri(coils, mask[:alpha].contiguous(), m_k[:alpha].contiguous(), y[:alpha].contiguous(),
                         nx, ny, r, mask_kind=mask_kind, mec=1, **kw)
    Z = torch.empty(q, n, dtype=torch.complex64, device=y.device)
    Z[:alpha] = first.Z
    zbar, U = first.zbar, first.U
    one = AltGDmin(nx, ny, nc, 1, r, m_max, mask_kind, FP32)
    for k in range(alpha, q):
        mk, mkk, yk = _frames(mask, m_k, y, k, k + 1)
        _bind(one, coils, mk, mkk, yk)
        yt = one.residual(zbar=zbar)
        _bind(one, coils, mk, mkk, yt)
        b = one.ls(U)
        ytt = one.residual(X=one.expand(U, b))
        e = one.mec_cgls(ytt, 3, 1e-36)
        Z[k:k + 1] = one.expand(U, b, zbar, e)
    return Z
