"""Shared set-up for the GPU parity tests: one problem, its inputs rounded to
complex64 for both sides, and the oracle evaluated on the rounded inputs."""
from __future__ import annotations

import sys

import numpy as np

import datagen
from oracle import operators as O

GPU_OK = False
try:
    import torch
    GPU_OK = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Case:
    """Inputs for one problem.  y comes from the oracle's FP64 operator
    (plus seeded noise), is rounded to complex64, and the oracle then uses
    the rounded y, coils and masks, so both sides see identical inputs."""

    def __init__(self, prob: datagen.Problem):
        self.prob = prob
        coils64 = prob.coils.astype(np.complex64)
        self.coils = coils64.astype(np.complex128)
        op_exact = O.Operator(prob.nx, prob.ny, self.coils, O.omegas(prob.kind, prob.masks, prob.nx))
        y = datagen.add_noise(op_exact.apply_A(prob.zstar), prob.noise, op_exact.m_k, prob.snr_db)
        self.y32 = y.astype(np.complex64)
        self.y = self.y32.astype(np.complex128)
        self.op = op_exact
        self.mask = prob.mask_array()
        self.m_k = prob.m_k()

    @property
    def kind_code(self):
        return 0 if self.prob.kind == "lines" else 1

    def gpu_ctx(self, precision=0, trunc_c=36.0, eta_cap_c=0.0, eps_exit=0.0, t_max=70):
        import paper_2212_09664_amd as ag
        p = self.prob
        ctx = ag.AltGDmin(p.nx, p.ny, p.nc, p.q, p.r, int(self.y.shape[2]), self.kind_code, precision,
                          trunc_c=trunc_c, eta_cap_c=eta_cap_c, eps_exit=eps_exit, t_max=t_max)
        dev = torch.device("cuda:0")
        ctx.set_problem(torch.from_numpy(self.coils.astype(np.complex64)).to(dev),
                        torch.from_numpy(self.mask).to(dev), torch.from_numpy(self.m_k).to(dev),
                        torch.from_numpy(self.y32).to(dev))
        return ctx


def to_gpu_U(U: np.ndarray):
    """n x r numpy -> (r, n) complex64 device tensor."""
    return torch.from_numpy(np.ascontiguousarray(U.T.astype(np.complex64))).to("cuda:0")


def from_gpu_U(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128).T


def from_gpu_B(t) -> np.ndarray:
    """(q, r) device tensor -> r x q numpy."""
    return t.detach().cpu().numpy().astype(np.complex128).T


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def proj_dist(U1, U2) -> float:
    """||P1 - P2||_F for the projectors onto span(U1), span(U2) (equal rank),
    as sqrt(2) ||(I - P1) Q2||_F after re-orthonormalising both bases in
    FP64 (no cancellation, unlike 2r - 2||U1^H U2||_F^2)."""
    Q1, _ = np.linalg.qr(U1.astype(np.complex128))
    Q2, _ = np.linalg.qr(U2.astype(np.complex128))
    return float(np.sqrt(2.0) * np.linalg.norm(Q2 - Q1 @ (Q1.conj().T @ Q2)))
