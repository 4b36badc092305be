"""Property checks shared by the oracle pin tests and the planted-mistake
tests.  Each returns a relative error; the pins assert it is at rounding
level, the planted-mistake tests assert it is not."""
import numpy as np

import datagen
from oracle import altgdmin as AG
from oracle import operators as O


def small_problem(kind="lines", seed=0, nx=8, ny=8, nc=3, q=6, r=2, backend="fft",
                  noisy=True):
    p = datagen.make_small(nx, ny, nc, q, r, seed=seed, kind=kind, n_lines=ny // 2,
                           m=nx * ny // 2, lowrank=False, coils="random", variable_m=True)
    op = O.from_problem(p, backend)
    Y = op.apply_A(p.zstar)
    if noisy:
        Y = datagen.add_noise(Y, p.noise, op.m_k, 20.0)
    rng = np.random.default_rng(seed + 100)
    U, _ = np.linalg.qr(datagen.crandn(rng, op.n, r))
    return p, op, Y, U, rng


def adjoint_error(op, rng):
    X = datagen.crandn(rng, op.n, op.q)
    Y = datagen.crandn(rng, op.q, op.nc, op.m_max)
    Y = np.where(np.arange(op.m_max)[None, None, :] < op.m_k[:, None, None], Y, 0)
    lhs = np.vdot(op.apply_A(X), Y)
    rhs = np.vdot(X, op.apply_AH(Y))
    return abs(lhs - rhs) / abs(lhs)


def fd_gradient_error(op, Y, U, rng, grad_fn=AG.gradient):
    """Central difference of f(U, B) with B fixed versus 2 Re tr(grad^H D)."""
    B = AG.ls_step(op, U, Y)
    # perturb B away from the minimiser so the gradient is not special
    B = B + 0.3 * datagen.crandn(rng, *B.shape)
    G = grad_fn(op, U, B, Y)
    D = datagen.crandn(rng, *U.shape)
    eps = 1e-6
    fp = AG.cost(op, U + eps * D, B, Y)
    fm = AG.cost(op, U - eps * D, B, Y)
    fd = (fp - fm) / (2 * eps)
    an = 2.0 * float(np.real(np.vdot(G, D)))
    return abs(fd - an) / abs(an)


def inv_error(op, Y, U, grad_fn=AG.gradient):
    """||U^H grad|| / ||grad|| at the LS-optimal B."""
    B = AG.ls_step(op, U, Y)
    G = grad_fn(op, U, B, Y)
    return np.linalg.norm(U.conj().T @ G) / np.linalg.norm(G)
