"""Error metrics (oracle, test infrastructure)."""
from __future__ import annotations

import numpy as np


def subspace_distance(U1: np.ndarray, U2: np.ndarray) -> float:
    """SD(U1, U2) = ||(I - U1 U1^H) U2||_F for orthonormal U1, U2 (Sec. II-A)."""
    return float(np.linalg.norm(U2 - U1 @ (U1.conj().T @ U2)))


def nmse(X: np.ndarray, Xstar: np.ndarray) -> float:
    """||X - X*||_F^2 / ||X*||_F^2 (the error of Table 1)."""
    return float(np.linalg.norm(X - Xstar) ** 2 / np.linalg.norm(Xstar) ** 2)


def nsmse(X: np.ndarray, Xstar: np.ndarray) -> float:
    """Normalised scale-invariant MSE (Sec. V-B):
    sum_k dist^2(x*_k, x_k) / ||X*||_F^2 with
    dist^2(x*, x) = ||x* - x (x^H x*) / ||x||^2||^2."""
    num = 0.0
    for k in range(Xstar.shape[1]):
        x, xs = X[:, k], Xstar[:, k]
        nx2 = float(np.vdot(x, x).real)
        if nx2 == 0.0:
            num += float(np.vdot(xs, xs).real)
            continue
        d = xs - x * (np.vdot(x, xs) / nx2)
        num += float(np.vdot(d, d).real)
    return num / float(np.linalg.norm(Xstar) ** 2)
