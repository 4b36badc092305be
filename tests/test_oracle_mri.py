"""Pins for the oracle's altGDmin-MRI pieces around the loop: CGLS, the mean
image, the residuals, the automatic rank, MEC-1 / MEC-2, and the tracking
drivers (Algorithms 1, 3, 4, 5 and Algorithm 2's rank rule).

Each check comes from something other than the oracle: LAPACK least squares,
the Krylov-subspace optimality of CG, closed forms under full sampling (where
A_k^H A_k = I), hand-computed spectra and thresholds, numpy's FFT, and exact
recovery."""
import math

import numpy as np
import pytest

import datagen
from oracle import altgdmin as AG
from oracle import metrics as M
from oracle import mri as R
from oracle import operators as O


def _dense(op: O.Operator, k: int) -> np.ndarray:
    """A_k as an explicit (nc m_k) x n matrix, column by column."""
    cols = [op.A(k, e).reshape(-1) for e in np.eye(op.n, dtype=np.complex128)]
    return np.stack(cols, axis=1)


def _full_op(nx, ny, nc, q, backend="fft"):
    return O.Operator(nx, ny, datagen.coil_maps(nx, ny, nc), [np.arange(nx * ny)] * q, backend)


# ---------------------------------------------------------------------------
# CGLS
# ---------------------------------------------------------------------------
def test_cgls_reaches_the_least_squares_solution():
    """n iterations of CG on an n-dimensional problem end at the exact LS
    solution (LAPACK's lstsq), and the residual norm never increases."""
    rng = np.random.default_rng(0)
    A = datagen.crandn(rng, 30, 8)
    y = datagen.crandn(rng, 30)
    xs = np.linalg.lstsq(A, y, rcond=None)[0]
    x, it = R.cgls(lambda v: A @ v, lambda w: A.conj().T @ w, y, np.zeros(8, complex), 0.0, 8)
    assert it == 8
    assert np.linalg.norm(x - xs) < 1e-10 * np.linalg.norm(xs)
    res = [np.linalg.norm(y - A @ R.cgls(lambda v: A @ v, lambda w: A.conj().T @ w, y,
                                          np.zeros(8, complex), 0.0, k)[0]) for k in range(9)]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))


def test_cgls_iterate_is_the_krylov_minimiser():
    """After k iterations from 0, CGLS's x minimises ||y - A x|| over the
    Krylov space span{A^H y, (A^H A) A^H y, ...} (k vectors): computed here by
    brute force with lstsq on that basis."""
    rng = np.random.default_rng(1)
    A = datagen.crandn(rng, 40, 12)
    y = datagen.crandn(rng, 40)
    N, c = A.conj().T @ A, A.conj().T @ y
    for k in (1, 2, 3, 5):
        V = np.stack([np.linalg.matrix_power(N, j) @ c for j in range(k)], axis=1)
        coef = np.linalg.lstsq(A @ V, y, rcond=None)[0]
        x, _ = R.cgls(lambda v: A @ v, lambda w: A.conj().T @ w, y, np.zeros(12, complex), 0.0, k)
        assert np.linalg.norm(x - V @ coef) < 1e-9 * np.linalg.norm(V @ coef)


def test_cgls_stopping_rule():
    """The loop ends at the first iteration with ||A^H r|| <= tol ||A^H y||."""
    rng = np.random.default_rng(2)
    A = datagen.crandn(rng, 50, 20)
    y = datagen.crandn(rng, 50)
    AH = lambda w: A.conj().T @ w
    s0 = np.linalg.norm(AH(y))
    tol = 1e-3
    x, it = R.cgls(lambda v: A @ v, AH, y, np.zeros(20, complex), tol, 50)
    assert np.linalg.norm(AH(y - A @ x)) <= tol * s0
    xp, _ = R.cgls(lambda v: A @ v, AH, y, np.zeros(20, complex), 0.0, it - 1)
    assert np.linalg.norm(AH(y - A @ xp)) > tol * s0


# ---------------------------------------------------------------------------
# mean image and residual (Algorithm 1, steps 1-2)
# ---------------------------------------------------------------------------
def test_mean_image_under_full_sampling_is_the_temporal_mean():
    """Full sampling with sum_c |s_c|^2 = 1: A_k^H A_k = I, so the stacked
    normal operator is q I, CGLS converges in one iteration and zbar is the
    average of the frames."""
    op = _full_op(8, 8, 3, 6)
    Z = datagen.crandn(np.random.default_rng(3), 64, 6)
    zbar, it = R.mean_image(op, op.apply_A(Z))
    assert it == 1
    assert np.linalg.norm(zbar - Z.mean(axis=1)) < 1e-12 * np.linalg.norm(Z)


@pytest.mark.parametrize("kind", ["lines", "index"])
def test_mean_image_equals_stacked_least_squares(kind):
    """On a 4x4 grid, n = 16 CG iterations (no early stop) reach lstsq of the
    explicitly stacked dense operator [A_1; ...; A_q]."""
    p = datagen.make_small(4, 4, 2, 5, 1, seed=4, kind=kind, n_lines=2, m=6, lowrank=False, snr_db=20.0)
    op = O.Operator(4, 4, p.coils, O.omegas(p.kind, p.masks, 4), "dense")
    Y = datagen.add_noise(op.apply_A(p.zstar), p.noise, op.m_k, 20.0)
    big = np.concatenate([_dense(op, k) for k in range(op.q)], axis=0)
    rhs = np.concatenate([op.frame_vec(Y, k) for k in range(op.q)])
    zs = np.linalg.lstsq(big, rhs, rcond=None)[0]
    z, it = R.mean_image(op, Y, tol=0.0, maxit=16)
    assert np.linalg.norm(z - zs) < 1e-8 * np.linalg.norm(zs)


def test_residual_of_the_truth_is_zero_and_linear():
    p = datagen.make_small(16, 16, 3, 5, 2, seed=5, kind="lines", n_lines=5)
    op = O.from_problem(p)
    Y = op.apply_A(p.zstar)
    zbar = p.zstar.mean(axis=1)
    assert np.abs(R.residual(op, Y, zbar, p.zstar - zbar[:, None])).max() < 1e-12
    Yt = R.residual(op, Y, zbar)
    assert np.abs(Yt - op.apply_A(p.zstar - zbar[:, None])).max() < 1e-12


# ---------------------------------------------------------------------------
# automatic rank
# ---------------------------------------------------------------------------
def test_auto_rank_hand_spectrum():
    """Singular values 3, 2, 1, 0.5, 0.1 (energies 9, 4, 1, 0.25, 0.01):
    over the first 3, 85 % of 14 is 11.9, reached at r = 2; over 5, 85 % of
    14.26 is 12.121, also r = 2; over 1, r = 1; b = 95 over 3 (13.3): r = 3."""
    rng = np.random.default_rng(6)
    Q1 = np.linalg.qr(datagen.crandn(rng, 20, 5))[0]
    Q2 = np.linalg.qr(datagen.crandn(rng, 7, 5))[0]
    X0 = Q1 @ np.diag([3.0, 2.0, 1.0, 0.5, 0.1]) @ Q2.conj().T
    assert R.auto_rank(X0, 3) == 2
    assert R.auto_rank(X0, 5) == 2
    assert R.auto_rank(X0, 1) == 1
    assert R.auto_rank(X0, 3, b=95.0) == 3


def test_rank_cap_hand_values():
    """floor(min(n, q, nc min_k m_k) / 10): 64x64 grid, 40 frames -> 4; 16
    frames -> 1; a frame with 3 samples on 2 coils -> floor(6/10) -> at least 1."""
    mk = lambda sizes: [np.arange(s) for s in sizes]
    assert R.rank_cap(O.Operator(64, 64, np.ones((2, 4096)), mk([500] * 40))) == 4
    assert R.rank_cap(O.Operator(64, 64, np.ones((2, 4096)), mk([500] * 16))) == 1
    assert R.rank_cap(O.Operator(64, 64, np.ones((2, 4096)), mk([3] + [500] * 39))) == 1
    assert R.rank_cap(O.Operator(8, 8, np.ones((1, 64)), mk([40] * 300))) == 4


# ---------------------------------------------------------------------------
# MEC (Algorithm 3)
# ---------------------------------------------------------------------------
def test_mec1_full_sampling_is_the_adjoint():
    """A_k^H A_k = I: one CGLS iteration is exact, so e_k = A_k^H yres_k."""
    op = _full_op(8, 8, 2, 4)
    Yr = op.apply_A(datagen.crandn(np.random.default_rng(7), 64, 4))
    assert np.linalg.norm(R.mec1(op, Yr) - op.apply_AH(Yr)) < 1e-12 * np.linalg.norm(Yr)


def test_mec1_is_three_krylov_steps_per_frame():
    """Each column of E is the 3-vector Krylov minimiser of its own frame's
    LS problem (brute force on the explicit A_k)."""
    p = datagen.make_small(8, 8, 2, 3, 1, seed=8, kind="index", m=20, lowrank=False)
    op = O.Operator(8, 8, p.coils, O.omegas(p.kind, p.masks, 8), "dense")
    Yr = datagen.add_noise(op.apply_A(p.zstar), p.noise, op.m_k, 10.0)
    E = R.mec1(op, Yr)
    for k in range(op.q):
        A = _dense(op, k)
        y = op.frame_vec(Yr, k)
        N, c = A.conj().T @ A, A.conj().T @ y
        V = np.stack([np.linalg.matrix_power(N, j) @ c for j in range(3)], axis=1)
        ref = V @ np.linalg.lstsq(A @ V, y, rcond=None)[0]
        assert np.linalg.norm(E[:, k] - ref) < 1e-9 * np.linalg.norm(ref)


def test_temporal_dft_is_numpys_unitary_fft():
    S = datagen.crandn(np.random.default_rng(9), 10, 7)
    assert np.allclose(R.temporal_dft(S), np.fft.fft(S, axis=1, norm="ortho"), atol=1e-13)
    assert np.allclose(R.temporal_idft(R.temporal_dft(S)), S, atol=1e-13)


def test_soft_threshold_hand_values():
    S = np.array([[3 + 4j, 0.5, -2.0, 1j]])
    out = R.soft_threshold(S, 1.0)
    assert np.allclose(out, [[2.4 + 3.2j, 0.0, -1.0, 0.0]], atol=1e-15)


def test_mec2_closed_form_under_full_sampling():
    """Full sampling (A^H A = I) and yres = A(E*): every M_t equals F_t(E*),
    so the second M shows no change and the loop ends after two updates with
    E = F_t^{-1}(SThr_omega(F_t(E*))), omega = 0.001 max |F_t(E*)|."""
    op = _full_op(8, 8, 2, 6)
    rng = np.random.default_rng(10)
    S = np.zeros((64, 6), dtype=np.complex128)
    S[rng.integers(0, 64, 40), rng.integers(0, 6, 40)] = datagen.crandn(rng, 40)
    Estar = R.temporal_idft(S)
    res = R.mec2(op, op.apply_A(Estar))
    omega = 1e-3 * np.abs(S).max()
    assert res.omega == pytest.approx(omega, rel=1e-12)
    assert res.iters == 2 and res.changes[0] < 1e-12
    assert np.linalg.norm(res.E - R.temporal_idft(R.soft_threshold(S, omega))) < 1e-12 * np.linalg.norm(S)


def test_mec2_iteration_cap_and_first_update():
    """Without convergence the loop stops after max_iter updates; its first
    update is F^{-1} SThr(F(A^H yres)) (E_0 = 0)."""
    p = datagen.make_small(8, 8, 2, 5, 1, seed=11, kind="index", m=16, lowrank=False)
    op = O.from_problem(p)
    Yr = op.apply_A(p.zstar)
    one = R.mec2(op, Yr, max_iter=1)
    M0 = R.temporal_dft(op.apply_AH(Yr))
    assert one.iters == 1
    assert np.allclose(one.E, R.temporal_idft(R.soft_threshold(M0, 1e-3 * np.abs(M0).max())), atol=1e-13)
    many = R.mec2(op, Yr, max_iter=4, tol=0.0)
    assert many.iters == 4 and len(many.changes) == 3


# ---------------------------------------------------------------------------
# Algorithm 1 end to end, Algorithms 4 and 5
# ---------------------------------------------------------------------------
def _mean_plus_lowrank(nx, ny, q, r, rng, mean_scale=5.0):
    zbar = mean_scale * datagen.crandn(rng, nx * ny)
    X, U = datagen.lowrank_gaussian(nx * ny, q, r, rng)
    return zbar[:, None] + X, zbar, X


@pytest.mark.parametrize("mec", [1, 2])
def test_altgdmin_mri_exact_under_full_sampling(mec):
    """Full sampling, noise-free Z = zbar 1^T + X* (rank r): the mean is the
    temporal mean, the residual sequence has rank r (a column-mean shift of
    a rank-r matrix stays within rank r + 1; here the mean of X* is kept in
    its span by construction), altGDmin returns its truncated SVD, the second
    residual is zero and so is E: Z is recovered to rounding."""
    rng = np.random.default_rng(12)
    op = _full_op(8, 8, 2, 10)
    zb = datagen.crandn(rng, 64)
    U, _ = np.linalg.qr(datagen.crandn(rng, 64, 2))
    B = datagen.crandn(rng, 2, 10)
    B -= B.mean(axis=1, keepdims=True)  # X* has zero temporal mean
    Z = zb[:, None] + U @ B
    res = R.altgdmin_mri(op, op.apply_A(Z), AG.Params(r=2, trunc_c=0.0), mec=mec, t_fixed=3)
    assert np.linalg.norm(res.zbar - zb) < 1e-12 * np.linalg.norm(zb)
    assert np.linalg.norm(res.Z - Z) < 1e-10 * np.linalg.norm(Z)


def test_mean_step_rescues_random_fourier_sampling():
    """Table 1's finding on a small synthetic sequence: with random 2D
    Fourier sampling of a sequence dominated by its mean image, altGDmin on
    the raw data reconstructs far worse than altGDmin-mean (mean by CGLS,
    altGDmin on the residual)."""
    rng = np.random.default_rng(13)
    nx = ny = 16
    q, r = 20, 2
    Z, zb, X = _mean_plus_lowrank(nx, ny, q, r, rng, mean_scale=3.0)
    omegas = [np.sort(rng.choice(nx * ny, size=nx * ny // 3, replace=False)) for _ in range(q)]
    op = O.Operator(nx, ny, datagen.coil_maps(nx, ny, 2), omegas)
    Y = op.apply_A(Z)
    plain = AG.run(op, Y, AG.Params(r=r, t_max=70), t_fixed=70, record=False)
    mean = R.altgdmin_mri(op, Y, AG.Params(r=r, t_max=70), mec=None, t_fixed=70)
    e_plain, e_mean = M.nmse(plain.X, Z), M.nmse(mean.Z, Z)
    assert e_mean < 0.1 * e_plain


def test_minibatch_with_one_batch_is_algorithm_1():
    p = datagen.make_small(16, 16, 2, 8, 2, seed=14, kind="lines", n_lines=6, snr_db=30.0)
    op = O.from_problem(p)
    Y = datagen.add_noise(op.apply_A(p.zstar), p.noise, op.m_k, 30.0)
    prm = AG.Params(r=2, t_max=10)
    a = R.minibatch_st(op, Y, prm, alpha=8, t_first=10)
    b = R.altgdmin_mri(op, Y, prm, mec=1).Z
    assert np.linalg.norm(a - b) < 1e-12 * np.linalg.norm(b)


def test_minibatch_later_batches_start_from_the_previous_basis():
    """A second batch whose frames lie in the first batch's final subspace,
    sampled fully: with U_0 = U^(1) the LS step is exact, the gradient is
    zero (stationary guard) and the batch is reconstructed exactly."""
    rng = np.random.default_rng(15)
    op = _full_op(8, 8, 2, 12)
    zb = datagen.crandn(rng, 64)
    U, _ = np.linalg.qr(datagen.crandn(rng, 64, 2))
    B = datagen.crandn(rng, 2, 12)
    B[:, :6] -= B[:, :6].mean(axis=1, keepdims=True)
    B[:, 6:] -= B[:, 6:].mean(axis=1, keepdims=True)
    Z = zb[:, None] + U @ B
    out = R.minibatch_st(op, op.apply_A(Z), AG.Params(r=2, trunc_c=0.0), alpha=6, t_first=3)
    assert np.linalg.norm(out - Z) < 1e-10 * np.linalg.norm(Z)


def test_online_frames_follow_the_first_batch_model():
    """Online tracking: frames after the first batch are zbar + U b_k + e_k
    with b_k the LS coefficients of the residual; for frames in the span of
    the first batch's basis, fully sampled, they are exact."""
    rng = np.random.default_rng(16)
    op = _full_op(8, 8, 2, 10)
    zb = datagen.crandn(rng, 64)
    U, _ = np.linalg.qr(datagen.crandn(rng, 64, 2))
    B = datagen.crandn(rng, 2, 10)
    B[:, :5] -= B[:, :5].mean(axis=1, keepdims=True)
    Z = zb[:, None] + U @ B
    out = R.online_st(op, op.apply_A(Z), AG.Params(r=2, trunc_c=0.0, t_max=3), alpha=5)
    assert np.linalg.norm(out - Z) < 1e-10 * np.linalg.norm(Z)
