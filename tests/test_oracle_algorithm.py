"""Pins for the oracle's altGDmin (Algorithm 2, Sec. III-B).

Every check here comes from something other than the oracle itself: hand
computation, closed forms, calculus (finite differences), invariances the
algebra implies, library routines for special cases, and exact recovery.
"""
import math

import numpy as np
import pytest

import datagen
from oracle import altgdmin as AG
from oracle import metrics as M
from oracle import operators as O
from oracle import variants as V

from oracle_checks import adjoint_error, fd_gradient_error, inv_error, small_problem


# ---------------------------------------------------------------------------
# initialisation, by hand
# ---------------------------------------------------------------------------
def test_backprojection_hand_example():
    """2x2 grid, one coil with s = 1, two frames.  F[(ky,kx),(y,x)] =
    (-1)^(ky y + kx x) / 2, so by hand:
      frame 1 samples DC (index 0) with y = 2 -> A^H y = [1, 1, 1, 1];
      frame 2 samples indices 1, 2, 3 with y = [2, 0, 0] -> A^H y = 2 F^H e_1
      = [1, -1, 1, -1]  (index 1 is kx = 1: the sign flips along x).
    m_1 = 1, m_2 = 3, mbar = 2: the columns are scaled by 1/sqrt(2) and
    1/sqrt(6).  gamma = 36 * 8 / (3 * 2) = 48 truncates nothing."""
    op = O.Operator(2, 2, np.ones((1, 4)), [np.array([0]), np.array([1, 2, 3])], "dense")
    Y = np.zeros((2, 1, 3), dtype=np.complex128)
    Y[0, 0, 0] = 2.0
    Y[1, 0, :] = [2.0, 0.0, 0.0]
    Ytr, gamma, frac = AG.truncation(op, Y, 36.0)
    assert gamma == pytest.approx(48.0, rel=1e-15) and frac == 0.0
    X0 = AG.backprojection(op, Ytr)
    assert np.allclose(X0[:, 0], np.array([1, 1, 1, 1]) / math.sqrt(2), atol=1e-15)
    assert np.allclose(X0[:, 1], np.array([1, -1, 1, -1]) / math.sqrt(6), atol=1e-15)
    U0 = AG.spectral_init(X0, 1)
    assert abs(abs(np.vdot(U0[:, 0], np.ones(4) / 2)) - 1) < 1e-14


def test_truncation_hand_example():
    """Two frames, two coils (coil 2 all zero), m_1 = 10, m_2 = 20, so
    m = max m_k = 20 and q = 2.  Frame 1: ten samples of value 1; frame 2:
    nineteen of value 1j and one of value 20.  sum |y|^2 = 29 + 400 = 429,
    gamma = 36 * 429 / 40 = 386.1, sqrt(gamma) = 19.65 < 20: exactly the
    one large sample is zeroed (1 of the 60 valid samples).  (Dividing by
    the mean mbar = 15 instead would give sqrt(514.8) = 22.7 and keep it.)"""
    om = [np.arange(10), np.arange(20)]
    op = O.Operator(5, 4, np.ones((2, 20)), om, "fft")
    Y = np.zeros((2, 2, 20), dtype=np.complex128)
    Y[0, 0, :10] = 1.0
    Y[1, 0, :19] = 1j
    Y[1, 0, 19] = 20.0
    Ytr, gamma, frac = AG.truncation(op, Y, 36.0)
    assert gamma == pytest.approx(386.1, rel=1e-14)
    assert Ytr[1, 0, 19] == 0 and np.all(Ytr[1, 0, :19] == 1j) and np.all(Ytr[0, 0, :10] == 1)
    assert frac == pytest.approx(1.0 / 60.0)
    # inclusive at the threshold: 36 samples of value 1 and one of value 18
    # give gamma = 36 * (36 + 324) / 40 = 324, sqrt(gamma) = 18 exactly, and
    # the sample of magnitude 18 is kept
    Y2 = np.zeros((2, 2, 20), dtype=np.complex128)
    Y2[0, 0, :10] = 1.0
    Y2[0, 1, :6] = 1.0
    Y2[1, 0, :20] = 1.0
    Y2[1, 1, 0] = -18.0
    Ytr2, gamma2, frac2 = AG.truncation(op, Y2, 36.0)
    assert gamma2 == 324.0 and frac2 == 0.0 and Ytr2[1, 1, 0] == -18.0
    Y2[1, 1, 0] = -18.0000001
    assert AG.truncation(op, Y2, 36.0)[0][1, 1, 0] == 0.0
    Ytr3, _, frac3 = AG.truncation(op, Y, 0.0)
    assert frac3 == 0.0 and np.array_equal(Ytr3, Y)


# ---------------------------------------------------------------------------
# operator-level algebra
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["lines", "index"])
def test_adjoint_identity_small(kind):
    _, op, _, _, rng = small_problem(kind)
    assert adjoint_error(op, rng) < 1e-12


@pytest.mark.parametrize("kind", ["lines", "index"])
@pytest.mark.parametrize("backend", ["dense", "fft"])
def test_normal_equations_and_cholesky(kind, backend):
    """b_k solves the normal equations (M^dagger, Sec. II-A); Gram + Cholesky
    equals lstsq."""
    _, op, Y, U, _ = small_problem(kind, backend=backend)
    B = AG.ls_step(op, U, Y)
    for k in range(op.q):
        Mk = op.AU(k, U)
        res = Mk.conj().T @ (Mk @ B[:, k] - op.frame_vec(Y, k))
        assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(Mk) * np.linalg.norm(op.frame_vec(Y, k))
    G, h = V.gram_rhs(op, U, Y)
    assert np.allclose(G, np.conj(np.transpose(G, (0, 2, 1))), atol=1e-14)
    assert np.all(np.linalg.eigvalsh(G) > 0)
    B2 = V.cholesky_solve(G, h)
    assert np.linalg.norm(B2 - B) < 1e-10 * np.linalg.norm(B)


@pytest.mark.parametrize("kind", ["lines", "index"])
def test_gradient_matches_finite_difference(kind):
    _, op, Y, U, rng = small_problem(kind, seed=3)
    assert fd_gradient_error(op, Y, U, rng) < 1e-7


def test_gradient_envelope_finite_difference():
    """g(U) = min_B f(U, B) has the same derivative as f with B held at its
    minimiser (Danskin): d/de g(U + e D) = 2 Re tr(grad^H D)."""
    _, op, Y, U, rng = small_problem("index", seed=4)
    B = AG.ls_step(op, U, Y)
    G = AG.gradient(op, U, B, Y)
    D = datagen.crandn(rng, *U.shape)
    eps = 1e-5
    fd = (V.min_cost(op, U + eps * D, Y) - V.min_cost(op, U - eps * D, Y)) / (2 * eps)
    an = 2.0 * float(np.real(np.vdot(G, D)))
    assert abs(fd - an) < 1e-6 * abs(an)


@pytest.mark.parametrize("kind", ["lines", "index"])
def test_gradient_is_orthogonal_to_U(kind):
    """U^H grad = sum_k (A_k U)^H (A_k U b_k - y_k) b_k^H = 0 at the LS b_k,
    for any masks, coils and noise."""
    _, op, Y, U, _ = small_problem(kind, seed=5)
    assert inv_error(op, Y, U) < 1e-12
    # also for a U that is not orthonormal
    assert inv_error(op, Y, U @ np.array([[2.0, 1j], [0.5, 1.0]])) < 1e-12


@pytest.mark.parametrize("kind", ["lines", "index"])
def test_folded_gradient_equals_literal(kind):
    _, op, Y, U, rng = small_problem(kind, seed=6)
    B = AG.ls_step(op, U, Y) + 0.1 * datagen.crandn(rng, U.shape[1], op.q)
    G1 = AG.gradient(op, U, B, Y)
    G2 = V.folded_gradient(op, U, B, Y)
    assert np.linalg.norm(G1 - G2) < 1e-12 * np.linalg.norm(G1)


@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 8), (8, 16)])
def test_hybrid_form_equals_full_2d(nx, ny):
    """Fully sampled readout lines: the kx-inverse-transformed data and the
    y-only transform give the same Gram, rhs, b_k and gradient."""
    p, op, Y, U, rng = small_problem("lines", seed=7, nx=nx, ny=ny)
    Yh = V.hybrid_data(Y, p.masks, nx)
    # norms are preserved line by line
    assert abs(np.linalg.norm(Yh) - np.linalg.norm(Y)) < 1e-12 * np.linalg.norm(Y)
    W = V.hybrid_basis(U, p.coils, nx, ny)
    Gh, hh = V.hybrid_gram_rhs(W, Yh, p.masks, nx)
    G, h = V.gram_rhs(op, U, Y)
    assert np.linalg.norm(Gh - G) < 1e-12 * np.linalg.norm(G)
    assert np.linalg.norm(hh - h) < 1e-12 * np.linalg.norm(h)
    B = V.cholesky_solve(Gh, hh)
    grad_h = V.hybrid_gradient(W, Yh, B, p.coils, p.masks, nx, ny)
    grad = AG.gradient(op, U, B, Y)
    assert np.linalg.norm(grad_h - grad) < 1e-12 * np.linalg.norm(grad)


# ---------------------------------------------------------------------------
# step size and QR
# ---------------------------------------------------------------------------
def test_qr_closed_forms():
    """With U^H U = I and U^H grad = 0: Uhat^H Uhat = I + eta^2 grad^H grad;
    CholeskyQR and LAPACK QR span the same space; the SD formula holds; at
    t = 1, eta * sigma_max(grad) = 0.14 exactly."""
    _, op, Y, U, _ = small_problem("index", seed=8)
    B = AG.ls_step(op, U, Y)
    G = AG.gradient(op, U, B, Y)
    eta = AG.step_size(G, 0.14)
    assert eta * np.linalg.norm(G, 2) == pytest.approx(0.14, rel=1e-14)
    Uhat = U - eta * G
    r = U.shape[1]
    assert np.allclose(Uhat.conj().T @ Uhat, np.eye(r) + eta ** 2 * (G.conj().T @ G), atol=1e-13)
    Uq = AG.qr_project(Uhat)
    Uc, R, sd2 = V.qr_closed_form(U, G, eta)
    assert np.allclose(Uc.conj().T @ Uc, np.eye(r), atol=1e-13)
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R).real > 0)
    assert M.subspace_distance(Uq, Uc) < 1e-12
    assert M.subspace_distance(U, Uq) ** 2 == pytest.approx(sd2, rel=1e-10)


def _cap_example():
    """2x2 grid, one coil s = 1, two frames, rank 1, warm start
    U_0 = [1, 1, 1, 1]/2, whose transform is 1 at DC and 0 elsewhere.
    Frame 1 samples {DC, index 1} with y = [1, 1]; frame 2 samples
    {DC, index 2} with y = [2, 1].  By hand: A_k U_0 = [1, 0], so b_1 = 1,
    b_2 = 2, B_0 = [1, 2], ||B_0||_2 = sqrt(5); the residuals are [0, -1]
    and grad = -(F^H e_1) 1 - (F^H e_2) 2 with F^H e_1 = [1,-1,1,-1]/2
    (kx = 1) and F^H e_2 = [1,1,-1,-1]/2 (ky = 1): grad = -[3, 1, -1, -3]/2,
    ||grad||_2 = sqrt(5).  n = 4, mbar = 2."""
    op = O.Operator(2, 2, np.ones((1, 4)), [np.array([0, 1]), np.array([0, 2])], "dense")
    Y = np.zeros((2, 1, 2), dtype=np.complex128)
    Y[0, 0, :] = [1.0, 1.0]
    Y[1, 0, :] = [2.0, 1.0]
    return op, Y, np.full((4, 1), 0.5, dtype=np.complex128)


@pytest.mark.parametrize("cap_c,eta_hand,capped", [
    (0.0, 0.14 / math.sqrt(5.0), None),    # no cap: Algorithm 2's rule
    (0.5, 0.14 / math.sqrt(5.0), False),   # cap c n/(mbar ||B_0||^2) = 0.5*4/(2*5) = 0.2 > 0.0626
    (0.1, 0.04, True),                     # cap 0.1*4/(2*5) = 0.04 < 0.0626: binds
])
def test_step_size_cap_hand_example(cap_c, eta_hand, capped):
    """The optional step-size cap (the conservative rule of Sec. III-B,
    parameter setting) on the hand example above, through the whole run."""
    op, Y, U0 = _cap_example()
    B = AG.ls_step(op, U0, Y)
    assert np.allclose(B, [[1.0, 2.0]], atol=1e-14)
    G = AG.gradient(op, U0, B, Y)
    assert np.allclose(G[:, 0], -np.array([3, 1, -1, -3]) / 2, atol=1e-14)
    res = AG.run(op, Y, AG.Params(r=1, trunc_c=0.0, eta_cap_c=cap_c), U0=U0, t_fixed=1)
    assert res.eta == pytest.approx(eta_hand, rel=1e-14)
    assert res.history.get("eta_capped") is capped
    # one step: U_1 = (U_0 - eta grad) / ||U_0 - eta grad||
    uh = U0[:, 0] + eta_hand * np.array([3, 1, -1, -3]) / 2
    assert abs(abs(np.vdot(res.U[:, 0], uh / np.linalg.norm(uh))) - 1) < 1e-14


def test_subspace_distance_closed_forms():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(datagen.crandn(rng, 10, 6))
    U1, U2 = Q[:, :3], Q[:, 3:]
    assert M.subspace_distance(U1, U1) < 1e-14
    assert M.subspace_distance(U1, U2) == pytest.approx(math.sqrt(3), rel=1e-14)
    rot = np.linalg.qr(datagen.crandn(rng, 3, 3))[0]
    assert M.subspace_distance(U1, U1 @ rot) < 1e-14


def test_nsmse_is_scale_invariant_and_bounded_by_nmse():
    rng = np.random.default_rng(1)
    Xs = datagen.crandn(rng, 20, 5)
    assert M.nsmse(Xs * (0.3 - 2j), Xs) < 1e-28
    X = Xs + 0.1 * datagen.crandn(rng, 20, 5)
    assert M.nsmse(X, Xs) <= M.nmse(X, Xs)
    assert M.nmse(np.zeros_like(Xs), Xs) == pytest.approx(1.0)


# ---------------------------------------------------------------------------
# whole-loop properties
# ---------------------------------------------------------------------------
def test_full_sampling_reduces_to_truncated_svd():
    """All locations sampled, sum_c |s_c|^2 = 1, no truncation: X_0 = Z*/n,
    U_0 = top-r left singular vectors of Z*, grad_0 = 0, the stationarity
    guard fires and X = U_0 U_0^H Z* (Eckart-Young)."""
    nx, ny, nc, q, r = 8, 8, 3, 7, 2
    rng = np.random.default_rng(2)
    Z = datagen.crandn(rng, nx * ny, q)
    op = O.Operator(nx, ny, datagen.coil_maps(nx, ny, nc), [np.arange(nx * ny)] * q, "fft")
    Y = op.apply_A(Z)
    X0 = AG.backprojection(op, Y)
    assert np.allclose(X0, Z / (nx * ny), atol=1e-14)
    res = AG.run(op, Y, AG.Params(r=r, trunc_c=0.0), t_fixed=5)
    u, s, _ = np.linalg.svd(Z)
    assert M.subspace_distance(u[:, :r], res.U0) < 1e-12
    assert res.iters == 0 and res.history.get("converged_at_start")
    X = res.U @ (res.U.conj().T @ Z)
    assert np.linalg.norm(X - Z) ** 2 == pytest.approx(np.sum(s[r:] ** 2), rel=1e-12)


def test_gauge_and_scale_invariance():
    """U_0 -> U_0 Q' (Q' unitary) leaves every X_t unchanged; y -> a y scales
    B by a and leaves U unchanged; A -> a A with y -> a y (a rescaled DFT)
    leaves U and B unchanged."""
    p, op, Y, U, rng = small_problem("lines", seed=9)
    prm = AG.Params(r=2, trunc_c=0.0)
    ref = AG.run(op, Y, prm, U0=U, t_fixed=6)
    Qp = np.linalg.qr(datagen.crandn(rng, 2, 2))[0]
    g = AG.run(op, Y, prm, U0=U @ Qp, t_fixed=6)
    assert np.linalg.norm(g.X - ref.X) < 1e-12 * np.linalg.norm(ref.X)
    a = 3.7 - 1.1j
    s = AG.run(op, a * Y, prm, U0=U, t_fixed=6)
    assert M.subspace_distance(s.U, ref.U) < 1e-12
    assert np.linalg.norm(s.X - a * ref.X) < 1e-12 * np.linalg.norm(a * ref.X)
    op2 = O.Operator(op.nx, op.ny, 2.5 * op.coils, op.omegas, "fft")
    f = AG.run(op2, 2.5 * Y, prm, U0=U, t_fixed=6)
    assert M.subspace_distance(f.U, ref.U) < 1e-12
    assert np.linalg.norm(f.B - ref.B) < 1e-12 * np.linalg.norm(ref.B)


@pytest.mark.parametrize("kind", ["lines", "index"])
def test_exact_recovery_noise_free(kind):
    """Noise-free, exactly rank-r data: SD(U_t, U*) falls geometrically to
    the FP64 floor and the reconstruction error vanishes."""
    nx, ny, nc, q, r = 16, 16, 4, 20, 2
    p = datagen.make_small(nx, ny, nc, q, r, seed=1, kind=kind, n_lines=8, m=nx * ny // 3)
    op = O.from_problem(p)
    Y = op.apply_A(p.zstar)
    res = AG.run(op, Y, AG.Params(r=r, t_max=330), Zstar=p.zstar, Ustar=p.ustar)
    sd = np.array(res.history["sd_star"])
    assert sd[-1] < 1e-10
    assert res.history["nmse"][-1] < 1e-18
    # geometric: log SD drops by a comparable amount over equal windows
    logs = np.log10(sd[:200:40])
    steps = -np.diff(logs)
    assert np.all(steps > 0.5) and steps.max() < 4 * steps.min()


def test_gaussian_measurement_regime():
    """The guarantee's setting (Sec. III-B): i.i.d. Gaussian A_k, exactly
    rank-r X*, mq well above (n + q) r: altGDmin recovers X*."""
    n, q, m, r = 100, 50, 40, 2
    rng = np.random.default_rng(11)
    mats = [datagen.crandn(rng, m, n) for _ in range(q)]
    op = O.MatrixOperator(mats)
    Z, Us = datagen.lowrank_gaussian(n, q, r, rng)
    Y = op.apply_A(Z)
    res = AG.run(op, Y, AG.Params(r=r, t_max=150), Zstar=Z, Ustar=Us)
    assert res.history["nmse"][-1] < 1e-12
    assert res.history["nmse"][-1] < 1e-6 * res.history["nmse"][0]


def test_exit_rule_fires_and_is_recorded():
    nx, ny, nc, q, r = 16, 16, 4, 20, 2
    p = datagen.make_small(nx, ny, nc, q, r, seed=1, kind="lines", n_lines=8)
    op = O.from_problem(p)
    Y = op.apply_A(p.zstar)
    res = AG.run(op, Y, AG.Params(r=r, t_max=70, eps_exit=0.01))
    sd = np.array(res.history["sd"]) / math.sqrt(r)
    t = res.iters
    assert t < 70 and sd[t - 1] < 0.01 and np.all(sd[: t - 1] >= 0.01)


def test_consecutive_exit_variant():
    """The Sec. VI variant of the exit rule: with exit_consec = c the loop
    ends at the first t whose last c steps all had SD/sqrt(r) < eps; with
    c = 1 it is Algorithm 2's rule.  Checked against the recorded SD
    sequence of a fixed-length run."""
    nx, ny, nc, q, r = 16, 16, 4, 20, 2
    p = datagen.make_small(nx, ny, nc, q, r, seed=2, kind="lines", n_lines=8, snr_db=30.0)
    op = O.from_problem(p)
    Y = datagen.add_noise(op.apply_A(p.zstar), p.noise, op.m_k, 30.0)
    eps = 0.01
    full = AG.run(op, Y, AG.Params(r=r, t_max=70, eps_exit=0.0), t_fixed=70)
    small = np.array(full.history["sd"]) / math.sqrt(r) < eps
    for c in (1, 2, 4):
        want = next(t + 1 for t in range(70) if t + 1 >= c and small[t + 1 - c: t + 1].all())
        res = AG.run(op, Y, AG.Params(r=r, t_max=70, eps_exit=eps, exit_consec=c))
        assert res.iters == want and res.history["exit_at"] == want
