"""Pins of the warm-start CNN oracle (FP64): each check compares it with
something other than itself — a library correlation, finite differences,
the projector form of the loss, closed forms of Adam — and planted mistakes
must fail them."""
import numpy as np
import pytest
from scipy.signal import correlate2d

import datagen
from oracle import cnn as C
from oracle import metrics as M
from oracle import operators as O


def _rand(rng, *shape):
    return rng.standard_normal(shape)


def test_conv_forward_matches_library_correlation():
    rng = np.random.default_rng(0)
    X, W, b = _rand(rng, 3, 7, 5), _rand(rng, 4, 3, 3, 3), _rand(rng, 4)
    Y = C.conv_forward(X, W, b)
    for o in range(4):
        ref = b[o] + sum(correlate2d(X[i], W[o, i], mode="same", boundary="fill") for i in range(3))
        assert np.allclose(Y[o], ref, atol=1e-12)


def test_im2col_adjoint_identity():
    rng = np.random.default_rng(1)
    X = _rand(rng, 2, 4, 6)
    Cm = _rand(rng, 18, 24)
    assert np.isclose(np.sum(C.im2col(X) * Cm), np.sum(X * C.col2im(Cm, 2, 4, 6)), rtol=1e-12)


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(2)
    X, W, b, dY = _rand(rng, 3, 5, 4), _rand(rng, 2, 3, 3, 3), _rand(rng, 2), _rand(rng, 2, 5, 4)
    dX, dW, db = C.conv_backward(X, W, dY)
    f = lambda X_, W_, b_: np.sum(dY * C.conv_forward(X_, W_, b_))
    eps = 1e-6
    for arr, grad, which in ((X, dX, 0), (W, dW, 1), (b, db, 2)):
        D = _rand(rng, *arr.shape)
        args_p = [X, W, b]
        args_m = [X, W, b]
        args_p[which] = arr + eps * D
        args_m[which] = arr - eps * D
        fd = (f(*args_p) - f(*args_m)) / (2 * eps)
        assert np.isclose(fd, np.sum(grad * D), rtol=1e-7, atol=1e-9)


def _orth(rng, n, r):
    Q, _ = np.linalg.qr(datagen.crandn(rng, n, r))
    return Q


def test_loss_equals_half_projector_distance_and_sd():
    rng = np.random.default_rng(3)
    n, r = 40, 3
    Mm = datagen.crandn(rng, n, r)
    Ut = _orth(rng, n, r)
    L, _ = C.projection_loss(Mm, Ut)
    Qm, _ = np.linalg.qr(Mm)
    PM, PU = Qm @ Qm.conj().T, Ut @ Ut.conj().T
    assert np.isclose(L, 0.5 * np.linalg.norm(PM - PU) ** 2, rtol=1e-10)
    L2, _ = C.projection_loss(Qm, Ut)
    assert np.isclose(L2, M.subspace_distance(Qm, Ut) ** 2, rtol=1e-10)
    # only the span matters: M -> M Q' for any invertible Q'
    Qp = datagen.crandn(rng, r, r)
    L3, _ = C.projection_loss(Mm @ Qp, Ut)
    assert np.isclose(L, L3, rtol=1e-9)
    # equal spans give zero loss
    L4, _ = C.projection_loss(Ut @ datagen.crandn(rng, r, r), Ut)
    assert abs(L4) < 1e-12


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(4)
    n, r = 30, 2
    Mm, Ut = datagen.crandn(rng, n, r), _orth(rng, n, r)
    L, G = C.projection_loss(Mm, Ut)
    eps = 1e-6
    D = datagen.crandn(rng, n, r)
    fd = (C.projection_loss(Mm + eps * D, Ut)[0] - C.projection_loss(Mm - eps * D, Ut)[0]) / (2 * eps)
    assert np.isclose(fd, 2 * np.real(np.vdot(G, D)), rtol=1e-7)
    # the gradient is orthogonal to span(M) from the left: M^H G = 0
    assert np.linalg.norm(Mm.conj().T @ G) < 1e-12 * np.linalg.norm(G) * n


def _tiny(rng, cin=4, width=3, r=1, H=5, Wd=6):
    X = _rand(rng, cin, H, Wd)
    Ut = _orth(rng, H * Wd, r)
    p = C.init_params(rng, cin, width, 2 * r)
    p = p + 0.05 * _rand(rng, p.size)  # non-zero biases too
    return X, Ut, p


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(5)
    X, Ut, p = _tiny(rng)
    L, g = C.loss_and_grad(p, X, Ut, 3, 1)
    eps = 1e-6
    for trial in range(3):
        D = _rand(rng, p.size)
        fd = (C.loss_and_grad(p + eps * D, X, Ut, 3, 1)[0] - C.loss_and_grad(p - eps * D, X, Ut, 3, 1)[0]) / (2 * eps)
        assert np.isclose(fd, g @ D, rtol=1e-6, atol=1e-10), trial
    # one coordinate in each layer
    sizes = [co * ci * 9 + co for ci, co in C.layer_channels(4, 3, 2)]
    offs = np.cumsum([0] + sizes[:-1])
    for o in offs:
        e = np.zeros(p.size)
        e[o + 1] = 1.0
        fd = (C.loss_and_grad(p + eps * e, X, Ut, 3, 1)[0] - C.loss_and_grad(p - eps * e, X, Ut, 3, 1)[0]) / (2 * eps)
        assert np.isclose(fd, g[o + 1], rtol=1e-5, atol=1e-10)


def test_parameter_count_of_the_workload_networks():
    # 2q -> 32 -> 32 -> 32 -> 2r
    assert C.param_count(96, 32, 12) == 49644   # q = 48, r = 6
    assert C.param_count(80, 32, 16) == 46192   # q = 40, r = 8


def test_adam_closed_form_for_a_constant_gradient():
    p0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = v = np.zeros(3)
    lr = 1e-2
    p1, m, v = C.adam_step(p0, g, m, v, lr, 1)
    # with bias correction the first steps move each parameter by lr * g / (|g| + eps)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    p2, m, v = C.adam_step(p1, g, m, v, lr, 2)
    assert np.allclose(p2, p1 - lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, (1 - 0.9 ** 2) * g) and np.allclose(v, (1 - 0.999 ** 2) * g * g)


def test_network_input_is_the_rms_normalised_back_projection():
    p = datagen.make_small(16, 8, 2, 3, 2, seed=6, kind="lines", n_lines=3, snr_db=30.0, variable_m=True)
    op = O.from_problem(p)
    Y = datagen.add_noise(op.apply_A(p.zstar), p.noise, op.m_k, p.snr_db)
    X = C.network_input(op, Y)
    assert X.shape == (6, 8, 16)
    assert np.isclose(np.sqrt(np.mean(X ** 2)), 1.0)
    AH = op.apply_AH(Y)
    s = AH[3, 1].real / X[2, 0, 3]
    assert np.allclose(X[2].ravel() * s, AH[:, 1].real) and np.allclose(X[3].ravel() * s, AH[:, 1].imag)


# planted mistakes --------------------------------------------------------------

def test_planted_missing_relu_mask_fails_finite_differences(monkeypatch):
    rng = np.random.default_rng(7)
    X, Ut, p = _tiny(rng, cin=3, width=4)
    real_backward = C.conv_backward

    def lg_no_mask(params, X_, U_, width, r, layers=4):
        Y, acts = C.forward(params, X_, width, 2 * r, layers, keep=True)
        L, dMb = C.projection_loss(C.output_to_M(Y), U_)
        wb = C.unpack(params, X_.shape[0], width, 2 * r, layers)
        d = C.M_grad_to_output(dMb, *X_.shape[1:])
        grads = [None] * layers
        for i in range(layers - 1, -1, -1):
            dX, dW, db = real_backward(acts[i], wb[i][0], d)  # mask dropped
            grads[i] = (dW, db)
            d = dX
        return L, C.pack(grads)

    L, g = lg_no_mask(p, X, Ut, 4, 1)
    eps = 1e-6
    D = _rand(rng, p.size)
    fd = (C.loss_and_grad(p + eps * D, X, Ut, 4, 1)[0] - C.loss_and_grad(p - eps * D, X, Ut, 4, 1)[0]) / (2 * eps)
    assert not np.isclose(fd, g @ D, rtol=1e-4)


def test_planted_missing_factor_two_fails_finite_differences():
    rng = np.random.default_rng(8)
    n, r = 20, 2
    Mm, Ut = datagen.crandn(rng, n, r), _orth(rng, n, r)
    _, G = C.projection_loss(Mm, Ut)
    Y = C.M_grad_to_output(G, 4, 5) / 2.0  # the planted mistake
    Yr = np.empty((2 * r, n))
    Yr[0::2], Yr[1::2] = Mm.real.T, Mm.imag.T
    D = _rand(rng, 2 * r, n)
    eps = 1e-6

    def L_of(Z):
        return C.projection_loss((Z[0::2] + 1j * Z[1::2]).T, Ut)[0]

    fd = (L_of(Yr + eps * D) - L_of(Yr - eps * D)) / (2 * eps)
    assert np.isclose(fd, np.sum(C.M_grad_to_output(G, 4, 5).reshape(2 * r, n) * D), rtol=1e-6)
    assert not np.isclose(fd, np.sum(Y.reshape(2 * r, n) * D), rtol=1e-2)


def test_bf16_round_hand_values_and_bounds():
    """bfloat16 keeps 8 significand bits: at 1 the spacing is 2^-7, ties go to
    the even neighbour; every result has a zero low half in binary32, is a
    fixed point, and lies within half a spacing (2^-9 relative) of x."""
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -9, 1 + 2.0 ** -7 + 2.0 ** -8, -2.5, np.pi, 0.0])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -7, 1 + 2.0 ** -6, -2.5, 3.140625, 0.0])
    assert np.array_equal(C.bf16_round(x), want)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(10000) * 10.0 ** rng.integers(-20, 20, 10000)
    z = C.bf16_round(y)
    assert np.all((z.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    assert np.array_equal(C.bf16_round(z), z)
    assert np.all(np.abs(z - y) <= 2.0 ** -8 * np.abs(y))


def test_rounded_convolution_is_the_convolution_of_rounded_operands():
    """With operand rounding the forward, the input gradient and the weight
    gradient are the plain ones evaluated on rounded operands (bias exact)."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3, 8, 8))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    dY = rng.standard_normal((4, 8, 8))
    R = C.bf16_round
    assert np.array_equal(C.conv_forward(X, W, b, rnd=R), C.conv_forward(R(X), R(W), b))
    got = C.conv_backward(X, W, dY, rnd=R)
    ref = C.conv_backward(R(X), R(W), R(dY))
    for g, h in zip(got, ref):
        assert np.array_equal(g, h)
    assert not np.allclose(C.conv_forward(X, W, b, rnd=R), C.conv_forward(X, W, b), rtol=1e-6)
