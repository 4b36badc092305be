"""FP64 oracle of the learned warm start: the CNN that maps zero-filled,
coil-combined frames to an initial basis, its projection loss, backward pass
and Adam update.  Test infrastructure only (used by tests/, the smoke check
and the benchmark's CPU baseline); nothing here is imported by the product
path.

Network (4 convolutions, 3x3, stride 1, zero "same" padding, with bias):
    input  2q planes: Re and Im of A_k^H y_k per frame, divided by the RMS of
           all 2q planes (no truncation, no 1/sqrt(m_k m) scaling);
    conv(2q -> w) ReLU, conv(w -> w) ReLU, conv(w -> w) ReLU, conv(w -> 2r);
    output M, n x r complex: channel 2j is Re M[:, j], channel 2j+1 Im M[:, j].
U0 is then the CholeskyQR of M (its span is all that matters).

Loss (the paper's subspace distance, its definition of SD with P = U U^H):
    L(M) = r - tr(G^-1 C C^H),  G = M^H M,  C = M^H U_tgt,
which equals 1/2 ||P_M - P_tgt||_F^2 for the orthogonal projectors onto
span(M) and span(U_tgt), and SD(M, U_tgt)^2 when M is orthonormal.  Its
Wirtinger gradient is dL/d conj(M) = -(I - P_M) U_tgt U_tgt^H M G^-1, and the
gradient with respect to the real output channels is (2 Re, 2 Im) of it.

Convolutions are written as explicit im2col matrices (rows ordered
(input channel, tap row, tap column)) multiplied by the weight matrix.  With
operand rounding (rnd = bf16_round) every convolution's two operands (data
and weights in the forward pass and the input gradient; output gradient and
data in the weight gradient) are first rounded to bfloat16, the arithmetic
of a BF16 matrix-core convolution with a wide accumulator; the products and
sums are then exact up to FP64 rounding.  Biases are not rounded.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """x rounded to the nearest bfloat16 (8 significand bits, ties to even),
    through binary32 (the bfloat16 format is the top half of a binary32
    word), returned as float64.  Finite inputs only."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(x):
    return x


def layer_channels(cin: int, width: int, cout: int, layers: int = 4):
    ch = [cin] + [width] * (layers - 1) + [cout]
    return [(ch[i], ch[i + 1]) for i in range(layers)]


def param_count(cin: int, width: int, cout: int, layers: int = 4) -> int:
    return sum(co * ci * 9 + co for ci, co in layer_channels(cin, width, cout, layers))


def unpack(params: np.ndarray, cin: int, width: int, cout: int, layers: int = 4):
    """Flat parameters -> [(W (co, ci, 3, 3), b (co,))], each layer W then b."""
    out, o = [], 0
    for ci, co in layer_channels(cin, width, cout, layers):
        W = params[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = params[o:o + co]
        o += co
        out.append((W, b))
    assert o == params.size
    return out


def pack(layers_wb) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers_wb])


def init_params(rng: np.random.Generator, cin: int, width: int, cout: int, layers: int = 4) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    wb = []
    for ci, co in layer_channels(cin, width, cout, layers):
        bound = np.sqrt(6.0 / (ci * 9))
        wb.append((rng.uniform(-bound, bound, size=(co, ci, 3, 3)), np.zeros(co)))
    return pack(wb)


def im2col(X: np.ndarray) -> np.ndarray:
    """(C, H, W) -> (C*9, H*W) with zero padding of one pixel."""
    C, H, Wd = X.shape
    Xp = np.zeros((C, H + 2, Wd + 2), dtype=X.dtype)
    Xp[:, 1:-1, 1:-1] = X
    cols = np.empty((C, 3, 3, H, Wd), dtype=X.dtype)
    for ty in range(3):
        for tx in range(3):
            cols[:, ty, tx] = Xp[:, ty:ty + H, tx:tx + Wd]
    return cols.reshape(C * 9, H * Wd)


def col2im(cols: np.ndarray, C: int, H: int, Wd: int) -> np.ndarray:
    """Adjoint of im2col: scatter-add the (C*9, H*W) columns back."""
    c5 = cols.reshape(C, 3, 3, H, Wd)
    Xp = np.zeros((C, H + 2, Wd + 2), dtype=cols.dtype)
    for ty in range(3):
        for tx in range(3):
            Xp[:, ty:ty + H, tx:tx + Wd] += c5[:, ty, tx]
    return Xp[:, 1:-1, 1:-1]


def conv_forward(X, W, b, rnd=_ident):
    C, H, Wd = X.shape
    co = W.shape[0]
    return (rnd(W).reshape(co, -1) @ im2col(rnd(X)) + b[:, None]).reshape(co, H, Wd)


def conv_backward(X, W, dY, rnd=_ident):
    """Gradients of sum(dY * conv(X, W, b)) with respect to X, W and b."""
    C, H, Wd = X.shape
    co = W.shape[0]
    d2 = rnd(dY).reshape(co, H * Wd)
    cols = im2col(rnd(X))
    dW = (d2 @ cols.T).reshape(W.shape)
    db = d2.sum(axis=1)
    dX = col2im(rnd(W).reshape(co, -1).T @ d2, C, H, Wd)
    return dX, dW, db


def forward(params, X, width, cout, layers: int = 4, keep: bool = False, rnd=_ident):
    """Network output (cout, H, W); with keep, also the layer inputs."""
    wb = unpack(params, X.shape[0], width, cout, layers)
    acts = [X]
    a = X
    for i, (W, b) in enumerate(wb):
        z = conv_forward(a, W, b, rnd)
        a = np.maximum(z, 0.0) if i < layers - 1 else z
        acts.append(a)
    return (a, acts) if keep else a


def output_to_M(Y: np.ndarray) -> np.ndarray:
    """(2r, H, W) -> n x r complex, pixel p = x + W*y."""
    r2, H, Wd = Y.shape
    Z = Y.reshape(r2, H * Wd)
    return (Z[0::2] + 1j * Z[1::2]).T


def M_grad_to_output(dMbar: np.ndarray, H: int, Wd: int) -> np.ndarray:
    """Wirtinger gradient dL/d conj(M) -> gradient over the real channels."""
    n, r = dMbar.shape
    out = np.empty((2 * r, n))
    out[0::2] = 2.0 * dMbar.real.T
    out[1::2] = 2.0 * dMbar.imag.T
    return out.reshape(2 * r, H, Wd)


def projection_loss(M: np.ndarray, Ut: np.ndarray):
    """L = r - tr(G^-1 C C^H) and dL/d conj(M) = -(I - P_M) Ut Ut^H M G^-1."""
    r = M.shape[1]
    G = M.conj().T @ M
    C = M.conj().T @ Ut
    Gi = np.linalg.inv(G)
    L = float(np.real(r - np.trace(Gi @ C @ C.conj().T)))
    UUhM = Ut @ (Ut.conj().T @ M)
    dMbar = -(UUhM - M @ (Gi @ (M.conj().T @ UUhM))) @ Gi
    return L, dMbar


def loss_and_grad(params, X, Ut, width, r, layers: int = 4, rnd=_ident):
    """Loss of one sequence and its gradient with respect to every parameter."""
    cin, H, Wd = X.shape
    Y, acts = forward(params, X, width, 2 * r, layers, keep=True, rnd=rnd)
    L, dMbar = projection_loss(output_to_M(Y), Ut)
    wb = unpack(params, cin, width, 2 * r, layers)
    d = M_grad_to_output(dMbar, H, Wd)
    grads = [None] * layers
    for i in range(layers - 1, -1, -1):
        W, b = wb[i]
        if i < layers - 1:
            d = d * (acts[i + 1] > 0)  # ReLU of layer i
        dX, dW, db = conv_backward(acts[i], W, d, rnd)
        grads[i] = (dW, db)
        d = dX
    return L, pack(grads)


def batch_loss_and_grad(params, Xs, Uts, width, r, layers: int = 4, rnd=_ident):
    """Mean loss and mean gradient over a batch of sequences."""
    Ls, gs = zip(*[loss_and_grad(params, X, U, width, r, layers, rnd) for X, U in zip(Xs, Uts)])
    return float(np.mean(Ls)), np.mean(gs, axis=0)


def adam_step(params, grads, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def network_input(op, Y: np.ndarray) -> np.ndarray:
    """2q planes (Re, Im of A_k^H y_k per frame), divided by their RMS."""
    X = op.apply_AH(Y)  # n x q
    nx, ny = op.nx, op.ny
    planes = np.empty((2 * X.shape[1], ny, nx))
    planes[0::2] = X.real.T.reshape(-1, ny, nx)
    planes[1::2] = X.imag.T.reshape(-1, ny, nx)
    rms = np.sqrt(np.mean(planes ** 2))
    return planes / rms if rms > 0 else planes
