"""The warm-start CNN on the GPU (through the C ABI) against the FP64 oracle:
forward output, loss and parameter gradients, Adam, the network input
(L1), and the spectral fallback of altgdmin_init_warm (L3, L5)."""
import numpy as np
import pytest

import datagen
from oracle import altgdmin as AG
from oracle import cnn as C
from oracle import variants as V

from gpu_cases import GPU_OK, Case, from_gpu_U, log, proj_dist, rel, to_gpu_U

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not GPU_OK, reason="needs a GPU")]

if GPU_OK:
    import torch

CASES = [
    # (nx, ny, q, r, width, batch)
    (16, 16, 5, 2, 8, 2),     # one-chunk channels, 1 output tile of 16 channels
    (24, 16, 20, 3, 20, 3),   # 40 input channels: two channel chunks; width not a multiple of 16
    (128, 128, 48, 6, 32, 2), # the warm-start workload's network
]


def _data(nx, ny, q, r, width, batch, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((batch, 2 * q, ny, nx)).astype(np.float32)
    Ut = []
    for b in range(batch):
        Q, _ = np.linalg.qr(datagen.crandn(rng, nx * ny, r))
        Ut.append(Q.astype(np.complex64))
    p = C.init_params(rng, 2 * q, width, 2 * r)
    p = (p + 0.02 * rng.standard_normal(p.size)).astype(np.float32)
    return X, np.array(Ut), p


@pytest.mark.parametrize("cfg", CASES, ids=[f"{c[0]}x{c[1]}_q{c[2]}_w{c[4]}" for c in CASES])
def test_forward_loss_and_gradients_match_oracle(cfg):
    """The convolutions run on BF16 matrix-core operands with FP32
    accumulation.  The reference is the oracle with the same operand rounding
    (oracle.cnn.bf16_round on both operands of every convolution); what
    remains is FP32 accumulation and the operands that round to the other
    bfloat16 neighbour because their FP32 activation differs from the FP64
    one in the last bits.  Such flips can show far above the FP32 level (a
    projected loss gradient can be a strongly cancelling sum), so each bound
    is five times the rounding oracle's own change under a 1e-6 relative
    perturbation of the input, and at least 1e-4 (output) or 5e-4
    (gradients, per layer and in total).  The distance to the plain FP64
    oracle, i.e. the effect of the BF16 operands themselves, is logged and
    only sanity-bounded (3e-2 output, 0.2 gradient)."""
    nx, ny, q, r, width, batch = cfg
    log(f"cnn {cfg}")
    import paper_2212_09664_amd as ag
    X, Ut, p = _data(nx, ny, q, r, width, batch, 1)
    net = ag.WsInit(nx, ny, q, r, width=width, batch=batch)
    assert net.param_count == p.size
    dev = torch.device("cuda:0")
    pg = torch.from_numpy(p).to(dev)
    xg = torch.from_numpy(X).to(dev)
    ug = torch.from_numpy(np.ascontiguousarray(np.transpose(Ut, (0, 2, 1)))).to(dev)  # (B, r, n)
    Mg = net.forward(pg, xg).cpu().numpy()
    loss, grads = net.loss_backward(pg, xg, ug)
    torch.cuda.synchronize()
    X64, p64, Ut64 = X.astype(np.float64), p.astype(np.float64), Ut.astype(np.complex128)
    Xp = X64 * (1.0 + 1e-6 * np.random.default_rng(2).standard_normal(X64.shape))
    for b in range(batch):
        Mb16 = C.output_to_M(C.forward(p64, X64[b], width, 2 * r, rnd=C.bf16_round))
        Mpert = C.output_to_M(C.forward(p64, Xp[b], width, 2 * r, rnd=C.bf16_round))
        M64 = C.output_to_M(C.forward(p64, X64[b], width, 2 * r))
        Mgb = Mg[b].T.astype(np.complex128)
        e, e64, sm = rel(Mgb, Mb16), rel(Mgb, M64), rel(Mpert, Mb16)
        log(f"  M[{b}] rel {e:.2e} (BF16-operand oracle, flip sensitivity {sm:.2e}), {e64:.2e} (FP64 oracle)")
        assert e <= max(1e-4, 5 * sm) and e64 < 3e-2
    Lref, gref = C.batch_loss_and_grad(p64, list(X64), list(Ut64), width, r, rnd=C.bf16_round)
    L64, g64 = C.batch_loss_and_grad(p64, list(X64), list(Ut64), width, r)
    _, gpert = C.batch_loss_and_grad(p64, list(Xp), list(Ut64), width, r, rnd=C.bf16_round)
    gl = float(loss.item())
    gg = grads.cpu().numpy().astype(np.float64)
    eg, eg64, sens = rel(gg, gref), rel(gg, g64), rel(gpert, gref)
    log(f"  loss {gl:.8f} vs {Lref:.8f} (FP64 oracle {L64:.8f}); grad rel {eg:.2e} "
        f"(flip sensitivity {sens:.2e}), FP64 oracle {eg64:.2e}")
    assert abs(gl - Lref) <= 1e-4 * max(1.0, abs(Lref))
    assert eg <= max(5e-4, 5 * sens) and eg64 < 0.2
    # per layer, so that a wrong small layer cannot hide behind a big one
    off = 0
    for ci, co in C.layer_channels(2 * q, width, 2 * r):
        k = co * ci * 9 + co
        el = rel(gg[off:off + k], gref[off:off + k])
        sl = rel(gpert[off:off + k], gref[off:off + k])
        log(f"    layer {ci}->{co}: rel {el:.2e} (flip sensitivity {sl:.2e})")
        assert el <= max(5e-4, 5 * sl), (ci, co, el, sl)
        off += k


def test_adam_matches_oracle():
    import paper_2212_09664_amd as ag
    rng = np.random.default_rng(2)
    net = ag.WsInit(16, 16, 5, 2, width=8, batch=1)
    n = net.param_count
    p = rng.standard_normal(n).astype(np.float32)
    dev = torch.device("cuda:0")
    pg = torch.from_numpy(p).to(dev)
    mg, vg = torch.zeros(n, device=dev), torch.zeros(n, device=dev)
    pr, mr, vr = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        net.adam_step(pg, torch.from_numpy(g).to(dev), mg, vg, 1e-3, step)
        pr, mr, vr = C.adam_step(pr, g.astype(np.float64), mr, vr, 1e-3, step)
    torch.cuda.synchronize()
    assert np.allclose(pg.cpu().numpy(), pr, rtol=1e-6, atol=1e-6)


def test_network_input_matches_oracle():
    p = datagen.make_small(32, 16, 3, 6, 2, seed=7, kind="lines", n_lines=5, snr_db=30.0, variable_m=True)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    Xg = ctx.cnn_input().cpu().numpy().astype(np.float64)
    Xr = C.network_input(cs.op, cs.y)
    e = rel(Xg, Xr)
    log(f"  planes rel {e:.2e}")
    assert e < 1e-5


def test_warm_init_keeps_the_lower_cost_basis():
    """A good guess (the noise-free signal subspace) is kept; a random one
    falls back to the spectral basis; the decision agrees with the oracle's
    costs f(U) = sum_k ||y_k||^2 - h_k^H G_k^-1 h_k."""
    p = datagen.make_small(32, 32, 3, 10, 2, seed=8, kind="lines", n_lines=8, lowrank=True, snr_db=40.0)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    Us = from_gpu_U(ctx.init())
    f_spec = V.min_cost(cs.op, np.linalg.qr(Us)[0], cs.y)
    rng = np.random.default_rng(9)
    Ugood, _ = np.linalg.qr(p.zstar @ datagen.crandn(rng, p.q, p.r))
    Ubad = datagen.crandn(rng, p.n, p.r)
    for M, label in ((Ugood @ datagen.crandn(rng, p.r, p.r), "good"), (Ubad, "random")):
        choice = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
        U = from_gpu_U(ctx.init_warm(to_gpu_U(M), choice=choice))
        ch = int(choice.item())
        f_cnn = V.min_cost(cs.op, np.linalg.qr(M)[0], cs.y)
        log(f"  {label}: f_cnn {f_cnn:.6e} f_spec {f_spec:.6e} choice {ch}")
        assert ch == int(f_cnn < f_spec)
        ref = M if ch else Us
        assert proj_dist(U, ref) < 1e-5
        assert np.allclose(U.conj().T @ U, np.eye(p.r), atol=2e-6)
    assert ch == 0  # the random guess lost
    # the step size is Algorithm 2's rule at the spectral basis, whichever basis is kept
    U = ctx.init()
    ctx.iterate(1, U, sync=True)
    eta_plain = ctx.get_eta()
    ctx.init_warm(to_gpu_U(Ugood))
    ctx.iterate(1, to_gpu_U(Ugood), sync=True)
    assert ctx.get_eta() == pytest.approx(eta_plain, rel=1e-6)


def test_warm_init_from_a_given_fallback_matches_init_warm():
    """altgdmin_init_warm_from, given the basis altgdmin_init computed, gives
    bitwise the basis, the choice and the next iterates of altgdmin_init_warm,
    for a kept and for a rejected guess, into a new buffer or in place."""
    p = datagen.make_small(32, 32, 3, 10, 2, seed=8, kind="lines", n_lines=8, lowrank=True, snr_db=40.0)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(9)
    Ugood, _ = np.linalg.qr(p.zstar @ datagen.crandn(rng, p.q, p.r))
    for M, kept in ((Ugood @ datagen.crandn(rng, p.r, p.r), 1), (datagen.crandn(rng, p.n, p.r), 0)):
        Mg = to_gpu_U(M)
        c0 = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
        U0 = ctx.init_warm(Mg, choice=c0)
        B0 = ctx.iterate(2, U0)
        torch.cuda.synchronize()
        assert int(c0.item()) == kept
        for in_place in (False, True):
            Ufb = ctx.init()
            c1 = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
            U1 = ctx.init_warm_from(Mg, Ufb, U=Ufb if in_place else None, choice=c1)
            B1 = ctx.iterate(2, U1)
            torch.cuda.synchronize()
            log(f"  kept {kept} in_place {in_place}: choice {int(c1.item())}")
            assert int(c1.item()) == kept
            assert torch.equal(U1, U0) and torch.equal(B1, B0)


@pytest.mark.parametrize("guess", ["zero", "nan"])
def test_warm_init_falls_back_when_the_guess_cannot_be_scored(guess):
    """A network output that cannot be scored (all zero: its Gram is
    singular even with the ridge; NaN: non-finite) counts as infinitely
    costly: the spectral basis is kept, no error is left set, and the loop
    then runs exactly as after the plain initialisation."""
    p = datagen.make_small(32, 32, 3, 10, 2, seed=8, kind="lines", n_lines=8, lowrank=True, snr_db=40.0)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    Uspec = ctx.init()
    Bspec = ctx.iterate(4, Uspec.clone())
    torch.cuda.synchronize()
    Uspec0 = ctx.init()
    M = torch.zeros(p.r, p.n, dtype=torch.complex64, device="cuda:0")
    if guess == "nan":
        M[:] = float("nan")
    choice = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    U = ctx.init_warm(M, choice=choice)
    st, frame = ctx.last_error()
    log(f"  {guess}: choice {int(choice.item())}, status {st}")
    assert st == 0 and int(choice.item()) == 0
    assert torch.equal(U, Uspec0)
    B, done = ctx.iterate(4, U, sync=True)
    assert done == 4
    # the step size comes from the warm start's own evaluation of the rule at
    # the spectral basis (same value up to rounding)
    assert rel(from_gpu_U(B.T.contiguous()), from_gpu_U(Bspec.T.contiguous())) < 1e-5
