"""GPU (HIP, through the C ABI) versus the FP64 oracle on identical inputs.

Tolerances: operators (A, A^H, W-derived G_k/h_k through b_k, the gradient)
at 1e-5 relative (the gradient normalised by the size of the terms it is a
difference of: ||sum_k A_k^H A_k U b_k b_k^H||_F); end to end, |NMSE_gpu -
NMSE_oracle| <= 1e-4 after the fixed iteration count.
"""
import math

import numpy as np
import pytest

import datagen
from oracle import altgdmin as AG
from oracle import metrics as M
from oracle import operators as O

from gpu_cases import GPU_OK, Case, from_gpu_B, from_gpu_U, log, proj_dist, rel, to_gpu_U

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not GPU_OK, reason="needs a GPU")]

if GPU_OK:
    import torch

OP_CASES = [
    # (nx, ny, nc, q, r, kind, lines/m, variable m_k)
    (64, 64, 4, 6, 3, "lines", 16, True),
    (32, 16, 3, 5, 2, "lines", 5, True),
    (16, 64, 2, 4, 2, "lines", 9, False),
    (128, 128, 3, 3, 2, "lines", 20, True),
    (256, 256, 2, 2, 2, "lines", 33, True),
    (32, 32, 3, 6, 3, "index", 300, True),
    (16, 64, 2, 5, 2, "index", 250, True),
    (128, 128, 2, 4, 4, "index", 2000, True),
]


def _case(cfg, seed=0, snr=30.0):
    nx, ny, nc, q, r, kind, lm, var = cfg
    p = datagen.make_small(nx, ny, nc, q, r, seed=seed, kind=kind, n_lines=lm, m=lm, lowrank=False,
                           snr_db=snr, coils="random", variable_m=var)
    return Case(p)


@pytest.mark.parametrize("cfg", OP_CASES, ids=[f"{c[0]}x{c[1]}_{c[5]}" for c in OP_CASES])
def test_apply_A_and_AH_match_oracle(cfg):
    log(f"apply_A/AH {cfg}")
    cs = _case(cfg)
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(5)
    X = datagen.crandn(rng, cs.prob.n, cs.prob.q).astype(np.complex64).astype(np.complex128)
    Xg = torch.from_numpy(np.ascontiguousarray(X.T.astype(np.complex64))).cuda()
    Yg = ctx.apply_A(Xg)
    Yref = cs.op.apply_A(X)
    Ygn = Yg.cpu().numpy().astype(np.complex128)
    assert rel(Ygn, Yref) < 1e-5
    # padding is written as zero
    for k in range(cs.prob.q):
        assert np.all(Ygn[k, :, cs.m_k[k]:] == 0)
    Xa = ctx.apply_AH(torch.from_numpy(cs.y32).cuda())
    Xref = cs.op.apply_AH(cs.y)
    assert rel(Xa.cpu().numpy().T.astype(np.complex128), Xref) < 1e-5
    # adjoint identity on the GPU's own operators
    Yr = datagen.crandn(rng, *cs.y.shape)
    Yr = np.where(np.arange(cs.y.shape[2])[None, None, :] < cs.m_k[:, None, None], Yr, 0).astype(np.complex64)
    AHY = ctx.apply_AH(torch.from_numpy(Yr).cuda()).cpu().numpy().T.astype(np.complex128)
    lhs = np.vdot(Ygn, Yr.astype(np.complex128))
    rhs = np.vdot(X, AHY)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("cfg", OP_CASES, ids=[f"{c[0]}x{c[1]}_{c[5]}" for c in OP_CASES])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "mixed"])
def test_ls_step_and_gradient_match_oracle(cfg, precision):
    log(f"gradient {cfg} precision={precision}")
    cs = _case(cfg, seed=1)
    ctx = cs.gpu_ctx(precision=precision)
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(datagen.crandn(rng, cs.prob.n, cs.prob.r))
    U = U.astype(np.complex64).astype(np.complex128)
    Bg, Gg = ctx.gradient(to_gpu_U(U))
    B = from_gpu_B(Bg)
    G = from_gpu_U(Gg)
    Bref = AG.ls_step(cs.op, U, cs.y)
    Gref = AG.gradient(cs.op, U, Bref, cs.y)
    conds = []
    FU = cs.op.transform_basis(U)
    for k in range(cs.prob.q):
        Mk = cs.op.AU(k, U, FU)
        conds.append(np.linalg.cond(Mk.conj().T @ Mk))
    tol_b = 1e-5 * max(1.0, max(conds) / 10.0)
    assert rel(B, Bref) < tol_b, (rel(B, Bref), max(conds))
    # grad = T1 - T2 with T1 = sum_k A_k^H A_k U b_k b_k^H, T2 = sum_k A_k^H y_k b_k^H:
    # normalise by the larger of the two terms
    t1 = np.linalg.norm(AG.gradient(cs.op, U, Bref, np.zeros_like(cs.y)))
    t2 = np.linalg.norm(AG.gradient(cs.op, np.zeros_like(U), Bref, cs.y))
    scale = max(t1, t2)
    err = np.linalg.norm(G - Gref) / scale
    log(f"  b rel {rel(B, Bref):.2e} (tol {tol_b:.1e}), grad rel/scale {err:.2e}, plain {rel(G, Gref):.2e}")
    assert err < 1e-5


def test_spectral_init_matches_oracle():
    log("init gauss64")
    cs = Case(datagen.make("gauss64", 0))
    ctx = cs.gpu_ctx()
    U0 = from_gpu_U(ctx.init())
    st = ctx.stats()
    Ytr, gamma, _ = AG.truncation(cs.op, cs.y, 36.0)
    X0 = AG.backprojection(cs.op, Ytr)
    s = np.linalg.svd(X0, compute_uv=False)
    Uref = AG.spectral_init(X0, cs.prob.r)
    assert st["gamma"] == pytest.approx(gamma, rel=1e-12)
    assert st["n_trunc"] == AG.truncation_count(cs.op, cs.y, 36.0)
    assert np.allclose(U0.conj().T @ U0, np.eye(cs.prob.r), atol=2e-6)
    gap = (s[cs.prob.r - 1] - s[cs.prob.r]) / s[0]
    d = proj_dist(U0, Uref)
    log(f"  projector distance {d:.2e}, relative gap {gap:.2e}")
    assert d < 1e-6 / gap


@pytest.mark.parametrize("cfg", [(32, 32, 3, 8, 3, "lines", 10, True), (32, 32, 3, 8, 3, "index", 400, True),
                                 (64, 32, 4, 12, 4, "lines", 12, False),
                                 # frame counts at the eigen-solver's and the Gram's boundaries:
                                 # q = 48 / 49 (real-tile / complex-tile Gram), q = 64 with r = 9
                                 # (matrix in LDS, workgroup back-transformation), q = 65 and 128
                                 # (packed lower triangle, the largest LDS footprint)
                                 (32, 32, 2, 48, 6, "lines", 10, True), (32, 32, 2, 49, 6, "lines", 10, True),
                                 (32, 32, 2, 64, 9, "lines", 10, True), (32, 32, 2, 65, 5, "lines", 10, True),
                                 (32, 32, 2, 128, 16, "lines", 10, True)],
                         ids=["lines32", "index32", "lines64x32", "q48", "q49", "q64r9", "q65", "q128r16"])
def test_spectral_init_small_shapes(cfg):
    log(f"init {cfg}")
    nx, ny, nc, q, r, kind, lm, var = cfg
    p = datagen.make_small(nx, ny, nc, q, r, seed=3, kind=kind, n_lines=lm, m=lm, lowrank=True,
                           snr_db=40.0, variable_m=var)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    U0 = from_gpu_U(ctx.init())
    Ytr, gamma, _ = AG.truncation(cs.op, cs.y, 36.0)
    X0 = AG.backprojection(cs.op, Ytr)
    s = np.linalg.svd(X0, compute_uv=False)
    Uref = AG.spectral_init(X0, r)
    gap = (s[r - 1] - s[r]) / s[0]
    d = proj_dist(U0, Uref)
    log(f"  projector distance {d:.2e}, relative gap {gap:.2e}, truncated {ctx.stats()['n_trunc']}")
    assert d < 1e-6 / gap
    assert ctx.stats()["n_trunc"] == AG.truncation_count(cs.op, cs.y, 36.0)


def _end_to_end(cs, T, trunc_c=36.0, precision=0):
    ctx = cs.gpu_ctx(precision=precision, trunc_c=trunc_c)
    U = ctx.init()
    Uprev = torch.empty_like(U)
    B, done = ctx.iterate(T, U, U_prev=Uprev, sync=True)
    assert done == T
    Xg = from_gpu_U(Uprev) @ from_gpu_B(B)
    ref = AG.run(cs.op, cs.y, AG.Params(r=cs.prob.r, trunc_c=trunc_c), t_fixed=T, record=False)
    return ctx, Xg, ref


def test_end_to_end_gauss64_20_iterations():
    """The exact-low-rank 64x64 workload (4 coils, 16 frames, rank 4,
    noise-free), 20 iterations."""
    log("end-to-end gauss64")
    cs = Case(datagen.make("gauss64", 0))
    ctx, Xg, ref = _end_to_end(cs, 20)
    n_gpu = M.nmse(Xg, cs.prob.zstar)
    n_ref = M.nmse(ref.X, cs.prob.zstar)
    log(f"  NMSE gpu {n_gpu:.6e} oracle {n_ref:.6e}; X rel {rel(Xg, ref.X):.2e}")
    assert abs(n_gpu - n_ref) <= 1e-4
    assert rel(Xg, ref.X) < 1e-3
    eta = ctx.get_eta()
    assert eta == pytest.approx(ref.eta, rel=1e-4)


@pytest.mark.parametrize("kind", ["lines", "index"])
def test_end_to_end_small_ragged(kind):
    log(f"end-to-end small {kind}")
    p = datagen.make_small(32, 16, 3, 10, 2, seed=4, kind=kind, n_lines=6, m=170, lowrank=True,
                           snr_db=35.0, variable_m=True)
    cs = Case(p)
    ctx, Xg, ref = _end_to_end(cs, 15)
    assert abs(M.nmse(Xg, p.zstar) - M.nmse(ref.X, p.zstar)) <= 1e-4
    assert rel(Xg, ref.X) < 1e-3


@pytest.mark.parametrize("r", [3, 5, 7, 8, 12, 16])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "mixed"])
def test_end_to_end_ranks_around_the_step_kernels(r, precision):
    """Ranks up to 8 run the QR step fused with the update (odd ranks take
    the 8-byte path of the partial-sum kernel and the strided rows of the
    update); ranks above 8 the separate step (one-wave factor of 16 rows) and
    update, with the QR Gram of three or four row tiles."""
    log(f"end-to-end r={r} precision={precision}")
    p = datagen.make_small(32, 32, 3, 20, r, seed=30 + r, kind="lines", n_lines=12, lowrank=True,
                           snr_db=40.0, variable_m=True)
    cs = Case(p)
    ctx, Xg, ref = _end_to_end(cs, 8, precision=precision)
    st = ctx.stats()
    n_gpu, n_ref = M.nmse(Xg, p.zstar), M.nmse(ref.X, p.zstar)
    log(f"  NMSE gpu {n_gpu:.6e} oracle {n_ref:.6e}; X rel {rel(Xg, ref.X):.2e}; t {st['t']}")
    assert st["t"] == 8
    assert abs(n_gpu - n_ref) <= 1e-4
    assert rel(Xg, ref.X) < 1e-3
    assert ctx.get_eta() == pytest.approx(ref.eta, rel=1e-4)


@pytest.mark.parametrize("r", [5, 8, 13, 16])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "mixed"])
def test_end_to_end_general_mask_ranks(r, precision):
    """General (index) masks at ranks that take each shape of the per-frame
    Gram (the W row and the sample's y as 2r + 2 real columns in one, two or
    three 16-column tiles) and of the fold's register tile (8, 16), with two
    sample chunks per frame (the second ragged) and a coil count below the
    eight coil slots of the Gram's grid."""
    log(f"end-to-end general mask r={r} precision={precision}")
    p = datagen.make_small(64, 32, 3, 20, r, seed=60 + r, kind="index", m=700, lowrank=True,
                           snr_db=40.0, variable_m=True)
    cs = Case(p)
    assert int(max(cs.m_k)) > 512  # two sample chunks of the Gram in the longest frames
    ctx, Xg, ref = _end_to_end(cs, 8, precision=precision)
    st = ctx.stats()
    n_gpu, n_ref = M.nmse(Xg, p.zstar), M.nmse(ref.X, p.zstar)
    log(f"  NMSE gpu {n_gpu:.6e} oracle {n_ref:.6e}; X rel {rel(Xg, ref.X):.2e}; t {st['t']}")
    assert st["t"] == 8
    assert abs(n_gpu - n_ref) <= 1e-4
    assert rel(Xg, ref.X) < 1e-3
    assert ctx.get_eta() == pytest.approx(ref.eta, rel=1e-4)


def test_end_to_end_general_mask_more_coils_than_xcds():
    """Twelve coils on general masks: the Gram's grid deals coil c to slot
    c mod 8 of two coil groups (slots 12..15 empty)."""
    log("end-to-end general mask, 12 coils")
    p = datagen.make_small(32, 32, 12, 12, 6, seed=71, kind="index", m=600, lowrank=True,
                           snr_db=40.0, variable_m=True)
    cs = Case(p)
    ctx, Xg, ref = _end_to_end(cs, 6)
    n_gpu, n_ref = M.nmse(Xg, p.zstar), M.nmse(ref.X, p.zstar)
    log(f"  NMSE gpu {n_gpu:.6e} oracle {n_ref:.6e}; X rel {rel(Xg, ref.X):.2e}")
    assert abs(n_gpu - n_ref) <= 1e-4
    assert rel(Xg, ref.X) < 1e-3
    assert ctx.get_eta() == pytest.approx(ref.eta, rel=1e-4)


@pytest.mark.parametrize("ny,r", [(64, 9), (64, 12), (128, 16), (64, 16), (256, 12)])
def test_end_to_end_fused_adjoint_gram_ranks_above_8(ny, r):
    """Image columns of 64 and 128 pixels: the adjoint transform also forms
    the QR Gram of [U grad] per column, here with three and four row tiles
    of the real embedding (ranks 9 to 16), which the separate QR step then
    sums over the columns."""
    log(f"end-to-end fused adjoint Gram ny={ny} r={r}")
    p = datagen.make_small(32, ny, 3, 20, r, seed=40 + r, kind="lines", n_lines=ny // 3, lowrank=True,
                           snr_db=40.0, variable_m=True)
    cs = Case(p)
    ctx, Xg, ref = _end_to_end(cs, 6)
    n_gpu, n_ref = M.nmse(Xg, p.zstar), M.nmse(ref.X, p.zstar)
    log(f"  NMSE gpu {n_gpu:.6e} oracle {n_ref:.6e}; X rel {rel(Xg, ref.X):.2e}")
    assert abs(n_gpu - n_ref) <= 1e-4
    assert rel(Xg, ref.X) < 1e-3
    assert ctx.get_eta() == pytest.approx(ref.eta, rel=1e-4)


def test_mixed_precision_end_to_end_gauss64():
    log("end-to-end gauss64 mixed")
    cs = Case(datagen.make("gauss64", 0))
    ctx, Xg, ref = _end_to_end(cs, 20, precision=1)
    assert abs(M.nmse(Xg, cs.prob.zstar) - M.nmse(ref.X, cs.prob.zstar)) <= 1e-4


@pytest.mark.parametrize("r", [5, 6, 7, 10])
def test_gradient_with_rank_below_the_register_tile(r):
    """Ranks below the kernels' register tile (4, 8, 16): the padded rows and
    columns of the per-line S_u must not enter the fold."""
    log(f"gradient r={r}")
    p = datagen.make_small(64, 64, 3, 12, r, seed=20 + r, kind="lines", n_lines=14, lowrank=False,
                           snr_db=30.0, coils="random", variable_m=True)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(r)
    U, _ = np.linalg.qr(datagen.crandn(rng, cs.prob.n, r))
    U = U.astype(np.complex64).astype(np.complex128)
    for rep in range(3):  # repeated launches see different leftover LDS contents
        Bg, Gg = ctx.gradient(to_gpu_U(U))
        G = from_gpu_U(Gg)
        assert np.all(np.isfinite(G))
    Bref = AG.ls_step(cs.op, U, cs.y)
    Gref = AG.gradient(cs.op, U, Bref, cs.y)
    t1 = np.linalg.norm(AG.gradient(cs.op, U, Bref, np.zeros_like(cs.y)))
    t2 = np.linalg.norm(AG.gradient(cs.op, np.zeros_like(U), Bref, cs.y))
    assert np.linalg.norm(G - Gref) / max(t1, t2) < 1e-5


@pytest.mark.parametrize("r", [4, 8])
def test_exit_rule_matches_oracle(r):
    """Algorithm 2's exit rule SD(U, U+)/sqrt(r) < 0.01 (with the exit rule
    on, the fused step's outcome goes through the commit kernel): the GPU
    stops at the oracle's iteration and returns the same X = U_{t-1} B_t.
    The seed is one where every SD of the oracle's run lies at least 1 %
    from the threshold (checked here), far beyond the GPU's error on SD."""
    log(f"exit rule r={r}")
    eps = 0.01
    p = datagen.make_small(32, 32, 3, 20, r, seed=43, kind="lines", n_lines=12, lowrank=True, snr_db=40.0,
                           variable_m=True)
    cs = Case(p)
    ref = AG.run(cs.op, cs.y, AG.Params(r=r, eps_exit=eps), record=True)
    sd = np.array(ref.history["sd"]) / np.sqrt(r)
    assert ref.history["exit_at"] == ref.iters and ref.iters < 70
    assert np.min(np.abs(sd - eps)) > 0.01 * eps
    ctx = cs.gpu_ctx(eps_exit=eps)
    U = ctx.init()
    Uprev = torch.empty_like(U)
    B, done = ctx.iterate(70, U, U_prev=Uprev, sync=True)
    st = ctx.stats()
    Xg = from_gpu_U(Uprev) @ from_gpu_B(B)
    log(f"  iterations gpu {done} oracle {ref.iters}; X rel {rel(Xg, ref.X):.2e}; sd/sqrt(r) gpu {st['sd'] / np.sqrt(r):.6f}")
    assert done == ref.iters and st["t"] == ref.iters and st["exited"] == 1
    assert st["sd"] / np.sqrt(r) == pytest.approx(sd[-1], rel=1e-3)
    assert rel(Xg, ref.X) < 1e-3


@pytest.mark.parametrize("r", [5, 8])
def test_step_commit_paths_agree(r):
    """Rank <= 8 runs the QR step fused with the update.  With the exit rule
    off, workgroup 0 commits t and eta itself; with it on, a one-thread
    kernel commits them after the step.  A threshold that never fires must
    leave the whole trajectory bitwise unchanged."""
    log(f"commit paths r={r}")
    p = datagen.make_small(32, 32, 3, 20, r, seed=44, kind="lines", n_lines=12, lowrank=True, snr_db=40.0,
                           variable_m=True)
    cs = Case(p)
    out = []
    for eps in (0.0, 1e-30):
        ctx = cs.gpu_ctx(eps_exit=eps)
        U = ctx.init()
        B, done = ctx.iterate(10, U, sync=True)
        out.append((U.clone(), B.clone(), done, ctx.get_eta(), ctx.stats()))
    (Ua, Ba, da, ea, sa), (Ub, Bb, db, eb, sb) = out
    assert da == db == 10 and sa["t"] == sb["t"] == 10
    assert sa["exited"] == 0 and sb["exited"] == 0
    assert torch.equal(Ua, Ub) and torch.equal(Ba, Bb)
    assert ea == eb and sa["f"] == sb["f"] and sa["sd"] == sb["sd"]


@pytest.mark.parametrize("bind", [True, False], ids=["cap_binds", "cap_loose"])
def test_step_size_cap_matches_oracle(bind):
    """The optional step-size cap eta <= c n / (mbar ||B_0||_2^2) (the
    conservative rule of Sec. III-B): c is chosen from the oracle's own
    uncapped eta so that the cap binds (half the rule's eta) or not (twice);
    the GPU's eta and trajectory match the oracle's."""
    p = datagen.make_small(32, 32, 3, 12, 3, seed=51, kind="lines", n_lines=10, lowrank=True, snr_db=40.0,
                           variable_m=True)
    cs = Case(p)
    T = 6
    free = AG.run(cs.op, cs.y, AG.Params(r=3), t_fixed=1, record=False)
    B0 = AG.ls_step(cs.op, free.U0, cs.y)
    cap1 = AG.step_size_cap(cs.op, B0, 1.0)
    c = (0.5 if bind else 2.0) * free.eta / cap1
    ref = AG.run(cs.op, cs.y, AG.Params(r=3, eta_cap_c=c), t_fixed=T, record=True)
    assert ref.history["eta_capped"] is bind
    ctx = cs.gpu_ctx(eta_cap_c=c)
    U = ctx.init()
    Uprev = torch.empty_like(U)
    B, done = ctx.iterate(T, U, U_prev=Uprev, sync=True)
    assert done == T
    Xg = from_gpu_U(Uprev) @ from_gpu_B(B)
    eta = ctx.get_eta()
    log(f"  c {c:.4e}: eta gpu {eta:.6e} oracle {ref.eta:.6e} (uncapped {free.eta:.6e}); X rel {rel(Xg, ref.X):.2e}")
    assert eta == pytest.approx(ref.eta, rel=1e-4)
    assert abs(M.nmse(Xg, p.zstar) - M.nmse(ref.X, p.zstar)) <= 1e-4
    assert rel(Xg, ref.X) < 1e-3


def test_statistics_survive_a_later_cost_call():
    """With the exit rule off the loop defers its statistics; a cost or
    gradient call in between (which reruns the per-frame solve) must not
    change what get_stats then reports for the last iteration."""
    p = datagen.make_small(32, 32, 3, 12, 4, seed=52, kind="lines", n_lines=10, lowrank=True, snr_db=40.0)
    cs = Case(p)
    want = None
    for eps in (1e-30, 0.0):  # commit kernel (statistics formed at once), then deferred
        ctx = cs.gpu_ctx(eps_exit=eps)
        U = ctx.init()
        ctx.iterate(5, U)
        other = to_gpu_U(np.linalg.qr(datagen.crandn(np.random.default_rng(3), p.n, p.r))[0])
        ctx.cost(other)
        ctx.gradient(other)
        st = ctx.stats()
        if want is None:
            want = st
    log(f"  f {st['f']:.9e} vs {want['f']:.9e}; sd {st['sd']:.6e} vs {want['sd']:.6e}")
    assert st["t"] == want["t"] == 5
    assert st["f"] == pytest.approx(want["f"], rel=1e-12)
    assert st["sd"] == pytest.approx(want["sd"], rel=1e-9)
    assert st["grad_norm"] == pytest.approx(want["grad_norm"], rel=1e-12)


def test_iteration_count_on_a_non_default_stream():
    """iterate(sync=True) reads the starting iteration count only after the
    stream's earlier work (init and the previous iterate) has finished."""
    p = datagen.make_small(64, 64, 4, 16, 4, seed=53, kind="lines", n_lines=16, lowrank=True, snr_db=40.0)
    cs = Case(p)
    s = torch.cuda.Stream()
    import paper_2212_09664_amd as ag
    ctx = ag.AltGDmin(p.nx, p.ny, p.nc, p.q, p.r, int(cs.y.shape[2]), 0, 0)
    dev = torch.device("cuda:0")
    with torch.cuda.stream(s):
        ctx.set_problem(torch.from_numpy(cs.coils.astype(np.complex64)).to(dev),
                        torch.from_numpy(cs.mask).to(dev), torch.from_numpy(cs.m_k).to(dev),
                        torch.from_numpy(cs.y32).to(dev), stream=s)
        U = ctx.init()
        counts = []
        for n in (7, 3, 5):
            _, done = ctx.iterate(n, U, sync=True)
            counts.append(done)
    log(f"  iterations reported {counts}")
    assert counts == [7, 3, 5]
    assert ctx.stats()["t"] == 15
