"""GPU (through the C ABI) versus the FP64 oracle for the steps around the
altGDmin loop: the mean image and residuals (Algorithm 1), the automatic
rank and the consecutive-exit variant (Algorithm 2's parameter setting,
Sec. VI), MEC-1 and MEC-2 (Algorithm 3), the whole pipeline and the
tracking drivers (Algorithms 4 and 5).

Tolerances: operators (the residual) 1e-5 relative; the iterative steps
(CG for the mean, per-frame CGLS, ISTA) are compared after the same number
of iterations at 1e-4 relative (their FP32 iterates drift from the FP64 ones
by the accumulated rounding of each iteration's reductions); end to end,
|NMSE_gpu - NMSE_oracle| <= 1e-4."""
import numpy as np
import pytest

import datagen
from oracle import altgdmin as AG
from oracle import metrics as M
from oracle import mri as R

from gpu_cases import GPU_OK, Case, log, rel

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not GPU_OK, reason="needs a GPU")]

if GPU_OK:
    import torch

CASES = [
    # (nx, ny, nc, q, r, kind, lines/m)
    (32, 32, 3, 10, 2, "lines", 10),
    (64, 32, 4, 12, 3, "lines", 9),
    (32, 32, 3, 8, 2, "index", 300),
]
IDS = [f"{c[0]}x{c[1]}_{c[5]}" for c in CASES]


def _case(cfg, seed=0, snr=30.0, mean_scale=3.0):
    """A mean-dominated sequence: Z* = zbar 1^T + (rank-r part) + noise."""
    nx, ny, nc, q, r, kind, lm = cfg
    p = datagen.make_small(nx, ny, nc, q, r, seed=seed, kind=kind, n_lines=lm, m=lm, lowrank=True,
                           snr_db=snr, variable_m=True)
    rng = np.random.default_rng(seed + 100)
    p.zstar = p.zstar + mean_scale * np.abs(p.zstar).mean() * datagen.crandn(rng, p.n)[:, None]
    return Case(p)


def _dev(cs):
    d = torch.device("cuda:0")
    return (torch.from_numpy(cs.coils.astype(np.complex64)).to(d), torch.from_numpy(cs.mask).to(d),
            torch.from_numpy(cs.m_k).to(d), torch.from_numpy(cs.y32).to(d))


def _np_img(t):
    """(q, n) or (n,) device tensor -> n x q (or n) complex128."""
    a = t.detach().cpu().numpy().astype(np.complex128)
    return a.T if a.ndim == 2 else a


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_mean_image_matches_oracle(cfg):
    """Same number of iterations on both sides (tolerance 0), then the
    paper's setting (1e-3, at most 10) with the same stopping iteration."""
    log(f"mean {cfg}")
    cs = _case(cfg)
    ctx = cs.gpu_ctx()
    for tol, maxit in ((0.0, 6), (1e-3, 10)):
        z, it = ctx.mean(tol, maxit, sync=True)
        zr, itr = R.mean_image(cs.op, cs.y, tol=tol, maxit=maxit)
        e = rel(_np_img(z), zr)
        log(f"  tol {tol}: iterations gpu {it} oracle {itr}; zbar rel {e:.2e}")
        assert it == itr
        assert e < 1e-4


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_residual_matches_oracle(cfg):
    cs = _case(cfg)
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(1)
    zb = datagen.crandn(rng, cs.prob.n).astype(np.complex64)
    X = datagen.crandn(rng, cs.prob.n, cs.prob.q).astype(np.complex64)
    zg = torch.from_numpy(zb).cuda()
    Xg = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    for a, b in ((zg, None), (None, Xg), (zg, Xg)):
        out = ctx.residual(zbar=a, X=b).cpu().numpy().astype(np.complex128)
        ref = R.residual(cs.op, cs.y, None if a is None else zb.astype(np.complex128),
                         None if b is None else X.astype(np.complex128))
        e = rel(out, ref)
        log(f"  residual rel {e:.2e}")
        assert e < 1e-5
        for k in range(cs.prob.q):
            assert np.all(out[k, :, cs.m_k[k]:] == 0)


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_mec1_matches_oracle(cfg):
    cs = _case(cfg)
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(2)
    Yr = cs.op.apply_A(0.05 * datagen.crandn(rng, cs.prob.n, cs.prob.q)).astype(np.complex64)
    E = ctx.mec_cgls(torch.from_numpy(Yr).cuda(), 3, 1e-36)
    Er = R.mec1(cs.op, Yr.astype(np.complex128))
    e = rel(_np_img(E), Er)
    log(f"  MEC-1 rel {e:.2e}")
    assert e < 1e-4


@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_mec2_matches_oracle(cfg):
    """ISTA: the same number of updates and the same E.  The stop test
    compares a relative change with the tolerance; every change of the
    oracle's run lies at least 5 % away from it (checked), so FP32 rounding
    cannot move the stopping iteration."""
    cs = _case(cfg)
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(3)
    S = np.zeros((cs.prob.n, cs.prob.q), dtype=np.complex128)
    idx = rng.integers(0, cs.prob.n, 60)
    S[idx, rng.integers(0, cs.prob.q, 60)] = datagen.crandn(rng, 60)
    Yr = (cs.op.apply_A(R.temporal_idft(S)) + 1e-3 * cs.op.apply_A(datagen.crandn(rng, cs.prob.n, cs.prob.q)))
    Yr = Yr.astype(np.complex64)
    # the paper's tolerance (no early stop here: every change stays above it)
    # and a looser one at which the loop stops early (changes >= 9 % away)
    for tol in (0.0025, 0.04):
        ref = R.mec2(cs.op, Yr.astype(np.complex128), tol=tol)
        E, it = ctx.mec_ista(torch.from_numpy(Yr).cuda(), 10, 1e-3, tol, sync=True)
        e = rel(_np_img(E), ref.E)
        log(f"  MEC-2 tol {tol}: updates gpu {it} oracle {ref.iters}; omega {ref.omega:.4e}; E rel {e:.2e}")
        assert min(abs(c - tol) for c in ref.changes) > 0.05 * tol
        assert it == ref.iters
        assert e < 1e-4


@pytest.mark.parametrize("name", ["cine256", "radial128"])
def test_mean_and_rank_at_full_size(name):
    """The workloads' own shapes: the mean image (the paper's settings) and
    the spectrum behind the automatic rank."""
    from test_gpu_workloads import _get
    cs = _get(name)
    ctx = cs.gpu_ctx()
    z, it = ctx.mean(1e-3, 10, sync=True)
    zr, itr = R.mean_image(cs.op, cs.y)
    e = rel(_np_img(z), zr)
    log(f"  {name} mean: iterations gpu {it} oracle {itr}; rel {e:.2e}")
    assert it == itr and e < 1e-4
    cap = R.rank_cap(cs.op)
    rr, rc = ctx.auto_rank(85.0)
    Ytr, _, _ = AG.truncation(cs.op, cs.y, 36.0)
    X0 = AG.backprojection(cs.op, Ytr)
    s2 = np.linalg.svd(X0, compute_uv=False)[:rc] ** 2
    g2 = np.array(ctx.rank_energy(rc))
    log(f"  {name} rank: r_cap gpu {rc} oracle {cap}; r gpu {rr} oracle {R.auto_rank(X0, cap)}; "
        f"energies rel {np.abs(g2 - s2).max() / s2[0]:.2e}")
    assert rc == cap
    assert np.abs(g2 - s2).max() <= 1e-5 * s2[0]
    assert rr == R.auto_rank(X0, cap)


def test_auto_rank_matches_oracle_with_margin():
    """A sequence of exact rank 3 plus weak noise, q = 40 frames (r_cap = 4):
    both sides pick the same r and no cumulative energy is within 1e-4 of
    the 85 % threshold."""
    p = datagen.make_small(32, 32, 4, 40, 3, seed=7, kind="lines", n_lines=14, lowrank=True, snr_db=40.0)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    rr, rc = ctx.auto_rank(85.0)
    Ytr, _, _ = AG.truncation(cs.op, cs.y, 36.0)
    X0 = AG.backprojection(cs.op, Ytr)
    cap = R.rank_cap(cs.op)
    s2 = np.linalg.svd(X0, compute_uv=False)[:cap] ** 2
    frac = np.cumsum(s2) / s2.sum()
    log(f"  r gpu {rr} oracle {R.auto_rank(X0, cap)}; cap {rc}/{cap}; cumulative {frac}")
    assert np.min(np.abs(frac - 0.85)) > 1e-4
    assert rc == cap and rr == R.auto_rank(X0, cap)


@pytest.mark.parametrize("consec", [2, 3])
@pytest.mark.parametrize("r", [4, 10])
def test_consecutive_exit_matches_oracle(consec, r):
    """The exit rule's Sec. VI variant on both step paths (rank <= 8: the
    fused step with its commit kernel; rank > 8: the separate step): the GPU
    stops at the oracle's iteration.  The seed keeps every SD/sqrt(r) at
    least 1 % away from the threshold."""
    eps = 0.01
    p = datagen.make_small(32, 32, 3, 20, r, seed={4: 46, 10: 44}[r], kind="lines", n_lines=14, lowrank=True,
                           snr_db=40.0, variable_m=True)
    cs = Case(p)
    ref = AG.run(cs.op, cs.y, AG.Params(r=r, eps_exit=eps, exit_consec=consec))
    sd = np.array(ref.history["sd"]) / np.sqrt(r)
    assert ref.iters < 70 and np.min(np.abs(sd - eps)) > 0.01 * eps
    import paper_2212_09664_amd as ag
    ctx2 = ag.AltGDmin(p.nx, p.ny, p.nc, p.q, p.r, int(cs.y.shape[2]), 0, 0, eps_exit=eps, exit_consec=consec)
    ctx2.set_problem(*_dev(cs))
    U = ctx2.init()
    Up = torch.empty_like(U)
    B, done = ctx2.iterate(70, U, U_prev=Up, sync=True)
    st = ctx2.stats()
    log(f"  consec {consec} r {r}: iterations gpu {done} oracle {ref.iters}")
    assert done == ref.iters and st["exited"] == 1
    X = _np_img(Up) @ B.cpu().numpy().astype(np.complex128).T  # (n, r) @ (r, q)
    assert rel(X, ref.X) < 1e-3


@pytest.mark.parametrize("mec", [1, 2])
@pytest.mark.parametrize("cfg", CASES, ids=IDS)
def test_pipeline_matches_oracle(cfg, mec):
    """Algorithm 1 end to end (mean, residual, altGDmin for 15 iterations,
    second residual, MEC) on both sides."""
    from paper_2212_09664_amd import mri
    cs = _case(cfg, seed=5)
    nx, ny, nc, q, r, kind, _ = cfg
    coils, mask, m_k, y = _dev(cs)
    out = mri.altgdmin_mri(coils, mask, m_k, y, nx, ny, r, mask_kind=0 if kind == "lines" else 1, mec=mec, T=15)
    ref = R.altgdmin_mri(cs.op, cs.y, AG.Params(r=r), mec=mec, t_fixed=15)
    Zg = _np_img(out.Z)
    ng, nr = M.nmse(Zg, cs.prob.zstar), M.nmse(ref.Z, cs.prob.zstar)
    log(f"  MEC-{mec}: NMSE gpu {ng:.6e} oracle {nr:.6e}; Z rel {rel(Zg, ref.Z):.2e}; mean iters "
        f"{out.mean_iters}/{ref.mean_iters}; mec iters {out.mec_iters}/{ref.mec_iters}")
    assert abs(ng - nr) <= 1e-4
    assert rel(Zg, ref.Z) < 1e-3
    assert out.mean_iters == ref.mean_iters and out.mec_iters == ref.mec_iters


def test_pipeline_with_auto_rank_matches_oracle():
    from paper_2212_09664_amd import mri
    p = datagen.make_small(32, 32, 4, 40, 3, seed=7, kind="lines", n_lines=14, lowrank=True, snr_db=40.0)
    cs = Case(p)
    coils, mask, m_k, y = _dev(cs)
    out = mri.altgdmin_mri(coils, mask, m_k, y, p.nx, p.ny, 8, mec=1, auto_rank=True, T=10)
    ref = R.altgdmin_mri(cs.op, cs.y, AG.Params(r=8), mec=1, auto=True, t_fixed=10)
    Zg = _np_img(out.Z)
    log(f"  auto rank gpu {out.r} oracle {ref.r}; NMSE gpu {M.nmse(Zg, p.zstar):.6e} oracle {M.nmse(ref.Z, p.zstar):.6e}")
    assert out.r == ref.r
    assert abs(M.nmse(Zg, p.zstar) - M.nmse(ref.Z, p.zstar)) <= 1e-4


def test_minibatch_tracking_matches_oracle():
    from paper_2212_09664_amd import mri
    cs = _case((32, 32, 3, 12, 2, "lines", 10), seed=9)
    coils, mask, m_k, y = _dev(cs)
    Zg = _np_img(mri.minibatch_st(coils, mask, m_k, y, 32, 32, 2, alpha=4, t_first=15, t_next=5))
    Zr = R.minibatch_st(cs.op, cs.y, AG.Params(r=2), alpha=4, t_first=15, t_next=5)
    ng, nr = M.nmse(Zg, cs.prob.zstar), M.nmse(Zr, cs.prob.zstar)
    log(f"  mini-batch: NMSE gpu {ng:.6e} oracle {nr:.6e}; Z rel {rel(Zg, Zr):.2e}")
    assert abs(ng - nr) <= 1e-4 and rel(Zg, Zr) < 1e-3


def test_online_tracking_matches_oracle():
    from paper_2212_09664_amd import mri
    cs = _case((32, 32, 3, 12, 2, "lines", 10), seed=10)
    coils, mask, m_k, y = _dev(cs)
    Zg = _np_img(mri.online_st(coils, mask, m_k, y, 32, 32, 2, alpha=6, T=15))
    Zr = R.online_st(cs.op, cs.y, AG.Params(r=2, t_max=15), alpha=6)
    ng, nr = M.nmse(Zg, cs.prob.zstar), M.nmse(Zr, cs.prob.zstar)
    log(f"  online: NMSE gpu {ng:.6e} oracle {nr:.6e}; Z rel {rel(Zg, Zr):.2e}")
    assert abs(ng - nr) <= 1e-4 and rel(Zg, Zr) < 1e-3
