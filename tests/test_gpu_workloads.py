"""GPU versus the FP64 oracle on the five workload shapes at their full sizes
(the sizes the throughput benchmark runs), in the library's production launch
configuration.

Per workload: the spectral initialisation (projector distance bounded by the
eigen-gap), the LS step and the gradient at a fixed orthonormal basis (the
operator tolerances of the small-case tests), a few whole iterations against
the oracle's trajectory, and — for the cine 256 x 256 workload — the full
70-iteration run checked by properties that hold at any size (orthonormal U,
U^H grad = 0, the final B equal to the oracle's LS solution for the GPU's own
U, NMSE below 2e-2).
"""
import json
import os

import numpy as np
import pytest

import datagen
from oracle import altgdmin as AG
from oracle import metrics as M

from gpu_cases import GPU_OK, Case, from_gpu_B, from_gpu_U, log, proj_dist, rel, to_gpu_U

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not GPU_OK, reason="needs a GPU")]

if GPU_OK:
    import torch

SEEDS = {"cine256": 1001, "radial128": 0, "cine256r16": 0, "cine128": 0, "gauss64": 0}
_CASES = {}


def _get(name):
    if name not in _CASES:
        _CASES[name] = Case(datagen.make(name, SEEDS[name]))
    return _CASES[name]


@pytest.mark.parametrize("name", ["cine256", "radial128", "cine256r16", "cine128"])
def test_spectral_init_full_size(name):
    log(f"init {name}")
    cs = _get(name)
    r = cs.prob.r
    ctx = cs.gpu_ctx()
    U0 = from_gpu_U(ctx.init())
    Ytr, gamma, _ = AG.truncation(cs.op, cs.y, 36.0)
    X0 = AG.backprojection(cs.op, Ytr)
    s = np.linalg.svd(X0, compute_uv=False)
    Uref = AG.spectral_init(X0, r)
    gap = (s[r - 1] - s[r]) / s[0]
    d = proj_dist(U0, Uref)
    log(f"  projector distance {d:.2e}, relative gap {gap:.2e}, gamma {ctx.stats()['gamma']:.6e} vs {gamma:.6e}")
    assert ctx.stats()["gamma"] == pytest.approx(gamma, rel=1e-12)
    assert ctx.stats()["n_trunc"] == AG.truncation_count(cs.op, cs.y, 36.0)
    assert np.allclose(U0.conj().T @ U0, np.eye(r), atol=5e-6)
    assert d < 1e-6 / gap


@pytest.mark.parametrize("name", ["cine256", "radial128", "cine256r16", "cine128"])
def test_ls_step_and_gradient_full_size(name):
    log(f"gradient {name}")
    cs = _get(name)
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(11)
    U, _ = np.linalg.qr(datagen.crandn(rng, cs.prob.n, cs.prob.r))
    U = U.astype(np.complex64).astype(np.complex128)
    Bg, Gg = ctx.gradient(to_gpu_U(U))
    B, G = from_gpu_B(Bg), from_gpu_U(Gg)
    FU = cs.op.transform_basis(U)
    Bref = AG.ls_step(cs.op, U, cs.y, FU=FU)
    Gref = AG.gradient(cs.op, U, Bref, cs.y, FU=FU)
    t1 = np.linalg.norm(AG.gradient(cs.op, U, Bref, np.zeros_like(cs.y), FU=FU))
    t2 = np.linalg.norm(AG.gradient(cs.op, np.zeros_like(U), Bref, cs.y))
    err = np.linalg.norm(G - Gref) / max(t1, t2)
    log(f"  b rel {rel(B, Bref):.2e}, grad rel/scale {err:.2e}, plain {rel(G, Gref):.2e}")
    assert rel(B, Bref) < 1e-5
    assert err < 1e-5


@pytest.mark.parametrize("name,T", [("cine256", 3), ("radial128", 4), ("cine128", 8), ("gauss64", 20)])
def test_iterations_full_size(name, T):
    log(f"iterations {name} T={T}")
    cs = _get(name)
    ctx = cs.gpu_ctx()
    U = ctx.init()
    Uprev = torch.empty_like(U)
    B, done = ctx.iterate(T, U, U_prev=Uprev, sync=True)
    assert done == T
    Xg = from_gpu_U(Uprev) @ from_gpu_B(B)
    ref = AG.run(cs.op, cs.y, AG.Params(r=cs.prob.r), t_fixed=T, record=False)
    n_gpu, n_ref = M.nmse(Xg, cs.prob.zstar), M.nmse(ref.X, cs.prob.zstar)
    log(f"  NMSE gpu {n_gpu:.6e} oracle {n_ref:.6e}; X rel {rel(Xg, ref.X):.2e}; eta {ctx.get_eta():.6e} vs {ref.eta:.6e}")
    assert abs(n_gpu - n_ref) <= 1e-4
    assert ctx.get_eta() == pytest.approx(ref.eta, rel=1e-4)


def test_cine256_full_run_properties():
    """The benchmark's own run: 70 iterations at 256x256x12x40, rank 8."""
    log("cine256 70 iterations")
    cs = _get("cine256")
    ctx = cs.gpu_ctx()
    U = ctx.init()
    Uprev = torch.empty_like(U)
    B, done = ctx.iterate(70, U, U_prev=Uprev, sync=True)
    assert done == 70
    Up, Un, Bg = from_gpu_U(Uprev), from_gpu_U(U), from_gpu_B(B)
    r = cs.prob.r
    assert np.allclose(Un.conj().T @ Un, np.eye(r), atol=5e-6)
    # B_70 is the LS solution for U_69: the oracle's, from the GPU's own U_69
    Up64 = Up.astype(np.complex64).astype(np.complex128)
    Bref = AG.ls_step(cs.op, Up64, cs.y)
    log(f"  final B rel {rel(Bg, Bref):.2e}")
    assert rel(Bg, Bref) < 1e-5
    nm = M.nmse(Up @ Bg, cs.prob.zstar)
    log(f"  NMSE {nm:.4e}")
    assert nm < 2e-2
    # the gradient at the final basis is orthogonal to it (normal equations),
    # to FP32 accuracy relative to the two terms it is the difference of
    Bn, Gn = ctx.gradient(U)
    G = from_gpu_U(Gn)
    Bo = AG.ls_step(cs.op, Un, cs.y)
    scale = max(np.linalg.norm(AG.gradient(cs.op, Un, Bo, np.zeros_like(cs.y))),
                np.linalg.norm(AG.gradient(cs.op, np.zeros_like(Un), Bo, cs.y)))
    log(f"  ||U^H grad|| / scale {np.linalg.norm(Un.conj().T @ G) / scale:.2e}")
    assert np.linalg.norm(Un.conj().T @ G) <= 1e-5 * scale


@pytest.mark.parametrize("name", ["cine256r16", "cine256"])
def test_mixed_form_error_table(name):
    """Both forms against the FP64 oracle on the same inputs: relative error
    of every output the loop produces (b_k, the gradient, X after a few
    iterations, eta, NMSE).  The mixed form runs its ky transforms as FP16
    hi+lo MFMA partial DFTs and its Grams / Cholesky in FP64."""
    cs = _get(name)
    rng = np.random.default_rng(13)
    U, _ = np.linalg.qr(datagen.crandn(rng, cs.prob.n, cs.prob.r))
    U = U.astype(np.complex64).astype(np.complex128)
    FU = cs.op.transform_basis(U)
    Bref = AG.ls_step(cs.op, U, cs.y, FU=FU)
    Gref = AG.gradient(cs.op, U, Bref, cs.y, FU=FU)
    t1 = np.linalg.norm(AG.gradient(cs.op, U, Bref, np.zeros_like(cs.y), FU=FU))
    t2 = np.linalg.norm(AG.gradient(cs.op, np.zeros_like(U), Bref, cs.y))
    T = 3
    ref = AG.run(cs.op, cs.y, AG.Params(r=cs.prob.r), t_fixed=T, record=False)
    n_ref = M.nmse(ref.X, cs.prob.zstar)
    rows = []
    for precision, form in ((0, "plain"), (1, "mixed")):
        ctx = cs.gpu_ctx(precision=precision)
        Bg, Gg = ctx.gradient(to_gpu_U(U))
        eb = rel(from_gpu_B(Bg), Bref)
        eg = np.linalg.norm(from_gpu_U(Gg) - Gref) / max(t1, t2)
        U0 = ctx.init()
        Up = torch.empty_like(U0)
        B, _ = ctx.iterate(T, U0, U_prev=Up, sync=True)
        Xg = from_gpu_U(Up) @ from_gpu_B(B)
        ex = rel(Xg, ref.X)
        ee = abs(ctx.get_eta() - ref.eta) / ref.eta
        dn = abs(M.nmse(Xg, cs.prob.zstar) - n_ref)
        rows.append((form, eb, eg, ex, ee, dn))
        log(f"  {name} {form:6s} b_k {eb:.2e}  grad {eg:.2e}  X_{T} {ex:.2e}  eta {ee:.2e}  |dNMSE| {dn:.2e}")
        assert eb < 1e-5 and eg < 1e-5 and ex < 1e-4 and ee < 1e-4 and dn < 1e-4


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", ["cine256", "radial128", "cine256r16", "cine128"])
def test_full_run_matches_oracle(name):
    """The whole reconstruction at the workload's fixed iteration count
    (cine256, cine256r16, cine128: 70; radial128: 50) against the FP64
    oracle's run on the same
    inputs (stored by tests/golden/make_fullrun_goldens.py, which calls only
    the oracle and the input generator): NMSE after every iteration within
    1e-4, eta within 1e-4 relative, the same gamma and the same truncated
    samples, and X_T at 256 seeded positions."""
    with open(os.path.join(GOLDEN, f"fullrun_{name}.json")) as fh:
        g = json.load(fh)
    log(f"full run {name} T={g['T']}")
    cs = _get(name)
    assert g["seed"] == SEEDS[name] and g["r"] == cs.prob.r
    assert float(np.sum(np.abs(cs.y) ** 2)) == pytest.approx(g["inputs"]["y_sq"], rel=1e-12)
    assert float(np.sum(np.abs(cs.prob.zstar) ** 2)) == pytest.approx(g["inputs"]["zstar_sq"], rel=1e-12)
    ctx = cs.gpu_ctx()
    U = ctx.init()
    st = ctx.stats()
    assert st["gamma"] == pytest.approx(g["gamma"], rel=1e-12)
    assert st["n_trunc"] == g["n_trunc"]
    dev = U.device
    zs = torch.from_numpy(np.ascontiguousarray(cs.prob.zstar.T)).to(dev)  # (q, n) complex128
    zz = float(torch.sum(torch.abs(zs) ** 2).item())
    Uprev = torch.empty_like(U)
    B = None
    nm = []
    for t in range(g["T"]):
        B = ctx.iterate(1, U, U_prev=Uprev)
        X = B.to(torch.complex128) @ Uprev.to(torch.complex128)  # (q, n)
        nm.append(float(torch.sum(torch.abs(X - zs) ** 2).item()) / zz)
    dn = np.abs(np.array(nm) - np.array(g["nmse"]))
    Xg = X.cpu().numpy().T
    rng = np.random.default_rng(12345)
    pp, kk = rng.integers(0, cs.prob.n, 256), rng.integers(0, cs.prob.q, 256)
    xs = np.array(g["x_samples_re"]) + 1j * np.array(g["x_samples_im"])
    ex = rel(Xg[pp, kk], xs)
    en = abs(np.linalg.norm(Xg) - g["x_norm"]) / g["x_norm"]
    eta = ctx.get_eta()
    log(f"  NMSE_T gpu {nm[-1]:.6e} oracle {g['nmse'][-1]:.6e}; max_t |dNMSE| {dn.max():.2e}; "
        f"X_T rel (256 samples) {ex:.2e}; ||X_T|| rel {en:.2e}; eta rel {abs(eta - g['eta']) / g['eta']:.2e}")
    assert dn.max() <= 1e-4
    assert eta == pytest.approx(g["eta"], rel=1e-4)
    assert ex < 1e-3 and en < 1e-4
