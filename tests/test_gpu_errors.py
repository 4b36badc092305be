"""Error paths of the C ABI, forced from the host (bad arguments, call
order, degenerate inputs that make a Gram singular, non-finite data, a
stationary start).  Every kernel still exits normally."""
import numpy as np
import pytest

import datagen

from gpu_cases import GPU_OK, Case, log, to_gpu_U

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not GPU_OK, reason="needs a GPU")]

if GPU_OK:
    import torch
    import paper_2212_09664_amd as ag


def test_bad_parameters_are_rejected_before_launch():
    log("bad params")
    with pytest.raises(ag.AltGDminError) as e:
        ag.AltGDmin(48, 64, 2, 4, 2, 48)          # nx not a power of two
    assert e.value.status == 1
    with pytest.raises(ag.AltGDminError):
        ag.AltGDmin(64, 64, 2, 4, 17, 64)         # r > 16
    with pytest.raises(ag.AltGDminError):
        ag.AltGDmin(64, 64, 2, 4, 2, 64, exit_consec=-1)
    with pytest.raises(ag.AltGDminError):
        ag.AltGDmin(64, 64, 2, 4, 2, 100)         # lines: m_max not a multiple of nx
    with pytest.raises(ag.AltGDminError):
        ag.AltGDmin(64, 64, 2, 4, 2, 64, eta_c=-1.0)


def test_iterate_before_init_is_a_state_error():
    log("state error")
    cs = Case(datagen.make_small(16, 16, 2, 4, 2, seed=0, n_lines=6))
    ctx = cs.gpu_ctx()
    U = torch.zeros(2, 256, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(ag.AltGDminError) as e:
        ctx.iterate(1, U)
    assert e.value.status == 2


def test_frame_with_too_few_samples_reports_not_pd_with_frame():
    """Frame 2 samples a single k-space location and the coil maps differ
    only by a constant phase, so A_2 U (nc x r) has rank 1 < r = 3 and
    G_2 = (A_2 U)^H (A_2 U) is singular."""
    log("not PD")
    nx = ny = 16
    q, r, nc = 4, 3, 2
    rng = np.random.default_rng(0)
    masks = [np.sort(rng.choice(nx * ny, 60, replace=False)).astype(np.int32) for _ in range(q)]
    masks[2] = np.array([17], dtype=np.int32)
    zstar, _ = datagen.lowrank_gaussian(nx * ny, q, r, rng)
    p = datagen.Problem("np", nx, ny, nc, q, r, "index", masks, datagen.coil_maps(nx, ny, nc, "flat"),
                        zstar, None, np.zeros((q, nc, 60), np.complex128))
    cs = Case(p)
    ctx = cs.gpu_ctx()
    rng2 = np.random.default_rng(1)
    U = to_gpu_U(np.linalg.qr(datagen.crandn(rng2, nx * ny, r))[0])
    ctx.init_from(U)
    with pytest.raises(ag.AltGDminError) as e:
        ctx.iterate(2, U, sync=True)
    assert e.value.status == 4 and e.value.frame == 2


def test_nonfinite_measurements_are_reported():
    log("non-finite")
    cs = Case(datagen.make_small(16, 16, 2, 4, 2, seed=0, n_lines=8))
    cs.y32[1, 0, 3] = np.nan
    ctx = cs.gpu_ctx()
    rng = np.random.default_rng(1)
    U = to_gpu_U(np.linalg.qr(datagen.crandn(rng, 256, 2))[0])
    ctx.init_from(U)
    with pytest.raises(ag.AltGDminError) as e:
        ctx.iterate(1, U, sync=True)
    assert e.value.status in (4, 5)


def test_out_of_range_mask_is_invalid():
    log("bad mask")
    cs = Case(datagen.make_small(16, 16, 2, 4, 2, seed=0, n_lines=8))
    cs.mask[1, 0] = 99
    ctx = cs.gpu_ctx()
    st, frame = ctx.last_error()
    assert st == 1 and frame == 1


def test_full_sampling_without_truncation_is_stationary():
    """Full sampling, sum |s_c|^2 = 1, no truncation: U_0 is already the
    top-r subspace of Z*, the gradient is zero and no step is taken."""
    log("stationary start")
    nx = ny = 16
    q, r, nc = 6, 2, 3
    rng = np.random.default_rng(2)
    masks = [np.arange(ny, dtype=np.int32) for _ in range(q)]
    p = datagen.Problem("full", nx, ny, nc, q, r, "lines", masks, datagen.coil_maps(nx, ny, nc, "ring"),
                        datagen.crandn(rng, nx * ny, q), None, np.zeros((q, nc, nx * ny), np.complex128))
    cs = Case(p)
    ctx = cs.gpu_ctx(trunc_c=0.0)
    U = ctx.init()
    B, done = ctx.iterate(5, U, sync=True)
    assert done == 0


def test_spectral_init_needs_r_at_most_q():
    """A context with r > q is valid (LS step, operators, the steps around
    the loop) but the spectral initialisation (top r of q singular vectors)
    refuses it before any launch."""
    p = datagen.make_small(32, 32, 2, 2, 2, seed=1, kind="lines", n_lines=8)
    cs = Case(p)
    ctx = ag.AltGDmin(p.nx, p.ny, p.nc, p.q, 4, int(cs.y.shape[2]))
    dev = torch.device("cuda:0")
    ctx.set_problem(torch.from_numpy(cs.coils.astype(np.complex64)).to(dev), torch.from_numpy(cs.mask).to(dev),
                    torch.from_numpy(cs.m_k).to(dev), torch.from_numpy(cs.y32).to(dev))
    with pytest.raises(ag.AltGDminError) as e:
        ctx.init()
    assert e.value.status == 1
    U, _ = np.linalg.qr(datagen.crandn(np.random.default_rng(0), p.n, 4))
    B = ctx.ls(torch.from_numpy(np.ascontiguousarray(U.T.astype(np.complex64))).to(dev))
    assert B.shape == (p.q, 4)
