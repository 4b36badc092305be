"""The entry point that allocates nothing (altgdmin_mean_noalloc): through
the C ABI, its result equals altgdmin_mean's (the same kernels in the same
order, so bitwise) and the FP64 oracle's mean image, on two calls in a row,
the second on a smaller problem; a problem whose scratch would exceed the
built-in array is refused before any launch."""
import ctypes

import numpy as np
import pytest

import datagen
from oracle import mri as R

from gpu_cases import GPU_OK, Case, log, rel

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not GPU_OK, reason="needs a GPU")]

if GPU_OK:
    import torch


def _run(cfg, seed):
    nx, ny, nc, q, kind, lm = cfg
    p = datagen.make_small(nx, ny, nc, q, 2, seed=seed, kind=kind, n_lines=lm, m=lm, lowrank=False,
                           snr_db=30.0, variable_m=True)
    cs = Case(p)
    ctx = cs.gpu_ctx()
    z_aux, it_aux = ctx.mean(1e-3, 10, sync=True)
    z = torch.full((p.n,), float("nan"), dtype=torch.complex64, device="cuda:0")
    it = ctx.mean_noalloc(z, 1e-3, 10, sync=True)
    zr, itr = R.mean_image(cs.op, cs.y)
    e = rel(z.cpu().numpy().astype(np.complex128), zr)
    log(f"  {cfg}: iterations {it} (aux {it_aux}, oracle {itr}); equal to the aux variant "
        f"{bool(torch.equal(z, z_aux))}; rel to oracle {e:.2e}")
    assert it == it_aux == itr
    assert torch.equal(z, z_aux)
    assert e < 1e-4


def test_noalloc_mean_twice_second_smaller():
    _run((64, 64, 6, 12, "lines", 16), seed=1)
    _run((32, 32, 3, 8, "index", 300), seed=2)


def test_noalloc_mean_refuses_problems_beyond_its_scratch():
    import paper_2212_09664_amd as ag
    # 512 x 512 with 8 coils needs 8 * 11 * 262144 bytes > 16 MiB
    ctx = ag.AltGDmin(512, 512, 8, 4, 2, 512 * 8)
    z = torch.zeros(512 * 512, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(ag.AltGDminError) as e:
        ctx.mean_noalloc(z)
    assert e.value.status == 7
