"""What the trained warm start gains over the method without it, on
held-out seeds of the two workloads it was trained for (the weights in
paper_2212_09664_amd/weights were trained by paper_2212_09664_amd.warmstart
on seeds 10000+, these seeds are from the held-out range 900000+).

Both arms run the same plain FP32 iteration with the same step size
(Algorithm 2's rule at the spectral basis); the warm arm starts from the
CNN's basis when its cost f(U) is lower.  Its first iterate must already be
closer to the sequence than the spectral run's, and it must reach
NMSE <= 2e-2 in fewer iterations."""
import os

import numpy as np
import pytest

from gpu_cases import GPU_OK, log

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not GPU_OK, reason="needs a GPU")]

if GPU_OK:
    import torch

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2212_09664_amd", "weights")


@pytest.mark.parametrize("workload,seeds", [("cine128", (900010, 900011, 900012)), ("cine256", (900010,))])
def test_trained_warm_start_reaches_the_target_sooner(workload, seeds):
    import paper_2212_09664_amd as ag
    from paper_2212_09664_amd import warmstart as W
    params = torch.from_numpy(np.load(os.path.join(WEIGHTS, f"wsinit_{workload}.npy"))).cuda()
    net = None
    for seed in seeds:
        d = W._gen((workload, seed))
        ctx, zstar = W._problem(ag, torch, d)
        if net is None:
            net = ag.WsInit(d["nx"], d["ny"], d["q"], d["r"], width=32, batch=1)
            assert net.param_count == params.numel()
        xbuf = torch.empty(1, 2 * d["q"], d["ny"], d["nx"], dtype=torch.float32, device="cuda:0")
        it_s, ms_s, _ = W.time_to_target(ag, torch, ctx, zstar)
        it_w, ms_w, kept = W.time_to_target(ag, torch, ctx, zstar, warm=(net, params, xbuf))
        log(f"  {workload} seed {seed}: spectral {it_s} it {ms_s:.2f} ms; warm {it_w} it {ms_w:.2f} ms; kept {kept}")
        assert it_s is not None and it_w is not None
        assert kept == 1
        assert it_w < it_s
