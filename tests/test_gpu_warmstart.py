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


def test_warm_start_with_the_forward_pass_on_a_second_stream():
    """warm_start with the network on a side stream (its forward pass beside
    the spectral initialisation) gives the basis and the choice that the
    single-stream init_warm gives, bit for bit, twice in a row."""
    import paper_2212_09664_amd as ag
    from paper_2212_09664_amd import warmstart as W
    workload, seed = "cine128", 900013
    params = torch.from_numpy(np.load(os.path.join(WEIGHTS, f"wsinit_{workload}.npy"))).cuda()
    d = W._gen((workload, seed))
    ctx, _ = W._problem(ag, torch, d)
    s = ctx.stream
    xbuf = torch.empty(1, 2 * d["q"], d["ny"], d["nx"], dtype=torch.float32, device="cuda:0")
    net1 = ag.WsInit(d["nx"], d["ny"], d["q"], d["r"], width=32, batch=1, stream=s)
    U1 = torch.empty(d["r"], d["nx"] * d["ny"], dtype=torch.complex64, device="cuda:0")
    c1 = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    W.warm_start(ctx, net1, params, xbuf, U1, choice=c1)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    net2 = ag.WsInit(d["nx"], d["ny"], d["q"], d["r"], width=32, batch=1, stream=side)
    M = torch.empty(1, d["r"], d["nx"] * d["ny"], dtype=torch.complex64, device="cuda:0")
    for rep in range(2):
        U2 = torch.full_like(U1, float("nan"))
        c2 = torch.full_like(c1, -1)
        W.warm_start(ctx, net2, params, xbuf, U2, M=M, choice=c2, side=side)
        torch.cuda.synchronize()
        log(f"  replay {rep}: choice {int(c2.item())} (single stream {int(c1.item())})")
        assert int(c2.item()) == int(c1.item())
        assert torch.equal(torch.view_as_real(U2), torch.view_as_real(U1))
