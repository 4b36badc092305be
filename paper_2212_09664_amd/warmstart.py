"""Training and evaluation of the learned warm start (include/wsinit.h) on
seeded synthetic sequences.

    python -m paper_2212_09664_amd.warmstart --workload cine128 --train 2000 --eval 200 \\
        --epochs 60 --out weights.npy --report report.json

Training pairs: for each training seed, the network input (the 2q
back-projected planes, altgdmin_cnn_input) and the target basis U_tgt from
the plain method after T_max = 70 iterations.  (Algorithm 2's exit rule,
SD(U, U+)/sqrt(r) < 0.01, fires after about 5 iterations on these
sequences, long before the basis has converged, so it is not used for the
targets.)  The loss is the squared subspace distance between span(M)
and span(U_tgt); Adam with a cosine learning-rate decay.  Every step runs
in the library's HIP kernels; this module only orchestrates.

Evaluation on held-out seeds: iterations and GPU time to NMSE <= 2e-2 for
the spectral initialisation and for the warm start (network input, forward
pass, init_warm with its cost-based fallback and the step size of
Algorithm 2's rule at the spectral basis), the fallback rate and the
held-out loss.  NMSE is evaluated off the clock.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _gen(args):
    """One seeded sequence on the CPU (worker process)."""
    import datagen
    workload, seed = args
    p = datagen.make(workload, seed)
    return dict(seed=seed, nx=p.nx, ny=p.ny, nc=p.nc, q=p.q, r=p.r, coils=p.coils.astype(np.complex64),
                mask=p.mask_array(), m_k=p.m_k(), zstar=p.zstar.astype(np.complex64),
                noise=p.noise.astype(np.complex64), snr=p.snr_db, kind=p.kind)


def _problem(ag, torch, d, eps_exit=0.0):
    """A context bound to one sequence; y = A(Z*) + noise synthesised on the GPU."""
    dev = torch.device("cuda:0")
    m_max = int(d["m_k"].max())
    kind = ag.MASK_LINES if d["kind"] == "lines" else ag.MASK_INDEX
    ctx = ag.AltGDmin(d["nx"], d["ny"], d["nc"], d["q"], d["r"], m_max, kind, ag.FP32, eps_exit=eps_exit, t_max=70)
    coils = torch.from_numpy(d["coils"]).to(dev)
    mask = torch.from_numpy(d["mask"]).to(dev)
    mk = torch.from_numpy(d["m_k"]).to(dev)
    ctx.set_problem(coils, mask, mk, None)
    zstar = torch.from_numpy(np.ascontiguousarray(d["zstar"].T)).to(dev)
    y = ctx.apply_A(zstar)
    w = torch.from_numpy(d["noise"]).to(dev)
    valid = (torch.arange(m_max, device=dev)[None, None, :] < mk[:, None, None])
    n_samp = int(valid.sum().item()) * d["nc"]
    sigma = torch.sqrt(torch.sum(torch.abs(y.to(torch.complex128)) ** 2) / (n_samp * 10 ** (d["snr"] / 10)))
    y = torch.where(valid, y + sigma.to(torch.float32) * w, torch.zeros_like(y))
    ctx.set_problem(coils, mask, mk, y.contiguous())
    return ctx, zstar


def generate(workload: str, seeds, pool, log=print):
    """Network inputs (N, 2q, ny, nx) and targets (N, r, n) on the GPU."""
    import torch
    import paper_2212_09664_amd as ag
    X = Ut = None
    iters = []
    t0 = time.time()
    for i, d in enumerate(pool.map(_gen, [(workload, s) for s in seeds], chunksize=4)):
        ctx, _ = _problem(ag, torch, d)
        if X is None:
            X = torch.empty(len(seeds), 2 * d["q"], d["ny"], d["nx"], dtype=torch.float32, device="cuda:0")
            Ut = torch.empty(len(seeds), d["r"], d["nx"] * d["ny"], dtype=torch.complex64, device="cuda:0")
        ctx.cnn_input(X[i])
        U = ctx.init()
        _, done = ctx.iterate(70, U, sync=True)
        Ut[i].copy_(U)
        iters.append(done)
        if (i + 1) % 200 == 0:
            log(f"  generated {i + 1}/{len(seeds)} ({time.time() - t0:.0f} s), mean iterations {np.mean(iters):.1f}")
    torch.cuda.synchronize()
    return X, Ut, iters


def he_uniform(rng, cin, width, cout, layers=4):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, FP32."""
    out = []
    ch = [cin] + [width] * (layers - 1) + [cout]
    for i in range(layers):
        bound = math.sqrt(6.0 / (ch[i] * 9))
        out.append(rng.uniform(-bound, bound, size=ch[i + 1] * ch[i] * 9))
        out.append(np.zeros(ch[i + 1]))
    return np.concatenate(out).astype(np.float32)


def train(X, Ut, r, width=32, epochs=60, batch=16, lr=1e-3, seed=0, log=print, Xv=None, Uv=None):
    import torch
    import paper_2212_09664_amd as ag
    N, c2q, ny, nx = X.shape
    q = c2q // 2
    net = ag.WsInit(nx, ny, q, r, width=width, batch=batch)
    rng = np.random.default_rng(seed)
    params = torch.from_numpy(he_uniform(rng, 2 * q, width, 2 * r)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grads = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float64, device="cuda:0")
    steps_per_epoch = N // batch
    total = epochs * steps_per_epoch
    step = 0
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        acc = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb = X.index_select(0, idx)
            ub = Ut.index_select(0, idx)
            net.loss_backward(params, xb, ub, grads, loss)
            step += 1
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total))
            net.adam_step(params, grads, m, v, lr_t, step)
            acc += loss
        tl = float(acc.item()) / steps_per_epoch
        msg = f"  epoch {ep + 1}/{epochs} train loss {tl:.4f}"
        if Xv is not None:
            vl = evaluate_loss(net, params, Xv, Uv, batch)
            msg += f"  held-out loss {vl:.4f}"
            hist.append((tl, vl))
        else:
            hist.append((tl, None))
        log(msg + f"  ({time.time() - t0:.0f} s)")
    return params, hist, net


def evaluate_loss(net, params, X, Ut, batch):
    import torch
    tot, cnt = 0.0, 0
    grads = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float64, device="cuda:0")
    for s in range(0, X.shape[0], batch):
        b = min(batch, X.shape[0] - s)
        net.loss_backward(params, X[s:s + b], Ut[s:s + b], grads, loss)
        tot += float(loss.item()) * b
        cnt += b
    return tot / cnt


def _nmse(U_prev, B, zstar, zz):
    import torch
    X = torch.matmul(B.to(torch.complex128), U_prev.to(torch.complex128))  # (q, n)
    return float(torch.sum(torch.abs(X - zstar.to(torch.complex128)) ** 2).item()) / zz


def warm_start(ctx, net, params, xbuf, U, M=None, choice=None, side=None):
    """The learned warm start into U: the network input (2q back-projected
    planes), the forward pass M = f(planes), then the cost-based pick
    between the spectral basis and QR(M) (altgdmin_init_warm).

    With `side`, a second stream that `net` was created on, the forward pass
    runs there beside the spectral initialisation, whose eigen-solver keeps
    one workgroup busy for most of its time: the spectral basis comes from
    init on the context's stream, and init_warm_from then scores both
    exactly as init_warm does.  M (B, r, n) may be given to avoid an
    allocation per call."""
    import torch
    s = ctx.stream
    if M is None:
        M = torch.empty(xbuf.shape[0], ctx.p.r, ctx.n, dtype=torch.complex64, device=xbuf.device)
    ctx.cnn_input(xbuf[0])
    if side is None:
        net.forward(params, xbuf, M)
        ctx.init_warm(M[0], U, choice)
        return U
    if net.stream.cuda_stream != side.cuda_stream:
        raise ValueError("warm_start: the network must run on the side stream")
    planes_ready = torch.cuda.Event()
    planes_ready.record(s)
    side.wait_event(planes_ready)
    net.forward(params, xbuf, M)
    guess_ready = torch.cuda.Event()
    guess_ready.record(side)
    ctx.init(U)
    s.wait_event(guess_ready)
    ctx.init_warm_from(M[0], U, U, choice)
    return U


def time_to_target(ag, torch, ctx, zstar, warm=None, target=2e-2, t_max=70):
    """(iterations, GPU ms, kept-learned flag) to NMSE <= target; the clock
    covers the initialisation (and, for the warm start, the network input
    and forward pass) and each iteration, not the NMSE evaluation."""
    stream = ctx.stream
    zz = float(torch.sum(torch.abs(zstar.to(torch.complex128)) ** 2).item())
    q, r, n = ctx.p.q, ctx.p.r, ctx.n
    U = torch.empty(r, n, dtype=torch.complex64, device="cuda:0")
    Up = torch.empty_like(U)
    B = torch.empty(q, r, dtype=torch.complex64, device="cuda:0")
    choice = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    if warm is None:
        ctx.init(U)
    else:
        net, params, xbuf = warm
        warm_start(ctx, net, params, xbuf, U, choice=choice)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    for t in range(1, t_max + 1):
        e0.record(stream)
        ctx.iterate(1, U, B, U_prev=Up)
        e1.record(stream)
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        if _nmse(Up, B, zstar, zz) <= target:
            return t, ms, int(choice.item())
    return None, ms, int(choice.item())


def evaluate(workload, seeds, net, params, pool, log=print):
    import torch
    import paper_2212_09664_amd as ag
    rows = []
    xbuf = None
    for i, d in enumerate(pool.map(_gen, [(workload, s) for s in seeds], chunksize=4)):
        ctx, zstar = _problem(ag, torch, d)
        if xbuf is None:
            xbuf = torch.empty(1, 2 * d["q"], d["ny"], d["nx"], dtype=torch.float32, device="cuda:0")
        # one untimed pass of each so that both paths are warm
        if i == 0:
            time_to_target(ag, torch, ctx, zstar)
            time_to_target(ag, torch, ctx, zstar, warm=(net, params, xbuf))
        it_s, ms_s, _ = time_to_target(ag, torch, ctx, zstar)
        it_w, ms_w, ch = time_to_target(ag, torch, ctx, zstar, warm=(net, params, xbuf))
        rows.append(dict(seed=d["seed"], iters_spectral=it_s, ms_spectral=ms_s, iters_warm=it_w, ms_warm=ms_w,
                         kept_learned=ch))
        if (i + 1) % 50 == 0:
            log(f"  evaluated {i + 1}/{len(seeds)}")
    return rows


def summarise(rows):
    def stat(key):
        v = [r[key] for r in rows if r[key] is not None]
        return dict(mean=float(np.mean(v)) if v else None, median=float(np.median(v)) if v else None, n=len(v))
    both = [r for r in rows if r["iters_spectral"] is not None and r["iters_warm"] is not None]
    return dict(
        n=len(rows),
        reached_spectral=sum(r["iters_spectral"] is not None for r in rows),
        reached_warm=sum(r["iters_warm"] is not None for r in rows),
        iters_spectral=stat("iters_spectral"), iters_warm=stat("iters_warm"),
        ms_spectral=stat("ms_spectral"), ms_warm=stat("ms_warm"),
        fallback_rate=float(np.mean([1 - r["kept_learned"] for r in rows])),
        warm_faster_fraction=float(np.mean([r["ms_warm"] < r["ms_spectral"] for r in both])) if both else None,
        mean_iteration_gain=float(np.mean([r["iters_spectral"] - r["iters_warm"] for r in both])) if both else None,
    )


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cine128")
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--eval", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--train-seed0", type=int, default=10_000)
    ap.add_argument("--eval-seed0", type=int, default=900_000)
    ap.add_argument("--out", default=None, help="trained parameters (.npy, float32)")
    ap.add_argument("--params", default=None, help="evaluate these parameters instead of training")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    # the CPU workers are forked before anything touches the GPU
    pool = ProcessPoolExecutor(max_workers=args.workers)
    list(pool.map(int, range(args.workers)))
    import torch

    def log(m):
        print(m, flush=True)

    report = dict(workload=args.workload, train=args.train, eval=args.eval, epochs=args.epochs, batch=args.batch,
                  lr=args.lr, width=args.width)
    t0 = time.time()
    eval_seeds = list(range(args.eval_seed0, args.eval_seed0 + args.eval))
    log(f"generating {args.eval} held-out sequences ({args.workload})")
    Xv, Uv, _ = generate(args.workload, eval_seeds, pool, log)
    r = Uv.shape[1]
    if args.params:
        import paper_2212_09664_amd as ag
        params = torch.from_numpy(np.load(args.params)).cuda()
        net = ag.WsInit(Xv.shape[3], Xv.shape[2], Xv.shape[1] // 2, r, width=args.width, batch=args.batch)
        hist = []
    else:
        log(f"generating {args.train} training sequences")
        X, Ut, iters = generate(args.workload, list(range(args.train_seed0, args.train_seed0 + args.train)),
                                pool, log)
        report["target_iterations_mean"] = float(np.mean(iters))
        log(f"training ({args.epochs} epochs, batch {args.batch})")
        params, hist, net = train(X, Ut, r, args.width, args.epochs, args.batch, args.lr, log=log, Xv=Xv, Uv=Uv)
        del X, Ut
        if args.out:
            np.save(args.out, params.cpu().numpy())
    report["history"] = hist
    report["heldout_loss"] = evaluate_loss(net, params, Xv, Uv, args.batch)
    log(f"held-out loss {report['heldout_loss']:.4f}; evaluating time to NMSE <= 2e-2")
    del Xv, Uv
    rows = evaluate(args.workload, eval_seeds, net, params, pool, log)
    pool.shutdown()
    report["summary"] = summarise(rows)
    report["rows"] = rows
    report["wall_s"] = time.time() - t0
    log(json.dumps(report["summary"]))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
