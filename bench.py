"""altGDmin throughput on one MI355X, with a roofline figure, the three forms
(plain, learned warm start, mixed precision + warm start) timed to the same
NMSE on the same inputs, and the FP64 CPU oracle timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form all|plain|mixed|warm|mixed_warm]
                    [--workload cine256|radial128|cine256r16|cine128|gauss64]

Workload (default): the 256x256, 12-coil, 40-frame cine-like sequence
(motion-ellipse phantom, ring coils, 1D Cartesian variable-density mask at
acceleration 8 with 8 centre lines redrawn per frame, 30 dB noise), rank 8,
70 iterations.

One step is a whole reconstruction: bind the problem (per-line inverse DFT
along kx of y, index tables, ||y_k||^2), truncated spectral initialisation,
then the workload's iterations.  value = iterations per second of the plain
FP32 form over the timed steps (whole job, inputs already resident in HBM).

Also reported:
* the steps around the loop (altGDmin-MRI: mean image, residuals, MEC-1,
  MEC-2, automatic rank), each timed with HIP events on the same inputs;
* the loop alone (iterate only), and per form the time to NMSE <= 2e-2:
  HIP events after setup, after init and after every iteration (median over
  10 replays); NMSE evaluated off the clock on a replay of the same
  deterministic run; the ratio of each form's time to the plain form's;
* roofline: the unit of work is one altGDmin iteration.  Its algorithmic
  bytes B_alg = 8 (2 Nc M + 2 Nc n + 5 n r) (y', coils and U read before and
  after the per-frame solve, the new U written, complex64) and flops F (the
  2 Nc r shared transforms, the per-line Grams, rhs, fold and residual
  contractions, the coil products and the QR Gram) are divided by the
  measured time of one iteration; the bound is whichever of B_alg / 8 TB/s
  and F / 157.3 TFLOP/s is larger.  The loop's most expensive kernel class
  is reported beside it with its own operand bytes.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD_TEXT = {
    "cine256": "cine256: 256x256 complex images, 12 ring coils, 40 frames, rank 8, "
               "1D Cartesian variable-density mask R=8 (8 centre lines, redrawn per frame), "
               "motion-ellipse phantom + 1% sparse residual, 30 dB noise, 70 iterations",
    "radial128": "radial128: 128x128, 8 ring coils, 100 frames, rank 10, 16 golden-angle spokes per frame "
                 "rasterised onto the grid, gamma-variate perfusion phantom, 25 dB noise, 50 iterations",
    "cine256r16": "cine256r16: 256x256, 16 ring coils, 64 frames, rank 16, 1D Cartesian variable-density "
                  "mask R=12 (8 centre lines), motion-ellipse phantom, 30 dB noise, 70 iterations",
    "cine128": "cine128: 128x128, 8 ring coils, 48 frames, rank 6, 1D Cartesian variable-density mask R=8, "
               "motion-ellipse phantom, 30 dB noise, 70 iterations",
    "gauss64": "gauss64: 64x64, 4 corner coils, 16 frames, rank 4, exact rank-4 Gaussian sequence, "
               "4 centre + 12 uniform lines per frame, noise-free, 20 iterations",
}
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
NMSE_TARGET = 2e-2


# ---------------------------------------------------------------------------
# the unit of work: one iteration
# ---------------------------------------------------------------------------
def iteration_bytes(prob) -> float:
    """B_alg of one iteration (complex64 = 8 B): y' (Nc M samples), the coil
    maps (Nc n) and U (n r) are read in both phases of the iteration (before
    and after the per-frame solve, which needs all of A_k U first), the new U
    is written (n r), and the QR reads U and the step twice more (2 n r)."""
    n, nc, r = prob.n, prob.nc, prob.r
    M = int(prob.m_k().sum())
    return 8.0 * (2 * nc * M + 2 * nc * n + 5 * n * r)


def iteration_flops(prob) -> float:
    """Flops of one iteration: 5 N log2 N per length-N complex FFT, 8 per
    complex multiply-add, Hermitian Grams counted once per pair.

    1D Cartesian (hybrid ky, x form): 2 Nc r transforms along y for every x
    column; per sampled line the Gram of Nc nx rows (r(r+1)/2 pairs), the rhs
    and the residual term of the fold (r per sample each), and the fold's
    W S_u product (r^2 per row of W).  General masks: 2 Nc r full 2D
    transforms; per sample the Gram pair products, rhs, residual and fold
    (r(r+1)/2 + 3 r).  Both: the coil products (2 Nc r n) and the Gram of
    [U grad] (2r(2r+1)/2 n)."""
    n, nc, r, nx, ny = prob.n, prob.nc, prob.r, prob.nx, prob.ny
    M = int(prob.m_k().sum())
    pairs = r * (r + 1) // 2
    if prob.kind == "lines":
        n_u = len(np.unique(np.concatenate(prob.masks)))
        fft = 2 * nc * r * 5 * n * np.log2(ny)
        contr = 8 * (n_u * nc * nx * pairs + 2 * nc * M * r + n_u * nc * nx * r * r)
    else:
        fft = 2 * nc * r * 5 * n * np.log2(n)
        contr = 8 * nc * M * (pairs + 3 * r)
    other = 8 * (2 * nc * r * n) + 8 * (2 * r * (2 * r + 1) // 2) * n
    return float(fft + contr + other)


def kernel_operand_bytes(kernel: str, prob) -> float:
    """Operand bytes of one launch of a loop kernel class (each operand it
    must read or write once, complex64), for the per-kernel view."""
    n, nc, r, nx = prob.n, prob.nc, prob.r, prob.nx
    M = int(prob.m_k().sum())
    if prob.kind == "lines":
        n_u = len(np.unique(np.concatenate(prob.masks)))
        W = nc * r * n_u * nx
    else:
        W = nc * r * n
    table = {
        "fwd_transform": n * r + nc * n + W,
        "gram_rhs": W + nc * M,
        "fold": 2 * W + nc * M,
        "adj_transform": W + nc * n + 2 * n * r,  # rank <= 8: also reads U for the QR Gram
        "qr_gram": 2 * n * r,
        "apply_qr": 3 * n * r,
    }
    return 8.0 * table[kernel]


LOOP_KERNELS = ("fwd_transform", "gram_rhs", "fold", "adj_transform", "qr_gram", "apply_qr")


def kernel_source_hash() -> str:
    """Hash of the HIP sources; a stored counter figure is valid only for it."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2212_09664_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch of each loop kernel class from the committed
    FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None when the
    summary is absent or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"altgdmin_{workload}_hbm_counters.txt")
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    out = {}
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 5 and f[0] == "traffic" and f[3] == "hash":
                if f[4] != want:
                    return None
                out[f[1]] = float(f[2])
    return out or None


# ---------------------------------------------------------------------------
# GPU side
# ---------------------------------------------------------------------------
def gpu_inputs(prob):
    """Inputs resident on the device; measurements synthesised with the
    library's own forward operator plus the seeded noise (R18)."""
    import torch
    import paper_2212_09664_amd as ag
    dev = torch.device("cuda:0")
    m_k = prob.m_k()
    m_max = int(m_k.max())
    kind = ag.MASK_LINES if prob.kind == "lines" else ag.MASK_INDEX
    ctx = ag.AltGDmin(prob.nx, prob.ny, prob.nc, prob.q, prob.r, m_max, kind, ag.FP32, t_max=prob.t_iters)
    coils = torch.from_numpy(prob.coils.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(prob.mask_array()).to(dev)
    mk = torch.from_numpy(m_k).to(dev)
    ctx.set_problem(coils, mask, mk, None)
    zstar = torch.from_numpy(np.ascontiguousarray(prob.zstar.T.astype(np.complex64))).to(dev)
    y_clean = ctx.apply_A(zstar)
    t = dict(coils=coils, mask=mask, m_k=mk, zstar=zstar)
    if prob.snr_db is None:
        y = y_clean
    else:
        w = torch.from_numpy(prob.noise.astype(np.complex64)).to(dev)
        valid = (torch.arange(m_max, device=dev)[None, None, :] < mk[:, None, None])
        n_samp = int(valid.sum().item()) * prob.nc
        sigma = torch.sqrt(torch.sum(torch.abs(y_clean.to(torch.complex128)) ** 2) /
                           (n_samp * 10.0 ** (prob.snr_db / 10.0)))
        y = torch.where(valid, y_clean + sigma.to(torch.float32) * w, torch.zeros_like(y_clean))
    t["y"] = y.contiguous()
    torch.cuda.synchronize()
    del ctx
    return t


class Form:
    """One form of the method on the shared inputs: its context, its
    initialisation (spectral, or learned with the spectral fallback) and its
    precision."""

    def __init__(self, prob, t, form: str, workload: str):
        import torch
        import paper_2212_09664_amd as ag
        self.prob, self.t, self.form = prob, t, form
        m_max = int(prob.m_k().max())
        precision = ag.MIXED if form in ("mixed", "mixed_warm") else ag.FP32
        kind = ag.MASK_LINES if prob.kind == "lines" else ag.MASK_INDEX
        self.ctx = ag.AltGDmin(prob.nx, prob.ny, prob.nc, prob.q, prob.r, m_max, kind, precision,
                               t_max=prob.t_iters)
        self.ws = torch.empty(self.ctx.workspace_bytes + 256, dtype=torch.uint8, device="cuda:0")
        self.bind()
        self.stream = self.ctx.stream
        self.U = torch.empty(prob.r, prob.n, dtype=torch.complex64, device="cuda:0")
        self.B = torch.empty(prob.q, prob.r, dtype=torch.complex64, device="cuda:0")
        self.warm = None
        if form in ("warm", "mixed_warm"):
            wpath = os.path.join(ROOT, "paper_2212_09664_amd", "weights", f"wsinit_{workload}.npy")
            if not os.path.exists(wpath):
                raise FileNotFoundError(f"no trained warm-start weights for {workload} ({wpath})")
            params = torch.from_numpy(np.load(wpath)).to("cuda:0")
            # the network runs on a second stream, beside the spectral
            # initialisation (default priority, like every stream here)
            self.side = torch.cuda.Stream()
            net = ag.WsInit(prob.nx, prob.ny, prob.q, prob.r, width=32, batch=1, stream=self.side)
            xbuf = torch.empty(1, 2 * prob.q, prob.ny, prob.nx, dtype=torch.float32, device="cuda:0")
            self.M = torch.empty(1, prob.r, prob.n, dtype=torch.complex64, device="cuda:0")
            self.warm = (net, params, xbuf)

    def bind(self):
        t = self.t
        self.ctx.set_problem(t["coils"], t["mask"], t["m_k"], t["y"], workspace=self.ws)

    def initialise(self):
        if self.warm is None:
            self.ctx.init(self.U)
        else:
            from paper_2212_09664_amd.warmstart import warm_start
            net, params, xbuf = self.warm
            warm_start(self.ctx, net, params, xbuf, self.U, M=self.M, side=self.side)

    def step(self, T):
        self.bind()
        self.initialise()
        self.ctx.iterate(T, self.U, self.B)

    def time_to_nmse(self, T, replays=10, warmups=3):
        """Run A (events after setup, init and every iteration; median of the
        replays) and run B (NMSE after every iteration, off the clock)."""
        import torch
        s = self.stream
        zs = self.t["zstar"].to(torch.complex128)
        zz = float(torch.sum(torch.abs(zs) ** 2).item())
        with torch.cuda.stream(s):
            # run B: the deterministic trajectory's NMSE
            self.bind()
            self.initialise()
            Up = torch.empty_like(self.U)
            nm = []
            for _ in range(T):
                self.ctx.iterate(1, self.U, self.B, U_prev=Up)
                X = self.B.to(torch.complex128) @ Up.to(torch.complex128)
                nm.append(float(torch.sum(torch.abs(X - zs) ** 2).item()) / zz)
            hit = next((i for i, v in enumerate(nm) if v <= NMSE_TARGET), None)
            stamps = []
            for rep in range(warmups + replays):
                evs = [torch.cuda.Event(enable_timing=True) for _ in range(T + 3)]
                torch.cuda.synchronize()
                evs[0].record(s)
                self.bind()
                evs[1].record(s)
                self.initialise()
                evs[2].record(s)
                for i in range(T):
                    self.ctx.iterate(1, self.U, self.B)
                    evs[3 + i].record(s)
                torch.cuda.synchronize()
                if rep >= warmups:
                    stamps.append([evs[0].elapsed_time(e) for e in evs[1:]])
        med = [statistics.median(col) for col in zip(*stamps)]
        return dict(nmse=nm, hit=hit, ttn_ms=(med[2 + hit] if hit is not None else None),
                    iters=(hit + 1 if hit is not None else None), setup_ms=med[0], init_ms=med[1] - med[0],
                    nmse_final=nm[-1])

    def loop_ms(self, T, reps=10):
        """Median over replays of the event time of iterate(T) alone."""
        import torch
        s = self.stream
        out = []
        with torch.cuda.stream(s):
            for _ in range(reps):
                self.bind()
                self.initialise()
                torch.cuda.synchronize()
                l0, l1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                l0.record(s)
                self.ctx.iterate(T, self.U, self.B)
                l1.record(s)
                torch.cuda.synchronize()
                out.append(l0.elapsed_time(l1))
        return statistics.median(out)


def headline(prob, t, args, workload):
    """The plain form's whole-step throughput, its loop, its dominant kernel
    class and its time to target."""
    import torch
    T = prob.t_iters
    f = Form(prob, t, "plain", workload)
    s = f.stream
    with torch.cuda.stream(s):
        for _ in range(args.warmup):
            f.step(T)
        torch.cuda.synchronize()
        # the loop's dominant kernel class: total event time per class over one step
        tot = {}
        for name in LOOP_KERNELS:
            f.ctx.set_timing(name)
            f.step(T)
            torch.cuda.synchronize()
            _, _, ms = f.ctx.kernel_time()
            tot[name] = ms
        f.ctx.set_timing("none")
        kernel = max(tot, key=tot.get)
        # the timed steps; an event pair around each step's loop gives the
        # iteration time inside the timed region
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        loop_evs = []
        torch.cuda.synchronize()
        ev0.record(s)
        for _ in range(args.steps):
            f.bind()
            f.initialise()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            f.ctx.iterate(T, f.U, f.B)
            b.record(s)
            loop_evs.append((a, b))
        ev1.record(s)
        torch.cuda.synchronize()
        total_ms = ev0.elapsed_time(ev1)
        loop = statistics.median(a.elapsed_time(b) for a, b in loop_evs)
        # the dominant class alone, with events around each of its launches
        f.ctx.set_timing(kernel)
        for _ in range(args.steps):
            f.step(T)
        kname, klaunch, kms = f.ctx.kernel_time()
        f.ctx.set_timing("none")
    ttn = f.time_to_nmse(T)
    return dict(total_ms=total_ms, loop_ms=loop, T=T, kname=kname, klaunch=klaunch,
                kavg_ms=kms / max(klaunch, 1), class_ms_per_step=tot, ttn=ttn)


def pipeline_timing(prob, t, reps=5, warmups=2):
    """The steps around the loop (altGDmin-MRI, Algorithm 1) on the same
    inputs, each bracketed by HIP events on the library's stream: the mean
    image (CG, tolerance 1e-3, at most 10 iterations), the first residual,
    the rebinding of the residual data, the spectral initialisation, the
    loop, the second residual, MEC-1 (3 CGLS iterations per frame) and MEC-2
    (ISTA, at most 10 updates), the output assembly, and the automatic-rank
    spectrum.  Medians over the replays; NMSE of each output off the clock."""
    import torch
    import paper_2212_09664_amd as ag
    T = prob.t_iters
    m_max = int(prob.m_k().max())
    kind = ag.MASK_LINES if prob.kind == "lines" else ag.MASK_INDEX
    ctx = ag.AltGDmin(prob.nx, prob.ny, prob.nc, prob.q, prob.r, m_max, kind, ag.FP32, t_max=T)
    ws = torch.empty(ctx.workspace_bytes + 256, dtype=torch.uint8, device="cuda:0")
    names = ["mean", "residual1", "rebind", "init", "loop", "residual2", "mec1", "expand", "mec2", "auto_rank"]
    times = {k: [] for k in names}
    s = torch.cuda.current_stream()
    zs = t["zstar"].to(torch.complex128)
    zz = float(torch.sum(torch.abs(zs) ** 2).item())
    nm = {}
    for rep in range(warmups + reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ctx.set_problem(t["coils"], t["mask"], t["m_k"], t["y"], workspace=ws)
        aux = ctx.aux()
        torch.cuda.synchronize()
        ev[0].record(s)
        zbar = ctx.mean(1e-3, 10)
        ev[1].record(s)
        yt = ctx.residual(zbar=zbar)
        ev[2].record(s)
        ctx.set_problem(t["coils"], t["mask"], t["m_k"], yt, workspace=ws)
        ev[3].record(s)
        U = ctx.init()
        ev[4].record(s)
        Up = torch.empty_like(U)
        B = ctx.iterate(T, U, U_prev=Up)
        ev[5].record(s)
        X = ctx.expand(Up, B)
        ytt = ctx.residual(X=X)
        ev[6].record(s)
        E1 = ctx.mec_cgls(ytt, 3, 1e-36)
        ev[7].record(s)
        Z1 = ctx.expand(Up, B, zbar, E1)
        ev[8].record(s)
        E2 = ctx.mec_ista(ytt, 10, 1e-3, 0.0025)
        ev[9].record(s)
        ctx.auto_rank(85.0)  # synchronises
        ev[10].record(s)
        torch.cuda.synchronize()
        if rep >= warmups:
            for i, k in enumerate(names):
                times[k].append(ev[i].elapsed_time(ev[i + 1]))
        if rep == 0:
            Z2 = ctx.expand(Up, B, zbar, E2)
            for key, Z in (("mri1", Z1), ("mri2", Z2), ("no_mec", ctx.expand(Up, B, zbar))):
                nm[key] = float(torch.sum(torch.abs(Z.to(torch.complex128) - zs) ** 2).item()) / zz
    med = {k: round(statistics.median(v), 4) for k, v in times.items()}
    total1 = sum(med[k] for k in ("mean", "residual1", "rebind", "init", "loop", "residual2", "mec1", "expand"))
    return {"ms": med, "altgdmin_mri1_ms": round(total1, 4),
            "altgdmin_mri2_ms": round(total1 - med["mec1"] + med["mec2"], 4),
            "nmse": {k: v for k, v in nm.items()}}


def other_form(prob, t, form, workload):
    T = prob.t_iters
    f = Form(prob, t, form, workload)
    return dict(loop_ms=f.loop_ms(T), ttn=f.time_to_nmse(T))


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle
# ---------------------------------------------------------------------------
def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, reps: int = 3):
    """The FP64 oracle (literal Algorithm 2) on the same workload and seed:
    the truncated spectral initialisation once, then `reps` single
    iterations from the spectral basis, each timed; the median iteration time
    scales the sample to one step of init + T iterations,
    value = T / (init + T * median)."""
    import datagen
    from oracle import altgdmin as AG
    from oracle import operators as O
    op = O.from_problem(prob)
    Y = datagen.add_noise(op.apply_A(prob.zstar), prob.noise, op.m_k, prob.snr_db)
    t0 = time.perf_counter()
    Ytr, _, _ = AG.truncation(op, Y, 36.0)
    U0 = AG.spectral_init(AG.backprojection(op, Ytr), prob.r)
    t_init = time.perf_counter() - t0
    its = []
    for _ in range(reps):
        t1 = time.perf_counter()
        AG.run(op, Y, AG.Params(r=prob.r), U0=U0, t_fixed=1, record=False)
        its.append(time.perf_counter() - t1)
    med = statistics.median(its)
    T = prob.t_iters
    return dict(value=T / (t_init + T * med), init_s=t_init, iter_s=its, median_iter_s=med, cores=O.WORKERS,
                cpu=cpu_model(), T=T)


# ---------------------------------------------------------------------------
# probes
# ---------------------------------------------------------------------------
def bandwidth_probe():
    """Rates of torch's own copy, sum and fill kernels (HIP events, 20
    launches after 3 warm-up ones) at sizes around a loop kernel's bytes: what
    a plain streaming kernel reaches with the data resident in the last-level
    cache (up to ~200 MB) and from HBM (larger)."""
    import torch

    def per_launch_us(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3
    rows = []
    for mb in (41, 64, 114, 256, 1024):
        a = torch.randn(mb * 2**20 // 4, device="cuda:0")
        b = torch.empty_like(a)
        nbytes = mb * 2**20
        us_c = per_launch_us(lambda: b.copy_(a))
        us_r = per_launch_us(lambda: a.sum())
        us_w = per_launch_us(lambda: b.fill_(1.0))
        rows.append({"MiB": mb, "copy_GBps": round(2 * nbytes / us_c / 1e3), "read_GBps": round(nbytes / us_r / 1e3),
                     "write_GBps": round(nbytes / us_w / 1e3)})
        del a, b
    print(json.dumps({"bandwidth_probe": rows}), flush=True)


def r4(v):
    return None if v is None else round(float(v), 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", choices=["all", "plain", "mixed", "warm", "mixed_warm"], default="all",
                    help="all (default): the plain form's throughput plus the time to NMSE <= 2e-2 of every "
                         "form on the same inputs; a single form: only that form's figures")
    ap.add_argument("--seed", type=int, default=1001)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true", help="skip the timing of the steps around the loop")
    ap.add_argument("--workload", choices=sorted(WORKLOAD_TEXT), default="cine256",
                    help="the headline figure is cine256; the others are for comparisons")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (scale reference for HBM byte counters)")
    ap.add_argument("--bandwidth-probe", action="store_true",
                    help="only time plain device copies, reads and writes of several sizes (practical ceilings)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method's x-column sharding is a design note, not code).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        # 256 MiB read + 256 MiB written by one copy kernel, five times
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 5}), flush=True)
        return
    if args.bandwidth_probe:
        bandwidth_probe()
        return
    import datagen
    workload = args.workload
    prob = datagen.make(workload, args.seed)
    t = gpu_inputs(prob)
    T = prob.t_iters
    forms = {}
    if args.form in ("all", "plain"):
        g = headline(prob, t, args, workload)
        forms["plain"] = dict(loop_ms=g["loop_ms"], ttn=g["ttn"])
        print(f"# plain: {args.steps} steps {g['total_ms']:.2f} ms, loop {g['loop_ms']:.3f} ms", flush=True)
    else:
        g = None
    extra = ["warm", "mixed", "mixed_warm"] if args.form == "all" else ([args.form] if args.form != "plain" else [])
    for form in extra:
        try:
            forms[form] = other_form(prob, t, form, workload)
            print(f"# {form}: loop {forms[form]['loop_ms']:.3f} ms", flush=True)
        except FileNotFoundError as e:
            print(f"# {form}: skipped ({e})", flush=True)
    plain_ttn = forms.get("plain", {}).get("ttn", {}).get("ttn_ms")
    form_rows = {}
    for name, fr in forms.items():
        tt = fr["ttn"]
        form_rows[name] = {
            "loop_iter_per_s": round(T / (fr["loop_ms"] * 1e-3), 2),
            "time_to_nmse_ms": r4(tt["ttn_ms"]), "iters_to_nmse": tt["iters"],
            "init_ms": r4(tt["init_ms"]), "setup_ms": r4(tt["setup_ms"]),
            "nmse_final": tt["nmse_final"],
            "ttn_vs_plain": (None if (plain_ttn is None or tt["ttn_ms"] is None) else round(tt["ttn_ms"] / plain_ttn, 4)),
        }
    head = g if g is not None else None
    main_form = "plain" if head is not None else extra[0]
    iter_ms = forms[main_form]["loop_ms"] / T
    b_alg = iteration_bytes(prob)
    flops = iteration_flops(prob)
    t_hbm = b_alg / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (FP32_PEAK_TFLOPS * 1e12)
    achieved_gbs = b_alg / (iter_ms * 1e-3) / 1e9
    achieved_tf = flops / (iter_ms * 1e-3) / 1e12
    traffic = measured_traffic(workload) if main_form == "plain" else None
    if t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tf / FP32_PEAK_TFLOPS, 4)}
    roof.update({
        "traffic": (round(sum(traffic[k] for k in LOOP_KERNELS if k in traffic)) if traffic else None),
        "unit_of_work": "one altGDmin iteration (the loop's kernels, summed)",
        "alg_bytes_per_iter": b_alg, "flops_per_iter": flops, "iter_ms": round(iter_ms, 5),
        "hbm_frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "fp32_frac": round(achieved_tf / FP32_PEAK_TFLOPS, 4),
    })
    if head is not None:
        kb = kernel_operand_bytes(head["kname"], prob)
        kach = kb / (head["kavg_ms"] * 1e-3) / 1e9
        roof["dominant_kernel"] = {
            "kernel": head["kname"], "operand_bytes_per_launch": kb, "avg_launch_ms": round(head["kavg_ms"], 5),
            "launches": head["klaunch"], "achieved": round(kach, 1), "unit": "GB/s",
            "frac": round(kach / HBM_PEAK_GBS, 4),
            "traffic": (traffic.get(head["kname"]) if traffic else None),
        }
        value = args.steps * T / (head["total_ms"] * 1e-3)
        ms_step = head["total_ms"] / args.steps
    else:
        value = T / (forms[main_form]["loop_ms"] * 1e-3)
        ms_step = forms[main_form]["loop_ms"]
    out = {
        "metric": "altGDmin iter/s + time-to-NMSE<=2e-2 at 256^2 x 12 coils x 40 frames vs plain",
        "value": round(value, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if main_form in ("plain", "warm") else "f32+f16x2+f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT[workload],
            "form": main_form,
            "step": f"bind + spectral init + {T} iterations",
        },
        "loop_iter_per_s": form_rows[main_form]["loop_iter_per_s"],
        "time_to_nmse_ms": form_rows[main_form]["time_to_nmse_ms"],
        "iters_to_nmse": form_rows[main_form]["iters_to_nmse"],
        "nmse_final": form_rows[main_form]["nmse_final"],
        "forms": form_rows,
        "roofline": roof,
    }
    if args.form == "all" and not args.no_pipeline:
        out["pipeline"] = pipeline_timing(prob, t)
        print(f"# pipeline: {out['pipeline']['ms']}", flush=True)
    if not args.no_cpu:
        cb = cpu_baseline(prob)
        out["cpu_baseline"] = {
            "value": round(cb["value"], 4), "unit": "iter/s", "cores": cb["cores"], "kind": "oracle",
            "cpu": cb["cpu"],
            "sample": f"FP64 NumPy/SciPy oracle (literal Algorithm 2) on the same workload and seed: the spectral "
                      f"init once ({cb['init_s']:.1f} s) and 3 single iterations "
                      f"({', '.join(f'{v:.2f}' for v in cb['iter_s'])} s; median {cb['median_iter_s']:.2f} s), "
                      f"scaled to one step of init + {cb['T']} iterations",
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
