"""Writes the oracle's full-length reference runs used by the GPU parity
tests (test infrastructure; calls only the FP64 oracle and the seeded input
generator).

    python tests/golden/make_fullrun_goldens.py [name ...]

For each workload: the inputs exactly as the GPU tests build them (coil maps
and measurements y = A(Z*) + noise rounded to complex64, then read back as
complex128 by the oracle), then Algorithm 2 with the truncated spectral
initialisation for the workload's fixed iteration count.  Stored per
workload (``fullrun_<name>.json``): the NMSE and cost after every iteration,
eta, gamma and the number of truncated samples, ||X_T||_F and X_T at 256
seeded positions, plus checksums of the inputs so that a changed generator
is caught instead of compared.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
from oracle import altgdmin as AG  # noqa: E402
from oracle import metrics as M  # noqa: E402
from oracle import operators as O  # noqa: E402

# workload, seed, fixed iteration count (the workloads' own T)
RUNS = {"cine256": (1001, 70), "radial128": (0, 50), "cine256r16": (0, 70), "cine128": (0, 70)}
N_SAMPLES = 256


def inputs(name: str, seed: int):
    prob = datagen.make(name, seed)
    coils = prob.coils.astype(np.complex64).astype(np.complex128)
    op = O.Operator(prob.nx, prob.ny, coils, O.omegas(prob.kind, prob.masks, prob.nx))
    y = datagen.add_noise(op.apply_A(prob.zstar), prob.noise, op.m_k, prob.snr_db)
    y = y.astype(np.complex64).astype(np.complex128)
    return prob, op, y


def sample_positions(n: int, q: int):
    rng = np.random.default_rng(12345)
    return rng.integers(0, n, N_SAMPLES), rng.integers(0, q, N_SAMPLES)


def input_checksums(prob, y):
    return {"y_sq": float(np.sum(np.abs(y) ** 2)), "zstar_sq": float(np.sum(np.abs(prob.zstar) ** 2)),
            "coils_sq": float(np.sum(np.abs(prob.coils) ** 2))}


def make(name: str) -> dict:
    seed, T = RUNS[name]
    prob, op, y = inputs(name, seed)
    t0 = time.perf_counter()
    res = AG.run(op, y, AG.Params(r=prob.r), t_fixed=T, Zstar=prob.zstar, record=True)
    pp, kk = sample_positions(prob.n, prob.q)
    X = res.X
    out = {
        "workload": name, "seed": seed, "T": T, "r": prob.r,
        "nmse": [float(v) for v in res.history["nmse"]],
        "f": [float(v) for v in res.history["f"]],
        "eta": float(res.eta), "gamma": float(res.gamma),
        "n_trunc": AG.truncation_count(op, y, 36.0),
        "x_norm": float(np.linalg.norm(X)),
        "x_samples_re": [float(v) for v in X[pp, kk].real],
        "x_samples_im": [float(v) for v in X[pp, kk].imag],
        "inputs": input_checksums(prob, y),
        "oracle_seconds": round(time.perf_counter() - t0, 1),
    }
    return out


def main(names):
    for name in names or sorted(RUNS):
        out = make(name)
        path = os.path.join(HERE, f"fullrun_{name}.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(f"{name}: NMSE_T {out['nmse'][-1]:.6e}, eta {out['eta']:.6e}, {out['oracle_seconds']} s -> {path}",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
