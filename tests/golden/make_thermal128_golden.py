"""Writes tests/golden/thermal128_fp64.npz: FP64 oracle values of the thermal
workload (128^3 cells, 10^3 tethered particles, kT = 1e-3, resonant standing
wave along x) after 100 and 500 IC steps, for the GPU parity test that runs
by default (tests/test_gpu_thermal128_golden.py).

Only the oracle computes: the inputs come from the seeded workload generator
(which holds none of the step's arithmetic) and every stored value is an
oracle output.  Stored per checkpoint: the four fields at a fixed sample of
cells (every cell of the 3 x 3 x 3 neighbourhood of each particle's starting
position, where the coupling acts, plus uniformly drawn cells), the largest
|value| of each field over the whole grid (the denominator of the relative
error), and every particle's q and u.

Run from the repository root:  python tests/golden/make_thermal128_golden.py
(one core, about a quarter of an hour).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ic_oracle as O  # noqa: E402
from paper_1307_0702_amd import workloads as W  # noqa: E402
from tests.oracle_state import make_state, modes_of  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "thermal128_fp64.npz")
CHECKPOINTS = (100, 500)
N_RANDOM = 40960
SAMPLE_SEED = 128500


def sample_cells(w):
    fl = w.fluid
    shape = (fl.nz, fl.ny, fl.nx)
    near = np.floor(np.asarray(w.particles.q) / fl.h + 0.5).astype(np.int64)
    d = np.array([[i, j, k] for k in (-1, 0, 1) for j in (-1, 0, 1) for i in (-1, 0, 1)])
    pts = (near[:, None, :] + d[None, :, :]).reshape(-1, 3)
    pts = np.mod(pts, [fl.nx, fl.ny, fl.nz])
    idx_near = (pts[:, 2] * fl.ny + pts[:, 1]) * fl.nx + pts[:, 0]
    rng = np.random.default_rng(SAMPLE_SEED)
    idx_rand = rng.integers(0, np.prod(shape), N_RANDOM)
    return np.unique(np.concatenate([idx_near, idx_rand])).astype(np.int64)


def main():
    w = W.thermal_128()
    st = make_state(w)
    prm = w.fluid.as_dict()
    modes = modes_of(w)
    idx = sample_cells(w)
    rec = {"cells": idx}
    t0 = time.time()
    for n in range(1, max(CHECKPOINTS) + 1):
        st, _ = O.ic_step(st, prm, modes)
        if n % 25 == 0:
            print(f"step {n}  {time.time() - t0:.0f} s", flush=True)
        if n in CHECKPOINTS:
            fields = [st["drho"]] + list(st["g"])
            rec[f"s{n}_fields"] = np.stack([f.reshape(-1)[idx] for f in fields])
            rec[f"s{n}_fmax"] = np.array([np.max(np.abs(f)) for f in fields])
            rec[f"s{n}_q"] = st["q"].copy()
            rec[f"s{n}_u"] = st["u"].copy()
    np.savez(OUT, **rec)
    print("wrote", OUT, "cells", len(idx))


if __name__ == "__main__":
    main()
