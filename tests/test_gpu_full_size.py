"""Parity at the full benchmark size: the paper-scale workload (256^3 cells,
10^4 tethered particles of split contrast, kT = 1e-3, modal drive) advanced
two steps in one ic_step call, in the launch configuration bench.py times
(default stage tile, particle prologue on the side stream, and in FP32 the
second step's noise generated beside the first step's stages), against two
FP64 oracle steps over the whole grid, element by element.

Bars: FP64 e <= 1e-12; FP32 e <= 2e-5 after two steps from an
FP32-representable state (the per-step FP32 bar of 1e-5, twice).  e is
max|x_gpu - x_oracle| / max|x_oracle| per field and for u; q is compared as a
periodic distance in units of h.  One oracle step takes ~15 s here.
"""
import time

import numpy as np
import pytest

from oracle import ic_oracle as O
from paper_1307_0702_amd import workloads as W
from tests.oracle_state import make_state, modes_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def workload():
    return W.paper_scale_256()


def _rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_paper_scale_two_steps_match_oracle(workload, prec, tol):
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation
    w = workload
    fl, p = w.fluid, w.particles
    drho, g = w.drho, w.g
    if prec == "fp32":
        drho = drho.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    print(f"full size {fl.shape} particles {p.n} {prec}: GPU", flush=True)
    sim = Simulation(fl, prec=prec, max_particles=p.n)
    sim.set_state(drho, g)
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing(modes_of(w))
    sim.step(2)
    gd, gg = sim.get_state()
    gq, gu = sim.get_particles()
    del sim

    w2 = W.Workload(w.name, fl, p, w.modes, drho, g, w.period_steps)
    st = make_state(w2)
    prm = fl.as_dict()
    for n in range(2):
        t0 = time.perf_counter()
        st, _ = O.ic_step(st, prm, modes_of(w))
        print(f"  oracle step {n + 1}: {time.perf_counter() - t0:.1f} s", flush=True)
    errs = {"drho": _rel(gd, st["drho"]), "u": _rel(gu, st["u"])}
    for a in range(3):
        errs["g%d" % a] = _rel(gg[a], st["g"][a])
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    dq = np.abs(gq - st["q"])
    errs["q"] = float(np.max(np.minimum(dq, L - dq)) / fl.h)
    print("  ", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)
