"""The thermal workload at full size over 500 steps, FP64, against stored
oracle values (tests/golden/thermal128_fp64.npz, written by
tests/golden/make_thermal128_golden.py from the oracle alone).

128^3 cells, 10^3 tethered particles of random mass and compressibility,
kT = 1e-3, resonant standing wave along x.  Checked after 100 and 500
steps: the four fields at the stored sample of cells (every cell of the
3 x 3 x 3 neighbourhood of each particle's starting position plus uniformly
drawn cells; relative to the largest |value| of the field over the whole
grid) and every particle's position (periodic distance in units of h) and
velocity.  Bar: 1e-12.
"""
import os

import numpy as np
import pytest

from paper_1307_0702_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "thermal128_fp64.npz")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_thermal_128_500_steps_match_stored_oracle_values():
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation
    ref = np.load(GOLDEN, allow_pickle=False)
    cells = ref["cells"]
    w = W.thermal_128()
    fl, p = w.fluid, w.particles
    sim = Simulation(fl, prec="fp64", max_particles=p.n)
    sim.set_state(w.drho, w.g)
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing([m.as_dict() for m in w.modes])
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    done = 0
    for n in (100, 500):
        print(f"thermal 128^3, 1000 particles, fp64: stepping to {n}", flush=True)
        sim.step(n - done)
        done = n
        drho, g = sim.get_state()
        q, u = sim.get_particles()
        fields = [drho] + list(g)
        want = ref[f"s{n}_fields"]
        fmax = ref[f"s{n}_fmax"]
        errs = {}
        for i, name in enumerate(("drho", "gx", "gy", "gz")):
            errs[name] = float(np.max(np.abs(fields[i].reshape(-1)[cells] - want[i])) / fmax[i])
        dq = np.abs(q - ref[f"s{n}_q"])
        errs["q"] = float(np.max(np.minimum(dq, L - dq)) / fl.h)
        errs["u"] = float(np.max(np.abs(u - ref[f"s{n}_u"])) / np.max(np.abs(ref[f"s{n}_u"])))
        print(f"  after {n} steps:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v <= 1e-12, (n, k, v)
