"""Parity at the full sizes of the three workloads, and at the largest grid
one field allows, in the launch
configuration bench.py times (default stage tile, particle prologue on the
side stream, and in FP32 the next step's noise generated beside the current
step's stages), against the FP64 oracle over the whole grid, element by
element:

- paper scale: 256^3 cells, 10^4 tethered particles of split contrast,
  kT = 1e-3, modal drive; two steps in one ic_step call (one oracle step
  takes ~13 s);
- thermal: 128^3 cells, 10^3 tethered particles, kT = 1e-3; FP64 checked
  after steps 1 and 10;
- standing wave: 32^3, kT = 0, the symmetric tethered pair under the
  resonant drive; FP64 checked after 100 steps;
- maximum grid: a random block with one particle repeated up to one field
  just under 4 GiB (1.016e9 FP32 cells, 5.12e8 FP64 cells), against the
  block's oracle steps repeated.

Bars: FP64 e <= 1e-12; FP32 e <= 1e-5 per step from an FP32-representable
state (2e-5 after two).  e is max|x_gpu - x_oracle| / max|x_oracle| per field
and for u; q is compared as a periodic distance in units of h.
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


def _sim(w, prec, drho, g):
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation
    fl, p = w.fluid, w.particles
    sim = Simulation(fl, prec=prec, max_particles=p.n)
    sim.set_state(drho, g)
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing(modes_of(w))
    return sim


def _errs(sim, st, fl):
    gd, gg = sim.get_state()
    gq, gu = sim.get_particles()
    errs = {"drho": _rel(gd, st["drho"]), "u": _rel(gu, st["u"])}
    for a in range(3):
        errs["g%d" % a] = _rel(gg[a], st["g"][a])
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    dq = np.abs(gq - st["q"])
    errs["q"] = float(np.max(np.minimum(dq, L - dq)) / fl.h)
    print("  ", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    return errs


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


@pytest.mark.parametrize("prec,tol,checks", [("fp64", 1e-12, (1, 10)), ("fp32", 1e-5, (1,))])
def test_thermal_128_matches_oracle(prec, tol, checks):
    w = W.thermal_128()
    fl = w.fluid
    drho, g = w.drho, w.g
    if prec == "fp32":
        drho = drho.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    print(f"thermal {fl.shape} particles {w.particles.n} {prec}", flush=True)
    sim = _sim(w, prec, drho, g)
    st = make_state(W.Workload(w.name, fl, w.particles, w.modes, drho, g, w.period_steps))
    prm = fl.as_dict()
    done = 0
    for c in checks:
        sim.step(c - done)
        for _ in range(c - done):
            st, _ = O.ic_step(st, prm, modes_of(w))
        done = c
        print(f"  after {c} steps", flush=True)
        for k, v in _errs(sim, st, fl).items():
            assert v <= tol, (c, k, v)


def test_standing_wave_32_hundred_steps_match_oracle():
    w = W.standing_wave_32()
    fl = w.fluid
    sim = _sim(w, "fp64", w.drho, w.g)
    st = make_state(w)
    prm = fl.as_dict()
    sim.step(100)
    for _ in range(100):
        st, _ = O.ic_step(st, prm, modes_of(w))
    for k, v in _errs(sim, st, fl).items():
        assert v <= 1e-12, (k, v)


@pytest.mark.parametrize("prec,block,tiles,tol", [
    # one field just under the 4 GiB limit of the stage kernel's 32-bit byte offsets
    ("fp32", (48, 48, 40), (21, 21, 25), 2e-5),    # 1008 x 1008 x 1000 = 1.016e9 cells
    ("fp64", (40, 40, 40), (20, 20, 20), 1e-12),   # 800^3 = 5.12e8 cells
])
def test_maximum_grid_matches_tiled_oracle(prec, block, tiles, tol):
    # A random block with one tethered particle, repeated periodically over
    # the largest grid one field allows (kT = 0, a drive whose wavelength is
    # the block).  By translation invariance two steps of the large grid are
    # the block's two oracle steps repeated: checked on 10^6 sampled cells
    # and on every particle.
    import torch
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation
    bx, by, bz = block
    tx, ty, tz = tiles
    nx, ny, nz = bx * tx, by * ty, bz * tz
    fb = W.Fluid(bx, by, bz, kT=0.0, seed=71)
    drho, g = W.random_fields(fb.shape, 71)
    if prec == "fp32":
        drho = drho.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(72)
    q0 = rng.uniform(0, 1, 3) * np.array([bx, by, bz])
    me0, kr0 = 4.0, 0.7
    mode_b = W.Mode(axis=0, shape="cos", m=1, x0=3.0, amp=2e-3, omega=0.25, phase=0.1)
    # the large problem
    fl = W.Fluid(nx, ny, nz, kT=0.0, seed=71)
    nb = tx * ty * tz
    b = np.arange(nb)
    off = np.stack([b % tx * bx, (b // tx) % ty * by, b // (tx * ty) * bz], axis=1).astype(np.float64)
    q = q0[None, :] + off
    print(f"maximum grid {prec}: {nx}x{ny}x{nz} = {nx * ny * nz:.3e} cells, {nb} particles", flush=True)
    sim = Simulation(fl, prec=prec, max_particles=nb)
    dev = sim.device
    for c, blk in enumerate([drho, g[0], g[1], g[2]]):
        sim.U[c].copy_(torch.as_tensor(blk, dtype=sim.dtype, device=dev).repeat(tz, ty, tx))
    eps = np.full(nb, ic.ic_eps_from_kappa_ratio(fl.cf, kr0))
    sim.set_particles(q, np.full(nb, me0), eps, ks=np.full(nb, 0.05), qeq=q + 0.3)
    md = mode_b.as_dict()
    md["m"] = tx
    sim.set_forcing([md])
    sim.step(2)
    sim.synchronize()
    # the block, two oracle steps
    p = W.Particles(q=q0[None, :], me=np.array([me0]), kappa_ratio=np.array([kr0]),
                    ks=np.array([0.05]), qeq=q0[None, :] + 0.3)
    wb = W.Workload("block", fb, p, [mode_b], drho, g, 0)
    st = make_state(wb)
    for _ in range(2):
        st, _ = O.ic_step(st, fb.as_dict(), modes_of(wb))
    idx = rng.integers(0, nx * ny * nz, size=1_000_000)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    got = sim.U.view(4, -1)[:, torch.as_tensor(idx, device=dev)].double().cpu().numpy()
    want = [st["drho"][z % bz, y % by, x % bx]] + [st["g"][a][z % bz, y % by, x % bx] for a in range(3)]
    full = [st["drho"], st["g"][0], st["g"][1], st["g"][2]]
    errs = {}
    for c, name in enumerate(["drho", "g0", "g1", "g2"]):
        errs[name] = float(np.max(np.abs(got[c] - want[c])) / np.max(np.abs(full[c])))
    gq, gu = sim.get_particles()
    L = np.array([nx, ny, nz], dtype=np.float64)
    dq = np.abs((gq - off) - st["q"][0])
    dq = np.minimum(dq, L - dq)
    errs["q"] = float(np.max(dq))
    errs["u"] = float(np.max(np.abs(gu - st["u"][0])) / np.max(np.abs(st["u"][0])))
    print("  ", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)
