"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Same seeded inputs on both sides; errors are e = max|x_gpu - x_oracle| /
max|x_oracle| per field (drho, gx, gy, gz, u; q as a periodic distance in
units of h).  Bar: FP64 e <= 1e-12 after several steps; FP32 e <= 1e-5 for
one step from the same FP32-representable state.
"""
import math

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


def _sim(w, prec="fp64", u=True):
    from paper_1307_0702_amd.ic import Simulation
    fl, p = w.fluid, w.particles
    sim = Simulation(fl, prec=prec, max_particles=max(p.n, 1))
    sim.set_state(w.drho, w.g)
    if p.n:
        from paper_1307_0702_amd import ic
        eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
        sim.set_particles(p.q, p.me, eps, u=p.u if u else None, ks=p.ks, qeq=p.qeq, fext=p.fext)
    if w.modes:
        sim.set_forcing(modes_of(w))
    return sim


def _rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


def _compare(sim, st, w, tol, label=""):
    drho, g = sim.get_state()
    errs = {"drho": _rel(drho, st["drho"])}
    for a in range(3):
        errs["g%d" % a] = _rel(g[a], st["g"][a])
    if w.particles.n:
        q, u = sim.get_particles()
        errs["u"] = _rel(u, st["u"])
        L = np.array([w.fluid.nx, w.fluid.ny, w.fluid.nz]) * w.fluid.h
        dq = np.abs(q - st["q"])
        dq = np.minimum(dq, L - dq)
        errs["q"] = np.max(dq) / w.fluid.h
    print(label, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (label, k, v)
    return errs


def _run_both(w, nsteps, prec="fp64", tol=1e-12, check_every=None):
    print(f"case {w.name} grid {w.fluid.shape} np {w.particles.n} kT {w.fluid.kT} prec {prec}",
          flush=True)
    sim = _sim(w, prec)
    st = make_state(w)
    prm = w.fluid.as_dict()
    modes = modes_of(w)
    for n in range(nsteps):
        sim.step(1)
        st, _ = O.ic_step(st, prm, modes)
        if check_every and (n + 1) % check_every == 0:
            _compare(sim, st, w, tol, f"step {n + 1}")
    _compare(sim, st, w, tol, f"step {nsteps}")
    return sim, st


def test_fp64_thermal_particles_ragged_multitile():
    # 3 x 3 x 2 stage tiles, ragged in every direction; overlapping kernels
    # allowed (Jacobi superposition of the no-slip corrections).
    w = W.small_random(nx=70, ny=20, nz=40, npart=12, seed=21, kT=1e-3)
    _run_both(w, 4, check_every=1)


def test_fp64_thermal_particles_whole_tiles():
    # nx, ny multiples of the 32 x 16 stage tile: the whole-tile kernels
    w = W.small_random(nx=64, ny=32, nz=20, npart=10, seed=27, kT=1e-3)
    _run_both(w, 3, check_every=1)


def test_fp32_whole_tiles_one_step():
    w = W.small_random(nx=32, ny=48, nz=18, npart=6, seed=37, kT=1e-3)
    w.drho = w.drho.astype(np.float32).astype(np.float64)
    w.g = w.g.astype(np.float32).astype(np.float64)
    _run_both(w, 1, prec="fp32", tol=1e-5)


def test_fp64_deterministic_no_particles():
    w = W.small_random(nx=33, ny=17, nz=35, npart=0, seed=5, kT=0.0)
    w.modes = []
    _run_both(w, 3)


def test_fp64_plane_drive_nonoverlapping_particles_10_steps():
    w = W.small_random(nx=24, ny=24, nz=24, npart=6, seed=8, kT=1e-3, min_sep=3.5)
    w.modes = [W.Mode(axis=2, shape="plane", m=1, x0=7.2, amp=4e-3, omega=0.3),
               W.Mode(axis=1, shape="cos", m=2, x0=0.0, amp=1e-3, omega=0.5, phase=1.0)]
    _run_both(w, 10, check_every=5)


def test_fp64_thermal_particles_500_steps():
    # the long horizon of the parity bar: thermal noise, six particles (some
    # kernels overlapping), a cosine and a plane drive; checked at 100 and 500
    w = W.small_random(nx=22, ny=18, nz=14, npart=6, seed=55, kT=1e-3)
    w.modes.append(W.Mode(axis=1, shape="plane", m=1, x0=5.0, amp=2e-3, omega=0.45, phase=0.2))
    _run_both(w, 500, check_every=100)


def test_fp64_grid_smaller_than_tile():
    w = W.small_random(nx=6, ny=5, nz=4, npart=2, seed=9, kT=1e-3)
    _run_both(w, 3)


def test_fp64_smallest_grid():
    # 4 cells per side, the smallest grid accepted: a particle's influence
    # box wraps onto itself on every axis, so all particles form one cluster
    w = W.small_random(nx=4, ny=4, nz=4, npart=3, seed=9, kT=1e-3)
    _run_both(w, 3, check_every=1)


def test_fp64_particles_on_periodic_seams():
    w = W.small_random(nx=36, ny=12, nz=34, npart=6, seed=13, kT=1e-3)
    L = np.array([36.0, 12.0, 34.0])
    w.particles.q[:] = np.array([[0.0, 0.0, 0.0], [35.999999, 11.5, 33.9], [31.5, 8.0, 32.0],
                                 [32.0, 7.5, 31.5], [0.5, 6.0, 16.0], [18.0, 0.25, 33.75]])
    w.particles.qeq[:] = w.particles.q
    _run_both(w, 3)


@pytest.mark.parametrize("centre", [(20.0, 18.0, 16.0), (0.0, 0.0, 0.0)])
def test_fp64_dense_cluster_matches_oracle(centre):
    # 600 particles packed in a cube of 6 h (in the middle of the box, or
    # across the periodic corner): more particles than the one-workgroup
    # clustering takes, tile lists longer than the union buffer (merged
    # whole), and a cluster of hundreds of members that one wave applies
    # member after member; overlapping kernels throughout (Jacobi reading)
    w = W.small_random(nx=40, ny=36, nz=32, npart=600, seed=21, kT=1e-3)
    rng = np.random.default_rng(5)
    p, fl = w.particles, w.fluid
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    p.q[:] = (np.array(centre) * fl.h + rng.uniform(-3.0, 3.0, size=p.q.shape) * fl.h) % L
    p.qeq[:] = p.q
    _run_both(w, 2, check_every=1)


def test_fp32_dense_cluster_one_step():
    # the same pack in FP32 storage (fields start from FP32 values)
    w = W.small_random(nx=40, ny=36, nz=32, npart=600, seed=23, kT=1e-3)
    rng = np.random.default_rng(6)
    p, fl = w.particles, w.fluid
    p.q[:] = np.array([20.0, 18.0, 16.0]) * fl.h + rng.uniform(-3.0, 3.0, size=p.q.shape) * fl.h
    p.qeq[:] = p.q
    w.drho = w.drho.astype(np.float32).astype(np.float64)
    w.g = w.g.astype(np.float32).astype(np.float64)
    _run_both(w, 1, prec="fp32", tol=1e-5)


def test_fp64_initial_velocity_from_no_slip():
    w = W.small_random(nx=20, ny=16, nz=12, npart=4, seed=3, kT=0.0, min_sep=3.5)
    w.particles.u = None
    _run_both(w, 2)


def test_fp32_one_step_from_fp32_state():
    w = W.small_random(nx=70, ny=20, nz=40, npart=12, seed=31, kT=1e-3)
    w.drho = w.drho.astype(np.float32).astype(np.float64)
    w.g = w.g.astype(np.float32).astype(np.float64)
    _run_both(w, 1, prec="fp32", tol=1e-5)


def test_fp32_deterministic_one_step():
    w = W.small_random(nx=40, ny=24, nz=33, npart=5, seed=41, kT=0.0)
    w.drho = w.drho.astype(np.float32).astype(np.float64)
    w.g = w.g.astype(np.float32).astype(np.float64)
    _run_both(w, 1, prec="fp32", tol=1e-5)


def test_avg_force_and_lambda_sums():
    w = W.small_random(nx=24, ny=20, nz=22, npart=5, seed=17, kT=1e-3)
    sim = _sim(w)
    st = make_state(w)
    prm = w.fluid.as_dict()
    st, sF, sL = O.run(st, prm, 5, modes_of(w))
    sim.step(5)
    f, lam, ns = sim.avg_force(reset=True)
    assert ns == 5
    assert _rel(f, sF / 5) < 1e-12
    assert _rel(lam, sL / 5) < 1e-10
    f2, _, ns2 = sim.avg_force()
    assert ns2 == 0 and np.all(f2 == 0)


def test_conserved_sums_match_oracle():
    w = W.small_random(nx=30, ny=14, nz=18, npart=4, seed=19, kT=1e-3)
    sim = _sim(w)
    st = make_state(w)
    c_gpu = sim.conserved()
    c_or = O.conserved(st, w.fluid.as_dict())
    assert np.allclose(c_gpu, c_or, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_interpolate_and_spread_match_oracle(kind):
    from paper_1307_0702_amd.ic import Simulation
    import torch
    fl = W.Fluid(37, 19, 34, h=0.8)
    rng = np.random.default_rng(kind)
    sim = Simulation(fl, prec="fp64", max_particles=64)
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    q = rng.random((50, 3)) * L
    q[0] = [0.0, 0.0, 0.0]
    q[1] = L - 1e-9
    field = rng.standard_normal(fl.shape)
    face = None if kind == 0 else kind - 1
    got = sim.interpolate(q, kind, field)
    want = O.interpolate(field, q, fl.h, face)
    assert _rel(got, want) < 1e-13
    f = rng.standard_normal(50)
    out = torch.zeros(fl.shape, dtype=torch.float64, device="cuda:0")
    sim.spread(q, f, kind, out)
    want_s = O.spread(f, q, fl.h, fl.shape, face)
    assert _rel(out.cpu().numpy(), want_s) < 1e-13


def test_interpolate_faces_is_the_three_face_kernels():
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation
    fl = W.Fluid(29, 21, 18, h=1.0)
    rng = np.random.default_rng(44)
    sim = Simulation(fl, prec="fp32", max_particles=8)
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    q = rng.random((40, 3)) * L
    g = rng.standard_normal((3,) + fl.shape).astype(np.float32)
    got = sim.interpolate(q, ic.IC_FACES, g)
    assert got.shape == (40, 3)
    for a in range(3):
        one = sim.interpolate(q, ic.IC_FACE_X + a, g[a])
        assert np.array_equal(got[:, a], one)
        want = O.interpolate(g[a].astype(np.float64), q, fl.h, a)
        assert _rel(got[:, a], want) < 1e-13
    # host positions and a host result: staged by the library, same values
    import torch
    gd = torch.as_tensor(g, device=sim.device).contiguous()
    qh = np.ascontiguousarray(q)
    out_h = np.zeros((40, 3))
    ic.ic_interpolate(sim.ctx, 40, qh, ic.IC_FACES, gd, out_h)
    assert np.array_equal(out_h, got)
    out_h1 = np.zeros(40)
    ic.ic_interpolate(sim.ctx, 40, torch.as_tensor(qh, device=sim.device), ic.IC_FACE_Y, gd[1], out_h1)
    assert np.array_equal(out_h1, got[:, 1])


def test_get_and_set_state_resume_bit_for_bit():
    # a snapshot taken after 3 steps and restored later (with the step
    # counter) reproduces the continued trajectory exactly
    import torch
    from paper_1307_0702_amd import ic
    w = W.small_random(nx=30, ny=18, nz=20, npart=5, seed=61, kT=1e-3)
    sim = _sim(w)
    sim.step(3)
    snap = [torch.empty_like(sim.U[i]) for i in range(4)]
    q = torch.empty((w.particles.n, 3), dtype=torch.float64, device=sim.device)
    u = torch.empty_like(q)
    ic.ic_get_state(sim.ctx, snap, q, u)
    sim.step(4)
    r1, g1 = sim.get_state()
    q1, u1 = sim.get_particles()
    sim.U.zero_()
    ic.ic_set_state(sim.ctx, snap, q, u)
    sim.set_step(3)
    sim.step(4)
    r2, g2 = sim.get_state()
    q2, u2 = sim.get_particles()
    assert np.array_equal(r1, r2) and np.array_equal(q1, q2) and np.array_equal(u1, u2)
    for c in range(3):
        assert np.array_equal(g1[c], g2[c])
    bad = q.clone()
    bad[2, 0] = float("inf")
    with pytest.raises(ic.ICError) as e:
        ic.ic_set_state(sim.ctx, None, bad, None)
    assert e.value.code == ic.IC_E_ARG


def test_bitwise_repeatable():
    w = W.small_random(nx=40, ny=16, nz=36, npart=10, seed=23, kT=1e-3)
    a = _sim(w)
    a.step(3)
    b = _sim(w)
    b.step(3)
    ra, ga = a.get_state()
    rb, gb = b.get_state()
    assert np.array_equal(ra, rb)
    for c in range(3):
        assert np.array_equal(ga[c], gb[c])
    assert np.array_equal(a.get_particles()[0], b.get_particles()[0])


def _same(a, b):
    ra, ga = a.get_state()
    rb, gb = b.get_state()
    assert np.array_equal(ra, rb)
    for c in range(3):
        assert np.array_equal(ga[c], gb[c])
    qa, ua = a.get_particles()
    qb, ub = b.get_particles()
    assert np.array_equal(qa, qb) and np.array_equal(ua, ub)
    assert a.conserved().tolist() == b.conserved().tolist()


def _large(seed=29):
    # >= 2^20 cells (two streams, background noise, step graphs), ragged in
    # y for the 32 x 32 and 32 x 8 noise tiles, more tiles than CUs
    return W.small_random(nx=130, ny=100, nz=90, npart=40, seed=seed, kT=1e-3)


def test_background_noise_is_bitwise_the_in_line_noise():
    # b draws every step's noise in line (setting the step counter forgets
    # any noise drawn ahead), a draws each next step's in the background
    from paper_1307_0702_amd import ic
    w = _large()
    a = _sim(w, prec="fp32")
    a.step(3)
    b = _sim(w, prec="fp32")
    for n in range(3):
        ic.ic_set_step(b.ctx, n)
        b.step(1)
    _same(a, b)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_particle_free_step_graph_is_bitwise_the_in_line_noise(prec):
    # no particles: the side stream carries only the next step's noise; 21
    # steps in one call (graph replays) against 21 steps each drawing its
    # noise in line
    from paper_1307_0702_amd import ic
    w = W.small_random(nx=130, ny=100, nz=90, npart=0, seed=43, kT=1e-3)
    a = _sim(w, prec=prec)
    a.step(21)
    b = _sim(w, prec=prec)
    for n in range(21):
        ic.ic_set_step(b.ctx, n)
        b.step(1)
    _same(a, b)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_step_graph_is_bitwise_the_launched_steps(prec):
    # 46 steps in one call: one launched step (the first step's noise is not
    # drawn ahead), 11 replays of the 4-step graph, one launched step;
    # against 46 calls of one step
    from paper_1307_0702_amd import ic
    w = _large(seed=37)
    a = _sim(w, prec=prec)
    a.step(46)
    b = _sim(w, prec=prec)
    for _ in range(46):
        b.step(1)
    _same(a, b)
    assert ic.ic_get_step(a.ctx) == 46
    # a changed forcing is recaptured, the particle count too
    modes = modes_of(w)
    modes[0]["amp"] *= 2.0
    for sim in (a, b):
        sim.set_forcing(modes)
    a.step(20)
    for _ in range(20):
        b.step(1)
    _same(a, b)
    p = w.particles
    from paper_1307_0702_amd import ic as _ic
    eps = np.array([_ic.ic_eps_from_kappa_ratio(w.fluid.cf, r) for r in p.kappa_ratio])
    for sim in (a, b):
        q, u = sim.get_particles()
        sim.set_particles(q[:30], p.me[:30], eps[:30], u=u[:30], ks=p.ks[:30], qeq=p.qeq[:30],
                          fext=p.fext[:30])
    a.step(17)
    for _ in range(17):
        b.step(1)
    _same(a, b)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_prepared_step_graph_is_bitwise_the_launched_steps(prec):
    # 3 steps (too few for the graph), the graph captured without running a
    # step, then 21 steps in one call (five replays of the 4-step graph and
    # one launched step); against 24 calls of one step
    from paper_1307_0702_amd import ic
    w = _large(seed=41)
    a = _sim(w, prec=prec)
    a.step(3)
    a.prepare()
    assert ic.ic_get_step(a.ctx) == 3
    a.prepare()   # nothing changed: the graph is kept
    a.step(21)
    b = _sim(w, prec=prec)
    for _ in range(24):
        b.step(1)
    _same(a, b)
    # a grid too small for the graph, and a profiled context: nothing to do
    s = _sim(W.small_random(nx=16, ny=12, nz=14, npart=2, seed=3, kT=1e-3), prec=prec)
    s.prepare()
    ic.ic_profile(a.ctx, 1)
    a.prepare()
    ic.ic_profile(a.ctx, 0)


def test_error_codes_from_device_paths():
    from paper_1307_0702_amd import ic
    w = W.small_random(nx=16, ny=16, nz=16, npart=2, seed=2, kT=0.0)
    sim = _sim(w)
    with pytest.raises(ic.ICError) as e:
        sim.set_particles(w.particles.q, np.array([-9.0, 0.0]), np.zeros(2))
    assert e.value.code == ic.IC_E_MASS
    with pytest.raises(ic.ICError) as e:
        sim.set_particles(w.particles.q, np.zeros(2), np.array([0.0, 100.0]))
    assert e.value.code == ic.IC_E_UNSTABLE
    with pytest.raises(ic.ICError) as e:
        sim.set_particles(np.zeros((5, 3)), np.zeros(5), np.zeros(5))
    assert e.value.code == ic.IC_E_CAPACITY


def test_non_finite_state_is_reported_and_every_kernel_exits():
    # A NaN density cell next to a particle makes J v, q^{n+1/2} and the
    # impulse non-finite.  The step replaces such positions by 0 before any
    # point index is formed (so every kernel exits normally), keeps the old
    # position, and the next synchronising call reports IC_E_ARG
    # ("non-finite state"), not IC_E_MASS.
    from paper_1307_0702_amd import ic
    w = W.small_random(nx=20, ny=16, nz=14, npart=3, seed=31, kT=0.0, min_sep=3.5)
    q0 = np.array(w.particles.q[0])
    i, j, k = (np.floor(q0 / w.fluid.h + 0.5).astype(int) % [w.fluid.nx, w.fluid.ny, w.fluid.nz])
    bad = w.drho.copy()
    bad[k, j, i] = np.nan
    sim = _sim(w)
    sim.set_state(bad, w.g)
    print("non-finite density next to particle 0, fp64", flush=True)
    sim.step(2)
    with pytest.raises(ic.ICError) as e:
        sim.get_particles()
    assert e.value.code == ic.IC_E_ARG
    assert "non-finite" in str(e.value)
    # the flag was cleared, positions stayed finite and inside the box
    q, _ = sim.get_particles()
    L = np.array([w.fluid.nx, w.fluid.ny, w.fluid.nz]) * w.fluid.h
    assert np.all(np.isfinite(q)) and np.all(q >= 0) and np.all(q < L)
    # a finite state steps normally again
    sim.set_state(w.drho, w.g)
    eps = np.array([ic.ic_eps_from_kappa_ratio(w.fluid.cf, r) for r in w.particles.kappa_ratio])
    p = w.particles
    sim.set_particles(p.q, p.me, eps, u=p.u, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.step(1)
    q, u = sim.get_particles()
    assert np.all(np.isfinite(q)) and np.all(np.isfinite(u))
    # J at a non-finite position is NaN, not an out-of-bounds gather
    out = sim.interpolate(np.array([[np.nan, 1.0, 1.0], [2.0, 3.0, 4.0]]), ic.IC_CELL, sim.U[0])
    assert np.isnan(out[0]) and np.isfinite(out[1])
