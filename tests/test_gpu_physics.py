"""Physics of the IC step on the GPU path, against closed forms of the paper.

The oracle cannot run the tens of thousands of steps these need, so they run
on the HIP path, which the parity tests tie to the oracle step by step.

* Radiation force (Sec. V, Eq. (1); Sec. VI protocol): two particles tethered
  at x0 +- 3L/8 from the pressure antinode of a resonantly driven standing
  wave.  Their springs inject opposite momenta, so the total stays zero.
  The mean spring force is compared with Gor'kov's
  F = c_f^2 drho^2 V k / (4 rho0) (f1 + 3/2 f2) sin(2 k z), using the measured
  wave amplitude.  f1 = 1 - kappa_p/kappa_f, f2 = 2 m_e / (2 m_e + 3 rho0 V).
  The springs are soft (tether frequency a sixth of the drive frequency at
  every box size), so the particles oscillate with the wave as Gor'kov's
  force assumes.  Regime: the paper's nu/(c h) = 0.0125; box sizes 32h to 64h
  for the finite-size check (Sec. VI studies the same dependence).
* Equilibrium fluctuations (Sec. IV E; App. A, convergence analysis):
  Var(drho) = rho0 kT/(c_f^2 h^3) per cell, Var(v) = kT/(rho0 h^3) per face,
  Var(J rho) = rho0 kT/(c_p^2 V) at a particle, and particle equipartition
  Var(u_a) = kT/m_p.
"""
import math

import numpy as np
import pytest

from paper_1307_0702_amd import workloads as W

pytestmark = pytest.mark.gpu

V = 8.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sim(w, prec):
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation
    fl, p = w.fluid, w.particles
    sim = Simulation(fl, prec=prec, max_particles=max(p.n, 1))
    sim.set_state(w.drho, w.g)
    if p.n:
        eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
        sim.set_particles(p.q, p.me, eps, u=p.u, ks=p.ks, qeq=p.qeq, fext=p.fext)
    if w.modes:
        sim.set_forcing([m.as_dict() for m in w.modes])
    return sim


def _amplitude(sim, w, nT):
    """Amplitude of the cos(k (x - x0)) density mode over one period."""
    fl = w.fluid
    x = np.arange(fl.nx) * fl.h
    c = np.cos(2 * math.pi * w.modes[0].m * (x - w.modes[0].x0) / (fl.nx * fl.h))
    a2 = []
    for _ in range(nT):
        sim.step(1)
        d, _ = sim.get_state()
        a = 2.0 / fl.nx * np.sum(d.mean(axis=(0, 1)) * c)
        a2.append(a * a)
    return math.sqrt(2.0 * np.mean(a2))


def radiation_force(me, kappa_ratio, eta=0.0125, amp=1e-3, ks=None, nwarm=None, nper=4,
                    prec="fp64", L=32, Lt=None, m=1):
    """Mean tether force on the symmetric pair and Gor'kov's value for it.
    The tether is soft, k_s = m_p (omega/6)^2 (reading R9), so its frequency
    stays a sixth of the drive frequency at every box size; the warm-up
    grows with the acoustic damping time, as L^2.  Lt: lateral box size (y, z;
    default L); the wave runs along x with wavelength L / m."""
    Lt = L if Lt is None else Lt
    lam = L / m
    fl = W.Fluid(L, Lt, Lt, kT=0.0, seed=1, eta=eta, zeta=eta)
    mode, nT = W.modal_drive(fl, amp, m=m)
    if ks is None:
        ks = (me + fl.rho0 * V) * (mode.omega / 6) ** 2
    if nwarm is None:
        nwarm = int(40000 * (L / 32) ** 2)
    drho, g = W.standing_wave_fields(fl, amp, m=m, omega=mode.omega)
    qeq = np.array([[3 * lam / 8, Lt / 2, Lt / 2], [lam - 3 * lam / 8, 0.0, 0.0]])
    k = 2 * math.pi / lam
    kd = 2.0 / fl.h * math.sin(k * fl.h / 2)
    # start each particle where the fluid around it is at t = 0 (one end of
    # its oscillation), so its mean position starts at the anchor
    q = qeq.copy()
    q[:, 0] -= amp * np.sin(k * (qeq[:, 0] - mode.x0)) / kd
    p = W.Particles(q=q, me=np.full(2, me), kappa_ratio=np.full(2, kappa_ratio),
                    ks=np.full(2, ks), qeq=qeq)
    w = W.Workload("pair", fl, p, [mode], drho, g, nT)
    print(f"radiation force: me={me} kappa_ratio={kappa_ratio} eta={eta} amp={amp} {prec} "
          f"L={L} Lt={Lt} m={m} steps={nwarm + nper * nT}", flush=True)
    sim = _sim(w, prec)
    sim.step(nwarm)
    sim.avg_force(reset=True)
    sim.step(nper * nT)
    f, _, _ = sim.avg_force(reset=True)
    mom = sim.conserved()[1:]
    a = _amplitude(sim, w, nT)
    f1 = 1 - kappa_ratio
    f2 = 2 * me / (2 * me + 3 * fl.rho0 * V)
    mag = fl.cf ** 2 * a * a * V * k / (4 * fl.rho0) * (f1 + 1.5 * f2)
    # z = +3L/8 and -3L/8 from the antinode: sin(2 k z) = -1 and +1
    gork = np.array([-mag, mag])
    print(f"  mean F_x {f[:, 0]}, Gor'kov {gork}, amplitude {a:.4e}, momentum {mom}", flush=True)
    return f, gork, mom, a


def test_radiation_force_dipolar():
    f, gork, mom, _ = radiation_force(me=V, kappa_ratio=1.0)       # f1 = 0, f2 = 0.4
    assert np.all(np.abs(mom) < 1e-9)
    assert np.allclose(f[:, 1:], 0.0)
    assert np.all(np.sign(f[:, 0]) == np.sign(gork))
    assert np.allclose(f[:, 0], gork, rtol=0.05)


def test_radiation_force_monopolar():
    # c_p = 2 c_f: kappa_p = kappa_f / 4, f1 = 0.75, in a box of 32 h.  At
    # this box size the paper reports monopolar deviations reaching roughly 10%
    # from Gor'kov (Sec. VI A); the model's force is about 10% low.
    f, gork, _, _ = radiation_force(me=0.0, kappa_ratio=0.25)
    assert np.all(np.sign(f[:, 0]) == np.sign(gork))
    r = f[:, 0] / gork
    assert np.all((r > 0.85) & (r < 0.95)), r


def test_radiation_force_soft_monopolar_particle():
    # kappa_p = 2 kappa_f (c_p = c_f / sqrt 2), neutrally buoyant: f1 = -1.
    # Unlike the stiff particle above, the soft one follows Gor'kov closely.
    f, gork, _, _ = radiation_force(me=0.0, kappa_ratio=2.0, nper=8)
    r = f[:, 0] / gork
    print(f"  soft monopolar ratio {r}", flush=True)
    assert np.all(np.abs(r - 1) < 0.04), r


OPEN_MONOPOLAR = ("open discrepancy with Sec. VI A: the paper's monopolar deviation (about 10% "
                  "at 32 h) tends to zero as the box grows; in this low-viscosity setup the "
                  "model's stiff-particle deficit stays near 10% in larger and wider boxes "
                  "(near 6% once the tether's reactive mass k_s/omega^2 is counted)")


@pytest.mark.xfail(strict=True, reason=OPEN_MONOPOLAR)
def test_radiation_force_lateral_box_size():
    # Wavelength fixed at 32h, box widened to 64h across the wave: periodic
    # images twice as far.  If the 32 h deficit were an image effect, as the
    # paper's finite-size argument has it, the ratio would move toward 1.
    f, gork, _, _ = radiation_force(me=0.0, kappa_ratio=0.25, Lt=64, nper=8)
    r = f[:, 0] / gork
    print(f"  32 x 64 x 64 monopolar ratio {r}", flush=True)
    assert np.all(np.abs(r - 1) < 0.05), r


def test_radiation_force_frequency_dependence_dipolar():
    # Box 64h, second mode (wavelength 32h): twice the frequency of the first
    # mode in the same box.  The dipolar ratio stays within a few per cent
    # of 1.
    f, gork, _, _ = radiation_force(me=V, kappa_ratio=1.0, L=64, m=2, nper=8)
    rd = f[:, 0] / gork
    print(f"  L = 64, m = 2: dipolar ratio {rd}", flush=True)
    assert np.all(np.abs(rd - 1) < 0.05), rd


@pytest.mark.xfail(strict=True, reason=OPEN_MONOPOLAR)
def test_radiation_force_frequency_dependence_monopolar():
    # Same box and mode for the stiff particle: the periodic images are twice
    # as far (in wavelengths) as in the 32 h box, so under the paper's
    # finite-size argument the deficit would have shrunk.
    f, gork, _, _ = radiation_force(me=0.0, kappa_ratio=0.25, L=64, m=2, nper=8)
    rm = f[:, 0] / gork
    print(f"  L = 64, m = 2: monopolar ratio {rm}", flush=True)
    assert np.all(np.abs(rm - 1) < 0.05), rm


@pytest.mark.parametrize("L", [48, 64])
def test_radiation_force_finite_size_dipolar(L):
    # Box sizes 48h and 64h (kR_a = 0.16 and 0.12 against 0.24 at 32h).
    f, gork, _, _ = radiation_force(me=V, kappa_ratio=1.0, L=L, nper=8)
    rd = f[:, 0] / gork
    print(f"  L = {L}: dipolar ratio {rd}", flush=True)
    assert np.all(np.abs(rd - 1) < 0.05), rd


@pytest.mark.xfail(strict=True, reason=OPEN_MONOPOLAR)
@pytest.mark.parametrize("L,bound", [(48, 0.07), (64, 0.05)])
def test_radiation_force_finite_size_monopolar(L, bound):
    # The paper: the about-10% monopolar deviation at 32 h tends to zero as
    # the box grows (Sec. VI A); at least as 1/L, it would be below 7% at
    # 48 h and 5% at 64 h.
    f, gork, _, _ = radiation_force(me=0.0, kappa_ratio=0.25, L=L, nper=8)
    rm = f[:, 0] / gork
    print(f"  L = {L}: monopolar ratio {rm}", flush=True)
    assert np.all(np.abs(rm - 1) < bound), rm


def test_radiation_force_negative_contrast():
    # m_p = rho0 V / 2, kappa_p = 2 kappa_f: f1 + 3/2 f2 = -1.75
    f, gork, _, _ = radiation_force(me=-0.5 * V, kappa_ratio=2.0)
    assert np.all(np.sign(f[:, 0]) == np.sign(gork))
    assert np.allclose(f[:, 0], gork, rtol=0.06)


def test_radiation_force_neutral_particle_and_amplitude_scaling():
    f0, _, _, a = radiation_force(me=0.0, kappa_ratio=1.0)
    # a neutral blob feels only a finite-size remainder: compare with the
    # dipolar force of an m_p = 2 rho0 V particle (f2 = 0.4) in the same wave
    L = 32
    ref = a * a * V * (2 * math.pi / L) / 4 * 1.5 * 0.4
    assert np.all(np.abs(f0[:, 0]) < 0.08 * ref)
    # the force is second order in the wave amplitude
    fa, _, _, _ = radiation_force(me=V, kappa_ratio=1.0)
    fb, _, _, _ = radiation_force(me=V, kappa_ratio=1.0, amp=5e-4)
    assert np.allclose(fb[:, 0] / fa[:, 0], 0.25, rtol=0.03)


@pytest.mark.parametrize("amp,bound", [(1e-3, 1e-3), (1e-2, 1e-4)])
def test_fp32_averaged_force_against_fp64(amp, bound):
    # Deterministic run (kT = 0): FP32 storage of the fields as deviations
    # from rho0 with FP64 particle state and accumulators, against all-FP64.
    # The radiation force is second order in the wave amplitude while the
    # fluxes it comes from are first order, so FP32 rounding of those fluxes
    # is amplified by 1/amplitude in the averaged force: 6.4e-4 relative at
    # drho = 1e-3, 8.7e-5 at the paper-scale drho = 1e-2 (measured).  The FP32
    # momentum drift (~1e-8 here) is not the cause: removing it every 10
    # steps leaves the difference unchanged.
    kw = dict(me=V, kappa_ratio=0.5, eta=0.5, nwarm=20000, nper=4, amp=amp)
    f64, _, m64, _ = radiation_force(prec="fp64", **kw)
    f32, _, m32, _ = radiation_force(prec="fp32", **kw)
    rel = np.max(np.abs(f32[:, 0] - f64[:, 0])) / np.max(np.abs(f64[:, 0]))
    print(f"  FP32 vs FP64 averaged force: relative difference {rel:.2e}; "
          f"momentum FP32 {m32[0]:.2e}, FP64 {m64[0]:.2e}", flush=True)
    assert np.all(np.sign(f32[:, 0]) == np.sign(f64[:, 0]))
    assert abs(m64[0]) < 1e-9 and abs(m32[0]) < 1e-4
    assert rel < bound


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_equilibrium_fluctuations_and_equipartition(prec):
    from paper_1307_0702_amd import ic
    fl = W.Fluid(32, 32, 32, kT=1e-3, seed=7)
    p = W.uniform_particles(fl, 8, 70, ks=0.0, min_sep=4.0)
    w = W.Workload("thermal-32", fl, p, [], np.zeros(fl.shape), np.zeros((3,) + fl.shape), 0)
    print(f"thermal equilibrium {prec}: 32^3, 8 particles, 22000 steps", flush=True)
    sim = _sim(w, prec)
    sim.step(2000)
    mp = p.me + fl.rho0 * V
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    us, dr, vv, jr = [], [], [], []
    for it in range(2000):
        sim.step(10)
        q, u = sim.get_particles()
        us.append(u.copy())
        if it % 20 == 0:
            d, gg = sim.get_state()
            dr.append(d.var())
            rf = fl.rho0 + 0.5 * (d + np.roll(d, -1, axis=2))
            vv.append((gg[0] / rf).var())
            jr.append(sim.interpolate(q, ic.IC_CELL, d))
    us = np.array(us)
    equi = (us ** 2).mean(axis=0) / (fl.kT / mp)[:, None]
    var_rho = np.mean(dr) / (fl.rho0 * fl.kT / fl.cf ** 2)
    var_v = np.mean(vv) / (fl.kT / fl.rho0)
    cp2 = fl.cf ** 2 + eps
    var_j = np.array(jr).var(axis=0) / (fl.rho0 * fl.kT / (cp2 * V))
    print(f"  Var(u) m_p/kT mean {equi.mean():.4f}; Var drho {var_rho:.4f}; Var v {var_v:.4f}; "
          f"Var(J rho) mean {var_j.mean():.4f}", flush=True)
    assert abs(equi.mean() - 1) < 0.03
    assert abs(var_rho - 1) < 0.02
    assert abs(var_v - 1) < 0.02
    assert abs(var_j.mean() - 1) < 0.06


def secondary_force(d, amp=1e-2, L=32, eta=0.0125, kappa_ratio=0.5, nper=8):
    """Two neutrally buoyant particles on the pressure-antinode plane of the
    standing wave (x = x0), a distance d apart along z, softly tethered: the
    mean tether forces and the point-source secondary (Bjerknes) force of
    Sec. VI, F = (9 / 4 pi) V^2 <p_in^2> omega^2 rho0 kappa_e^2 / (9 d^2)
    (attractive for particles pulsating in phase), <p_in^2> = (c_f^2 a)^2 / 2
    at the antinode, kappa_e = kappa_p - kappa_f."""
    fl = W.Fluid(L, L, L, kT=0.0, seed=1, eta=eta, zeta=eta)
    mode, nT = W.modal_drive(fl, amp)
    drho, g = W.standing_wave_fields(fl, amp, omega=mode.omega)
    centre = np.array([mode.x0, L / 2, L / 2])
    qeq = np.array([centre - [0, 0, d / 2], centre + [0, 0, d / 2]])
    ks = V * (mode.omega / 6) ** 2
    p = W.Particles(q=qeq.copy(), me=np.zeros(2), kappa_ratio=np.full(2, kappa_ratio),
                    ks=np.full(2, ks), qeq=qeq)
    w = W.Workload("pair-antinode", fl, p, [mode], drho, g, nT)
    print(f"secondary force: d={d} kappa_ratio={kappa_ratio} amp={amp} L={L}", flush=True)
    sim = _sim(w, "fp64")
    sim.step(int(40000 * (L / 32) ** 2))
    sim.avg_force(reset=True)
    sim.step(nper * nT)
    f, _, _ = sim.avg_force(reset=True)
    a = _amplitude(sim, w, nT)
    ke = (kappa_ratio - 1.0) / (fl.rho0 * fl.cf ** 2)
    p2 = (fl.cf ** 2 * a) ** 2 / 2
    theory = 9 / (4 * math.pi) * V ** 2 * p2 * mode.omega ** 2 * fl.rho0 * ke ** 2 / (9 * d ** 2)
    print(f"  mean force {f.tolist()}, point-source value {theory:.4e}, amplitude {a:.4e}", flush=True)
    return f, theory


def test_secondary_force_between_compressible_particles():
    # Attraction along the line of centres, equal and opposite, no primary
    # force on the antinode plane, weaker at larger distance.  Its size is
    # 2.4x the point-source value at d = 2.5h here (measured), within a
    # factor [1.5, 3.5] below.
    f25, t25 = secondary_force(2.5)
    f4, t4 = secondary_force(4.0)
    for f in (f25, f4):
        assert f[0, 2] > 0 and f[1, 2] < 0                     # attraction
        assert abs(f[0, 2] + f[1, 2]) < 1e-6 * abs(f[0, 2])   # equal and opposite
        assert np.all(np.abs(f[:, :2]) < 1e-6 * abs(f[0, 2]))
    assert f25[0, 2] > f4[0, 2]
    r = f25[0, 2] / t25
    assert 1.5 < r < 3.5, r


def gibbs_boltzmann(nwarm, nrun, every=200):
    """Free dipolar particles in a thermal standing wave: the time average of
    cos(2 k xi) (xi = x - x0 from the pressure antinode) against the
    Boltzmann average in the acoustic potential U = U0 cos(2 k xi) + const,
    U0 = V p_a^2 (f1 + 3/2 f2) / (8 rho0 c_f^2) (Sec. V, Eq. (1) integrated;
    Sec. VI), <cos> = -I1(U0/kT) / I0(U0/kT).  Returns (measured, its
    standard error over particles, Boltzmann value, U0/kT)."""
    from scipy.special import i0, i1
    w = W.gibbs_boltzmann_32()
    fl, mode = w.fluid, w.modes[0]
    sim = _sim(w, "fp64")
    k = 2 * math.pi * mode.m / (fl.nx * fl.h)
    sim.step(nwarm)
    cs = []
    for _ in range(nrun // every):
        sim.step(every)
        q, _ = sim.get_particles()
        cs.append(np.cos(2 * k * (q[:, 0] - mode.x0)))
    a = _amplitude(sim, w, w.period_steps)
    cs = np.array(cs)
    f2 = 2 * w.particles.me[0] / (2 * w.particles.me[0] + 3 * fl.rho0 * V)
    u0 = V * (fl.cf ** 2 * a) ** 2 * (1.5 * f2) / (8 * fl.rho0 * fl.cf ** 2) / fl.kT
    per = cs.mean(axis=0)
    return float(per.mean()), float(per.std() / math.sqrt(len(per))), float(-i1(u0) / i0(u0)), u0


def test_gibbs_boltzmann_position_distribution():
    # Particles start spread uniformly along the wave and collect around the
    # pressure nodes; the measured average (-0.339 +- 0.043 over 6e5 steps,
    # U0/kT = 0.75) matches the Boltzmann value (-0.350).  The shorter run
    # here is checked to three standard errors, and against the uniform
    # distribution's 0.
    m, se, th, u0 = gibbs_boltzmann(50000, 300000)
    print(f"  <cos 2k xi> {m:.4f} +- {se:.4f}, Boltzmann {th:.4f}, U0/kT {u0:.3f}", flush=True)
    assert 0.4 < u0 < 1.5
    assert abs(m - th) < 3 * max(se, 0.03)
    assert m < -0.1                      # well away from a uniform spread



def test_force_sweeps_of_the_paper_figures_as_one_ensemble():
    # Sec. VI force figures: the force along the wave for a dense particle
    # (f2 = 0.4) and a stiff one (c_p = 2 c_f), and its maximum against
    # c_p / c_f and rho_p / rho0 -- 26 boxes of 32^3 advanced together in
    # HIP-graph launches (ensemble).  Gor'kov with the measured amplitude.
    from paper_1307_0702_amd.ensemble import Ensemble
    cases = W.force_sweeps_32()
    ens = Ensemble([w for _, _, w in cases], prec="fp64", tune=False)
    nT = cases[0][2].period_steps
    chunk = nT // 3
    ens.capture(chunk)
    ens.run(-(-40000 // chunk))
    for s in ens.sims:
        s.avg_force(reset=True)
    ens.run(8 * nT // chunk)
    forces = [s.avg_force(reset=True)[0] for s in ens.sims]
    a2 = np.zeros(len(cases))
    for _ in range(3):                  # a third of a period apart: exact mean of a^2
        ens.run(1)
        for i, (s, (_, _, w)) in enumerate(zip(ens.sims, cases)):
            d, _ = s.get_state()
            x = np.arange(w.fluid.nx) * w.fluid.h
            c = np.cos(2 * math.pi * (x - w.modes[0].x0) / (w.fluid.nx * w.fluid.h))
            a = 2.0 / w.fluid.nx * np.sum(d.mean(axis=(0, 1)) * c)
            a2[i] += a * a / 3
    ens.release()
    res = {}
    for (name, par, w), f, m2 in zip(cases, forces, a2):
        fl, p = w.fluid, w.particles
        k = 2 * math.pi / (fl.nx * fl.h)
        f1 = 1.0 - p.kappa_ratio[0]
        f2 = 2 * p.me[0] / (2 * p.me[0] + 3 * fl.rho0 * V)
        x = (p.qeq[0, 0] - w.modes[0].x0) % (fl.nx * fl.h)
        gk = fl.cf ** 2 * 2 * m2 * V * k / (4 * fl.rho0) * (f1 + 1.5 * f2) * math.sin(2 * k * x)
        res.setdefault(name, []).append((par, f[0, 0], gk))
    scale = max(abs(f[0, 0]) for f in forces)
    for f in forces:
        assert abs(f[0, 0] + f[1, 0]) < 1e-6 * scale        # the mirrored pair's forces cancel
    for name, rows in res.items():
        print(f"  {name}: " + ", ".join(f"{par:g}: {fx / gk:.3f}" if abs(gk) > 1e-15 else f"{par:g}: node"
                                       for par, fx, gk in rows), flush=True)
    fmax = max(abs(fx) for _, fx, _ in res["position-dipolar"])
    for name, lo, hi in (("position-dipolar", 0.94, 1.06), ("position-monopolar", 0.82, 0.95)):
        for par, fx, gk in res[name]:
            if par == 8.0:                    # the pressure node: sin 2kx = 0
                assert abs(fx) < 0.03 * fmax, (name, fx)
            else:
                assert lo < fx / gk < hi, (name, par, fx / gk)
    for par, fx, gk in res["sound-speed-ratio"]:
        # soft particles (c_p < c_f) follow Gor'kov, stiff ones carry the
        # monopolar deficit
        lo, hi = (0.9, 1.1) if par < 1 else (0.78, 0.95)
        assert lo < fx / gk < hi, (par, fx / gk)
    soft = [abs(fx) for par, fx, _ in res["sound-speed-ratio"] if par < 1]
    assert soft == sorted(soft, reverse=True)          # grows as c_p / c_f -> 0
    for par, fx, gk in res["density-ratio"]:
        assert 0.92 < fx / gk < 1.08, (par, fx / gk)
