"""Force measurements of Sec. VI on the HIP path (used by bench.py and the
GPU tests).

table1_run: the Table I configuration of one force figure in the paper's
units (plane drive, h = 10, c_f = 4): the measured amplitude of the driven
density mode and, with the symmetric tethered pair, the window mean of
-F_tether and Gor'kov's force (Sec. V, Eq. (1)) with that amplitude.

gorkov_single_32: one tethered particle in the deterministic 32^3 standing
wave at eta = zeta = 0.5 (m_p = 2 rho0 V, kappa_p = kappa_f / 2, at x = 4
from the antinode), 1000 steps, the spring force averaged over the last two
whole drive periods, against Gor'kov's value.
"""
from __future__ import annotations

import math

import numpy as np

from . import ic
from . import workloads as W


def _gorkov(fl, amp, me, kappa_ratio, z, m_tether=0.0):
    """Gor'kov's primary force F = c_f^2 amp^2 V k / (4 rho0) (f1 + 3/2 f2)
    sin(2 k z), z measured from the pressure antinode, for the fundamental
    mode along x.  m_tether: a mass taken off the excess mass in f2 (the
    tether's reactive mass, see tether_mass)."""
    V = 8.0 * fl.h ** 3
    k = 2.0 * math.pi / (fl.nx * fl.h)
    f1 = 1.0 - kappa_ratio
    me = me - m_tether
    f2 = 2.0 * me / (2.0 * me + 3.0 * fl.rho0 * V)
    return fl.cf ** 2 * amp * amp * V * k / (4.0 * fl.rho0) * (f1 + 1.5 * f2) * np.sin(2.0 * k * z)


def tether_mass(ks, omega):
    """Reactive mass of a tether at the drive frequency: over one drive
    period the spring force -k_s (q - q_eq) of a particle oscillating with
    the wave is k_s/omega^2 times its acceleration, so the particle answers
    the wave as one with excess mass m_e - k_s/omega^2 (a dipolar term of
    its own in Gor'kov's f2, whatever the particle's compressibility)."""
    return ks / omega ** 2


def _mode_amplitude_tracker(sim, fl, x0=0.0):
    """Per-step accumulator of the squared cos(k (x - x0)) density-mode
    amplitude, on the device (no copy of the state per step)."""
    t = sim.torch
    k = 2.0 * math.pi / (fl.nx * fl.h)
    c = t.cos(k * (t.arange(fl.nx, dtype=t.float64, device=sim.device) * fl.h - x0))
    acc = t.zeros((), dtype=t.float64, device=sim.device)

    def add():
        a = 2.0 / fl.nx * (sim.U[0].double().mean(dim=(0, 1)) * c).sum()
        acc.add_(a * a)

    return add, acc


def _sim(w, prec):
    fl, p = w.fluid, w.particles
    sim = ic.Simulation(fl, prec=prec, max_particles=max(p.n, 1))
    sim.set_state(w.drho, w.g)
    if p.n:
        eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
        sim.set_particles(p.q, p.me, eps, u=p.u, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing([m.as_dict() for m in w.modes])
    return sim


def table1_run(fig, particles=True, nwarm=40000, nper=10, prec="fp64", log=None, **kw):
    """Returns dict(amp=measured mode amplitude, printed=Table I's value,
    force=[2][3] mean -F_tether or None, gorkov=[2] Gor'kov's F_x or None,
    gorkov_tether=[2] the same with the tethers' reactive mass).  kw go to
    workloads.table1 (n, ks_scale, cp); nwarm is the warm-up for the 32^3
    box and grows as L^2 with it (the resonant mode's decay time)."""
    w = W.table1(fig, particles, **kw)
    nwarm = int(round(nwarm * (w.fluid.nx / 32) ** 2 / w.period_steps)) * w.period_steps
    fl, p = w.fluid, w.particles
    sim = _sim(w, prec)
    if log:
        log(f"table I {fig}: {p.n} particles, dt {fl.dt:.6f}, {nwarm} + {nper} x "
            f"{w.period_steps} steps")
    sim.step(nwarm)
    if p.n:
        sim.avg_force(reset=True)
    add, acc = _mode_amplitude_tracker(sim, fl)
    n = nper * w.period_steps
    for _ in range(n):
        sim.step(1)
        add()
    amp = math.sqrt(2.0 * float(acc) / n)
    out = dict(fig=fig, amp=amp, printed=W.TABLE1[fig]["drho"], force=None, gorkov=None,
               gorkov_tether=None)
    if p.n:
        f, _, _ = sim.avg_force(reset=True)
        L = fl.nx * fl.h
        z = (p.qeq[:, 0] - w.modes[0].x0 + L / 2) % L - L / 2
        out["force"] = f
        out["gorkov"] = _gorkov(fl, amp, p.me[0], p.kappa_ratio[0], z)
        out["gorkov_tether"] = _gorkov(fl, amp, p.me[0], p.kappa_ratio[0], z,
                                       tether_mass(p.ks[0], w.modes[0].omega))
    return out


def gorkov_single_32(prec="fp64", nsteps=1000, navg_periods=2):
    """One tethered particle in the 32^3 standing wave at eta = zeta = 0.5
    (the deterministic FP64 configuration): mean -F_tether_x over the last
    navg_periods whole drive periods of nsteps steps, the measured wave
    amplitude over the same window, and Gor'kov's force with it."""
    fl = W.Fluid(32, 32, 32, kT=0.0, seed=1)
    V = 8.0
    mode, nT = W.modal_drive(fl, 1e-3)
    drho, g = W.standing_wave_fields(fl, 1e-3, omega=mode.omega)
    q = np.array([[4.0, 16.0, 16.0]])
    ks = W.soft_tether(fl, mode.omega, 2.0 * V)
    p = W.Particles(q=q, me=np.array([V]), kappa_ratio=np.array([0.5]), ks=np.array([ks]),
                    qeq=q.copy())
    w = W.Workload("gorkov-single-32", fl, p, [mode], drho, g, nT)
    sim = _sim(w, prec)
    navg = navg_periods * nT
    sim.step(nsteps - navg)
    sim.avg_force(reset=True)
    add, acc = _mode_amplitude_tracker(sim, fl)
    for _ in range(navg):
        sim.step(1)
        add()
    f, _, ns = sim.avg_force(reset=True)
    amp = math.sqrt(2.0 * float(acc) / navg)
    gk = float(_gorkov(fl, amp, V, 0.5, np.array([4.0]))[0])
    mom = sim.conserved()[1:]
    return dict(force=f[0].tolist(), gorkov=gk, ratio=float(f[0, 0] / gk), amp=amp,
                averaged_steps=int(ns), warmup_steps=nsteps - navg, period_steps=nT,
                total_momentum=mom.tolist())
