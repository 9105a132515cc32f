"""Host-side pieces of the radiation-force experiments (no GPU).

* The tether's reactive mass: a particle held by a spring k_s and moved at
  the drive frequency omega answers a periodic force as a free particle of
  mass m - k_s/omega^2.  Checked against a direct integration of the driven,
  damped oscillator m x'' = -k_s x - c x' + F0 cos(omega t) (its steady
  amplitude is F0 / |k_s - m omega^2 + i c omega|), so the mass shift that
  the comparisons with Gor'kov's force use is the one the mechanics gives.
* Gor'kov's force with that mass: f2 of m_e - k_s/omega^2, f1 unchanged.
* The Table I configuration in other box sizes: driven at the box's
  discrete resonance (2 c_f / h) sin(pi h / L), a period of whole steps,
  the symmetric pair at +-3L/8 from the driven plane, tether scaled.
"""
import math

import numpy as np
import pytest

from paper_1307_0702_amd import experiments as E
from paper_1307_0702_amd import workloads as W


def _steady_amplitude(m, k, c, omega, f0, periods=200, steps_per_period=400):
    # classical RK4 on (x, v); the amplitude over the last ten periods
    dt = 2 * math.pi / omega / steps_per_period

    def f(t, y):
        x, v = y
        return np.array([v, (-k * x - c * v + f0 * math.cos(omega * t)) / m])

    y = np.zeros(2)
    t = 0.0
    xs = []
    n = periods * steps_per_period
    for i in range(n):
        k1 = f(t, y)
        k2 = f(t + dt / 2, y + dt / 2 * k1)
        k3 = f(t + dt / 2, y + dt / 2 * k2)
        k4 = f(t + dt, y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        t += dt
        if i >= n - 10 * steps_per_period:
            xs.append(y[0])
    return 0.5 * (max(xs) - min(xs))


@pytest.mark.parametrize("k_over_m_omega2", [1.0 / 36, 1.0 / 9, 0.25])
def test_tether_acts_as_a_mass_shift_at_the_drive_frequency(k_over_m_omega2):
    m, omega, f0 = 3.0, 0.7, 1e-3
    k = k_over_m_omega2 * m * omega ** 2
    c = 0.05 * m * omega                       # light damping, as the fluid gives
    amp = _steady_amplitude(m, k, c, omega, f0)
    m_eff = m - E.tether_mass(k, omega)
    # a free particle of mass m_eff with the same damping
    want = f0 / abs(-m_eff * omega ** 2 + 1j * c * omega)
    assert amp == pytest.approx(want, rel=2e-3)
    # and not the spring-free mass
    assert abs(amp / (f0 / abs(-m * omega ** 2 + 1j * c * omega)) - 1) > 0.9 * k_over_m_omega2


def test_gorkov_with_the_tether_mass():
    fl = W.Fluid(32, 32, 32, h=10.0, cf=4.0)
    V = 8.0 * fl.h ** 3
    z = np.array([30.0, -50.0])
    for me, kr in ((8000.0, 1.0), (0.0, 0.25), (-2000.0, 2.0)):
        mt = 444.0
        got = E._gorkov(fl, 3e-3, me, kr, z, m_tether=mt)
        k = 2 * math.pi / (fl.nx * fl.h)
        f2 = 2 * (me - mt) / (2 * (me - mt) + 3 * fl.rho0 * V)
        want = fl.cf ** 2 * 9e-6 * V * k / (4 * fl.rho0) * ((1 - kr) + 1.5 * f2) * np.sin(2 * k * z)
        assert np.allclose(got, want, rtol=1e-14, atol=0)
        assert np.allclose(E._gorkov(fl, 3e-3, me - mt, kr, z), got, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", [32, 48, 64])
def test_table1_in_other_box_sizes(n):
    w = W.table1("force3", n=n, ks_scale=0.25)
    fl, p, mode = w.fluid, w.particles, w.modes[0]
    L = n * fl.h
    omega = W.TABLE1["force3"]["omega"] if n == 32 else 2 * fl.cf / fl.h * math.sin(math.pi * fl.h / L)
    assert mode.omega == omega
    assert mode.shape == "plane" and mode.amp == 0.005
    assert w.period_steps * fl.dt * omega == pytest.approx(2 * math.pi, rel=1e-14)
    assert np.allclose(p.qeq[:, 0], [3 * L / 8, L - 3 * L / 8])
    V = 8.0 * fl.h ** 3
    assert np.allclose(p.ks, 0.25 * fl.rho0 * V * (omega / 6) ** 2, rtol=1e-14)
    assert np.allclose(p.kappa_ratio, (4.0 / 8.0) ** 2)
    # the printed frequency of the 32^3 box is its discrete resonance
    assert W.TABLE1["force3"]["omega"] == pytest.approx(
        2 * fl.cf / fl.h * math.sin(math.pi / 32), abs=5e-7)
