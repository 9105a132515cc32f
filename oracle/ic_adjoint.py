"""Plain FP64 adjoint (reverse mode) of the deterministic fluid part of the IC
step, for checking the HIP adjoint.

TEST INFRASTRUCTURE ONLY, like ic_oracle: only the test suite imports it.

Scope: kT = 0 and no particles, i.e. the three SSP-RK3 stages of App. A with
the conservative staggered flux of ic_oracle.fluid_increment and the imposed
pressure p_ext = sum_m A_m prof_m sin(omega_m t + phase_m) (Sec. VI).  For a
loss L of the state after N steps, step_vjp maps dL/dU^{n+1} to dL/dU^n and
accumulates dL/dA_m.  Each function is the transpose of the corresponding
forward map, written term by term from ic_oracle.fluid_increment: a shift
x -> x[i + s] transposes to y -> y[i - s].
"""
from __future__ import annotations

import math

import numpy as np

from . import ic_oracle as O


def _at(a, alpha, s):
    return O._at(a, alpha, s)


def fluid_increment_vjp(drho, g, prm, lr, lg):
    """(dDelta/d(drho, g))^T (lr, lg) for Delta = fluid_increment(drho, g, prm,
    p_extra, 0, None) (independent of p_extra), and the adjoint of p_extra.

    Returns (mu_drho, [mu_g0, mu_g1, mu_g2], mu_p)."""
    h, dt, rho0, cf = prm["h"], prm["dt"], prm["rho0"], prm["cf"]
    eta, zeta = prm["eta"], prm["zeta"]
    lam = zeta - 2.0 * eta / 3.0
    k = dt / h
    rf = [rho0 + 0.5 * (drho + _at(drho, a, 1)) for a in range(3)]
    v = [g[a] / rf[a] for a in range(3)]
    mu_g = [np.zeros_like(drho) for _ in range(3)]
    mu_v = [np.zeros_like(drho) for _ in range(3)]
    mu_r = np.zeros_like(drho)

    # mass: d_drho = -k sum_a (g_a - g_a[i-a])
    for a in range(3):
        mu_g[a] += -k * (lr - _at(lr, a, 1))

    # momentum: d_g_a = -k (C_a[i+a] - C_a + sum_b (E_ab - E_ab[i-b]))
    muC = [-k * (_at(lg[a], a, -1) - lg[a]) for a in range(3)]
    mu_p = muC[0] + muC[1] + muC[2]
    mu_r += cf * cf * mu_p
    mu_div = -lam * mu_p
    for a in range(3):
        A = 0.25 * (g[a] + _at(g[a], a, -1))
        B = v[a] + _at(v[a], a, -1)
        t = 0.25 * B * muC[a]
        mu_g[a] += t + _at(t, a, 1)
        t = A * muC[a]
        mu_v[a] += t + _at(t, a, 1)
        mu_v[a] += -2.0 * eta / h * (muC[a] - _at(muC[a], a, 1))
        mu_v[a] += (mu_div - _at(mu_div, a, 1)) / h
    for a in range(3):
        for b in range(3):
            if b == a:
                continue
            muE = -k * (lg[a] - _at(lg[a], b, 1))
            P = g[a] + _at(g[a], b, 1)
            Q = v[b] + _at(v[b], a, 1)
            t = 0.25 * Q * muE
            mu_g[a] += t + _at(t, b, -1)
            t = 0.25 * P * muE
            mu_v[b] += t + _at(t, a, -1)
            mu_v[a] += -eta / h * (_at(muE, b, -1) - muE)
            mu_v[b] += -eta / h * (_at(muE, a, -1) - muE)

    # v_a = g_a / rf_a, rf_a = rho0 + (drho + drho[i+a]) / 2
    for a in range(3):
        mu_g[a] += mu_v[a] / rf[a]
        mu_rf = -mu_v[a] * v[a] / rf[a]
        mu_r += 0.5 * mu_rf + 0.5 * _at(mu_rf, a, -1)
    return mu_r, mu_g, mu_p


def drive_profiles(modes, shape, h):
    """prof_m at cell centres, one (nz, ny, nx) array per mode (amplitude 1,
    time factor 1)."""
    out = []
    for md in modes or []:
        one = dict(md)
        one["amp"] = 1.0
        one["omega"] = 0.0
        one["phase"] = math.pi / 2
        out.append(O.external_pressure([one], 0.0, shape, h))
    return out


def step_forward(drho, g, prm, modes, n):
    """One deterministic particle-free step; returns the stage inputs and the
    result (the oracle's RK3 combination)."""
    shape = drho.shape
    dt = prm["dt"]
    tn = n * dt
    ts = [tn, tn + dt, tn + 0.5 * dt]
    zero = [np.zeros(shape)] * 3

    def dU(r, gg, s):
        p = O.external_pressure(modes, ts[s], shape, prm["h"])
        return O.fluid_increment(r, gg, prm, p, zero, None)

    r0, g0 = drho, list(g)
    dr, dg = dU(r0, g0, 0)
    r1, g1 = r0 + dr, [g0[a] + dg[a] for a in range(3)]
    dr, dg = dU(r1, g1, 1)
    r2 = 0.75 * r0 + 0.25 * (r1 + dr)
    g2 = [0.75 * g0[a] + 0.25 * (g1[a] + dg[a]) for a in range(3)]
    dr, dg = dU(r2, g2, 2)
    r3 = (1.0 / 3.0) * r0 + (2.0 / 3.0) * (r2 + dr)
    g3 = [(1.0 / 3.0) * g0[a] + (2.0 / 3.0) * (g2[a] + dg[a]) for a in range(3)]
    return [(r0, g0), (r1, g1), (r2, g2)], (r3, g3), ts


def step_vjp(drho, g, prm, modes, n, lr, lg, profiles=None):
    """Reverse of step n (from U^n = (drho, g)): returns dL/dU^n given
    (lr, lg) = dL/dU^{n+1}, and dL/dA_m for the drive amplitudes."""
    stages, _, ts = step_forward(drho, g, prm, modes, n)
    if profiles is None:
        profiles = drive_profiles(modes, drho.shape, prm["h"])
    dA = np.zeros(len(modes or []))

    def apply(stage, lr_, lg_, w, s):
        r, gg = stages[stage]
        mr, mg, mp = fluid_increment_vjp(r, gg, prm, lr_, lg_)
        for m, md in enumerate(modes or []):
            dA[m] += w * math.sin(md["omega"] * ts[s] + md.get("phase", 0.0)) * \
                float(np.sum(mp * profiles[m]))
        return lr_ + mr, [lg_[a] + mg[a] for a in range(3)]

    # U3 = U0/3 + 2/3 (U2 + D(U2))
    r2, g2 = apply(2, lr, lg, 2.0 / 3.0, 2)
    r2, g2 = 2.0 / 3.0 * r2, [2.0 / 3.0 * x for x in g2]
    r0 = lr / 3.0
    g0 = [x / 3.0 for x in lg]
    # U2 = 3/4 U0 + 1/4 (U1 + D(U1))
    r1, g1 = apply(1, r2, g2, 0.25, 1)
    r1, g1 = 0.25 * r1, [0.25 * x for x in g1]
    r0 = r0 + 0.75 * r2
    g0 = [g0[a] + 0.75 * g2[a] for a in range(3)]
    # U1 = U0 + D(U0)
    rr, gg = apply(0, r1, g1, 1.0, 0)
    return r0 + rr, [g0[a] + gg[a] for a in range(3)], dA


def run_grad(drho, g, prm, modes, nsteps, cr, cg, n0=0):
    """Gradient of L = <cr, drho^N> + sum_a <cg_a, g_a^N> after nsteps steps
    from step n0, with respect to the initial state and the drive amplitudes
    (every intermediate state kept)."""
    states = [(drho, list(g))]
    for s in range(nsteps):
        _, (r, gg), _ = step_forward(states[-1][0], states[-1][1], prm, modes, n0 + s)
        states.append((r, gg))
    profiles = drive_profiles(modes, drho.shape, prm["h"])
    lr, lg = cr.copy(), [x.copy() for x in cg]
    dA = np.zeros(len(modes or []))
    for s in reversed(range(nsteps)):
        r, gg = states[s]
        lr, lg, d = step_vjp(r, gg, prm, modes, n0 + s, lr, lg, profiles)
        dA += d
    return lr, lg, dA, states[-1]
