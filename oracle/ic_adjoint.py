"""Plain FP64 adjoint (reverse mode) of the deterministic fluid part of the IC
step, for checking the HIP adjoint.

TEST INFRASTRUCTURE ONLY, like ic_oracle: only the test suite imports it.

Scope: kT = 0.  Fluid only (step_vjp, run_grad): the three SSP-RK3 stages of
App. A with the conservative staggered flux of ic_oracle.fluid_increment and
the imposed pressure p_ext = sum_m A_m prof_m sin(omega_m t + phase_m) (Sec.
VI).  For a loss L of the state after N steps, step_vjp maps dL/dU^{n+1} to
dL/dU^n and accumulates dL/dA_m.  Each function is the transpose of the
corresponding forward map, written term by term from
ic_oracle.fluid_increment: a shift x -> x[i + s] transposes to y -> y[i - s].

With particles (step_vjp_particles, run_grad_particles): the whole IC step of
ic_oracle.ic_step (App. A, substeps 1-7) reversed, substep 7 first and the RK
stages from the third to the first, including the dependence of the kernel
weights on the particle positions through phi' (phi is C^1, App. A), and the
gradients with respect to the excess masses m_e, the energies eps_pf, the
tether constants k_s and the drive amplitudes.  The forward pass is re-run
here with the oracle's own functions, keeping the intermediates.
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


# ---------------------------------------------------------------------------
# Particle coupling.
# ---------------------------------------------------------------------------

def phi_prime(r):
    """d phi / d r of the 3-point function (App. A), r in units of h:
    -r / sqrt(1 - 3 r^2) for |r| <= 1/2, and
    -sign(r) (1/2 + (1 - |r|) / (2 sqrt(1 - 3 (1 - |r|)^2))) for
    1/2 < |r| <= 3/2; zero beyond."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    out = np.zeros_like(r)
    inner = a <= 0.5
    outer = (a > 0.5) & (a <= 1.5)
    ri = r[inner]
    out[inner] = -ri / np.sqrt(1.0 - 3.0 * ri * ri)
    s = 1.0 - a[outer]
    out[outer] = -np.sign(r[outer]) * (0.5 + s / (2.0 * np.sqrt(1.0 - 3.0 * s * s)))
    return out


def stencil_grad(q, h, shape, face_axis):
    """Indices (K, J, I), weights W = prod_alpha phi and their gradients
    dW[b] = d W / d q_b (each (N, 3, 3, 3)) of the 27 kernel points of each
    particle, for cell-centred (face_axis None) or alpha-face fields."""
    nz, ny, nx = shape
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    per = []
    for ax, n in enumerate((nx, ny, nz)):
        s = 0.5 if face_axis == ax else 0.0
        near = np.floor(q[:, ax] / h - s + 0.5)
        rel = near[:, None] + np.array([-1.0, 0.0, 1.0])
        r = q[:, ax, None] / h - (rel + s)
        per.append((np.mod(rel.astype(np.int64), n), O.phi(r), phi_prime(r) / h))
    (ix, wx, dx), (iy, wy, dy), (iz, wz, dz) = per
    idx = (iz[:, :, None, None], iy[:, None, :, None], ix[:, None, None, :])

    def prod(fz, fy, fx):
        return fz[:, :, None, None] * fy[:, None, :, None] * fx[:, None, None, :]

    W = prod(wz, wy, wx)
    dW = [prod(wz, wy, dx), prod(wz, dy, wx), prod(dz, wy, wx)]
    return idx, W, dW


def _gather(field, idx, W):
    return np.sum(W * field[idx], axis=(1, 2, 3))


def _scatter(out, idx, vals):
    np.add.at(out, tuple(np.broadcast_arrays(*idx)), vals)


def _per(x):
    """(N,) -> (N, 1, 1, 1) for broadcasting against stencil arrays."""
    return np.asarray(x)[:, None, None, None]


def step_forward_particles(state, prm, modes):
    """One deterministic IC step with particles, as ic_oracle.ic_step
    computes it, keeping what the reverse pass needs."""
    h, dt, rho0 = prm["h"], prm["dt"], prm["rho0"]
    drho, g = state["drho"], list(state["g"])
    shape = drho.shape
    nz, ny, nx = shape
    Lbox = np.array([nx * h, ny * h, nz * h])
    V = O.kernel_volume(h)
    n = int(state["n"])
    q = np.asarray(state["q"], dtype=np.float64).reshape(-1, 3)
    u = np.asarray(state["u"], dtype=np.float64).reshape(-1, 3)
    me, eps = np.asarray(state["me"], float), np.asarray(state["eps"], float)
    ks = np.asarray(state["ks"], float)
    qeq = np.asarray(state["qeq"], float).reshape(-1, 3)
    fext = np.asarray(state["fext"], float).reshape(-1, 3)

    # substeps 1-2
    U1 = O._velocity_at(g, drho, q, prm)
    qh = O._wrap(q + 0.5 * dt * U1, Lbox)
    Jv_old = O._velocity_at(g, drho, qh, prm)
    dq = O._min_image(qh - qeq, Lbox)
    F = -ks[:, None] * dq + fext
    force_faces = [O.spread(F[:, a], qh, h, shape, a) for a in range(3)]
    # substep 3
    tn = n * dt
    ts = [tn, tn + dt, tn + 0.5 * dt]

    def dU(d, gg, s):
        p_part, _ = O.pressure(d, qh, eps, prm)
        p_ext = O.external_pressure(modes, ts[s], shape, h)
        return O.fluid_increment(d, gg, prm, p_part + p_ext, force_faces, None)

    r0, g0 = drho, g
    dr, dg = dU(r0, g0, 0)
    r1, g1 = r0 + dr, [g0[a] + dg[a] for a in range(3)]
    dr, dg = dU(r1, g1, 1)
    r2 = 0.75 * r0 + 0.25 * (r1 + dr)
    g2 = [0.75 * g0[a] + 0.25 * (g1[a] + dg[a]) for a in range(3)]
    dr, dg = dU(r2, g2, 2)
    r3 = (1.0 / 3.0) * r0 + (2.0 / 3.0) * (r2 + dr)
    g3 = [(1.0 / 3.0) * g0[a] + (2.0 / 3.0) * (g2[a] + dg[a]) for a in range(3)]
    # substeps 4-6
    rf3 = [rho0 + 0.5 * (r3 + O._at(r3, a, 1)) for a in range(3)]
    Vt = np.zeros_like(q)
    mf = np.zeros_like(q)
    for a in range(3):
        Vt[:, a] = O.interpolate(g3[a] / rf3[a], qh, h, a)
        mf[:, a] = V * O.interpolate(rf3[a], qh, h, a)
    u_new = u + (mf / (me[:, None] + mf)) * (Vt - u)
    g_new = [g3[a] + rf3[a] * (V * O.spread(u_new[:, a] - Vt[:, a], qh, h, shape, a))
             for a in range(3)]
    # substep 7
    Jv_new = O._velocity_at(g_new, r3, qh, prm)
    q_new = O._wrap(q + 0.5 * dt * (Jv_new + Jv_old), Lbox)
    return dict(q=q, u=u, me=me, eps=eps, ks=ks, qh=qh, dq=dq, F=F, ts=ts,
                stages=[(r0, g0), (r1, g1), (r2, g2)], r3=r3, g3=g3, rf3=rf3, Vt=Vt, mf=mf,
                u_new=u_new, g_new=g_new, q_new=q_new)


def step_vjp_particles(state, prm, modes, lr, lg, lq, lu, lF=None, profiles=None):
    """Reverse of one IC step with particles (kT = 0).

    (lr, lg, lq, lu) = dL/d(drho, g, q, u) after the step; lF = dL/dF^{n+1/2}
    of this step's tether-plus-external force (a loss on the force itself,
    e.g. the radiation-force estimator), or None.  Returns a dict with
    lr, lg, lq, lu = dL/d(state before the step) and the parameter gradients
    dme, deps, dks (per particle) and dA (per drive mode) of this step."""
    h, dt, rho0 = prm["h"], prm["dt"], prm["rho0"]
    k = dt / h
    V = O.kernel_volume(h)
    fw = step_forward_particles(state, prm, modes)
    drho, g = state["drho"], list(state["g"])
    shape = drho.shape
    q, u, me, eps, ks = fw["q"], fw["u"], fw["me"], fw["eps"], fw["ks"]
    qh, F = fw["qh"], fw["F"]
    r3, g3, rf3, g_new = fw["r3"], fw["g3"], fw["rf3"], fw["g_new"]
    Vt, mf, u_new = fw["Vt"], fw["mf"], fw["u_new"]
    N = len(q)
    h3 = h ** 3
    lqh = np.zeros((N, 3))
    lFt = np.zeros((N, 3)) if lF is None else np.array(lF, dtype=np.float64).reshape(-1, 3)
    lq_out = np.array(lq, dtype=np.float64).reshape(-1, 3).copy()
    lu = np.array(lu, dtype=np.float64).reshape(-1, 3)
    lr3 = np.array(lr, dtype=np.float64).copy()
    lgn = [np.array(lg[a], dtype=np.float64).copy() for a in range(3)]
    lrf3 = [np.zeros(shape) for _ in range(3)]
    st_qh = [stencil_grad(qh, h, shape, a) for a in range(3)]

    # substep 7: q^{n+1} = q^n + dt/2 (J v^{n+1} + J v^n), both at q^{n+1/2}
    lJ = 0.5 * dt * lq_out
    for a in range(3):
        idx, W, dW = st_qh[a]
        rfv, gnv = rf3[a][idx], g_new[a][idx]
        _scatter(lgn[a], idx, _per(lJ[:, a]) * W / rfv)
        _scatter(lrf3[a], idx, -_per(lJ[:, a]) * W * gnv / (rfv * rfv))
        for b in range(3):
            lqh[:, b] += lJ[:, a] * np.sum(dW[b] * gnv / rfv, axis=(1, 2, 3))
    # substep 6: g^{n+1} = g~ + rho_face V S (u^{n+1} - V~)
    du = u_new - Vt
    ldu = np.zeros((N, 3))
    for a in range(3):
        idx, W, dW = st_qh[a]
        lgv, rfv = lgn[a][idx], rf3[a][idx]
        ldu[:, a] = V / h3 * np.sum(W * lgv * rfv, axis=(1, 2, 3))
        _scatter(lrf3[a], idx, lgv * W * _per(V * du[:, a] / h3))
        for b in range(3):
            lqh[:, b] += V * du[:, a] / h3 * np.sum(dW[b] * lgv * rfv, axis=(1, 2, 3))
    lg3 = lgn
    # substeps 4-5: u^{n+1} = u^n + c (V~ - u^n), c = m_f / (m_e + m_f)
    lun = lu + ldu
    lVt = -ldu
    mt = me[:, None] + mf
    c = mf / mt
    lu_out = lun * (1.0 - c)
    lVt = lVt + c * lun
    lc = lun * (Vt - u)
    lmf = lc * me[:, None] / (mt * mt)
    dme = -np.sum(lc * mf / (mt * mt), axis=1)
    for a in range(3):
        idx, W, dW = st_qh[a]
        rfv, g3v = rf3[a][idx], g3[a][idx]
        _scatter(lg3[a], idx, _per(lVt[:, a]) * W / rfv)
        _scatter(lrf3[a], idx, -_per(lVt[:, a]) * W * g3v / (rfv * rfv) + _per(V * lmf[:, a]) * W)
        for b in range(3):
            lqh[:, b] += lVt[:, a] * np.sum(dW[b] * g3v / rfv, axis=(1, 2, 3))
            lqh[:, b] += V * lmf[:, a] * np.sum(dW[b] * rfv, axis=(1, 2, 3))
    for a in range(3):
        lr3 += 0.5 * lrf3[a] + 0.5 * O._at(lrf3[a], a, -1)

    # substep 3, the RK stages backwards; each stage increment also carries
    # the particle pressure S(eps V J drho_s) and the spread force dt S F
    if profiles is None:
        profiles = drive_profiles(modes, shape, h)
    dA = np.zeros(len(modes or []))
    deps = np.zeros(N)
    cidx, cW, cdW = stencil_grad(qh, h, shape, None)
    ts = fw["ts"]

    def apply(stage, lr_, lg_, w, s):
        r, gg = fw["stages"][stage]
        mr, mg, mp = fluid_increment_vjp(r, gg, prm, lr_, lg_)
        for m, md in enumerate(modes or []):
            dA[m] += w * math.sin(md["omega"] * ts[s] + md.get("phase", 0.0)) * \
                float(np.sum(mp * profiles[m]))
        # particle pressure: p_i += sum_p W_p(i)/h^3 eps_p V sum_j W_p(j) r_j
        mpv, rv = mp[cidx], r[cidx]
        P = np.sum(cW * mpv, axis=(1, 2, 3)) / h3
        Jr = np.sum(cW * rv, axis=(1, 2, 3))
        _scatter(mr, cidx, cW * _per(eps * V * P))
        deps[:] += w * V * Jr * P
        for b in range(3):
            lqh[:, b] += w * eps * V * (Jr * np.sum(cdW[b] * mpv, axis=(1, 2, 3)) / h3 +
                                        P * np.sum(cdW[b] * rv, axis=(1, 2, 3)))
        # spread force: d g_a += dt W_a F_a / h^3
        for a in range(3):
            idx, W, dW = st_qh[a]
            lgv = lg_[a][idx]
            lFt[:, a] += w * dt / h3 * np.sum(W * lgv, axis=(1, 2, 3))
            for b in range(3):
                lqh[:, b] += w * dt / h3 * F[:, a] * np.sum(dW[b] * lgv, axis=(1, 2, 3))
        return lr_ + mr, [lg_[a] + mg[a] for a in range(3)]

    r2, g2 = apply(2, lr3, lg3, 2.0 / 3.0, 2)
    r2, g2 = 2.0 / 3.0 * r2, [2.0 / 3.0 * x for x in g2]
    r0, g0 = lr3 / 3.0, [x / 3.0 for x in lg3]
    r1, g1 = apply(1, r2, g2, 0.25, 1)
    r1, g1 = 0.25 * r1, [0.25 * x for x in g1]
    r0, g0 = r0 + 0.75 * r2, [g0[a] + 0.75 * g2[a] for a in range(3)]
    rr, gg = apply(0, r1, g1, 1.0, 0)
    lr0, lg0 = r0 + rr, [g0[a] + gg[a] for a in range(3)]

    # substep 2: F = -k_s minimg(q^{n+1/2} - q_eq) + f_ext
    lqh += -ks[:, None] * lFt
    dks = -np.sum(lFt * fw["dq"], axis=1)
    # J^{n+1/2} v^n and substep 1 (J^n v^n at q^n) read the state before the step
    rf0 = [rho0 + 0.5 * (drho + O._at(drho, a, 1)) for a in range(3)]
    lrf0 = [np.zeros(shape) for _ in range(3)]

    def velocity_vjp(x, lv):
        """Transpose of x -> J_a(g_a / rho_face_a) at x for all a; returns
        the position gradient."""
        out = np.zeros((N, 3))
        for a in range(3):
            idx, W, dW = stencil_grad(x, h, shape, a)
            rfv, gv = rf0[a][idx], g[a][idx]
            _scatter(lg0[a], idx, _per(lv[:, a]) * W / rfv)
            _scatter(lrf0[a], idx, -_per(lv[:, a]) * W * gv / (rfv * rfv))
            for b in range(3):
                out[:, b] += lv[:, a] * np.sum(dW[b] * gv / rfv, axis=(1, 2, 3))
        return out

    lqh += velocity_vjp(qh, lJ)
    lq_out += lqh
    lq_out += velocity_vjp(q, 0.5 * dt * lqh)
    for a in range(3):
        lr0 += 0.5 * lrf0[a] + 0.5 * O._at(lrf0[a], a, -1)
    return dict(lr=lr0, lg=lg0, lq=lq_out, lu=lu_out, dme=dme, deps=deps, dks=dks, dA=dA)


def run_grad_particles(state, prm, modes, nsteps, cr=None, cg=None, cq=None, cu=None, cF=None):
    """Gradient of L = <cr, drho^N> + sum_a <cg_a, g_a^N> + <cq, q^N> +
    <cu, u^N> + sum_n <cF, F^{n+1/2}> over nsteps steps (every intermediate
    state kept; None = zero).  cF weighting every step's force equally makes
    L the sum behind the averaged tether force.  Returns the reversed seeds
    (dict as step_vjp_particles, accumulated over the steps) and the final
    state."""
    states = [dict(state)]
    for _ in range(nsteps):
        nxt, _ = O.ic_step(states[-1], prm, modes)
        states.append(nxt)
    shape = state["drho"].shape
    N = len(np.asarray(state["q"]).reshape(-1, 3))
    z3 = np.zeros((N, 3))
    out = dict(lr=np.zeros(shape) if cr is None else np.array(cr, float),
               lg=[np.zeros(shape) for _ in range(3)] if cg is None else [np.array(x, float) for x in cg],
               lq=z3.copy() if cq is None else np.array(cq, float).reshape(-1, 3),
               lu=z3.copy() if cu is None else np.array(cu, float).reshape(-1, 3),
               dme=np.zeros(N), deps=np.zeros(N), dks=np.zeros(N), dA=np.zeros(len(modes or [])))
    profiles = drive_profiles(modes, shape, prm["h"])
    for s in reversed(range(nsteps)):
        r = step_vjp_particles(states[s], prm, modes, out["lr"], out["lg"], out["lq"], out["lu"],
                               cF, profiles)
        for key in ("lr", "lg", "lq", "lu"):
            out[key] = r[key]
        for key in ("dme", "deps", "dks", "dA"):
            out[key] = out[key] + r[key]
    return out, states[-1]
