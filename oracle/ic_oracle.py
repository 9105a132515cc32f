"""Plain FP64 CPU oracle of one inertial-coupling (IC) time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this module: only the test suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP kernels.

What it computes follows Balboa Usabiaga & Delgado-Buscalioni, "A minimal
model for acoustic forces on Brownian particles" (arXiv:1307.0702):

* the 3-point Roma-Peskin function phi and the tensor-product kernel
  theta_h (App. A, "Spatial discretization");
* the discrete averaging J and spreading S operators on a staggered grid
  (Sec. II, Eqs. Jdis/Sdis; App. A, "Spatial discretization");
* the particle pressure pi = p(rho) + S Omega with
  Omega = eps_pf V (J rho - rho0) (Sec. III, Eqs. pressure/omega);
* the fluctuating isothermal Navier-Stokes flux with the Landau-Lifshitz
  stochastic stress (Sec. IV B, Eqs. consvDens/consvMom/totp and the
  stochastic-stress equation);
* the seven substeps of the IC time step and the three-stage SSP-RK3 fluid
  update with the weak-third-order noise combinations and stage pressures
  (App. A, "Temporal discretization").

Everything is FP64 and written array-wide with numpy.  Grid arrays have shape
(nz, ny, nx), so index [k, j, i] is the cell at r = (i h, j h, k h); the flat
cell index is c = (k ny + j) nx + i.  A vector component alpha lives on the
alpha-faces: g[alpha][k, j, i] sits at r_i + (h/2) e_alpha.

Readings of points the paper leaves open (the spatial discretisation of the
fluid solver is deferred by the paper to another reference) are marked
"Reading:" in the code; each one is listed with its reason in the design
notes of the repository.

Parity unpinned: how the no-slip corrections of particles whose kernels
overlap superpose (the Jacobi reading in ic_step) has no closed form or
printed value to check it against beyond what stays exact with overlap (total
momentum conservation and the fluid-force identity of lambda, both pinned);
every other part of the step is pinned by the tests of the oracle.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "phi", "kernel_points", "interpolate", "spread", "philox4x32_10",
    "uniform23", "box_muller", "cell_normals", "stochastic_stress",
    "pressure", "fluid_increment", "ic_step", "run", "conserved",
    "eps_from_kappa_ratio", "kernel_volume",
]

# Paper axis alpha (0=x, 1=y, 2=z) -> numpy axis of an (nz, ny, nx) array.
_NP_AXIS = (2, 1, 0)


def _at(a, alpha, s):
    """Value of a periodic grid array at index i + s e_alpha."""
    return np.roll(a, -s, axis=_NP_AXIS[alpha])


# ---------------------------------------------------------------------------
# Kernel: App. A, "Spatial discretization" (3-point function of Roma and
# Peskin), Sec. II (linear consistency and kernel volume conditions).
# ---------------------------------------------------------------------------

def phi(r):
    """The 3-point interpolating function phi(r), r in units of h."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    inner = r <= 0.5
    outer = (r > 0.5) & (r <= 1.5)
    ri = r[inner]
    out[inner] = (1.0 + np.sqrt(1.0 - 3.0 * ri * ri)) / 3.0
    ro = r[outer]
    out[outer] = (5.0 - 3.0 * ro - np.sqrt(1.0 - 3.0 * (1.0 - ro) ** 2)) / 6.0
    return out


def kernel_volume(h):
    """Kernel volume V = 8 h^3 of the tensor-product 3-point kernel (Sec. II,
    "Kernel volume")."""
    return 8.0 * h ** 3


def kernel_points(q, h, n, face):
    """Grid points along one axis that phi reaches from coordinate(s) q.

    Cell centres sit at x_i = i h and faces at x_i = (i + 1/2) h (App. A,
    "Spatial discretization").  Reading: the three points are the nearest
    point and its two neighbours; phi vanishes at |r| = 3/2, so a tie at
    that distance cannot change a result.

    Returns (idx, w): idx are the periodic indices (int64, shape (..., 3)),
    w = phi((q - x_idx)/h) (shape (..., 3)).
    """
    q = np.asarray(q, dtype=np.float64)
    s = 0.5 if face else 0.0
    near = np.floor(q / h - s + 0.5)
    rel = near[..., None] + np.array([-1.0, 0.0, 1.0])
    w = phi(q[..., None] / h - (rel + s))
    idx = np.mod(rel.astype(np.int64), n)
    return idx, w


def _stencil(q, h, shape, face_axis):
    """Indices and tensor-product weights of the 27 kernel points of each
    particle.  face_axis = None for cell-centred fields, alpha for fields on
    alpha-faces.  Weights are h^3 theta_h = prod_alpha phi."""
    nz, ny, nx = shape
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    ix, wx = kernel_points(q[:, 0], h, nx, face_axis == 0)
    iy, wy = kernel_points(q[:, 1], h, ny, face_axis == 1)
    iz, wz = kernel_points(q[:, 2], h, nz, face_axis == 2)
    K = iz[:, :, None, None]
    J = iy[:, None, :, None]
    I = ix[:, None, None, :]
    W = wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]
    return (K, J, I), W


def interpolate(field, q, h, face_axis=None):
    """Averaging operator J: J f = sum_i h^3 theta_h(q - r_i) f(r_i)
    (Sec. II, Eq. Jdis), with the staggered positions of App. A."""
    if len(q) == 0:
        return np.zeros(0)
    idx, W = _stencil(q, h, field.shape, face_axis)
    return np.sum(W * field[idx], axis=(1, 2, 3))


def spread(values, q, h, shape, face_axis=None, out=None):
    """Spreading operator S: adds theta_h(q - r_i) F to every grid point
    (Sec. II, Eq. Sdis), i.e. w F / h^3 with w = prod phi."""
    if out is None:
        out = np.zeros(shape)
    if len(q) == 0:
        return out
    idx, W = _stencil(q, h, shape, face_axis)
    vals = W * (np.asarray(values, dtype=np.float64)[:, None, None, None] / h ** 3)
    np.add.at(out, tuple(np.broadcast_arrays(*idx)), vals)
    return out


def eps_from_kappa_ratio(cf, kappa_ratio):
    """eps_pf from kappa_p/kappa_f: c_p^2 = c_f^2 + eps_pf and kappa = 1/(rho0
    c^2) (Sec. III, Eqs. part_svel/ke) give eps_pf = c_f^2 (kappa_f/kappa_p - 1)."""
    return cf * cf * (1.0 / np.asarray(kappa_ratio, dtype=np.float64) - 1.0)


# ---------------------------------------------------------------------------
# Random numbers.  The paper does not name its generator.  Reading: the
# counter-based Philox-4x32-10 generator (Salmon, Moraes, Dror and Shaw,
# SC'11) keyed by the seed, with counter (cell, step, call, replica), then
# the Box-Muller transform.  Implemented here from its published definition.
# ---------------------------------------------------------------------------

_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox-4x32 with 10 rounds.  Each round multiplies counter words 0 and 2
    by the two multipliers, keeps the 64-bit products' halves and mixes in the
    key; the key is bumped by the Weyl constants between rounds."""
    c = [np.asarray(x).astype(np.uint64) & _MASK32 for x in (c0, c1, c2, c3)]
    c = np.broadcast_arrays(*c)
    c = [x.copy() for x in c]
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _PHILOX_M0 * c[0]
        p1 = _PHILOX_M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
        k0 = (k0 + _PHILOX_W0) & 0xFFFFFFFF
        k1 = (k1 + _PHILOX_W1) & 0xFFFFFFFF
    return [x.astype(np.uint32) for x in c]


def uniform23(x):
    """Uniform in (0, 1) from the top 23 bits of a 32-bit word:
    ((x >> 9) + 1/2) 2^-23.  It needs 24 significant bits, so it is exact in
    both FP32 and FP64, and it is never 0 or 1."""
    x = np.asarray(x).astype(np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def box_muller(u1, u2):
    """Box-Muller: two independent standard normals from two uniforms."""
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def cell_normals(seed, step, replica, ncell):
    """The 12 standard normals of every cell for one time step: W_A then W_B,
    six components each in the order xx, yy, zz, xy, xz, yz.

    Philox calls j = 0, 1, 2 use counter (c, step mod 2^32, j, replica) and key
    (seed low 32 bits, seed high 32 bits); word m = 4 j + l of the 12 output
    words gives uniform u_m, and normals (z_2p, z_2p+1) come from Box-Muller
    of (u_2p, u_2p+1).  Reading of the layout: z_0..z_5 are W_A (xx, yy, zz,
    xy, xz, yz); z_8, z_9, z_10, z_11, z_6, z_7 are W_B (xx, yy, zz, xy, xz,
    yz), so the last RK stage, which needs W_A only, needs calls 0 and 1.
    Returns (W_A, W_B), each shaped (6, ncell).
    """
    cid = np.arange(ncell, dtype=np.uint64)
    k0, k1 = int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF
    words = []
    for j in range(3):
        words += philox4x32_10(cid, int(step) & 0xFFFFFFFF, j, int(replica), k0, k1)
    u = [uniform23(w) for w in words]
    z = []
    for p in range(6):
        a, b = box_muller(u[2 * p], u[2 * p + 1])
        z += [a, b]
    z = np.array(z)
    return z[:6], z[[8, 9, 10, 11, 6, 7]]


def stochastic_stress(Z, prm):
    """Discrete Landau-Lifshitz stochastic stress (Sec. IV B, stochastic
    stress equation) from six standard normals per cell (xx, yy, zz, xy, xz,
    yz), each shaped like the grid.

    Reading: the symmetrised tensor is (W + W^T)/sqrt(2) (diagonal sqrt(2)
    Z_aa, off-diagonal Z_ab), which gives the Landau-Lifshitz covariance
    2 kT [eta (d_ik d_jl + d_il d_jk) + (zeta - 2 eta/3) d_ij d_kl]; the
    space-time delta becomes 1/(h^3 dt) per cell and step.  Diagonal entries
    sit at cell centres, the off-diagonal ones at the cell's edges.

    Returns (diag[3], off) with off keyed by (alpha, beta), alpha < beta.
    """
    h, dt, kT, eta, zeta = prm["h"], prm["dt"], prm["kT"], prm["eta"], prm["zeta"]
    amp = 1.0 / math.sqrt(h ** 3 * dt)
    a = math.sqrt(2.0 * eta * kT)
    b = math.sqrt(zeta * kT / 3.0) - a / 3.0
    trace = math.sqrt(2.0) * (Z[0] + Z[1] + Z[2])
    diag = [amp * (a * math.sqrt(2.0) * Z[al] + b * trace) for al in range(3)]
    off = {(0, 1): amp * a * Z[3], (0, 2): amp * a * Z[4], (1, 2): amp * a * Z[5]}
    return diag, off


# ---------------------------------------------------------------------------
# Pressure and forcing.
# ---------------------------------------------------------------------------

def external_pressure(modes, t, shape, h):
    """Imposed pressure p_ext at cell centres at time t.

    'plane': amp sin(omega t + phase) on the single plane of cells whose
    index along `axis` is the nearest to x0 (Sec. VI, Eq. pext, with the
    Kronecker-delta reading given there).
    'cos': amp cos(2 pi m (x - x0)/L) sin(omega t + phase), a single standing
    mode (reading: a modal drive that excites only the resonant mode)."""
    nz, ny, nx = shape
    out = np.zeros(shape)
    n_of = (nx, ny, nz)
    for md in modes or []:
        ax = md["axis"]
        n = n_of[ax]
        x = np.arange(n) * h
        if md["shape"] == "plane":
            prof = np.zeros(n)
            prof[int(math.floor(md["x0"] / h + 0.5)) % n] = 1.0
        else:
            L = n * h
            prof = np.cos(2.0 * math.pi * md["m"] * (x - md["x0"]) / L)
        amp = md["amp"] * math.sin(md["omega"] * t + md.get("phase", 0.0))
        bshape = [1, 1, 1]
        bshape[_NP_AXIS[ax]] = n
        out = out + amp * prof.reshape(bshape)
    return out


def pressure(drho, q, eps, prm):
    """Particle part of the pressure functional: sum_p S_p Omega_p with
    Omega_p = eps_p V (J_p rho - rho0) (Sec. III, Eqs. pressure/omega; the
    stage pressures of App. A).  Reading: J_p rho - rho0 is evaluated as
    J_p(rho - rho0), equal by the partition of unity."""
    h = prm["h"]
    if len(q) == 0:
        return np.zeros(drho.shape), np.zeros(0)
    omega = np.asarray(eps) * kernel_volume(h) * interpolate(drho, q, h)
    return spread(omega, q, h, drho.shape), omega


# ---------------------------------------------------------------------------
# Fluid flux and the stage increment Delta U = -dt div F (App. A, "Temporal
# discretization"; Sec. IV B, Eqs. consvDens/consvMom/totp).
#
# Reading (the paper defers the fluid discretisation to another reference):
# a conservative centred staggered-grid form.
#   * rho_face = rho0 + (drho_i + drho_{i+alpha})/2, v = g / rho_face.
#   * Mass: d(drho)_i = -dt/h sum_a (g^a_i - g^a_{i-a}).
#   * Momentum on alpha-face i: flux Pi^{ab} = pi d_ab + g^a v^b - sigma - Sigma;
#     diagonal fluxes at cell centres, off-diagonal ones at edges.
#   * Centre flux of cell i: pi_i + (avg of g^a over the 2 alpha-faces)
#     (avg of v^a over the same) - sigma^aa_i - Sigma^aa_i, with
#     sigma^aa = 2 eta d_a v^a + (zeta - 2 eta/3) div v.
#   * Edge (a, b) of cell i at r_i + (h/2)(e_a + e_b): flux of a-momentum along
#     b = (avg of g^a over the two a-faces along b) (avg of v^b over the two
#     b-faces along a) - eta (d_b v^a + d_a v^b) - Sigma^ab.
#   The viscous part is then eta lap v + (zeta + eta/3) grad div v, as in the
#   viscous-stress equation of Sec. IV B.
# ---------------------------------------------------------------------------

def fluid_increment(drho, g, prm, p_extra, force_faces, Z):
    """Delta U(U) = -dt div F(U) for one RK stage.

    drho     : (nz,ny,nx) density deviation rho - rho0
    g        : list of 3 face arrays (momentum density components)
    p_extra  : particle pressure plus imposed pressure at cell centres
    force_faces : list of 3 face arrays, the spread external force S F
    Z        : 6 normals per cell (combination for this stage) or None
    """
    h, dt, rho0, cf = prm["h"], prm["dt"], prm["rho0"], prm["cf"]
    eta, zeta = prm["eta"], prm["zeta"]
    rho_face = [rho0 + 0.5 * (drho + _at(drho, a, 1)) for a in range(3)]
    v = [g[a] / rho_face[a] for a in range(3)]

    # Mass: conservation of mass, flux g.
    d_drho = -(dt / h) * sum(g[a] - _at(g[a], a, -1) for a in range(3))

    if Z is not None:
        diag_s, off_s = stochastic_stress(Z, prm)
    else:
        diag_s, off_s = [0.0, 0.0, 0.0], {(0, 1): 0.0, (0, 2): 0.0, (1, 2): 0.0}

    pi = cf * cf * drho + p_extra
    div_v = sum(v[b] - _at(v[b], b, -1) for b in range(3)) / h

    centre = []
    for a in range(3):
        g_avg = 0.5 * (g[a] + _at(g[a], a, -1))
        v_avg = 0.5 * (v[a] + _at(v[a], a, -1))
        sig = 2.0 * eta * (v[a] - _at(v[a], a, -1)) / h + (zeta - 2.0 * eta / 3.0) * div_v
        centre.append(pi + g_avg * v_avg - sig - diag_s[a])

    def edge_flux(a, b):
        """Flux of a-momentum across the b-direction, on edge (a, b) of cell i."""
        g_a = 0.5 * (g[a] + _at(g[a], b, 1))
        v_b = 0.5 * (v[b] + _at(v[b], a, 1))
        sig = eta * ((_at(v[a], b, 1) - v[a]) / h + (_at(v[b], a, 1) - v[b]) / h)
        return g_a * v_b - sig - off_s[(min(a, b), max(a, b))]

    d_g = []
    for a in range(3):
        div_flux = _at(centre[a], a, 1) - centre[a]
        for b in range(3):
            if b != a:
                e = edge_flux(a, b)
                div_flux = div_flux + (e - _at(e, b, -1))
        d_g.append(-(dt / h) * div_flux + dt * force_faces[a])
    return d_drho, d_g


# ---------------------------------------------------------------------------
# The IC time step (App. A, "Temporal discretization", substeps 1-7).
# ---------------------------------------------------------------------------

def _wrap(q, L):
    return np.mod(q, L)


def _min_image(d, L):
    return d - L * np.floor(d / L + 0.5)


def _velocity_at(g, drho, q, prm):
    """J_alpha (g^alpha / rho_face^alpha) for every particle, shape (N, 3)."""
    h, rho0 = prm["h"], prm["rho0"]
    out = np.zeros((len(q), 3))
    for a in range(3):
        rho_face = rho0 + 0.5 * (drho + _at(drho, a, 1))
        out[:, a] = interpolate(g[a] / rho_face, q, h, a)
    return out


def ic_step(state, prm, modes=None):
    """Advance (drho, g, q, u) from t^n = n dt to t^{n+1}.

    state: dict with drho, g (list of 3), n (step counter), and particle
    arrays q (N,3), u (N,3), me (N,), eps (N,), ks (N,), qeq (N,3),
    fext (N,3).  Returns (new_state, diag) where diag holds per-particle
    q_half, F (= F^{n+1/2}), lam (= lambda averaged over the step).
    """
    h, dt, rho0 = prm["h"], prm["dt"], prm["rho0"]
    drho = state["drho"]
    g = state["g"]
    nz, ny, nx = drho.shape
    shape = drho.shape
    Lbox = np.array([nx * h, ny * h, nz * h])
    V = kernel_volume(h)
    n = int(state["n"])
    t_n = n * dt

    q = np.asarray(state["q"], dtype=np.float64).reshape(-1, 3)
    u = np.asarray(state["u"], dtype=np.float64).reshape(-1, 3)
    npart = len(q)
    me = np.asarray(state["me"], dtype=np.float64)
    eps = np.asarray(state["eps"], dtype=np.float64)
    ks = np.asarray(state["ks"], dtype=np.float64)
    qeq = np.asarray(state["qeq"], dtype=np.float64).reshape(-1, 3)
    fext = np.asarray(state["fext"], dtype=np.float64).reshape(-1, 3)

    # Substep 1: q^{n+1/2} = q^n + dt/2 J^n v^n.
    q_half = _wrap(q + 0.5 * dt * _velocity_at(g, drho, q, prm), Lbox)
    # v^n averaged at q^{n+1/2}, needed by substep 7 (reading: taken before
    # the fluid moves, so no copy of v^n is kept).
    Jv_old = _velocity_at(g, drho, q_half, prm)

    # Substep 2: F^{n+1/2} = F(q^{n+1/2}, t^{n+1/2}); tethers
    # U = (1/2) k_s |q - q_eq|^2 (Sec. VI) with the minimum image, plus a
    # constant force.
    F = -ks[:, None] * _min_image(q_half - qeq, Lbox) + fext
    force_faces = [spread(F[:, a], q_half, h, shape, a) for a in range(3)]

    # Substep 3: three SSP-RK3 stages with q^{n+1/2} and F^{n+1/2} fixed.
    if prm["kT"] > 0.0:
        WA, WB = cell_normals(prm["seed"], n, prm.get("replica", 0), nx * ny * nz)
        WA = WA.reshape(6, nz, ny, nx)
        WB = WB.reshape(6, nz, ny, nx)
        s3 = math.sqrt(3.0)
        Zs = [WA - s3 * WB, WA + s3 * WB, WA]
    else:
        Zs = [None, None, None]
    t_stage = [t_n, t_n + dt, t_n + 0.5 * dt]

    def dU(d, gg, s):
        p_part, _ = pressure(d, q_half, eps, prm)
        p_ext = external_pressure(modes, t_stage[s], shape, h)
        return fluid_increment(d, gg, prm, p_part + p_ext, force_faces, Zs[s])

    r0, g0 = drho, g
    dr, dg = dU(r0, g0, 0)
    r1 = r0 + dr
    g1 = [g0[a] + dg[a] for a in range(3)]
    dr, dg = dU(r1, g1, 1)
    r2 = 0.75 * r0 + 0.25 * (r1 + dr)
    g2 = [0.75 * g0[a] + 0.25 * (g1[a] + dg[a]) for a in range(3)]
    dr, dg = dU(r2, g2, 2)
    r3 = (1.0 / 3.0) * r0 + (2.0 / 3.0) * (r2 + dr)
    g3 = [(1.0 / 3.0) * g0[a] + (2.0 / 3.0) * (g2[a] + dg[a]) for a in range(3)]

    # Substeps 4-5: impulse and particle velocity.  Reading: per component
    # alpha, m_f = V J_alpha(rho_face^alpha) so that the fluid and particle
    # momentum changes cancel exactly on the staggered grid.
    V_t = np.zeros((npart, 3))
    m_f = np.zeros((npart, 3))
    for a in range(3):
        rho_face = rho0 + 0.5 * (r3 + _at(r3, a, 1))
        V_t[:, a] = interpolate(g3[a] / rho_face, q_half, h, a)
        m_f[:, a] = V * interpolate(rho_face, q_half, h, a)
    if npart and np.any(me[:, None] + m_f <= 0.0):
        raise FloatingPointError("m_e + m_f <= 0")
    u_new = u + (m_f / (me[:, None] + m_f)) * (V_t - u) if npart else u.copy()

    # Substep 6: v^{n+1} = v~ + V S (u^{n+1} - J v~), applied to g with the
    # face density of rho^{n+1} (unchanged by this substep).
    g_new = []
    for a in range(3):
        rho_face = rho0 + 0.5 * (r3 + _at(r3, a, 1))
        dv = V * spread(u_new[:, a] - V_t[:, a], q_half, h, shape, a)
        g_new.append(g3[a] + rho_face * dv)

    # Substep 7: q^{n+1} = q^n + dt/2 J^{n+1/2}(v^{n+1} + v^n).
    Jv_new = _velocity_at(g_new, r3, q_half, prm)
    q_new = _wrap(q + 0.5 * dt * (Jv_new + Jv_old), Lbox)

    lam = me[:, None] * (u_new - u) / dt - F
    new = dict(state)
    new.update(drho=r3, g=g_new, q=q_new, u=u_new, n=n + 1)
    diag = dict(q_half=q_half, F=F, lam=lam, Jv_old=Jv_old, V_tilde=V_t, m_f=m_f)
    return new, diag


def run(state, prm, nsteps, modes=None, tether_force_sum=None):
    """Apply ic_step nsteps times.  Returns the final state and the FP64 sums
    over the steps of -F_tether^{n+1/2} = k_s minimg(q^{n+1/2} - q_eq)
    (the spring force estimator of the radiation force, Sec. VI) and of
    lambda."""
    npart = len(np.asarray(state["q"]).reshape(-1, 3))
    sF = np.zeros((npart, 3))
    sL = np.zeros((npart, 3))
    for _ in range(nsteps):
        state, d = ic_step(state, prm, modes)
        sF += d["F"] - np.asarray(state["fext"]).reshape(-1, 3)
        sL += d["lam"]
    return state, -sF, sL


def conserved(state, prm):
    """Total mass sum h^3 drho and total momentum sum h^3 g + sum m_e u
    (Sec. IV C, total momentum density p = m_e S u + g)."""
    h = prm["h"]
    mass = h ** 3 * float(np.sum(state["drho"]))
    mom = [h ** 3 * float(np.sum(state["g"][a])) for a in range(3)]
    me = np.asarray(state["me"], dtype=np.float64)
    u = np.asarray(state["u"], dtype=np.float64).reshape(-1, 3)
    for a in range(3):
        mom[a] += float(np.sum(me * u[:, a]))
    return np.array([mass] + mom)
