"""Seeded synthetic inputs for the inertial-coupling step.

This module only draws and lays out inputs: fluid parameters, particle sets,
initial fields and forcing descriptions.  It holds none of the step's
arithmetic and imports nothing from the rest of the package, so the test
suite can feed the very same arrays to the HIP path and to the CPU oracle.

Grid arrays have shape (nz, ny, nx) (x fastest in memory); particle arrays are
(N, 3) with columns x, y, z.

Workloads (all synthetic: the paper measures nothing on external data):
  * "standing-wave-32"  : 32^3, kT = 0, a symmetric pair of tethered
    particles in a modal standing wave of density amplitude 1e-3 (the
    deterministic radiation-force case; FP64).
  * "thermal-128"       : 128^3, kT = 1e-3, 1000 particles, wave 1e-2.
  * "paper-scale-256"   : 256^3, kT = 1e-3, 10^4 particles, half of each
    acoustic-contrast sign, wave 1e-2 (the benchmark workload).
Shared fluid: h = 1, rho0 = 1, c_f = 1, eta = zeta = 0.5, dt = 0.1, V = 8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Fluid:
    nx: int
    ny: int
    nz: int
    h: float = 1.0
    rho0: float = 1.0
    cf: float = 1.0
    eta: float = 0.5
    zeta: float = 0.5
    kT: float = 0.0
    dt: float = 0.1
    seed: int = 0
    replica: int = 0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def as_dict(self):
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, h=self.h, rho0=self.rho0,
                    cf=self.cf, eta=self.eta, zeta=self.zeta, kT=self.kT, dt=self.dt,
                    seed=self.seed, replica=self.replica)


@dataclass
class Particles:
    q: np.ndarray                 # (N, 3) positions
    me: np.ndarray                # (N,) excess mass m_p - rho0 V
    kappa_ratio: np.ndarray       # (N,) kappa_p / kappa_f
    ks: np.ndarray                # (N,) tether spring constants
    qeq: np.ndarray               # (N, 3) tether anchors
    fext: np.ndarray = None       # (N, 3) constant external force
    u: np.ndarray = None          # (N, 3) initial velocity (None: J v)

    def __post_init__(self):
        n = len(self.q)
        if self.fext is None:
            self.fext = np.zeros((n, 3))

    @property
    def n(self):
        return len(self.q)


@dataclass
class Mode:
    """One imposed pressure drive: amp * profile(x_axis) * sin(omega t + phase).
    shape "cos": profile cos(2 pi m (x - x0)/L); shape "plane": 1 on the plane
    of cells nearest x0, 0 elsewhere."""
    axis: int
    shape: str
    m: int
    x0: float
    amp: float
    omega: float
    phase: float = 0.0

    def as_dict(self):
        return dict(axis=self.axis, shape=self.shape, m=self.m, x0=self.x0,
                    amp=self.amp, omega=self.omega, phase=self.phase)


@dataclass
class Workload:
    name: str
    fluid: Fluid
    particles: Particles
    modes: list = field(default_factory=list)
    drho: np.ndarray = None
    g: np.ndarray = None           # (3, nz, ny, nx)
    period_steps: int = 0


# ----------------------------------------------------------------------------
# Field initialisers
# ----------------------------------------------------------------------------

def random_fields(shape, seed, drho_scale=1e-2, g_scale=1e-2):
    """Gaussian random density deviation and momentum, for parity tests."""
    rng = np.random.default_rng(seed)
    drho = drho_scale * rng.standard_normal(shape)
    g = g_scale * rng.standard_normal((3,) + tuple(shape))
    return drho, g


def standing_wave_fields(fl: Fluid, amp, axis=0, m=1, x0=0.0, omega=None, t=0.0):
    """Density and momentum of a linear standing sound wave along `axis`,
    drho = amp cos(k (x - x0)) cos(omega t) at cell centres and
    g = amp (omega / k_d) sin(k (x_face - x0)) sin(omega t) on the faces,
    k = 2 pi m / L and k_d = (2/h) sin(k h / 2) the staggered-grid wavenumber.
    This is the state a resonantly driven mode settles into, so runs start
    near it instead of waiting for the transient."""
    n = (fl.nx, fl.ny, fl.nz)[axis]
    L = n * fl.h
    k = 2.0 * math.pi * m / L
    kd = 2.0 / fl.h * math.sin(k * fl.h / 2.0)
    if omega is None:
        omega = fl.cf * kd
    x = np.arange(n) * fl.h
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    prof =(amp * np.cos(k * (x - x0)) * math.cos(omega * t)).reshape(bshape)
    drho = np.broadcast_to(prof, fl.shape).copy()
    g = np.zeros((3,) + fl.shape)
    gp = (amp * (omega / kd) * np.sin(k * (x + 0.5 * fl.h - x0)) * math.sin(omega * t)).reshape(bshape)
    g[axis] = np.broadcast_to(gp, fl.shape)
    return drho, g


def discrete_sound_frequency(fl: Fluid, axis=0, m=1):
    """omega_d = c_f k_d of mode m along `axis` on the staggered grid."""
    n = (fl.nx, fl.ny, fl.nz)[axis]
    k = 2.0 * math.pi * m / (n * fl.h)
    return fl.cf * 2.0 / fl.h * math.sin(k * fl.h / 2.0)


def period_steps(fl: Fluid, omega):
    """Whole number of steps closest to one drive period."""
    return int(round(2.0 * math.pi / (omega * fl.dt)))


def modal_drive(fl: Fluid, drho_amp, axis=0, m=1, x0=0.0):
    """A cosine pressure drive whose period is a whole number of steps, with
    the amplitude P = drho_amp nu_L omega that gives density amplitude
    drho_amp at resonance (nu_L = (4 eta/3 + zeta)/rho0)."""
    om_d = discrete_sound_frequency(fl, axis, m)
    nT = period_steps(fl, om_d)
    omega = 2.0 * math.pi / (nT * fl.dt)
    nu_l = (4.0 * fl.eta / 3.0 + fl.zeta) / fl.rho0
    return Mode(axis=axis, shape="cos", m=m, x0=x0, amp=drho_amp * nu_l * omega,
                omega=omega), nT


# ----------------------------------------------------------------------------
# Particle sets
# ----------------------------------------------------------------------------

def uniform_particles(fl: Fluid, n, seed, mass_range=(0.5, 2.0), kappa_range=(0.5, 2.0),
                      ks=0.0, min_sep=None):
    """n particles uniform in the box; m_p/(rho0 V) ~ U[mass_range],
    kappa_p/kappa_f ~ U[kappa_range]; tethered at their start positions with
    spring constant ks.  If min_sep is given, positions are redrawn until
    every pair is at least min_sep apart along some axis (periodic), so the
    kernels do not overlap."""
    rng = np.random.default_rng(seed)
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    V = 8.0 * fl.h ** 3
    if min_sep is None:
        q = rng.random((n, 3)) * L
    else:
        pts = []
        tries = 0
        while len(pts) < n:
            tries += 1
            if tries > 100000:
                raise RuntimeError("cannot place non-overlapping particles")
            c = rng.random(3) * L
            ok = True
            for p in pts:
                d = np.abs(c - p)
                d = np.minimum(d, L - d)
                if np.all(d < min_sep):
                    ok = False
                    break
            if ok:
                pts.append(c)
        q = np.array(pts).reshape(n, 3)
    mp = rng.uniform(*mass_range, size=n) * fl.rho0 * V
    kr = rng.uniform(*kappa_range, size=n)
    return Particles(q=q, me=mp - fl.rho0 * V, kappa_ratio=kr,
                     ks=np.full(n, float(ks)), qeq=q.copy())


def split_contrast_particles(fl: Fluid, n, seed, ks, threshold=0.05):
    """n particles, half with Gor'kov contrast f1 + 1.5 f2 > threshold and half
    with < -threshold (f1 = 1 - kappa_p/kappa_f, f2 = 2 m_e/(2 m_e + 3 rho0 V)),
    drawn as in uniform_particles and rejection-sampled."""
    rng = np.random.default_rng(seed)
    L = np.array([fl.nx, fl.ny, fl.nz]) * fl.h
    V = 8.0 * fl.h ** 3
    want = n // 2
    pos, neg = [], []
    while len(pos) < want or len(neg) < n - want:
        mp = rng.uniform(0.5, 2.0) * fl.rho0 * V
        kr = rng.uniform(0.5, 2.0)
        me = mp - fl.rho0 * V
        phi_c = (1.0 - kr) + 1.5 * (2.0 * me / (2.0 * me + 3.0 * fl.rho0 * V))
        if phi_c > threshold and len(pos) < want:
            pos.append((me, kr))
        elif phi_c < -threshold and len(neg) < n - want:
            neg.append((me, kr))
    props = np.array(pos + neg)
    q = rng.random((n, 3)) * L
    return Particles(q=q, me=props[:, 0].copy(), kappa_ratio=props[:, 1].copy(),
                     ks=np.full(n, float(ks)), qeq=q.copy())


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def soft_tether(fl: Fluid, omega, mp_min):
    """Spring constant whose tether frequency is a sixth of the drive
    frequency for the lightest particle: the particles then oscillate with
    the wave (as the radiation force assumes) while the spring holds their
    mean position."""
    return mp_min * (omega / 6.0) ** 2


def standing_wave_32(x=4.0):
    """32^3, kT = 0: a symmetric pair of particles with m_p = 2 rho0 V and
    kappa_p = kappa_f/2, tethered at x0 + x and x0 - x from the pressure
    antinode x0 = 0 (y, z = L/2 and 0, so the springs' momenta cancel);
    cosine drive along x with density amplitude 1e-3, whole-step period;
    fluid starts on the driven standing wave."""
    fl = Fluid(32, 32, 32, kT=0.0, seed=1)
    V = 8.0
    mode, nT = modal_drive(fl, 1e-3)
    drho, g = standing_wave_fields(fl, 1e-3, omega=mode.omega)
    q = np.array([[x, 16.0, 16.0], [32.0 - x, 0.0, 0.0]])
    ks = soft_tether(fl, mode.omega, 2.0 * V)
    p = Particles(q=q, me=np.full(2, 2.0 * V - V), kappa_ratio=np.full(2, 0.5),
                  ks=np.full(2, ks), qeq=q.copy())
    return Workload("standing-wave-32", fl, p, [mode], drho, g, nT)


# Sec. VI, Table I: the paper's own force runs.  Fig. "force" (dipolar):
# zeta = 1, omega = 0.0784137, m_e = 8000, c_p = 4, measured drho 0.00240249;
# Fig. "force3" (monopolar): zeta = 0.5, omega = 0.0784134, m_e = 0, c_p = 8,
# measured drho 0.00339202.  Shared: h = 10, 32^3 cells, rho0 = 1, eta = 0.5,
# c_f = 4, Kronecker-plane pressure drive of amplitude 0.005.
TABLE1 = {
    "force": dict(zeta=1.0, omega=0.0784137, me=8000.0, cp=4.0, drho=0.00240249),
    "force3": dict(zeta=0.5, omega=0.0784134, me=0.0, cp=8.0, drho=0.00339202),
}


def table1(fig, particles=True, steps_per_period=320, dp=0.005, n=32, ks_scale=1.0, cp=None):
    """The Table I configuration of figure `fig` ("force" or "force3") in the
    paper's units, with the paper-literal plane drive p_ext = dp sin(omega t)
    on the cells of the plane x = 0 (Sec. VI, Eq. pext; the wave runs along x
    here).  No time step is printed: dt = 2 pi / (omega steps_per_period), so
    a drive period is a whole number of steps (c_f dt / h = 0.100).  The
    fluid starts on the resonant mode's linear steady state,
    drho = D cos(k x) cos(omega t) with D = 2 (h/L) dp / (nu_L omega) (the
    k = 2 pi / L part of the plane drive is 2 (h/L) dp cos(k x)); the other
    modes the plane excites start at rest.  With particles: the symmetric
    pair of Sec. VI at (3L/8, L/2, L/2) and (-3L/8, 0, 0) from the driven
    plane, m_e and c_p of the figure (or `cp`), on soft tethers (reading R9)
    scaled by ks_scale.  n != 32: the same in an n^3 box, driven at its
    discrete resonance (2 c_f / h) sin(pi h / L), which is what the printed
    frequencies are for n = 32 (reading R7)."""
    t = TABLE1[fig]
    omega = t["omega"]
    if n != 32:
        omega = discrete_sound_frequency(Fluid(n, n, n, h=10.0, cf=4.0))
    fl = Fluid(n, n, n, h=10.0, rho0=1.0, cf=4.0, eta=0.5, zeta=t["zeta"], kT=0.0,
               dt=2.0 * math.pi / (omega * steps_per_period), seed=1)
    L = fl.nx * fl.h
    mode = Mode(axis=0, shape="plane", m=1, x0=0.0, amp=dp, omega=omega)
    nu_l = (4.0 * fl.eta / 3.0 + fl.zeta) / fl.rho0
    D = 2.0 * (fl.h / L) * dp / (nu_l * omega)
    drho, g = standing_wave_fields(fl, D, omega=omega)
    V = 8.0 * fl.h ** 3
    if particles:
        qeq = np.array([[3 * L / 8, L / 2, L / 2], [L - 3 * L / 8, 0.0, 0.0]])
        mp = t["me"] + fl.rho0 * V
        p = Particles(q=qeq.copy(), me=np.full(2, t["me"]),
                      kappa_ratio=np.full(2, (fl.cf / (cp or t["cp"])) ** 2),
                      ks=np.full(2, ks_scale * soft_tether(fl, omega, mp)), qeq=qeq)
    else:
        p = Particles(q=np.zeros((0, 3)), me=np.zeros(0), kappa_ratio=np.zeros(0),
                      ks=np.zeros(0), qeq=np.zeros((0, 3)))
    return Workload("table1-" + fig, fl, p, [mode], drho, g, steps_per_period)


def thermal_128(n=1000, seed=2):
    fl = Fluid(128, 128, 128, kT=1e-3, seed=seed)
    mode, nT = modal_drive(fl, 1e-2)
    drho, g = standing_wave_fields(fl, 1e-2, omega=mode.omega)
    p = uniform_particles(fl, n, seed, ks=soft_tether(fl, mode.omega, 4.0))
    return Workload("thermal-128", fl, p, [mode], drho, g, nT)


def paper_scale_256(n=10000, seed=3):
    fl = Fluid(256, 256, 256, kT=1e-3, seed=seed)
    mode, nT = modal_drive(fl, 1e-2)
    drho, g = standing_wave_fields(fl, 1e-2, omega=mode.omega)
    p = split_contrast_particles(fl, n, seed, ks=soft_tether(fl, mode.omega, 4.0))
    return Workload("paper-scale-256", fl, p, [mode], drho, g, nT)


def gibbs_boltzmann_32(n_side=3, drho_amp=0.1, kT=1e-3, seed=5):
    """32^3 in the paper's low-viscosity regime (eta = zeta = 0.0125), kT = 1e-3,
    a resonant standing wave along x (drive amplitude for drho_amp without
    particles; the free particles damp it to about a third), and
    n_side x n_side free particles with m_p = 2 rho0 V, kappa_p = kappa_f
    (Gor'kov contrast f2 = 0.4) on a lattice in y, z, at x drawn uniformly:
    they collect around the pressure nodes as their Boltzmann distribution
    in the acoustic potential says."""
    fl = Fluid(32, 32, 32, kT=kT, seed=seed, eta=0.0125, zeta=0.0125)
    mode, nT = modal_drive(fl, drho_amp)
    drho, g = standing_wave_fields(fl, drho_amp, omega=mode.omega)
    rng = np.random.default_rng(seed)
    L = fl.nx * fl.h
    yz = np.array([[(i + 0.5) * L / n_side, (j + 0.5) * L / n_side]
                   for i in range(n_side) for j in range(n_side)])
    n = len(yz)
    q = np.column_stack([rng.uniform(0, L, n), yz])
    V = 8.0 * fl.h ** 3
    p = Particles(q=q, me=np.full(n, V), kappa_ratio=np.ones(n), ks=np.zeros(n), qeq=q.copy())
    return Workload("gibbs-boltzmann-32", fl, p, [mode], drho, g, nT)


def adjoint_64(n=16, seed=5, amp=2.3e-4):
    """64^3, kT = 0, the fluid at rest: n particles drawn as in
    uniform_particles (masses and compressibilities on both sides of the
    fluid's), tethered at their start positions; four cosine pressure drives
    along x with m = 1..4 wavelengths in the box, each at its own discrete
    resonance rounded to a whole-step period, pressure amplitude amp each.
    period_steps is the period of the m = 1 drive."""
    fl = Fluid(64, 64, 64, kT=0.0, seed=seed)
    modes = []
    for m in range(1, 5):
        om = discrete_sound_frequency(fl, 0, m)
        modes.append(Mode(axis=0, shape="cos", m=m, x0=0.0, amp=amp,
                          omega=2.0 * math.pi / (period_steps(fl, om) * fl.dt)))
    nT = period_steps(fl, modes[0].omega)
    p = uniform_particles(fl, n, seed, ks=soft_tether(fl, modes[0].omega, 4.0))
    drho = np.zeros(fl.shape)
    g = np.zeros((3,) + fl.shape)
    return Workload("adjoint-64", fl, p, modes, drho, g, nT)


def force_pair_32(me, kappa_ratio, x, eta=0.0125, amp=1e-3, L=32):
    """The radiation-force protocol of Sec. VI on an L^3 box in the paper's
    low-viscosity regime: a resonant cosine drive along x (Delta rho = amp,
    whole-step period), the fluid on the driven standing wave, and a
    symmetric pair at x0 + x (y, z = L/2) and x0 - x (y, z = 0) with excess
    mass me and kappa_p / kappa_f = kappa_ratio, softly tethered (k_s =
    m_p (omega/6)^2).  Each particle starts where the fluid around it is at
    t = 0, one end of its oscillation, so its mean position starts at the
    anchor."""
    fl = Fluid(L, L, L, kT=0.0, seed=1, eta=eta, zeta=eta)
    mode, nT = modal_drive(fl, amp)
    drho, g = standing_wave_fields(fl, amp, omega=mode.omega)
    V = 8.0 * fl.h ** 3
    Lx = fl.nx * fl.h
    qeq = np.array([[(mode.x0 + x) % Lx, L / 2, L / 2], [(mode.x0 - x) % Lx, 0.0, 0.0]])
    k = 2.0 * math.pi / Lx
    kd = 2.0 / fl.h * math.sin(k * fl.h / 2.0)
    q = qeq.copy()
    q[:, 0] -= amp * np.sin(k * (qeq[:, 0] - mode.x0)) / kd
    ks = (me + fl.rho0 * V) * (mode.omega / 6.0) ** 2
    p = Particles(q=q, me=np.full(2, float(me)), kappa_ratio=np.full(2, float(kappa_ratio)),
                  ks=np.full(2, ks), qeq=qeq)
    return Workload("force-pair-32", fl, p, [mode], drho, g, nT)


def force_sweeps_32():
    """The sweeps behind the paper's force figures (Sec. VI), as a list of
    (sweep, parameter, workload): the force along the wave for a dense
    particle (m_e = rho0 V, kappa_p = kappa_f) and a stiff one (c_p = 2 c_f,
    m_e = 0) at x = 2, 4, ..., 14 from the antinode (wavelength 32); and at
    x = 4 (where sin 2kx = 1) the force against c_p / c_f for neutrally
    buoyant particles and against rho_p / rho0 for particles as compressible
    as the fluid."""
    V = 8.0
    out = []
    for x in range(2, 16, 2):
        out.append(("position-dipolar", float(x), force_pair_32(V, 1.0, float(x))))
        out.append(("position-monopolar", float(x), force_pair_32(0.0, 0.25, float(x))))
    for cr in (0.4, 0.6, 0.8, 1.25, 1.5, 2.0, 3.0):
        out.append(("sound-speed-ratio", cr, force_pair_32(0.0, 1.0 / (cr * cr), 4.0)))
    for dr in (0.5, 1.5, 2.0, 3.0, 5.0):
        out.append(("density-ratio", dr, force_pair_32((dr - 1.0) * V, 1.0, 4.0)))
    return out


def ensemble(n=64, seed=4000, sizes=(32, 48, 64), max_particles=50, kT=1e-3):
    """n independent thermal replicas: grid edge drawn from `sizes`, 1 to
    max_particles free particles with m_p/(rho0 V) ~ U[0.5, 2] and
    kappa_p/kappa_f ~ U[0.5, 2], noise seed seed + r and replica id r."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        e = int(rng.choice(sizes))
        npart = int(rng.integers(1, max_particles + 1))
        fl = Fluid(e, e, e, kT=kT, seed=seed + r, replica=r)
        p = uniform_particles(fl, npart, seed + 10000 + r, ks=0.0)
        out.append(Workload(f"replica-{r}", fl, p, [], np.zeros(fl.shape),
                            np.zeros((3,) + fl.shape), 0))
    return out


def small_random(nx=20, ny=12, nz=10, npart=6, seed=11, kT=1e-3, min_sep=None):
    """A small ragged grid with random fields and particles, for parity."""
    fl = Fluid(nx, ny, nz, kT=kT, seed=seed)
    drho, g = random_fields(fl.shape, seed)
    p = uniform_particles(fl, npart, seed + 1, ks=0.3, min_sep=min_sep)
    rng = np.random.default_rng(seed + 2)
    p.u = 1e-2 * rng.standard_normal((npart, 3))
    p.fext = 1e-3 * rng.standard_normal((npart, 3))
    p.qeq = p.q + rng.uniform(-0.5, 0.5, size=(npart, 3))
    mode = Mode(axis=0, shape="cos", m=1, x0=1.5, amp=3e-3, omega=0.2, phase=0.3)
    return Workload("small-random", fl, p, [mode], drho, g, 0)
