"""The FP64 reverse-mode oracle (oracle/ic_adjoint.py) against finite
differences of the forward oracle: transpose identities for the stage
increment and gradients of a loss after several RK3 steps."""
import numpy as np

from oracle import ic_adjoint as A
from oracle import ic_oracle as O

PRM = dict(h=1.0, dt=0.1, rho0=1.0, cf=1.0, eta=0.5, zeta=0.5, kT=0.0)


def _state(shape, seed, amp=0.1):
    rng = np.random.default_rng(seed)
    return amp * rng.standard_normal(shape), [amp * rng.standard_normal(shape) for _ in range(3)]


def _dot(a, b):
    return float(np.sum(a * b))


def _inc(r, g, p):
    z = [np.zeros(r.shape)] * 3
    return O.fluid_increment(r, g, PRM, p, z, None)


def test_increment_transpose_matches_central_differences():
    shape = (7, 5, 6)
    r, g = _state(shape, 1)
    lr, lg = _state(shape, 2, 1.0)
    dr, dg = _state(shape, 3, 1.0)
    p = 0.05 * np.random.default_rng(4).standard_normal(shape)
    mr, mg, _ = A.fluid_increment_vjp(r, g, PRM, lr, lg)
    eps = 1e-6
    ap = _inc(r + eps * dr, [g[a] + eps * dg[a] for a in range(3)], p)
    am = _inc(r - eps * dr, [g[a] - eps * dg[a] for a in range(3)], p)
    jvp = _dot(lr, (ap[0] - am[0]) / (2 * eps)) + sum(
        _dot(lg[a], (ap[1][a] - am[1][a]) / (2 * eps)) for a in range(3))
    vjp = _dot(mr, dr) + sum(_dot(mg[a], dg[a]) for a in range(3))
    assert abs(jvp - vjp) <= 1e-8 * abs(vjp)


def test_increment_transpose_each_term_against_pressure_and_momentum_alone():
    # perturb only the momentum of one axis, then only the density: each
    # group of terms is checked on its own
    shape = (6, 7, 5)
    r, g = _state(shape, 11)
    lr, lg = _state(shape, 12, 1.0)
    mr, mg, _ = A.fluid_increment_vjp(r, g, PRM, lr, lg)
    p = np.zeros(shape)
    eps = 1e-6
    rng = np.random.default_rng(13)
    for which in ("rho", 0, 1, 2):
        d = rng.standard_normal(shape)
        if which == "rho":
            ap, am = _inc(r + eps * d, g, p), _inc(r - eps * d, g, p)
            vjp = _dot(mr, d)
        else:
            gp = [g[a] + (eps * d if a == which else 0) for a in range(3)]
            gm = [g[a] - (eps * d if a == which else 0) for a in range(3)]
            ap, am = _inc(r, gp, p), _inc(r, gm, p)
            vjp = _dot(mg[which], d)
        jvp = _dot(lr, (ap[0] - am[0]) / (2 * eps)) + sum(
            _dot(lg[a], (ap[1][a] - am[1][a]) / (2 * eps)) for a in range(3))
        assert abs(jvp - vjp) <= 1e-8 * abs(vjp), which


def test_pressure_adjoint_is_exact_for_the_linear_drive_term():
    shape = (5, 6, 7)
    r, g = _state(shape, 21)
    lr, lg = _state(shape, 22, 1.0)
    _, _, mp = A.fluid_increment_vjp(r, g, PRM, lr, lg)
    q = np.random.default_rng(23).standard_normal(shape)
    a1 = _inc(r, g, q)
    a0 = _inc(r, g, np.zeros(shape))
    jvp = _dot(lr, a1[0] - a0[0]) + sum(_dot(lg[a], a1[1][a] - a0[1][a]) for a in range(3))
    assert abs(jvp - _dot(mp, q)) <= 1e-12 * abs(jvp)


def test_multistep_gradient_matches_central_differences():
    shape = (6, 5, 8)
    r, g = _state(shape, 31, 0.05)
    modes = [dict(axis=0, shape="cos", m=1, x0=0.5, amp=2e-3, omega=0.3, phase=0.2),
             dict(axis=2, shape="plane", m=1, x0=3.0, amp=1e-3, omega=0.7, phase=0.0)]
    cr, cg = _state(shape, 32, 1.0)
    nsteps, n0 = 4, 7
    gr, gg, gA, _ = A.run_grad(r, g, PRM, modes, nsteps, cr, cg, n0=n0)

    def loss(r0, g0, mds):
        rr, gx = r0, list(g0)
        for s in range(nsteps):
            _, (rr, gx), _ = A.step_forward(rr, gx, PRM, mds, n0 + s)
        return _dot(cr, rr) + sum(_dot(cg[a], gx[a]) for a in range(3))

    eps = 1e-6
    for m in range(2):
        mp = [dict(md) for md in modes]
        mm = [dict(md) for md in modes]
        mp[m]["amp"] += eps
        mm[m]["amp"] -= eps
        fd = (loss(r, g, mp) - loss(r, g, mm)) / (2 * eps)
        assert abs(fd - gA[m]) <= 1e-7 * abs(fd) + 1e-12, (m, fd, gA[m])
    rng = np.random.default_rng(33)
    dr, dg = rng.standard_normal(shape), [rng.standard_normal(shape) for _ in range(3)]
    fd = (loss(r + eps * dr, [g[a] + eps * dg[a] for a in range(3)], modes) -
          loss(r - eps * dr, [g[a] - eps * dg[a] for a in range(3)], modes)) / (2 * eps)
    an = _dot(gr, dr) + sum(_dot(gg[a], dg[a]) for a in range(3))
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_step_forward_is_the_oracle_step_without_particles():
    shape = (5, 6, 4)
    r, g = _state(shape, 41, 0.05)
    modes = [dict(axis=1, shape="cos", m=1, x0=0.0, amp=1e-3, omega=0.4, phase=0.0)]
    prm = dict(PRM, nx=4, ny=6, nz=5, seed=0, replica=0)
    st = dict(drho=r, g=list(g), n=3, q=np.zeros((0, 3)), u=np.zeros((0, 3)), me=np.zeros(0),
              eps=np.zeros(0), ks=np.zeros(0), qeq=np.zeros((0, 3)), fext=np.zeros((0, 3)))
    new, _ = O.ic_step(st, prm, modes)
    _, (r3, g3), _ = A.step_forward(r, g, prm, modes, 3)
    assert np.array_equal(new["drho"], r3)
    for a in range(3):
        assert np.array_equal(new["g"][a], g3[a])
