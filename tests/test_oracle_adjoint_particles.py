"""The FP64 reverse mode of the whole IC step with particles
(oracle/ic_adjoint.py: phi_prime, step_vjp_particles, run_grad_particles)
against what fixes it independently of itself:

- phi' against the derivative identities of the 3-point function (App. A):
  the kernel's partition of unity, first moment and sum of squares are
  constant in r, so sum phi' = 0, sum (r - i) phi' = -1, sum phi phi' = 0;
  phi'(1/2) = -1 from both sides, phi'(3/2) = 0 (phi is C^1), and central
  differences of phi;
- every block of the reversed step against central differences of the
  forward oracle (ic_oracle.ic_step), one input group and one output seed at
  a time, so a dropped term or a wrong sign in any substep fails on its own;
- a three-step gradient of the summed tether force (the radiation-force
  estimator of Sec. VI) with respect to m_e, eps_pf, k_s and the drive
  amplitudes, against central differences.
"""
import numpy as np
import pytest

from oracle import ic_adjoint as A
from oracle import ic_oracle as O

PRM = dict(h=1.0, dt=0.1, rho0=1.0, cf=1.0, eta=0.5, zeta=0.5, kT=0.0, seed=0, replica=0)
SHAPE = (9, 7, 8)   # (nz, ny, nx)
MODES = [dict(axis=0, shape="cos", m=1, x0=0.5, amp=2e-3, omega=0.3, phase=0.2),
         dict(axis=2, shape="plane", m=1, x0=3.0, amp=1e-3, omega=0.7, phase=0.0)]


def _state(seed=1, amp=0.05):
    rng = np.random.default_rng(seed)
    # particles 0 and 1 have overlapping kernel supports
    q = np.array([[2.3, 3.1, 4.4], [3.6, 3.9, 4.13], [6.2, 1.4, 6.7]])
    return dict(drho=amp * rng.standard_normal(SHAPE), g=[amp * rng.standard_normal(SHAPE) for _ in range(3)],
                n=5, q=q, u=0.02 * rng.standard_normal((3, 3)), me=np.array([2.0, -3.0, 0.5]),
                eps=np.array([0.6, -0.4, 1.2]), ks=np.array([0.3, 0.0, 1.0]),
                qeq=q + np.array([[0.2, -0.1, 0.05], [0.0, 0.0, 0.0], [-0.3, 0.1, 0.2]]),
                fext=np.array([[0.0, 0.0, 0.0], [1e-3, -2e-3, 0.0], [0.0, 5e-4, 0.0]]))


def _seeds(seed):
    rng = np.random.default_rng(seed)
    return dict(cr=rng.standard_normal(SHAPE), cg=[rng.standard_normal(SHAPE) for _ in range(3)],
                cq=rng.standard_normal((3, 3)), cu=rng.standard_normal((3, 3)),
                cF=rng.standard_normal((3, 3)))


def _loss(st, modes, c, nsteps=1):
    L = 0.0
    for _ in range(nsteps):
        st, d = O.ic_step(st, PRM, modes)
        L += float(np.sum(c["cF"] * d["F"]))
    L += float(np.sum(c["cr"] * st["drho"])) + sum(float(np.sum(c["cg"][a] * st["g"][a])) for a in range(3))
    L += float(np.sum(c["cq"] * st["q"])) + float(np.sum(c["cu"] * st["u"]))
    return L


def _perturbed(st, key, d, e):
    s = dict(st)
    if key == "g":
        s["g"] = [st["g"][a] + e * d[a] for a in range(3)]
    else:
        s[key] = st[key] + e * d
    return s


def _direction(st, key, rng):
    if key == "g":
        return [rng.standard_normal(SHAPE) for _ in range(3)]
    return rng.standard_normal(np.shape(st[key]))


def _dot(key, grad, d):
    if key == "g":
        return sum(float(np.sum(grad[a] * d[a])) for a in range(3))
    return float(np.sum(grad * d))


GRAD_OF = dict(drho="lr", g="lg", q="lq", u="lu", me="dme", eps="deps", ks="dks")


def test_phi_prime_identities_and_special_values():
    r = np.linspace(-2.0, 2.0, 40001)
    e = 1e-6
    fd = (O.phi(r + e) - O.phi(r - e)) / (2 * e)
    away = (np.abs(np.abs(r) - 0.5) > 1e-4) & (np.abs(np.abs(r) - 1.5) > 1e-4)
    assert np.max(np.abs(A.phi_prime(r) - fd)[away]) < 1e-7
    assert A.phi_prime(np.array([0.5]))[0] == pytest.approx(-1.0, abs=1e-15)
    assert A.phi_prime(np.array([0.5 + 1e-12]))[0] == pytest.approx(-1.0, abs=1e-5)
    assert A.phi_prime(np.array([-0.5]))[0] == pytest.approx(1.0, abs=1e-15)
    assert A.phi_prime(np.array([1.5, -1.5, 0.0, 1.7]))[:] == pytest.approx([0.0, 0.0, 0.0, 0.0], abs=1e-15)
    x = np.linspace(-0.5, 0.5, 2001)
    d = np.array([-1.0, 0.0, 1.0])
    rr = x[:, None] - d[None, :]
    p, dp = O.phi(rr), A.phi_prime(rr)
    assert np.max(np.abs(dp.sum(1))) < 1e-12
    assert np.max(np.abs((rr * dp).sum(1) + 1.0)) < 1e-12
    assert np.max(np.abs((p * dp).sum(1))) < 1e-12


def test_stencil_gradient_matches_differences_of_the_weights():
    rng = np.random.default_rng(3)
    q = rng.uniform(0.0, 7.0, (5, 3))
    for face in (None, 0, 1, 2):
        idx, W, dW = A.stencil_grad(q, 1.0, SHAPE, face)
        for b in range(3):
            e = np.zeros(3)
            e[b] = 1e-6
            _, Wp, _ = A.stencil_grad(q + e, 1.0, SHAPE, face)
            _, Wm, _ = A.stencil_grad(q - e, 1.0, SHAPE, face)
            assert np.max(np.abs((Wp - Wm) / 2e-6 - dW[b])) < 1e-7


def test_forward_replay_is_the_oracle_step():
    st = _state()
    new, diag = O.ic_step(st, PRM, MODES)
    fw = A.step_forward_particles(st, PRM, MODES)
    assert np.array_equal(fw["r3"], new["drho"])
    for a in range(3):
        assert np.array_equal(fw["g_new"][a], new["g"][a])
    assert np.array_equal(fw["q_new"], new["q"])
    assert np.array_equal(fw["u_new"], new["u"])
    assert np.array_equal(fw["F"], diag["F"])


@pytest.mark.parametrize("seed_key", ["cr", "cg", "cq", "cu", "cF"])
@pytest.mark.parametrize("key", ["drho", "g", "q", "u", "me", "eps", "ks"])
def test_one_step_block_matches_central_differences(key, seed_key):
    st = _state()
    full = _seeds(20)
    c = {k: (v if k == seed_key else (np.zeros_like(v) if k != "cg" else [np.zeros(SHAPE)] * 3))
         for k, v in full.items()}
    r = A.step_vjp_particles(st, PRM, MODES, c["cr"], c["cg"], c["cq"], c["cu"], c["cF"])
    rng = np.random.default_rng([ord(ch) for ch in key + seed_key])
    d = _direction(st, key, rng)
    # e = 1e-5 keeps the rounding of O(1) outputs (~1e-15 / e) and the
    # curvature error (~e^2) both below the bar
    e = 1e-5
    fd = (_loss(_perturbed(st, key, d, e), MODES, c) - _loss(_perturbed(st, key, d, -e), MODES, c)) / (2 * e)
    an = _dot(key, r[GRAD_OF[key]], d)
    assert abs(fd - an) <= 2e-6 * max(abs(fd), abs(an)) + 1e-10, (key, seed_key, fd, an)


def test_three_step_force_gradient_matches_central_differences():
    # L = x-force of particle 0 and z-force of particle 2 summed over three
    # steps: the shape of the averaged tether-force loss
    st = _state(seed=7)
    c = _seeds(21)
    for k in ("cr", "cq", "cu"):
        c[k] = np.zeros_like(c[k])
    c["cg"] = [np.zeros(SHAPE)] * 3
    c["cF"] = np.zeros((3, 3))
    c["cF"][0, 0] = -1.0
    c["cF"][2, 2] = -1.0
    out, _ = A.run_grad_particles(st, PRM, MODES, 3, cF=c["cF"])
    e = 1e-5
    for key in ("me", "eps", "ks", "q"):
        d = _direction(st, key, np.random.default_rng(5))
        fd = (_loss(_perturbed(st, key, d, e), MODES, c, 3) - _loss(_perturbed(st, key, d, -e), MODES, c, 3)) / (2 * e)
        an = _dot(key, out[GRAD_OF[key]], d)
        assert abs(fd - an) <= 2e-6 * abs(fd) + 1e-11, (key, fd, an)
    for m in range(len(MODES)):
        mp = [dict(md) for md in MODES]
        mm = [dict(md) for md in MODES]
        mp[m]["amp"] += e
        mm[m]["amp"] -= e
        fd = (_loss(dict(st), mp, c, 3) - _loss(dict(st), mm, c, 3)) / (2 * e)
        assert abs(fd - out["dA"][m]) <= 2e-6 * abs(fd) + 1e-11, (m, fd, out["dA"][m])


def test_particle_free_reverse_agrees_with_the_fluid_only_reverse():
    st = _state()
    for key in ("q", "u", "qeq", "fext"):
        st[key] = np.zeros((0, 3))
    for key in ("me", "eps", "ks"):
        st[key] = np.zeros(0)
    c = _seeds(22)
    r = A.step_vjp_particles(st, PRM, MODES, c["cr"], c["cg"], np.zeros((0, 3)), np.zeros((0, 3)))
    lr, lg, dA = A.step_vjp(st["drho"], st["g"], PRM, MODES, st["n"], c["cr"], c["cg"])
    assert np.allclose(r["lr"], lr, rtol=0, atol=1e-14)
    for a in range(3):
        assert np.allclose(r["lg"][a], lg[a], rtol=0, atol=1e-14)
    assert np.allclose(r["dA"], dA, rtol=1e-13)
