"""Pins of the oracle's kernel, J and S against what the paper fixes.

Sec. II (linear consistency, kernel volume, Faxen radius) and App. A
("Spatial discretization": the 3-point function and staggered positions).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import ic_oracle as O

OFFSETS = np.linspace(0.0, 1.0, 2001)


def test_phi_special_values():
    # App. A, 3-point function: phi(0)=2/3, phi(1/2)=1/2 from both branches,
    # phi(1)=1/6, phi(3/2)=0, symmetric, zero beyond 3/2.
    assert O.phi(0.0) == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert O.phi(0.5) == pytest.approx(0.5, abs=1e-15)
    assert O.phi(np.nextafter(0.5, 1.0)) == pytest.approx(0.5, abs=1e-12)
    assert O.phi(1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert O.phi(1.5) == pytest.approx(0.0, abs=1e-15)
    assert O.phi(1.6) == 0.0 and O.phi(-7.0) == 0.0
    r = np.linspace(-2, 2, 401)
    assert np.array_equal(O.phi(r), O.phi(-r))


def test_phi_is_c1():
    # Both branches meet with slope -1 at |r| = 1/2 and slope 0 at |r| = 3/2.
    e = 1e-7
    for r0, slope in [(0.5, -1.0), (1.5, 0.0)]:
        left = (O.phi(r0) - O.phi(r0 - e)) / e
        right = (O.phi(r0 + e) - O.phi(r0)) / e
        assert left == pytest.approx(slope, abs=1e-5)
        assert right == pytest.approx(slope, abs=1e-5)


def test_phi_moment_conditions():
    # Sec. II, Eqs. k1/k2/kvol in 1-D: sum phi = 1, sum r phi = 0,
    # sum phi^2 = 1/2 (the 1-D norm the paper quotes), for every offset.
    for o in OFFSETS:
        r = np.arange(-3, 4) - o
        p = O.phi(r)
        assert abs(p.sum() - 1.0) < 4e-16 * 4, o
        assert abs((r * p).sum()) < 4e-16 * 8, o
        assert abs((p * p).sum() - 0.5) < 4e-16 * 4, o


def test_kernel_volume_is_8h3():
    # Sec. II, "Kernel volume": tensor product gives V = 8 h^3, i.e.
    # sum_i h^3 theta^2 = 1/V for any q (3-D, arbitrary h).
    rng = np.random.default_rng(0)
    h = 0.7
    shape = (9, 8, 10)
    for _ in range(20):
        q = rng.random(3) * np.array([10, 8, 9]) * h
        idx, W = O._stencil(q[None, :], h, shape, None)
        s = np.sum((W / h ** 3) ** 2) * h ** 3
        assert s == pytest.approx(1.0 / O.kernel_volume(h), rel=1e-14)


def test_faxen_radius():
    # Sec. II, Eq. faxen: R_F^2 = 3 J[(r-q)^2] gives R_F = 0.945 h on
    # average over particle positions, varying by a few percent.
    m2 = []
    for o in OFFSETS[:-1]:
        r = np.arange(-3, 4) - o
        m2.append(np.sum(O.phi(r) * r * r))
    rf = np.sqrt(3.0 * np.array(m2))
    assert rf.mean() == pytest.approx(0.945, abs=1e-3)
    assert 0.86 < rf.min() and rf.max() <= 1.0 + 1e-12


def _dense_interp(field, q, h, face_axis):
    """J f as the plain sum over every grid point (Sec. II, Eq. Jdis) with
    minimum-image displacements, no stencil selection."""
    nz, ny, nx = field.shape
    L = np.array([nx, ny, nz]) * h
    out = 0.0
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        r = np.array([i, j, k], dtype=float) * h
        if face_axis is not None:
            r[face_axis] += 0.5 * h
        d = q - r
        d -= L * np.floor(d / L + 0.5)
        w = np.prod(O.phi(d / h))
        out += w * field[k, j, i]
    return out


@pytest.mark.parametrize("face_axis", [None, 0, 1, 2])
def test_interpolate_matches_dense_definition(face_axis):
    rng = np.random.default_rng(1 + (face_axis or 0))
    h = 1.3
    shape = (5, 6, 7)
    f = rng.standard_normal(shape)
    L = np.array([7, 6, 5]) * h
    # include points right on cell centres, faces and the periodic seam
    qs = [rng.random(3) * L for _ in range(6)]
    qs += [np.array([0.0, 0.0, 0.0]), np.array([3.0, 2.5, 4.5]) * h,
           L - 1e-12, np.array([6.5, 0.5, 0.5]) * h]
    q = np.array(qs)
    got = O.interpolate(f, q, h, face_axis)
    for p in range(len(q)):
        assert got[p] == pytest.approx(_dense_interp(f, q[p], h, face_axis), abs=1e-13)


@pytest.mark.parametrize("face_axis", [None, 0, 2])
def test_spread_is_adjoint_of_interpolate(face_axis):
    # Sec. II, Eq. adj: F . (J v) = sum_i h^3 v_i . (S F)_i, and
    # sum_i h^3 (S F)_i = F, J (S 1) = 1/V.
    rng = np.random.default_rng(5)
    h = 0.9
    shape = (6, 5, 7)
    L = np.array([7, 5, 6]) * h
    q = rng.random((4, 3)) * L
    F = rng.standard_normal(4)
    v = rng.standard_normal(shape)
    SF = O.spread(F, q, h, shape, face_axis)
    lhs = np.sum(F * O.interpolate(v, q, h, face_axis))
    rhs = h ** 3 * np.sum(v * SF)
    assert lhs == pytest.approx(rhs, rel=1e-13)
    assert h ** 3 * SF.sum() == pytest.approx(F.sum(), rel=1e-13)
    one = O.spread(np.ones(1), q[:1], h, shape, face_axis)
    assert O.interpolate(one, q[:1], h, face_axis)[0] == pytest.approx(
        1.0 / O.kernel_volume(h), rel=1e-13)


def test_interpolate_linear_field_exactly():
    # Sec. II, Eqs. k1/k2: any linear field is interpolated exactly (away
    # from the periodic seam, where the field is linear over the stencil).
    h = 0.5
    shape = (12, 12, 12)
    kk, jj, ii = np.meshgrid(np.arange(12), np.arange(12), np.arange(12), indexing="ij")
    a, b = 0.3, np.array([0.7, -1.1, 0.4])
    for face_axis in [None, 1]:
        x = ii * h + (0.5 * h if face_axis == 0 else 0.0)
        y = jj * h + (0.5 * h if face_axis == 1 else 0.0)
        z = kk * h + (0.5 * h if face_axis == 2 else 0.0)
        f = a + b[0] * x + b[1] * y + b[2] * z
        rng = np.random.default_rng(2)
        q = 2.0 + rng.random((10, 3)) * 2.0
        got = O.interpolate(f, q, h, face_axis)
        assert np.allclose(got, a + q @ b, atol=1e-13)


def test_eps_kappa_conversion():
    # Sec. III, Eqs. part_svel/ke: c_p = 2 c_f gives kappa_e = -3/4 kappa_f
    # (the value quoted in Sec. VI A), and f1 = -kappa_e/kappa_f.
    cf = 4.0
    cp = 8.0
    eps = cp * cp - cf * cf
    kappa_ratio = (cf / cp) ** 2
    assert O.eps_from_kappa_ratio(cf, kappa_ratio) == pytest.approx(eps)
    kappa_e = -eps / (cp * cp)
    assert kappa_e == pytest.approx(-0.75)
    assert 1.0 - kappa_ratio == pytest.approx(-kappa_e)
