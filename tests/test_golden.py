"""The oracle against numbers the paper prints (tests/golden/paper_values.txt)."""
import math
import os

import numpy as np

from oracle import ic_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("|")[0].strip()
        if line and not line.startswith("#"):
            name, value, tol = line.split()
            out[name] = (float(value), float(tol))
    return out


def _mode_frequency(nx, h, cf):
    """Frequency of the slowest x sound mode of the oracle's spatial operator
    (inviscid, no noise, no particles): the increment of a density cosine
    and of a momentum sine span a 2 x 2 block [[0, a], [b, 0]] whose
    eigenvalues are +- i sqrt(-a b)."""
    prm = dict(h=h, dt=1.0, rho0=1.0, cf=cf, eta=0.0, zeta=0.0, kT=0.0)
    shape = (4, 4, nx)
    k = 2 * math.pi / (nx * h)
    x = np.arange(nx) * h
    amp = 1e-9
    zero = np.zeros(shape)
    faces = [zero, zero, zero]
    drho = amp * np.broadcast_to(np.cos(k * x), shape).copy()
    d1, g1 = O.fluid_increment(drho, [zero, zero, zero], prm, zero, faces, None)
    gx = amp * np.broadcast_to(np.sin(k * (x + 0.5 * h)), shape).copy()
    d2, _ = O.fluid_increment(zero, [gx, zero, zero], prm, zero, faces, None)
    b = g1[0][0, 0, 0] / (amp * math.sin(k * 0.5 * h))   # momentum sine from density cosine
    a = d2[0, 0, 0] / amp                               # density cosine from momentum sine
    return math.sqrt(-a * b)


def test_table1_wave_frequencies_are_the_oracles_discrete_sound_mode():
    g = _golden()
    w = _mode_frequency(nx=32, h=10.0, cf=4.0)
    for name in ("table1_omega_force", "table1_omega_force3"):
        val, tol = g[name]
        assert abs(w - val) <= tol * val, (name, w, val)
    # and not the continuum value 2 pi c / L printed in the table caption
    assert abs(w - 2 * math.pi * 4.0 / 320.0) > 1e-4


def test_acoustic_radius_of_the_kernel_volume():
    val, tol = _golden()["acoustic_radius_over_h"]
    r = (3 * O.kernel_volume(1.0) / (4 * math.pi)) ** (1 / 3)
    assert abs(r - val) <= tol * val


def test_faxen_radius_of_the_kernel():
    val, tol = _golden()["faxen_radius_over_h"]
    # mean over sub-cell offsets of sqrt(3 m2), m2 the kernel's second moment
    offs = (np.arange(2000) + 0.5) / 2000
    rf = []
    for s in offs:
        idx, w = O.kernel_points(np.array([s]), 1.0, 10, False)
        r = s - (idx[0].astype(float))
        r = (r + 5) % 10 - 5
        rf.append(math.sqrt(3 * np.sum(w[0] * r * r)))
    assert abs(np.mean(rf) - val) <= tol * val


def test_table1_printed_amplitudes_are_the_workload_values():
    # the GPU test of Table I reads these; the workload builder carries the
    # same numbers
    from paper_1307_0702_amd import workloads as W
    g = _golden()
    for fig in ("force", "force3"):
        assert g["table1_drho_" + fig][0] == W.TABLE1[fig]["drho"]
