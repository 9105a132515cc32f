"""Pins of the oracle's random numbers.

The paper does not name its generator; the reading is Philox-4x32-10
(Salmon et al., SC'11) plus Box-Muller.  The oracle's Philox is checked word
for word against the independent implementation that ships with ROCm's
rocRAND (its header-only engine compiled for the host), and the normals
against their defining statistics.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ic_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(123)
    rows = [(0, 0, 0, 0, 0, 0), (1, 2, 3, 4, 5, 6),
            (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(200):
        k = rng.integers(0, 2 ** 32, size=2)
        c = rng.integers(0, 2 ** 32, size=4)
        c[1] = c[1] % (2 ** 30)   # the reference engine takes c0,c1 as a 64-bit offset/4
        rows.append((int(k[0]), int(k[1]), int(c[0]), int(c[1]), int(c[2]), int(c[3])))
    inp = "\n".join(" ".join(str(x) for x in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(x) for x in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(rows)
    for r, want in zip(rows, ref):
        got = O.philox4x32_10(r[2], r[3], r[4], r[5], r[0], r[1])
        assert tuple(int(x) for x in got) == want, r


def test_philox_vectorised_equals_scalar():
    c0 = np.arange(50, dtype=np.uint64) * 977 + 3
    vec = O.philox4x32_10(c0, 7, 2, 1, 0xDEADBEEF, 0x12345678)
    for i in range(0, 50, 7):
        sc = O.philox4x32_10(int(c0[i]), 7, 2, 1, 0xDEADBEEF, 0x12345678)
        assert [int(v[i]) for v in vec] == [int(s) for s in sc]


def test_uniform23_range_and_exactness():
    x = np.array([0, 511, 512, 0xFFFFFFFF, 0x80000000, 0x7FFFFFFF, 12345678], dtype=np.uint32)
    u = O.uniform23(x)
    assert u[0] == 2.0 ** -24 and u[1] == u[0]
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    assert np.all((u > 0) & (u < 1))
    # exactly representable in FP32 as well
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)


def test_cell_normals_statistics():
    # Standard normals: mean 0, variance 1, fourth moment 3, no correlation
    # between the 12 streams or between neighbouring cells (5 sigma).
    n = 200000
    WA, WB = O.cell_normals(seed=99, step=5, replica=0, ncell=n)
    Z = np.concatenate([WA, WB])
    assert Z.shape == (12, n)
    se = 5.0 / math.sqrt(n)
    assert np.all(np.abs(Z.mean(axis=1)) < se)
    assert np.all(np.abs(Z.var(axis=1) - 1.0) < 5.0 * math.sqrt(2.0 / n))
    assert np.all(np.abs((Z ** 4).mean(axis=1) - 3.0) < 5.0 * math.sqrt(96.0 / n))
    C = np.corrcoef(Z)
    off = C[~np.eye(12, dtype=bool)]
    assert np.all(np.abs(off) < se * 1.2)
    lag = np.array([np.corrcoef(z[:-1], z[1:])[0, 1] for z in Z])
    assert np.all(np.abs(lag) < se * 1.2)


def test_cell_normals_keyed_by_step_seed_replica():
    a = O.cell_normals(1, 0, 0, 64)[0]
    assert not np.allclose(a, O.cell_normals(1, 1, 0, 64)[0])
    assert not np.allclose(a, O.cell_normals(2, 0, 0, 64)[0])
    assert not np.allclose(a, O.cell_normals(1, 0, 1, 64)[0])
    assert np.array_equal(a, O.cell_normals(1, 0, 0, 64)[0])
    # the stream of a cell does not depend on the grid size
    assert np.array_equal(O.cell_normals(1, 3, 0, 100)[1][:, :64], O.cell_normals(1, 3, 0, 64)[1])
