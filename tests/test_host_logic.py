"""Host-side logic that needs no GPU: the default stage-tile extent, the
workspace layouts (two noise sets, the adjoint workspace), the benchmark's
refusal of more than one GPU and its traffic bookkeeping."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _params(**kw):
    from paper_1307_0702_amd import ic
    d = dict(nx=8, ny=8, nz=8, prec=ic.IC_FP64, h=1.0, rho0=1.0, cf=1.0, eta=0.5, zeta=0.5,
             kT=0.0, dt=0.1, seed=1, replica=0, max_particles=4)
    d.update(kw)
    return ic.ic_params(*[d[k] for k, _ in ic.ic_params._fields_])


def _policy(nx, ny, nz, prec):
    # rounds of resident blocks (3 per CU in FP32, 2 in FP64, 256 CUs) times
    # planes marched (tz plus 3 halo planes); ties go to the larger extent
    cap = 256 * (3 if prec == 1 else 2)
    best, cost = None, None
    for tz in (32, 16, 8, 4):
        blocks = -(-nx // 32) * -(-ny // 16) * -(-nz // tz)
        c = -(-blocks // cap) * (min(tz, nz) + 3)
        if cost is None or c < cost:
            best, cost = tz, c
    return best


@pytest.mark.parametrize("shape,prec", [((256, 256, 256), 1), ((256, 256, 256), 2),
                                         ((128, 128, 128), 1), ((32, 32, 32), 1),
                                         ((1008, 1008, 1000), 1), ((70, 20, 40), 2)])
def test_default_tile_extent(shape, prec):
    from paper_1307_0702_amd import ic
    nx, ny, nz = shape
    ctx = ic.ic_create(_params(nx=nx, ny=ny, nz=nz, prec=prec), 0)
    assert ic.ic_get_tile(ctx) == _policy(nx, ny, nz, prec)
    ic.ic_set_tile(ctx, 8)
    assert ic.ic_get_tile(ctx) == 8
    with pytest.raises(ic.ICError) as e:
        ic.ic_set_tile(ctx, 12)
    assert e.value.code == ic.IC_E_ARG
    ic.ic_destroy(ctx)


def test_thermal_workspace_holds_two_noise_sets():
    from paper_1307_0702_amd import ic
    n = 64
    cold = ic.ic_workspace_size(_params(nx=n, ny=n, nz=n, kT=0.0))
    hot = ic.ic_workspace_size(_params(nx=n, ny=n, nz=n, kT=1e-3))
    assert hot - cold == 18 * n ** 3 * 8      # 2 x 9 FP64 fields (256-byte multiples here)


def test_adjoint_workspace_size():
    from paper_1307_0702_amd import ic
    n = 64
    def up(b):
        return (b + 255) // 256 * 256

    for npart in (4, 1000):
        got = ic.ic_adjoint_workspace_size(_params(nx=n, ny=n, nz=n, max_particles=npart))
        fields = 16 * n ** 3 * 8
        partial = ic.IC_MAX_MODES * (n ** 3 // 256) * 8
        # per particle: five [N][3] and three [N] doubles
        particles = 5 * up(24 * npart) + 3 * up(8 * npart)
        assert got == fields + partial + particles


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_traffic_only_for_the_profiled_source(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    t, note = bench.measured_traffic("fp32")
    if t is None:
        pytest.skip("the counter summary was taken on another kernel source: " + note)
    assert t > 7e8
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 64)
    t2, note2 = bench.measured_traffic("fp32")
    assert t2 is None and "changed" in note2
