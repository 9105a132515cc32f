"""Host-side logic that needs no GPU: the default stage-tile extent, the
workspace layouts (two noise sets, the adjoint workspace), the benchmark's
refusal of more than one GPU, its traffic bookkeeping and its kernel-trace
timeline summary."""
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


def test_timeline_summary_of_a_synthetic_trace(tmp_path, capsys):
    # two precisions' worth of steps in one trace: the summary takes the
    # first run's steps after the warm-up, offsets from each step's first
    # sweep, medians over the steps
    sys.path.insert(0, ROOT)
    import bench
    rows = []

    def add(name, s, e):
        rows.append(dict(Kernel_Name=name, Start_Timestamp=str(int(s * 1000)),
                         End_Timestamp=str(int(e * 1000))))

    sweep0 = "void ic::(anonymous namespace)::stage_kernel<float, 0, true, true>(ic::(anonymous namespace)::StageArgs<float>)"
    sweep1 = "void ic::(anonymous namespace)::stage_kernel<float, 1, true, true>(ic::(anonymous namespace)::StageArgs<float>)"
    for n in range(6):          # 2 warm-up + 4 timed steps of 1000 us, the sweeps at +0 and +400
        t = 1000.0 * n + (3.0 if n == 3 else 0.0)
        add("void ic::(anonymous namespace)::k_step_begin(ic::StepState*, DriveArgs)", t - 10, t - 8)
        add(sweep0, t, t + 300)
        add(sweep1, t + 400, t + 700)
    for n in range(2):          # a second precision afterwards is not counted
        t = 10000.0 + 1000.0 * n
        add(sweep0.replace("float", "double"), t, t + 900)
    path = tmp_path / "trace.csv"
    with open(path, "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for r in rows:
            f.write('"%s",%s,%s\n' % (r["Kernel_Name"], r["Start_Timestamp"], r["End_Timestamp"]))
    bench.timeline_summary(str(path), 2, 4)
    out = capsys.readouterr().out.splitlines()
    assert out[0].startswith("# float, median over 3 steps")
    body = {l[:48].strip(): l[48:].split() for l in out[2:]}
    assert [float(x) for x in body["stage_kernel<float, 0, true, true>"]] == [0.0, 300.0, 300.0]
    assert [float(x) for x in body["stage_kernel<float, 1, true, true>"]] == [400.0, 700.0, 300.0]
    assert float(body["next step's first sweep"][0]) == 1000.0
