#!/usr/bin/env python3
"""Throughput of the inertial-coupling (IC) step on one MI355X.

Workload (default): the paper-scale configuration, a 256^3 periodic staggered
grid with 10^4 tethered particles (half of each acoustic-contrast sign),
kT = 1e-3 (thermal Landau-Lifshitz noise on), a cosine standing-wave drive
along x with density amplitude 1e-2; h = 1, rho0 = 1, c_f = 1,
eta = zeta = 0.5, dt = 0.1.  Synthetic, seeded inputs already resident in HBM
when the timed region starts.

A step is one full IC step (substeps 1-7 with three SSP-RK3 sweeps of the
grid).  value = cells * steps / wall time of the timed region (FP32 storage
of the fields as deviations from rho0, FP64 particle state and
accumulators); the FP64 run of the same workload is reported beside it.

roofline: the dominant kernel is the fluid-stage kernel (three launches per
step).  Its algorithmic HBM traffic is 32 words per cell-update (stage 1:
read 4 + write 4; stages 2 and 3: read 4 + 4 + write 4), i.e. 128 B (FP32)
or 256 B (FP64); achieved = those bytes / the summed duration of the stage
launches, measured with HIP events on the stream the kernels run on, over
the timed region.  Peak = 8 TB/s.

cpu_baseline: the FP64 numpy oracle (as it stands) timed for one step on a
256 x 256 x 64 slab of the same workload (2500 particles at the same
density), on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s + % HBM roofline at 256^3/1e4 particles; FP32 vs FP64; adjoint cost"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1307_0702_amd import workloads as W
    if name == "paper-scale-256":
        return W.paper_scale_256()
    if name == "thermal-128":
        return W.thermal_128()
    if name == "standing-wave-32":
        return W.standing_wave_32()
    raise SystemExit(f"unknown workload {name}")


def run_gpu(w, prec, steps, warmup):
    import torch

    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation

    fl, p = w.fluid, w.particles
    sim = Simulation(fl, prec=prec, max_particles=max(p.n, 1))
    sim.set_state(w.drho, w.g)
    if p.n:
        eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
        sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    if w.modes:
        sim.set_forcing([m.as_dict() for m in w.modes])
    log(f"[bench] {prec}: warmup {warmup} steps")
    sim.step(warmup)
    sim.synchronize()
    ic.ic_profile_read(sim.ctx)            # discard
    ic.ic_profile(sim.ctx, 1)
    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    stage_ms, launches = ic.ic_profile_read(sim.ctx)
    ic.ic_profile(sim.ctx, 0)
    ncell = fl.nx * fl.ny * fl.nz
    esz = 4 if prec == "fp32" else 8
    bytes_alg = 32 * esz * ncell * steps
    c = sim.conserved()
    finite = bool(np.all(np.isfinite(c)))
    res = dict(
        ms_per_step=wall * 1e3 / steps,
        event_ms_per_step=ev_ms / steps,
        cell_updates_per_s=ncell * steps / wall,
        particle_updates_per_s=p.n * steps / wall,
        stage_ms_per_launch=stage_ms / max(launches, 1),
        stage_launches=launches,
        stage_achieved_gbs=bytes_alg / (stage_ms * 1e-3) / 1e9 if stage_ms > 0 else None,
        step_achieved_gbs=bytes_alg / wall / 1e9,
        finite=finite,
    )
    log(f"[bench] {prec}: {res['ms_per_step']:.3f} ms/step, stage kernel "
        f"{res['stage_ms_per_launch']:.3f} ms/launch, {res['stage_achieved_gbs']:.0f} GB/s")
    del sim
    torch.cuda.empty_cache()
    return res


def cpu_baseline(w_full):
    """One oracle step on a 256 x 256 x 64 slab of the workload."""
    from oracle import ic_oracle as O
    from paper_1307_0702_amd import workloads as W

    fl = W.Fluid(w_full.fluid.nx, w_full.fluid.ny, 64, kT=w_full.fluid.kT, seed=w_full.fluid.seed)
    npart = int(round(w_full.particles.n * fl.nz / w_full.fluid.nz))
    p = W.split_contrast_particles(fl, npart, seed=fl.seed, ks=10.0)
    mode, _ = W.modal_drive(fl, 1e-2)
    drho, g = W.standing_wave_fields(fl, 1e-2, omega=mode.omega)
    eps = O.eps_from_kappa_ratio(fl.cf, p.kappa_ratio)
    st = dict(drho=drho, g=[g[0], g[1], g[2]], n=0, q=p.q, u=np.zeros((npart, 3)), me=p.me,
              eps=eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    prm = fl.as_dict()
    log(f"[bench] cpu baseline: oracle, 1 step on {fl.nx}x{fl.ny}x{fl.nz}, {npart} particles")
    c0 = time.process_time()
    t0 = time.perf_counter()
    O.ic_step(st, prm, [mode.as_dict()])
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    ncell = fl.nx * fl.ny * fl.nz
    log(f"[bench] cpu baseline: {wall:.1f} s")
    return dict(value=ncell / wall, unit="cell-updates/s", cores=max(1, int(round(cpu / wall))),
                kind="oracle",
                sample=f"1 FP64 oracle step on a {fl.nx}x{fl.ny}x{fl.nz} slab of the workload "
                       f"({npart} particles, same density, kT and drive); {wall:.1f} s wall")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="paper-scale-256")
    ap.add_argument("--prec", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is a "
              "single-GPU build, see the design notes for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"[bench] building inputs for {args.workload}")
    w = make_workload(args.workload)
    fl = w.fluid
    res = {}
    precs = ["fp32", "fp64"] if args.prec == "both" else [args.prec]
    for prec in precs:
        res[prec] = run_gpu(w, prec, args.steps, args.warmup)
    main_prec = precs[0]
    r = res[main_prec]
    esz = 4 if main_prec == "fp32" else 8
    roof = dict(bound="hbm", achieved=r["stage_achieved_gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(r["stage_achieved_gbs"] / HBM_PEAK_GBS) if r["stage_achieved_gbs"] else None,
                traffic=None, kernel="stage_kernel", bytes_per_cell_update=32 * esz)
    out = dict(
        metric=METRIC,
        value=r["cell_updates_per_s"],
        unit="cell-updates/s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=r["ms_per_step"],
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f32" if main_prec == "fp32" else "f64",
        data="synthetic",
        config=dict(workload=w.name, grid=[fl.nx, fl.ny, fl.nz], particles=w.particles.n,
                    kT=fl.kT, dt=fl.dt, storage="fields as deviations from rho0; particles FP64"),
        particle_updates_per_s=r["particle_updates_per_s"],
        roofline=roof,
    )
    if "fp64" in res and main_prec != "fp64":
        r64 = res["fp64"]
        out["fp64"] = dict(value=r64["cell_updates_per_s"], ms_per_step=r64["ms_per_step"],
                           roofline=dict(bound="hbm", achieved=r64["stage_achieved_gbs"],
                                         peak=HBM_PEAK_GBS, unit="GB/s",
                                         frac=r64["stage_achieved_gbs"] / HBM_PEAK_GBS,
                                         bytes_per_cell_update=256))
        out["speedup_fp32_over_fp64"] = r["cell_updates_per_s"] / r64["cell_updates_per_s"]
    out["finite"] = all(x["finite"] for x in res.values())
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
