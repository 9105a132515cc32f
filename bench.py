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
step).  Its algorithmic HBM traffic is 32 words per cell-update over the
three launches (stage 1: read 4 + write 4; stages 2 and 3: read 4 + 4 +
write 4), i.e. 128 B (FP32) or 256 B (FP64) per cell-update; achieved = those
bytes / the summed duration of the stage launches, measured with HIP events
recorded on the stream the kernels run on, over the timed region.
Peak = 8 TB/s.  traffic = HBM bytes per stage launch from rocprofv3
FETCH_SIZE and WRITE_SIZE counters, each scaled by what the same counter
reads for a plain 1 GiB device copy; it is read from the committed counter
summary and reported only while the kernel source still matches the one the
counters were taken on.

cpu_baseline: the FP64 numpy oracle (as it stands) timed for one full step of
the same workload on the host (about 15 s of CPU work; the particles start at
rest instead of at J v, which does not change the work done).

Helper modes (they serve the profiles kept beside this file):
  --copy-probe              1 GiB device-to-device copies (counter calibration
                            and the achievable copy bandwidth)
  --stats-summary CSV       condense a rocprofv3 --stats kernel table
  --pmc-summary F W CF CW   condense FETCH_SIZE / WRITE_SIZE passes of the bench
                            (F, W) and of the copy probe (CF, CW)
  --instr-summary DIR       condense an SQ instruction-counter pass
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s + % HBM roofline at 256^3/1e4 particles; FP32 vs FP64; adjoint cost"
HBM_PEAK_GBS = 8000.0
WORDS_PER_CELL_UPDATE = 32          # over the three stage launches of one step
ADJ_WORDS_PER_CELL = 72             # one reversed step (recomputation included)
STAGES = 3
KERNEL_SRC = os.path.join(ROOT, "paper_1307_0702_amd", "csrc", "ic_device.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "stage_kernel_256cube_1e4p_pmc.txt")
COPY_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def make_workload(name):
    from paper_1307_0702_amd import workloads as W
    if name == "paper-scale-256":
        return W.paper_scale_256()
    if name == "thermal-128":
        return W.thermal_128()
    if name == "standing-wave-32":
        return W.standing_wave_32()
    if name == "adjoint-64":
        return W.adjoint_64()
    raise SystemExit(f"unknown workload {name}")


def run_gpu(w, prec, steps, warmup, graph=True, one_by_one=False):
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
    if one_by_one:
        # every step launched one by one (ic_profile keeps ic_step off its
        # graph), so a kernel trace holds only the schedule of the profiled pass
        ic.ic_profile(sim.ctx, 1)
    # the step graph that an ic_step call of 5 steps or more replays is
    # captured here (no step is run), not inside the timed call; the warm-up
    # then follows without a pause
    sim.prepare()
    log(f"[bench] {prec}: warmup {warmup} steps")
    sim.step(warmup)
    sim.synchronize()
    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # the timed steps: one ic_step call, as a user makes it (on grids of
    # >= 2^20 cells it replays its 4-step graph and launches the rest)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    # the stage-kernel launch time: the same steps launched one by one with
    # HIP events around every stage launch on the context stream (ic_profile
    # keeps ic_step off its graph), right after the timed steps
    nprof = min(steps, 50)
    ic.ic_profile_read(sim.ctx)            # discard
    ic.ic_profile(sim.ctx, 1)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    sim.step(nprof)
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - tp
    stage_ms, launches = ic.ic_profile_read(sim.ctx)
    ic.ic_profile(sim.ctx, 0)
    ncell = fl.nx * fl.ny * fl.nz
    esz = 4 if prec == "fp32" else 8
    bytes_alg = WORDS_PER_CELL_UPDATE * esz * ncell * nprof
    c = sim.conserved()
    finite = bool(np.all(np.isfinite(c)))
    res = dict(
        ms_per_step=wall * 1e3 / steps,
        event_ms_per_step=ev_ms / steps,
        cell_updates_per_s=ncell * steps / wall,
        particle_updates_per_s=p.n * steps / wall,
        launched_ms_per_step=prof_wall * 1e3 / nprof,
        stage_ms_per_launch=stage_ms / max(launches, 1),
        stage_launches=launches,
        stage_achieved_gbs=bytes_alg / (stage_ms * 1e-3) / 1e9 if stage_ms > 0 else None,
        step_achieved_gbs=WORDS_PER_CELL_UPDATE * esz * ncell * steps / wall / 1e9,
        alg_bytes_per_launch=bytes_alg / max(launches, 1),
        finite=finite,
    )
    # the same steps replayed from one HIP graph (single-stream steps)
    res["graph_ms_per_step"] = None
    if graph:
        g = ic.ic_graph_create([sim.ctx], 50)
        ic.ic_graph_launch(g, stream.cuda_stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ic.ic_graph_launch(g, stream.cuda_stream)
        torch.cuda.synchronize()
        res["graph_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / 50
        ic.ic_graph_destroy(g)
    log(f"[bench] {prec}: {res['ms_per_step']:.3f} ms/step ({res['launched_ms_per_step']:.3f} "
        f"launched one by one), stage kernel {res['stage_ms_per_launch']:.3f} ms/launch, "
        f"{res['stage_achieved_gbs']:.0f} GB/s")
    del sim
    torch.cuda.empty_cache()
    return res


def run_ensemble(prec, steps, warmup):
    """64 thermal replicas (grid edges 32/48/64, 1-50 particles, own seeds and
    replica ids): aggregate cell-updates/s of member-after-member eager steps
    and of HIP-graph launches of all members (one launch per 50 steps)."""
    import torch

    from paper_1307_0702_amd import workloads as W
    from paper_1307_0702_amd.ensemble import Ensemble

    ws = W.ensemble()
    log(f"[bench] ensemble: {len(ws)} replicas, tuning tiles")
    ens = Ensemble(ws, prec=prec, tune=True)
    cells = ens.cells
    ens.run_serial(warmup)
    ens.synchronize()
    t0 = time.perf_counter()
    ens.run_serial(steps)
    ens.synchronize()
    t_serial = time.perf_counter() - t0
    tz_batch = ens.tune_batch()
    log(f"[bench] ensemble: batched graph tile extent {tz_batch}")
    # 50-step graphs replayed: measured 2.37e9 cell-updates/s against 1.75e9
    # for one 200-step graph (FP32, 4 hardware queues; more queues were slower)
    chunk = 50 if steps % 50 == 0 else steps
    ens.capture(chunk)
    ens.run()
    ens.synchronize()
    t0 = time.perf_counter()
    ens.run(steps // chunk)
    ens.synchronize()
    t_graph = time.perf_counter() - t0
    tiles = {"batched_graph": tz_batch}
    out = dict(metric="ensemble cell-updates/s", value=cells * steps / t_graph,
               unit="cell-updates/s", n_gpus=1, steps=steps, warmup=warmup,
               ms_per_step=t_graph * 1e3 / steps, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32" if prec == "fp32" else "f64", data="synthetic",
               config=dict(workload="ensemble-64", replicas=len(ws), cells=cells,
                           particles=sum(w.particles.n for w in ws), kT=ws[0].fluid.kT,
                           tile_z_by_edge=tiles),
               serial_value=cells * steps / t_serial,
               graph_speedup=t_serial / t_graph)
    # whole-step roofline of the graph launch: the stage kernels' 32 words
    # per cell-update over the replayed steps, against the HBM peak (the
    # replicas' 8.2e6 cells take 131 MB per FP32 state copy and about 1 GB
    # with the stage copies and noise fields, beyond the 256 MB last-level
    # cache, so HBM is the bound that applies)
    esz = 4 if prec == "fp32" else 8
    gbs = cells * steps * WORDS_PER_CELL_UPDATE * esz / t_graph / 1e9
    out["roofline"] = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                           frac=gbs / HBM_PEAK_GBS, traffic=None, kernel="whole step (graph replay)",
                           bytes_per_cell_update=WORDS_PER_CELL_UPDATE * esz)
    ens.release()
    del ens
    torch.cuda.empty_cache()
    return out


def run_adjoint(prec, steps, warmup):
    """Reverse mode on the deterministic 256^3 fluid (kT = 0, no particles,
    the paper-scale drive): time of one adjoint step (stage inputs recomputed,
    three transposed stages) against one forward step."""
    import torch

    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation

    w = make_workload("paper-scale-256")
    fl = w.fluid
    fl.kT = 0.0
    sim = Simulation(fl, prec=prec, max_particles=1)
    sim.set_state(w.drho, w.g)
    sim.set_forcing([m.as_dict() for m in w.modes])
    adj = Adjoint(sim)
    U = sim.U.clone()
    lam = torch.randn_like(sim.U)

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            fn(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    timed(lambda i: sim.step(1), warmup)
    fwd = timed(lambda i: sim.step(1), steps)
    timed(lambda i: adj.step(i, U, lam), warmup)
    rev = timed(lambda i: adj.step(i, U, lam), steps)
    ncell = fl.nx * fl.ny * fl.nz
    # algorithmic traffic of one reversed step: the two recomputed forward
    # stages (8 + 12 words per cell) and the three transposed stages, each
    # reading its input state and incoming adjoint and writing its outgoing
    # adjoint, with the accumulator written (third), read and written
    # (second) or read (first): 16 + 20 + 16 words -- 72 words per cell
    esz = 4 if prec == "fp32" else 8
    gbs = ADJ_WORDS_PER_CELL * esz * ncell / (rev * 1e-3) / 1e9
    out = dict(metric="adjoint cell-updates/s", value=ncell / (rev * 1e-3), unit="cell-updates/s",
               n_gpus=1, steps=steps, warmup=warmup, ms_per_step=rev, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32" if prec == "fp32" else "f64",
               data="synthetic",
               config=dict(workload="adjoint-256", grid=[fl.nx, fl.ny, fl.nz], particles=0, kT=0.0),
               forward_ms_per_step=fwd, adjoint_over_forward=rev / fwd,
               roofline=dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=gbs / HBM_PEAK_GBS, traffic=None, kernel="whole reversed step",
                             bytes_per_cell=ADJ_WORDS_PER_CELL * esz),
               finite=bool(torch.isfinite(lam).all()))
    del adj, sim
    torch.cuda.empty_cache()
    return out


def adjoint_step_cost(prec, nfwd=500, nrev=200):
    """One reversed step with particles against one forward step on the
    adjoint-64 workload (64^3, 16 tethered particles, four drives, kT = 0),
    each timed over back-to-back steps: (forward ms, reversed ms)."""
    import torch

    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation

    w = make_workload("adjoint-64")
    fl, p = w.fluid, w.particles
    sim = Simulation(fl, prec=prec, max_particles=p.n)
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing([m.as_dict() for m in w.modes])
    adj = Adjoint(sim)
    U, qs, us = adj.snapshot()
    lam = torch.randn_like(sim.U)
    lq = torch.randn((p.n, 3), dtype=torch.float64, device=sim.device)
    lu = torch.randn_like(lq)
    lF = torch.randn_like(lq)

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            fn(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    timed(lambda i: sim.step(1), 50)
    fwd = timed(lambda i: sim.step(1), nfwd)
    timed(lambda i: adj.step(i, U, lam, qs, us, lq, lu, lF), 20)
    rev = timed(lambda i: adj.step(i, U, lam, qs, us, lq, lu, lF), nrev)
    del adj, sim
    torch.cuda.empty_cache()
    return fwd, rev


def run_adjoint_particles(prec, periods, fd_check):
    """Reverse mode with particles: 64^3, kT = 0, 16 tethered particles, four
    resonant drives along x.  L = the x-component of the spring-force
    estimator <-F_tether> averaged over the particles and over `periods`
    periods of the m = 1 drive; its gradient with respect to the four drive
    amplitudes, m_p and kappa_p/kappa_f of every particle comes from a
    checkpointed reversal (checkpoint every 64 steps).  Reports the cost of
    one reversed step against one forward step, of the whole gradient
    against the forward run, and (fd_check) directional derivatives against
    central differences of the GPU forward run."""
    import torch

    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint, rollout_particles
    from paper_1307_0702_amd.ic import Simulation

    w = make_workload("adjoint-64")
    fl, p = w.fluid, w.particles
    nsteps = periods * w.period_steps
    md = [m.as_dict() for m in w.modes]
    sim = Simulation(fl, prec=prec, max_particles=p.n)
    kr = np.asarray(p.kappa_ratio, dtype=np.float64)
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in kr])
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing(md)
    adj = Adjoint(sim)
    dev = sim.device
    q0 = torch.empty((p.n, 3), dtype=torch.float64, device=dev)
    u0 = torch.empty_like(q0)
    ic.ic_copy_particles(sim.ctx, q0, u0)
    U0 = torch.zeros((4,) + sim.shape, dtype=sim.dtype, device=dev)

    # one step each way, timed back to back on a context of its own
    fwd, rev = adjoint_step_cost(prec)

    amps = torch.tensor([m["amp"] for m in md], dtype=torch.float64)
    me = torch.tensor(p.me, dtype=torch.float64)
    epst = torch.tensor(eps, dtype=torch.float64)
    fixed = dict(ks=p.ks, qeq=p.qeq, fext=p.fext)

    def loss(amps_, me_, eps_, every=64):
        _, _, _, F = rollout_particles(adj, U0, q0, u0, amps_, me_, eps_, md, 0, nsteps, every, **fixed)
        return -F[:, 0].mean()     # mean x-component of -F_tether (f_ext = 0)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.no_grad():
        L0 = float(loss(amps, me, epst))
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    xs = [amps.clone().requires_grad_(True), me.clone().requires_grad_(True),
          epst.clone().requires_grad_(True)]
    t0 = time.perf_counter()
    L = loss(*xs)
    L.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    dA, dme, deps = (x.grad.numpy() for x in xs)
    dkr = -fl.cf ** 2 / kr ** 2 * deps          # eps = cf^2 (1/r - 1)
    # the same gradient with the whole trajectory kept in device memory
    every_all = adj.auto_every(nsteps)
    ys = [x.detach().clone().requires_grad_(True) for x in xs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss(*ys, every="auto").backward()
    torch.cuda.synchronize()
    t_grad_all = time.perf_counter() - t0
    same = max(float((y.grad - x.grad).abs().max() / x.grad.abs().max()) for x, y in zip(xs, ys))
    out = dict(metric="adjoint particle-steps/s", value=p.n * nsteps / t_grad, unit="particle-steps/s",
               n_gpus=1, steps=nsteps, warmup=0, ms_per_step=t_grad * 1e3 / nsteps,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32" if prec == "fp32" else "f64", data="synthetic",
               config=dict(workload="adjoint-64", grid=[fl.nx, fl.ny, fl.nz], particles=p.n, kT=0.0,
                           drives=4, periods=periods, checkpoint_every=64),
               forward_step_ms=fwd, adjoint_step_ms=rev, adjoint_step_over_forward_step=rev / fwd,
               forward_run_s=t_fwd, gradient_run_s=t_grad, gradient_over_forward_run=t_grad / t_fwd,
               trajectory_in_memory=dict(every=every_all, state_bytes=adj.state_bytes(),
                                         gradient_run_s=t_grad_all,
                                         gradient_over_forward_run=t_grad_all / t_fwd,
                                         max_rel_diff_to_every_64=same),
               loss=L0, dL_damp=dA.tolist(), dL_dmp=dme.tolist(), dL_dkappa_ratio=dkr.tolist())
    if fd_check:
        rng = np.random.default_rng(7)
        fd = {}
        # steps large enough that 2 h dL stands well above the rounding of
        # positions accumulated over the run (L is quadratic in the drive
        # amplitudes, so their central difference has no curvature error)
        for name, i, h in (("amp", 0, 1e-2 * float(amps.abs().max())), ("m_p", 1, 1e-3),
                           ("eps", 2, 1e-3)):
            base = [amps, me, epst]
            d = torch.as_tensor(rng.standard_normal(tuple(base[i].shape)), dtype=torch.float64)
            ap = [b if j != i else b + h * d for j, b in enumerate(base)]
            am = [b if j != i else b - h * d for j, b in enumerate(base)]
            with torch.no_grad():
                f = (float(loss(*ap)) - float(loss(*am))) / (2 * h)
            an = float((xs[i].grad * d).sum())
            fd[name] = dict(fd=f, adjoint=an, rel=abs(f - an) / max(abs(f), 1e-300))
            log(f"[bench] adjoint-64 {prec} {name}: fd {f:.10e} adjoint {an:.10e}")
        out["central_differences"] = fd
    del adj, sim
    torch.cuda.empty_cache()
    return out


def run_force_sweeps(nwarm=40000, nper=8):
    """The force figures of Sec. VI as one ensemble (FP64, kT = 0): every
    configuration of workloads.force_sweeps_32 (26 symmetric pairs on 32^3
    boxes) advances in the same HIP-graph launches.  After nwarm steps the
    mean tether force is taken over nper drive periods, and each box's wave
    amplitude from 3 samples a third of a period apart (the mean of a^2 over
    them is exact for a sinusoid).  Gor'kov: F = c_f^2 a^2 V k (f1 + 3/2 f2) sin(2 k x) / (4 rho0)
    with the measured amplitude a."""
    import torch

    from paper_1307_0702_amd import workloads as W
    from paper_1307_0702_amd.ensemble import Ensemble

    cases = W.force_sweeps_32()
    ens = Ensemble([w for _, _, w in cases], prec="fp64", tune=False)
    nT = cases[0][2].period_steps
    assert nT % 3 == 0
    chunk = nT // 3                          # steps per graph launch
    nwarm = -(-nwarm // chunk) * chunk
    t0 = time.perf_counter()
    ens.capture(chunk)
    log(f"[bench] force sweeps: {len(cases)} boxes, {nwarm} + {nper * nT} steps")
    ens.run(nwarm // chunk)
    for s_ in ens.sims:
        s_.avg_force(reset=True)
    ens.run(nper * nT // chunk)
    forces = [s_.avg_force(reset=True)[0] for s_ in ens.sims]
    a2 = np.zeros(len(cases))
    for _ in range(3):
        ens.run(1)
        for i, (s_, (_, _, w)) in enumerate(zip(ens.sims, cases)):
            d, _ = s_.get_state()
            x = np.arange(w.fluid.nx) * w.fluid.h
            c = np.cos(2 * math.pi * (x - w.modes[0].x0) / (w.fluid.nx * w.fluid.h))
            a = 2.0 / w.fluid.nx * np.sum(d.mean(axis=(0, 1)) * c)
            a2[i] += a * a / 3
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ens.release()
    sweeps = {}
    for (name, par, w), f, m2 in zip(cases, forces, a2):
        fl, p = w.fluid, w.particles
        V = 8.0 * fl.h ** 3
        amp = math.sqrt(2.0 * m2)
        k = 2 * math.pi / (fl.nx * fl.h)
        f1 = 1.0 - p.kappa_ratio[0]
        f2 = 2 * p.me[0] / (2 * p.me[0] + 3 * fl.rho0 * V)
        x = (p.qeq[0, 0] - w.modes[0].x0) % (fl.nx * fl.h)
        gork = fl.cf ** 2 * amp * amp * V * k / (4 * fl.rho0) * (f1 + 1.5 * f2) * math.sin(2 * k * x)
        sweeps.setdefault(name, []).append(dict(
            param=par, force=float(f[0, 0]), force_partner=float(f[1, 0]), gorkov=gork,
            ratio=float(f[0, 0] / gork) if abs(gork) > 1e-18 else None, amplitude=amp))
    steps = nwarm + nper * nT + nT
    return dict(metric="radiation force sweeps against Gor'kov", value=len(cases) * 32 ** 3 * steps / wall,
                unit="cell-updates/s", n_gpus=1, steps=steps, warmup=nwarm, ms_per_step=wall * 1e3 / steps,
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload="force-sweeps-32", boxes=len(cases), grid=[32, 32, 32], kT=0.0,
                            eta=0.0125, amplitude=1e-3, average_periods=nper),
                sweeps=sweeps)


def run_force_precision(steps, kT=0.0):
    """The paper-scale configuration (256^3, 10^4 tethered particles of split
    contrast, standing wave of amplitude 1e-2) with kT = 0 by default: FP32
    (fields as deviations from rho0, FP64 particles and accumulators) against
    all-FP64, the spring-force estimator of the radiation force averaged over
    the last 7 whole drive periods of `steps` steps, and the FP32 speed-up.
    With kT > 0 both runs draw the same noise (same Philox streams), and the
    difference is that of two thermal trajectories from the same start."""
    import torch

    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.ic import Simulation

    w = make_workload("paper-scale-256")
    fl, p = w.fluid, w.particles
    fl.kT = kT
    nT = w.period_steps
    navg = 7 * nT
    nwarm = max(steps - navg, 0)
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    out = {}
    for prec in ("fp64", "fp32"):
        sim = Simulation(fl, prec=prec, max_particles=p.n)
        sim.set_state(w.drho, w.g)
        sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
        sim.set_forcing([m.as_dict() for m in w.modes])
        log(f"[bench] force precision {prec}: {nwarm} + {navg} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(nwarm)
        sim.avg_force(reset=True)
        sim.step(navg)
        f, _, ns = sim.avg_force(reset=True)
        torch.cuda.synchronize()
        out[prec] = (f, (time.perf_counter() - t0) / (nwarm + navg), ns)
        del sim
        torch.cuda.empty_cache()
    f64, t64, _ = out["fp64"]
    f32, t32, ns = out["fp32"]
    rel_max = float(np.max(np.abs(f32 - f64)) / np.max(np.abs(f64)))
    rel_rms = float(np.sqrt(np.mean((f32 - f64) ** 2) / np.mean(f64 ** 2)))
    return dict(metric="FP32 speed-up over FP64 at the averaged radiation force error",
                value=t64 / t32, unit="x", n_gpus=1, steps=nwarm + navg, warmup=0,
                ms_per_step=t32 * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32", data="synthetic",
                config=dict(workload="paper-scale-256-kT0" if kT == 0 else "paper-scale-256",
                            grid=[fl.nx, fl.ny, fl.nz], particles=p.n, kT=kT, averaged_steps=ns,
                            period_steps=nT),
                fp64_ms_per_step=t64 * 1e3, force_rel_err_max=rel_max, force_rel_err_rms=rel_rms,
                mean_abs_force_fp64=float(np.mean(np.abs(f64))))


def run_gibbs_boltzmann(steps, warmup):
    """Free dipolar particles in a thermal standing wave (32^3, kT = 1e-3):
    the distribution of their phase 2 k xi against the Boltzmann
    distribution in the acoustic potential (8 bins), and <cos 2 k xi>."""
    import math

    from scipy.special import i0, i1

    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd import workloads as W
    from paper_1307_0702_amd.ic import Simulation

    V = 8.0
    w = W.gibbs_boltzmann_32()
    fl, mode, p = w.fluid, w.modes[0], w.particles
    sim = Simulation(fl, prec="fp64", max_particles=p.n)
    sim.set_state(w.drho, w.g)
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq)
    sim.set_forcing([mode.as_dict()])
    k = 2 * math.pi * mode.m / (fl.nx * fl.h)
    t0 = time.perf_counter()
    sim.step(warmup)
    ph = []
    every = 200
    for i in range(steps // every):
        sim.step(every)
        q, _ = sim.get_particles()
        ph.append((2 * k * (q[:, 0] - mode.x0)) % (2 * math.pi))
        if (i + 1) % 500 == 0:
            log(f"[bench] gibbs-boltzmann: {(i + 1) * every} of {steps} steps")
    wall = time.perf_counter() - t0
    # amplitude of the driven density mode over one period
    x = np.arange(fl.nx) * fl.h
    c = np.cos(k * (x - mode.x0))
    a2 = []
    for _ in range(w.period_steps):
        sim.step(1)
        d, _ = sim.get_state()
        a2.append((2.0 / fl.nx * np.sum(d.mean(axis=(0, 1)) * c)) ** 2)
    a = math.sqrt(2.0 * np.mean(a2))
    ph = np.array(ph)
    f2 = 2 * w.particles.me[0] / (2 * w.particles.me[0] + 3 * fl.rho0 * V)
    u0 = V * (fl.cf ** 2 * a) ** 2 * (1.5 * f2) / (8 * fl.rho0 * fl.cf ** 2) / fl.kT
    per = np.cos(ph).mean(axis=0)
    hist, edges = np.histogram(ph.ravel(), bins=8, range=(0, 2 * math.pi), density=True)
    mid = 0.5 * (edges[1:] + edges[:-1])
    # bin averages of exp(-u0 cos) / (2 pi I0(u0))
    fine = np.linspace(0, 2 * math.pi, 8 * 64, endpoint=False) + math.pi / (8 * 64)
    boltz = (np.exp(-u0 * np.cos(fine)) / (2 * math.pi * i0(u0))).reshape(8, 64).mean(axis=1)
    return dict(metric="Gibbs-Boltzmann position distribution in a standing wave",
                value=float(per.mean()), unit="<cos 2k xi>", n_gpus=1, steps=steps, warmup=warmup,
                ms_per_step=wall * 1e3 / (steps + warmup), higher_is_better=False, scaling="weak",
                vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload=w.name, grid=[fl.nx, fl.ny, fl.nz], particles=w.particles.n,
                            kT=fl.kT, eta=fl.eta),
                std_error=float(per.std() / math.sqrt(len(per))),
                boltzmann=float(-i1(u0) / i0(u0)), u0_over_kT=float(u0), amplitude=float(a),
                pdf_measured=[round(float(x), 4) for x in hist],
                pdf_boltzmann=[round(float(x), 4) for x in boltz],
                pdf_bin_centres=[round(float(x), 4) for x in mid])


def measured_traffic(prec):
    """HBM bytes per stage launch from the committed counter summary, or None
    when the summary is missing or was taken on another kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None, "no counter summary"
    vals = {}
    with open(PMC_SUMMARY) as f:
        for line in f:
            m = re.match(r"^(\w+):\s*(\S+)", line)
            if m:
                vals[m.group(1)] = m.group(2)
    if vals.get("source_sha256") != kernel_source_sha():
        return None, "kernel changed since the counters were taken"
    key = f"traffic_bytes_per_stage_launch_{prec}"
    if key not in vals:
        return None, "no counters for " + prec
    return float(vals[key]), "rocprofv3 FETCH_SIZE x%s + WRITE_SIZE x%s" % (
        vals.get("fetch_scale", "?"), vals.get("write_scale", "?"))


def roofline(r, prec):
    traffic, note = measured_traffic(prec)
    esz = 4 if prec == "fp32" else 8
    ach = r["stage_achieved_gbs"]
    return dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(ach / HBM_PEAK_GBS) if ach else None, traffic=traffic,
                kernel="stage_kernel", launches_per_step=STAGES,
                alg_bytes_per_launch=r["alg_bytes_per_launch"],
                bytes_per_cell_update=WORDS_PER_CELL_UPDATE * esz,
                traffic_source=note,
                step_frac=r["step_achieved_gbs"] / HBM_PEAK_GBS,
                launch_timing=("HIP events around each stage launch on the context stream, over "
                               f"{r['stage_launches'] // STAGES} steps launched one by one right "
                               "after the timed steps (the timed call replays a step graph, "
                               "where no events sit between kernels)"),
                launched_ms_per_step=r["launched_ms_per_step"],
                # counter bytes over the same launch time: the second view
                measured_gbs=(traffic / (r["stage_ms_per_launch"] * 1e-3) / 1e9) if traffic else None,
                measured_frac=(traffic / (r["stage_ms_per_launch"] * 1e-3) / 1e9 / HBM_PEAK_GBS)
                if traffic else None)


def host_cpu():
    """CPU model and the number of cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def run_table1(log_fn):
    """Table I (Sec. VI) in the paper's units: the driven density amplitude
    of each force figure without particles against the printed value, and
    the symmetric pair's mean spring force against Gor'kov's."""
    from paper_1307_0702_amd.experiments import table1_run

    rows = {}
    for fig in ("force", "force3"):
        r0 = table1_run(fig, particles=False, log=log_fn)
        r1 = table1_run(fig, particles=True, log=log_fn)
        rows[fig] = dict(drho_measured=r0["amp"], drho_printed=r0["printed"],
                         drho_rel_err=r0["amp"] / r0["printed"] - 1,
                         force_x=r1["force"][:, 0].tolist(), gorkov_x=r1["gorkov"].tolist(),
                         ratio=(r1["force"][:, 0] / r1["gorkov"]).tolist(),
                         gorkov_with_tether_mass_x=r1["gorkov_tether"].tolist(),
                         ratio_with_tether_mass=(r1["force"][:, 0] / r1["gorkov_tether"]).tolist(),
                         drho_with_particles=r1["amp"])
        log_fn(f"[bench] table I {fig}: drho {r0['amp']:.6e} vs printed {r0['printed']:.6e}; "
               f"F/F_Gorkov {rows[fig]['ratio']}")
    return dict(metric="Table I: driven density amplitude and radiation force in the paper's units",
                value=rows["force3"]["drho_rel_err"], unit="relative error of drho (Fig. force3)",
                higher_is_better=False, n_gpus=1, dtype="f64", data="synthetic",
                config=dict(workload="table1", grid=[32, 32, 32], h=10.0, cf=4.0, eta=0.5,
                            drive="Kronecker plane, 0.005"),
                figures=rows)


def cpu_baseline(w):
    """One FP64 oracle step of the full workload (same fields, particles,
    drive and noise key) on the host."""
    from oracle import ic_oracle as O

    fl, p = w.fluid, w.particles
    eps = O.eps_from_kappa_ratio(fl.cf, p.kappa_ratio)
    st = dict(drho=w.drho.copy(), g=[c.copy() for c in w.g], n=0, q=p.q.copy(),
              u=np.zeros((p.n, 3)), me=p.me, eps=eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    log(f"[bench] cpu baseline: oracle, 1 step on {fl.nx}x{fl.ny}x{fl.nz}, {p.n} particles")
    c0 = time.process_time()
    t0 = time.perf_counter()
    O.ic_step(st, fl.as_dict(), [m.as_dict() for m in w.modes])
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    ncell = fl.nx * fl.ny * fl.nz
    log(f"[bench] cpu baseline: {wall:.1f} s")
    model, ncores = host_cpu()
    return dict(value=ncell / wall, unit="cell-updates/s", cores=max(1, int(round(cpu / wall))),
                kind="oracle",
                sample=f"1 FP64 oracle step (numpy, as it stands) of the full workload: "
                       f"{fl.nx}x{fl.ny}x{fl.nz} cells, {p.n} particles; {wall:.1f} s wall",
                cpu_model=model, host_cores_available=ncores)


def copy_probe():
    import torch
    n = COPY_BYTES // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps(dict(copy_bytes=COPY_BYTES, ms=dt * 1e3,
                          gbs_read_plus_write=2 * COPY_BYTES / dt / 1e9)), flush=True)


def _short(name):
    name = re.sub(r"\(ic::\(anonymous namespace\)::\w+(<\w+>)?\)", "", name)
    name = name.replace("ic::(anonymous namespace)::", "").replace("void ", "")
    return name[:60]


def stats_summary(path):
    rows = list(csv.DictReader(open(path)))
    print("%-60s %7s %12s %8s" % ("kernel", "calls", "avg_us", "pct"))
    for r in rows[:24]:
        print("%-60s %7s %12.1f %8s" % (_short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
                                       r["Percentage"]))


def timeline_summary(path, first_step, nsteps):
    """Median schedule of one step from a rocprofv3 kernel trace of this
    script: every kernel's start and end relative to the start of the step's
    first stage sweep, over the timed steps of the first run in the trace
    (steps first_step .. first_step + nsteps - 2 of that precision, i.e. after
    the warm-up and before the profiled pass)."""
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"]))
                for r in csv.DictReader(open(path)))
    first = [i for i, x in enumerate(ev) if x[2].startswith("stage_kernel<") and ", 0," in x[2]]
    prec = ev[first[0]][2].split("<")[1].split(",")[0]
    first = [i for i in first if ev[i][2].startswith("stage_kernel<" + prec + ",")]
    rows = {}
    steps = range(first_step, min(first_step + nsteps, len(first)) - 1)
    for j in steps:
        t0, t1 = ev[first[j]][0], ev[first[j + 1]][0]
        seen = {}
        for s, e, name in ev:
            # the step: from its k_step_begin (just before the sweep) up to the
            # next step's
            if t0 - 20000 <= s < t1 - 20000:
                k = (name, seen.get(name, 0))
                seen[name] = k[1] + 1
                rows.setdefault(k, []).append(((s - t0) / 1e3, (e - t0) / 1e3))
    print(f"# {prec}, median over {len(steps)} steps; us from the start of the first sweep")
    print("%-48s %9s %9s %9s" % ("kernel", "start_us", "end_us", "dur_us"))
    out = []
    for (name, n), v in rows.items():
        if len(v) < len(steps) // 2:
            continue
        st = float(np.median([a for a, _ in v]))
        en = float(np.median([b for _, b in v]))
        out.append((st, en, name))
    for st, en, name in sorted(out):
        print("%-48s %9.1f %9.1f %9.1f" % (name[:48], st, en, en - st))
    nxt = float(np.median([(ev[first[j + 1]][0] - ev[first[j]][0]) / 1e3 for j in steps]))
    print("%-48s %9.1f" % ("next step's first sweep", nxt))


def _pmc(dirname):
    per = {}
    for fn in os.listdir(dirname):
        if fn.endswith("counter_collection.csv"):
            for r in csv.DictReader(open(os.path.join(dirname, fn))):
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return per


def pmc_summary(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir):
    kib = 1024.0

    def copy_reading(d):
        vals = [v for k, vs in _pmc(d).items() if "copyBuffer" in k for v in vs]
        big = [v for v in vals if v * kib > COPY_BYTES / 8]
        return float(np.median(big))

    cf, cw = copy_reading(cal_fetch_dir), copy_reading(cal_write_dir)
    fs, ws = COPY_BYTES / (cf * kib), COPY_BYTES / (cw * kib)
    print(f"copy_probe_fetch_kib: {cf:.1f}")
    print(f"copy_probe_write_kib: {cw:.1f}")
    print(f"fetch_scale: {fs:.4f}")
    print(f"write_scale: {ws:.4f}")
    print(f"source_sha256: {kernel_source_sha()}")
    F, Wr = _pmc(fetch_dir), _pmc(write_dir)
    print("%-44s %6s %12s %12s %14s" % ("kernel", "n", "FETCH_KiB", "WRITE_KiB", "bytes/launch"))
    stage = {"float": [], "double": []}
    for k in sorted(F, key=lambda s: -np.mean(F[s])):
        if k not in Wr:
            continue
        f, wv = float(np.mean(F[k])), float(np.mean(Wr[k]))
        tb = (f * fs + wv * ws) * kib
        print("%-44s %6d %12.1f %12.1f %14.4g" % (_short(k)[:44], len(F[k]), f, wv, tb))
        m = re.search(r"stage_kernel<(float|double), (\d)", k)
        if m:
            stage[m.group(1)].append((len(F[k]), tb))
    for t, prec in (("float", "fp32"), ("double", "fp64")):
        if stage[t]:
            n = sum(c for c, _ in stage[t])
            avg = sum(c * b for c, b in stage[t]) / n
            print(f"traffic_bytes_per_stage_launch_{prec}: {avg:.6g}")


def instr_summary(dirname):
    """Per-wave instruction counts and VALU busy fraction per kernel from an
    SQ counter pass (SQ_WAVES, SQ_INSTS_VALU/SALU/LDS, SQ_ACTIVE_INST_VALU,
    SQ_BUSY_CYCLES, SQ_WAIT_INST_ANY)."""
    agg = {}
    for fn in os.listdir(dirname):
        if fn.endswith("counter_collection.csv"):
            for r in csv.DictReader(open(os.path.join(dirname, fn))):
                d = agg.setdefault(_short(r["Kernel_Name"])[:40], {})
                d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    print("%-40s %7s %9s %9s %8s %8s %9s" % ("kernel", "waves", "VALU/wv", "SALU/wv", "LDS/wv",
                                             "VALUbusy", "wait/wv"))
    for k in sorted(agg):
        a = {c: sum(x) / len(x) for c, x in agg[k].items()}
        w = a.get("SQ_WAVES", 0)
        if not w or "SQ_INSTS_VALU" not in a:
            continue
        # 4 cycles per wave64 VALU instruction on a SIMD16; 1024 SIMDs; the
        # busy-cycle counter sums the 32 shader engines
        busy = a["SQ_ACTIVE_INST_VALU"] * 4 / 1024 / (a["SQ_BUSY_CYCLES"] / 32)
        print("%-40s %7.0f %9.0f %9.0f %8.0f %7.0f%% %9.0f" % (
            k, w, a["SQ_INSTS_VALU"] / w, a["SQ_INSTS_SALU"] / w, a["SQ_INSTS_LDS"] / w,
            100 * busy, a["SQ_WAIT_INST_ANY"] / w))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="paper-scale-256")
    ap.add_argument("--prec", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--periods", type=int, default=20,
                    help="adjoint-64: drive periods the loss averages over")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the reverse-mode step cost in the default line")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-replayed step (a kernel trace then holds only the timed launches)")
    ap.add_argument("--one-by-one", action="store_true",
                    help="launch the warm-up and timed steps one by one too, as the profiled pass "
                         "is (for kernel traces; ms_per_step is then that schedule's)")
    ap.add_argument("--no-force-precision", action="store_true",
                    help="skip the FP32-against-FP64 averaged-force leg of the default line")
    ap.add_argument("--force-steps", type=int, default=20000,
                    help="steps of each run of the averaged-force precision leg")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--stats-summary", metavar="CSV")
    ap.add_argument("--timeline-summary", metavar="TRACE_CSV",
                    help="median schedule of one step from a rocprofv3 kernel trace of this "
                         "script (give the run's --steps and --warmup)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH", "WRITE", "CAL_FETCH", "CAL_WRITE"))
    ap.add_argument("--instr-summary", metavar="DIR")
    args = ap.parse_args()
    if args.instr_summary:
        return instr_summary(args.instr_summary)
    if args.stats_summary:
        return stats_summary(args.stats_summary)
    if args.timeline_summary:
        return timeline_summary(args.timeline_summary, args.warmup, args.steps)
    if args.pmc_summary:
        return pmc_summary(*args.pmc_summary)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the IC step here "
              "is a single-GPU build; the design notes describe how it would shard.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        return copy_probe()
    if args.workload == "ensemble-64":
        print(json.dumps(run_ensemble("fp32" if args.prec == "both" else args.prec, args.steps,
                                      args.warmup)), flush=True)
        return
    if args.workload == "gibbs-boltzmann":
        print(json.dumps(run_gibbs_boltzmann(args.steps, args.warmup)), flush=True)
        return
    if args.workload == "force-sweeps-32":
        print(json.dumps(run_force_sweeps()), flush=True)
        return
    if args.workload == "table1":
        print(json.dumps(run_table1(log)), flush=True)
        return
    if args.workload == "gorkov-single-32":
        from paper_1307_0702_amd.experiments import gorkov_single_32
        r = gorkov_single_32()
        log(f"[bench] one particle, eta = zeta = 0.5: F_x {r['force'][0]:.4e}, Gor'kov "
            f"{r['gorkov']:.4e}, ratio {r['ratio']:.3f}")
        print(json.dumps(dict(metric="averaged spring force against Gor'kov, one particle",
                              value=r["ratio"], unit="F / F_Gorkov", n_gpus=1, dtype="f64",
                              data="synthetic", higher_is_better=False,
                              config=dict(workload="gorkov-single-32", grid=[32, 32, 32], eta=0.5,
                                          zeta=0.5, particles=1, steps=1000), **r)), flush=True)
        return
    if args.workload == "force-precision-256":
        print(json.dumps(run_force_precision(args.steps)), flush=True)
        return
    if args.workload == "force-precision-256-thermal":
        print(json.dumps(run_force_precision(args.steps, kT=1e-3)), flush=True)
        return
    if args.workload == "adjoint-64":
        for prec in (["fp32", "fp64"] if args.prec == "both" else [args.prec]):
            print(json.dumps(run_adjoint_particles(prec, args.periods, fd_check=prec == "fp64")),
                  flush=True)
        return
    if args.workload == "adjoint-256":
        for prec in (["fp32", "fp64"] if args.prec == "both" else [args.prec]):
            print(json.dumps(run_adjoint(prec, args.steps, args.warmup)), flush=True)
        return
    log(f"[bench] building inputs for {args.workload}")
    w = make_workload(args.workload)
    fl = w.fluid
    res = {}
    precs = ["fp32", "fp64"] if args.prec == "both" else [args.prec]
    for prec in precs:
        res[prec] = run_gpu(w, prec, args.steps, args.warmup, graph=not args.no_graph,
                            one_by_one=args.one_by_one)
    main_prec = precs[0]
    r = res[main_prec]
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
        graph_ms_per_step=r["graph_ms_per_step"],
        roofline=roofline(r, main_prec),
    )
    if args.one_by_one:
        out["schedule"] = "every step launched one by one"
    if not args.no_adjoint:
        # the reverse-mode cost of the metric: one reversed step with
        # particles against one forward step (adjoint-64 workload)
        adj = {}
        for prec in precs:
            f_ms, r_ms = adjoint_step_cost(prec)
            adj[prec] = dict(forward_step_ms=f_ms, adjoint_step_ms=r_ms, ratio=r_ms / f_ms)
            log(f"[bench] adjoint-64 {prec}: forward {f_ms:.3f} ms, reversed {r_ms:.3f} ms, ratio {r_ms / f_ms:.2f}")
        out["adjoint"] = dict(workload="adjoint-64 (64^3, 16 tethered particles, four drives, kT = 0)", **adj)
    if "fp64" in res and main_prec != "fp64":
        r64 = res["fp64"]
        out["fp64"] = dict(value=r64["cell_updates_per_s"], ms_per_step=r64["ms_per_step"],
                           graph_ms_per_step=r64["graph_ms_per_step"],
                           roofline=roofline(r64, "fp64"))
        out["speedup_fp32_over_fp64"] = r["cell_updates_per_s"] / r64["cell_updates_per_s"]
    out["finite"] = all(x["finite"] for x in res.values())
    if not args.no_force_precision and w.name == "paper-scale-256":
        # the metric's precision claim: FP32 against FP64 on this
        # configuration at kT = 0, averaged spring forces over 7 periods
        fp = run_force_precision(args.force_steps)
        out["force_precision"] = dict(
            workload="paper-scale-256 at kT = 0", steps=fp["steps"],
            averaged_steps=fp["config"]["averaged_steps"],
            force_rel_err_max=fp["force_rel_err_max"], force_rel_err_rms=fp["force_rel_err_rms"],
            fp32_ms_per_step=fp["ms_per_step"], fp64_ms_per_step=fp["fp64_ms_per_step"],
            speedup_fp32_over_fp64=fp["value"])
        log(f"[bench] force precision: rel err {fp['force_rel_err_max']:.2e} (max), "
            f"speed-up {fp['value']:.2f}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
