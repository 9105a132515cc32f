"""Ensembles of independent IC runs in one HIP-graph launch.

An ensemble is a list of workloads (replicas with their own noise seed or
replica id, contrast sweeps, uneven grids and particle counts).  Each gets its
own context; `Ensemble.capture(nsteps)` records nsteps steps of every context
into one graph with one dependency chain per context (ic_graph_create), so a
single `Ensemble.run` launch advances all of them and the chains run
concurrently on the GPU.  Small grids cannot fill the chip alone; together
they can.

`autotune_tile` is the tile-shape tuner for a context stepped on its own: for
each grid shape it times the step at every allowed z extent of the stage
tile (4, 8, 16, 32 planes) and keeps the fastest.  Results are cached per
(grid, precision, particles).  `Ensemble.tune_batch` tunes the extent for the
batched graph instead, where the members together fill the GPU: it times
graph replays with one extent for every member and keeps the fastest.
"""
from __future__ import annotations

import time

import numpy as np

from . import ic

TILE_CHOICES = (4, 8, 16, 32)
_tile_cache = {}


def _make_sim(w, prec):
    fl, p = w.fluid, w.particles
    sim = ic.Simulation(fl, prec=prec, max_particles=max(p.n, 1))
    sim.set_state(w.drho, w.g)
    if p.n:
        eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
        sim.set_particles(p.q, p.me, eps, u=p.u, ks=p.ks, qeq=p.qeq, fext=p.fext)
    if w.modes:
        sim.set_forcing([m.as_dict() for m in w.modes])
    return sim


def autotune_tile(w, prec="fp32", steps=10, warmup=2):
    """Fastest stage-tile z extent for workload w's grid and particle count."""
    key = (w.fluid.shape, prec, w.particles.n)
    if key in _tile_cache:
        return _tile_cache[key]
    sim = _make_sim(w, prec)
    best, best_t = None, float("inf")
    for tz in TILE_CHOICES:
        if tz > 2 * w.fluid.nz:
            continue
        sim.set_tile(tz)
        sim.step(warmup)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        t = time.perf_counter() - t0
        if t < best_t:
            best, best_t = tz, t
    del sim
    _tile_cache[key] = best
    return best


class Ensemble:
    def __init__(self, workloads, prec="fp32", tune=True):
        self.workloads = list(workloads)
        self.sims = [_make_sim(w, prec) for w in self.workloads]
        self.tiles = []
        for w, s in zip(self.workloads, self.sims):
            tz = autotune_tile(w, prec) if tune else s.tile()
            s.set_tile(tz)
            self.tiles.append(tz)
        self.graph = None
        self.nsteps = 0

    @property
    def cells(self):
        return sum(w.fluid.nx * w.fluid.ny * w.fluid.nz for w in self.workloads)

    def tune_batch(self, nsteps=10, replays=3):
        """Stage-tile z extent for the batched graph: the same extent for
        every member, the one whose graph replays run fastest.  The steps
        taken while timing advance the members (callers tune before their
        measured or compared steps)."""
        import torch
        best, best_t = None, float("inf")
        for tz in TILE_CHOICES:
            for s in self.sims:
                s.set_tile(tz)
            self.capture(nsteps)
            self.run()
            self.synchronize()
            t0 = time.perf_counter()
            self.run(replays)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if t < best_t:
                best, best_t = tz, t
        for s in self.sims:
            s.set_tile(best)
        self.tiles = [best] * len(self.sims)
        self.release()
        return best

    def capture(self, nsteps):
        self.release()
        self.graph = ic.ic_graph_create([s.ctx for s in self.sims], nsteps)
        self.nsteps = nsteps

    def run(self, replays=1):
        """replays x nsteps steps of every member in one graph launch each."""
        stream = self.sims[0].stream.cuda_stream
        for _ in range(replays):
            ic.ic_graph_launch(self.graph, stream)

    def run_serial(self, nsteps):
        """The same steps, member after member, without the graph."""
        for s in self.sims:
            s.step(nsteps)

    def synchronize(self):
        for s in self.sims:
            s.synchronize()

    def release(self):
        if self.graph is not None:
            ic.ic_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
