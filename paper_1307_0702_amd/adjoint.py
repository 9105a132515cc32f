"""Gradients through the deterministic IC fluid step (kT = 0, no particles).

`Adjoint` owns the reverse-mode workspace of a Simulation and runs the
adjoint steps of libic.so (ic_adjoint_step) backwards over a trajectory.
Forward states are kept only at checkpoints every `every` steps; each segment
is re-stepped forward from its checkpoint before it is reversed, so memory is
(N / every + every) states for N steps.

`rollout` wraps this in a torch.autograd.Function: the output is the state
after nsteps steps from U0 with drive amplitudes `amps`, and backward returns
dL/dU0 and dL/damps.
"""
from __future__ import annotations

import numpy as np

from . import ic


class Adjoint:
    def __init__(self, sim):
        t = sim.torch
        self.sim = sim
        nbytes = ic.ic_adjoint_workspace_size(sim.params)
        with t.cuda.device(sim.device):
            self._raw = t.empty(nbytes + 256, dtype=t.uint8, device=sim.device)
            off = (-self._raw.data_ptr()) % 256
            self.ws = self._raw[off:off + nbytes]
            ic.ic_bind_adjoint(sim.ctx, self.ws, nbytes)

    def step(self, n, U, lam):
        """lam := dL/dU^n from lam = dL/dU^{n+1}; U = U^n (4 device fields)."""
        ic.ic_adjoint_step(self.sim.ctx, n, [U[i] for i in range(4)], [lam[i] for i in range(4)])

    def drive_grad(self, nmodes, reset=False):
        return ic.ic_adjoint_drive(self.sim.ctx, nmodes, reset)

    def forward(self, U0, n0, nsteps, every=64):
        """Steps the simulation from U0 at step n0; returns the final state
        and the checkpoints {step: state}."""
        sim = self.sim
        sim.U.copy_(U0)
        sim.set_step(n0)
        ckpt = {}
        for s in range(nsteps):
            if s % every == 0:
                ckpt[n0 + s] = sim.U.clone()
            sim.step(1)
        return sim.U.clone(), ckpt

    def backward(self, lam, n0, nsteps, ckpt, every=64):
        """lam (4 device fields, dL/dU^{n0+nsteps}) becomes dL/dU^{n0} in
        place; returns it.  The drive gradient accumulates in the workspace
        (drive_grad).  Re-stepping overwrites the bound state and the step
        counter."""
        sim = self.sim
        starts = sorted(ckpt)
        for c0 in reversed(starts):
            seg = min(every, n0 + nsteps - c0)
            states = [ckpt[c0]]
            sim.U.copy_(ckpt[c0])
            sim.set_step(c0)
            for _ in range(seg - 1):
                sim.step(1)
                states.append(sim.U.clone())
            for k in reversed(range(seg)):
                self.step(c0 + k, states[k], lam)
        return lam


class _Rollout:
    fn = None


def rollout(adj, U0, amps, modes, n0, nsteps, every=64):
    """U^{n0+nsteps} from U0 (a (4, nz, ny, nx) device tensor) with the drive
    amplitudes amps (a CPU float64 tensor, one per mode; the other mode
    fields from `modes`), differentiable in U0 and amps."""
    import torch

    if _Rollout.fn is None:
        class Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, U0_, amps_, adj_, modes_, n0_, nsteps_, every_):
                md = [dict(m) for m in modes_]
                for m, a in zip(md, amps_.tolist()):
                    m["amp"] = a
                adj_.sim.set_forcing(md)
                UN, ck = adj_.forward(U0_.detach(), n0_, nsteps_, every_)
                ctx.adj, ctx.ck, ctx.n0, ctx.ns, ctx.every = adj_, ck, n0_, nsteps_, every_
                ctx.nmodes = len(md)
                ctx.md = md
                return UN

            @staticmethod
            def backward(ctx, gout):
                a = ctx.adj
                a.sim.set_forcing(ctx.md)
                a.drive_grad(ctx.nmodes, reset=True)
                lam = gout.detach().to(a.sim.dtype).contiguous().clone()
                a.backward(lam, ctx.n0, ctx.ns, ctx.ck, ctx.every)
                dA = a.drive_grad(ctx.nmodes, reset=True)
                return lam, torch.as_tensor(np.asarray(dA), dtype=torch.float64), None, None, None, None, None

        _Rollout.fn = Fn
    return _Rollout.fn.apply(U0, amps, adj, modes, n0, nsteps, every)
