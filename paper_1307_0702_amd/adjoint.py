"""Gradients through the deterministic IC step (kT = 0).

`Adjoint` owns the reverse-mode workspace of a Simulation and runs the
adjoint steps of libic.so backwards over a trajectory: ic_adjoint_step for a
particle-free context, ic_adjoint_step_particles (the whole step with the
particle coupling) when particles are set.  Forward states (fields, and
particle positions and velocities) are kept only at checkpoints every
`every` steps; each segment is re-stepped forward from its checkpoint before
it is reversed, so memory is (N / every + every) states for N steps.

`rollout` wraps the particle-free case in a torch.autograd.Function: the
output is the state after nsteps steps from U0 with drive amplitudes `amps`,
and backward returns dL/dU0 and dL/damps.  `rollout_particles` does the same
with particles: outputs the state, positions, velocities and the mean force
F^{n+1/2} = -k_s minimg(q^{n+1/2} - q_eq) + f_ext over the steps (the
radiation-force estimator of Sec. VI), differentiable also in the initial
positions and velocities, the excess masses m_e and the energies eps_pf.
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

    def __del__(self):
        # the context must not keep pointers into the workspace torch frees
        sim = getattr(self, "sim", None)
        if sim is not None and getattr(sim, "ctx", None) is not None:
            try:
                sim.synchronize()
                ic.ic_bind_adjoint(sim.ctx, None, 0)
            except Exception:
                pass

    def step(self, n, U, lam, q=None, u=None, lq=None, lu=None, lF=None):
        """lam := dL/dU^n from lam = dL/dU^{n+1}; U = U^n (4 device fields).
        With particles set, also q, u = the particle state of step n and
        lq, lu := dL/d(q, u)^n from dL/d(q, u)^{n+1} ([np][3] float64 device
        tensors), lF = dL/dF^{n+1/2} of this step or None."""
        if self.sim.np == 0:
            ic.ic_adjoint_step(self.sim.ctx, n, [U[i] for i in range(4)], [lam[i] for i in range(4)])
        else:
            ic.ic_adjoint_step_particles(self.sim.ctx, n, [U[i] for i in range(4)], q, u,
                                         [lam[i] for i in range(4)], lq, lu, lF)

    def drive_grad(self, nmodes, reset=False):
        return ic.ic_adjoint_drive(self.sim.ctx, nmodes, reset)

    def particle_grad(self, reset=False):
        """Accumulated (dL/dm_e, dL/deps_pf, dL/dk_s) per particle."""
        return ic.ic_adjoint_particle_grad(self.sim.ctx, self.sim.np, reset)

    def snapshot(self):
        """(U, q, u) of the bound state, copies on the device (q, u None
        without particles)."""
        sim = self.sim
        U = sim.U.clone()
        if sim.np == 0:
            return U, None, None
        t = sim.torch
        q = t.empty((sim.np, 3), dtype=t.float64, device=sim.device)
        u = t.empty_like(q)
        ic.ic_copy_particles(sim.ctx, q, u)
        return U, q, u

    def restore(self, state, n):
        U, q, u = state
        self.sim.U.copy_(U)
        if q is not None:
            ic.ic_load_particles(self.sim.ctx, q, u)
        self.sim.set_step(n)

    def state_bytes(self):
        """Device bytes of one checkpoint (fields, positions, velocities)."""
        sim = self.sim
        return sim.U.numel() * sim.U.element_size() + 2 * 3 * 8 * sim.np

    def auto_every(self, nsteps, fraction=0.5):
        """Checkpoint spacing for nsteps steps: 1 (every state kept, no
        re-stepping in the reversal) when the whole trajectory fits in
        `fraction` of the free device memory, else 64."""
        free, _ = self.sim.torch.cuda.mem_get_info(self.sim.device)
        return 1 if nsteps * self.state_bytes() <= fraction * free else 64

    def forward(self, U0, n0, nsteps, every=64, q0=None, u0=None):
        """Steps the simulation from U0 (and, with particles, q0, u0) at step
        n0; returns the final fields and the checkpoints {step: (U, q, u)}.
        every="auto" picks the spacing with auto_every.  The final particle
        state is in self.final."""
        if every == "auto":
            every = self.auto_every(nsteps)
        self.every = every
        self.restore((U0, q0, u0), n0)
        ckpt = {}
        for s in range(nsteps):
            if s % every == 0:
                ckpt[n0 + s] = self.snapshot()
            self.sim.step(1)
        self.final = self.snapshot()
        return self.final[0], ckpt

    def backward(self, lam, n0, nsteps, ckpt, every=64, lq=None, lu=None, lF=None):
        """lam (4 device fields, dL/dU^{n0+nsteps}) becomes dL/dU^{n0} in
        place, and with particles lq, lu likewise; lF (dL/dF^{n+1/2}, the
        same for every step) or None.  Returns lam.  The drive and particle
        parameter gradients accumulate in the workspace (drive_grad,
        particle_grad).  Re-stepping overwrites the bound state and the step
        counter."""
        sim = self.sim
        if every == "auto":
            every = self.every
        starts = sorted(ckpt)
        for c0 in reversed(starts):
            seg = min(every, n0 + nsteps - c0)
            states = [ckpt[c0]]
            if seg > 1:
                self.restore(ckpt[c0], c0)
                for _ in range(seg - 1):
                    sim.step(1)
                    states.append(self.snapshot())
            for k in reversed(range(seg)):
                U, q, u = states[k]
                self.step(c0 + k, U, lam, q, u, lq, lu, lF)
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
                ctx.adj, ctx.ck, ctx.n0, ctx.ns, ctx.every = adj_, ck, n0_, nsteps_, adj_.every
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


class _RolloutParticles:
    fn = None


def rollout_particles(adj, U0, q0, u0, amps, me, eps, modes, n0, nsteps, every=64,
                      ks=None, qeq=None, fext=None):
    """(U, q, u) after nsteps steps from (U0, q0, u0) and the mean of
    F^{n+1/2} over the steps ([np][3]), with drive amplitudes amps and
    particle parameters me, eps (CPU float64 tensors); U0 (4, nz, ny, nx),
    q0, u0 ([np][3] float64) on the device.  Differentiable in U0, q0, u0,
    amps, me and eps; ks, qeq, fext (numpy or None) are held fixed."""
    import torch

    if _RolloutParticles.fn is None:
        class Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, U0_, q0_, u0_, amps_, me_, eps_, adj_, modes_, n0_, nsteps_, every_, fixed_):
                sim = adj_.sim
                md = [dict(m) for m in modes_]
                for m, a in zip(md, amps_.tolist()):
                    m["amp"] = a
                sim.set_forcing(md)
                ks_, qeq_, fext_ = fixed_
                q_host = q0_.detach().cpu().numpy()
                u_host = u0_.detach().cpu().numpy()
                me_h, eps_h = me_.detach().numpy().copy(), eps_.detach().numpy().copy()
                sim.set_particles(q_host, me_h, eps_h, u=u_host, ks=ks_, qeq=qeq_, fext=fext_)
                # the particle set and parameters of this trajectory: backward
                # re-steps and reverses with them, whatever the shared context
                # holds by then (another rollout may have run in between)
                ctx.particles = (q_host, me_h, eps_h, u_host,
                                 None if ks_ is None else np.array(ks_, dtype=np.float64),
                                 None if qeq_ is None else np.array(qeq_, dtype=np.float64),
                                 None if fext_ is None else np.array(fext_, dtype=np.float64))
                UN, ck = adj_.forward(U0_.detach(), n0_, nsteps_, every_, q0_.detach(), u0_.detach())
                tether, _, _ = sim.avg_force(reset=True)   # mean of k_s minimg(q^{n+1/2} - q_eq)
                f0 = np.zeros((sim.np, 3)) if fext_ is None else np.asarray(fext_, dtype=np.float64)
                Fmean = torch.as_tensor(f0 - tether, dtype=torch.float64, device=U0_.device)
                ctx.adj, ctx.ck, ctx.n0, ctx.ns, ctx.every = adj_, ck, n0_, nsteps_, adj_.every
                ctx.md = md
                _, qN, uN = adj_.final
                return UN, qN, uN, Fmean

            @staticmethod
            def backward(ctx, gU, gq, gu, gF):
                a = ctx.adj
                sim = a.sim
                q_h, me_h, eps_h, u_h, ks_h, qeq_h, fext_h = ctx.particles
                sim.set_particles(q_h, me_h, eps_h, u=u_h, ks=ks_h, qeq=qeq_h, fext=fext_h)
                a.sim.set_forcing(ctx.md)
                a.drive_grad(len(ctx.md), reset=True)
                a.particle_grad(reset=True)
                dev = sim.device

                def z(g, shape, dtype):
                    if g is None:
                        return torch.zeros(shape, dtype=dtype, device=dev)
                    return g.detach().to(device=dev, dtype=dtype).contiguous().clone()

                lam = z(gU, (4,) + sim.shape, sim.dtype)
                lq = z(gq, (sim.np, 3), torch.float64)
                lu = z(gu, (sim.np, 3), torch.float64)
                lF = None if gF is None else (gF.detach().to(device=dev, dtype=torch.float64) / ctx.ns).contiguous()
                a.backward(lam, ctx.n0, ctx.ns, ctx.ck, ctx.every, lq, lu, lF)
                dA = a.drive_grad(len(ctx.md), reset=True)
                dme, deps, _ = a.particle_grad(reset=True)
                t64 = torch.float64
                return (lam, lq, lu, torch.as_tensor(np.asarray(dA), dtype=t64),
                        torch.as_tensor(dme, dtype=t64), torch.as_tensor(deps, dtype=t64),
                        None, None, None, None, None, None)

        _RolloutParticles.fn = Fn
    return _RolloutParticles.fn.apply(U0, q0, u0, amps, me, eps, adj, modes, n0, nsteps, every,
                                      (ks, qeq, fext))
