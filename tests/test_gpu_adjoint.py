"""Reverse mode of the deterministic IC fluid step (ic_adjoint_*), through the
C ABI, against the FP64 reverse-mode oracle (oracle/ic_adjoint.py) and
against central differences of the GPU forward step.

Bars: FP64 max|x_gpu - x_oracle| / max|x_oracle| <= 1e-12 per field for one
step and <= 1e-11 over a checkpointed multi-step reversal; FP32 <= 1e-5 for
one step (stage inputs recomputed in FP32); drive-amplitude gradients to the
same relative bars.
"""
import numpy as np
import pytest

from oracle import ic_adjoint as OA
from paper_1307_0702_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


MODES = [dict(axis=0, shape="cos", m=1, x0=1.5, amp=3e-3, omega=0.2, phase=0.3),
         dict(axis=2, shape="plane", m=1, x0=4.0, amp=2e-3, omega=0.7, phase=0.0),
         dict(axis=1, shape="cos", m=2, x0=0.0, amp=1e-3, omega=0.35, phase=1.1)]


def _setup(nx, ny, nz, prec, seed, modes=MODES):
    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation
    fl = W.Fluid(nx, ny, nz, kT=0.0, seed=seed)
    drho, g = W.random_fields(fl.shape, seed)
    lr, lg = W.random_fields(fl.shape, seed + 1, 1.0, 1.0)
    if prec == "fp32":
        # FP32-representable inputs on both sides
        drho, g = drho.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
        lr, lg = lr.astype(np.float32).astype(np.float64), lg.astype(np.float32).astype(np.float64)
    sim = Simulation(fl, prec=prec, max_particles=1)
    if modes:
        sim.set_forcing(modes)
    return fl, sim, Adjoint(sim), drho, g, lr, lg


def _dev(sim, drho, g):
    t = sim.torch
    U = t.empty((4,) + sim.shape, dtype=sim.dtype, device=sim.device)
    U[0].copy_(t.as_tensor(drho))
    for a in range(3):
        U[1 + a].copy_(t.as_tensor(g[a]))
    return U


def _rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def _errs(lam, er, eg):
    got = lam.detach().cpu().double().numpy()
    e = {"drho": _rel(got[0], er)}
    for a in range(3):
        e["g%d" % a] = _rel(got[1 + a], eg[a])
    return e


@pytest.mark.parametrize("prec,shape,tol", [
    ("fp64", (37, 21, 11), 1e-12),
    ("fp64", (64, 32, 20), 1e-12),
    ("fp64", (5, 4, 4), 1e-12),
    ("fp32", (37, 21, 11), 1e-5),
    ("fp32", (64, 32, 40), 1e-5),
])
def test_one_adjoint_step_matches_oracle(prec, shape, tol):
    from paper_1307_0702_amd import ic
    nx, ny, nz = shape
    print(f"adjoint step vs oracle {prec} {shape}", flush=True)
    fl, sim, adj, drho, g, lr, lg = _setup(nx, ny, nz, prec, 700 + nx)
    n = 5
    U = _dev(sim, drho, g)
    lam = _dev(sim, lr, lg)
    bound_before = sim.U.clone()
    sim.set_step(17)
    adj.step(n, U, lam)
    dA = adj.drive_grad(len(MODES), reset=True)
    sim.synchronize()
    er, eg, eA = OA.step_vjp(drho, list(g), fl.as_dict(), MODES, n, lr, list(lg))
    errs = _errs(lam, er, eg)
    errs["dA"] = _rel(dA, eA)
    print("  ", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    # the bound state and the step counter are untouched
    assert sim.torch.equal(sim.U, bound_before)
    assert ic.ic_get_step(sim.ctx) == 17


def test_adjoint_without_drives_matches_oracle():
    fl, sim, adj, drho, g, lr, lg = _setup(24, 17, 9, "fp64", 91, modes=[])
    U = _dev(sim, drho, g)
    lam = _dev(sim, lr, lg)
    adj.step(0, U, lam)
    er, eg, _ = OA.step_vjp(drho, list(g), fl.as_dict(), [], 0, lr, list(lg))
    errs = _errs(lam, er, eg)
    print("  ", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= 1e-12


def test_checkpointed_reversal_matches_oracle_run_grad():
    fl, sim, adj, drho, g, lr, lg = _setup(40, 24, 18, "fp64", 811)
    n0, nsteps = 3, 8
    U0 = _dev(sim, drho, g)
    UN, ck = adj.forward(U0, n0, nsteps, every=3)
    assert sorted(ck) == [3, 6, 9]
    lam = _dev(sim, lr, lg)
    adj.drive_grad(len(MODES), reset=True)
    adj.backward(lam, n0, nsteps, ck, every=3)
    dA = adj.drive_grad(len(MODES), reset=True)
    er, eg, eA, (rN, gN) = OA.run_grad(drho, list(g), fl.as_dict(), MODES, nsteps, lr, list(lg), n0=n0)
    fwd = UN.cpu().numpy()
    ferr = max([_rel(fwd[0], rN)] + [_rel(fwd[1 + a], gN[a]) for a in range(3)])
    errs = _errs(lam, er, eg)
    errs["dA"] = _rel(dA, eA)
    errs["forward"] = ferr
    print("  ", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= 1e-11, (k, v)


def test_rollout_gradients_match_central_differences_of_the_gpu_forward():
    import torch
    from paper_1307_0702_amd.adjoint import rollout
    fl, sim, adj, drho, g, lr, lg = _setup(24, 20, 16, "fp64", 905)
    n0, nsteps = 2, 6
    U0 = _dev(sim, drho, g)
    C = _dev(sim, lr, lg)
    amps = torch.tensor([m["amp"] for m in MODES], dtype=torch.float64)

    def loss(U0_, amps_):
        return float((rollout(adj, U0_, amps_, MODES, n0, nsteps, every=4) * C).sum())

    U0r = U0.clone().requires_grad_(True)
    ar = amps.clone().requires_grad_(True)
    out = rollout(adj, U0r, ar, MODES, n0, nsteps, every=4)
    (out * C).sum().backward()
    gU, gA = U0r.grad, ar.grad
    rng = np.random.default_rng(906)
    d = torch.as_tensor(1e-2 * rng.standard_normal(U0.shape), device=U0.device)
    eps = 1e-3
    fd = (loss(U0 + eps * d, amps) - loss(U0 - eps * d, amps)) / (2 * eps)
    an = float((gU * d).sum())
    print(f"  state: fd {fd:.12e} adjoint {an:.12e}", flush=True)
    assert abs(fd - an) <= 1e-8 * abs(an)
    for m in range(len(MODES)):
        e = torch.zeros_like(amps)
        e[m] = 1e-5
        fd = (loss(U0, amps + e) - loss(U0, amps - e)) / 2e-5
        print(f"  amp {m}: fd {fd:.12e} adjoint {float(gA[m]):.12e}", flush=True)
        assert abs(fd - float(gA[m])) <= 1e-6 * abs(fd) + 1e-9


def test_adjoint_error_paths():
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation
    fl = W.Fluid(16, 16, 16, kT=0.0, seed=3)
    sim = Simulation(fl, prec="fp64", max_particles=4)
    U = sim.U.clone()
    lam = sim.U.clone()
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_step(sim.ctx, 0, list(U), list(lam))
    assert e.value.code == ic.IC_E_STATE          # workspace not bound
    adj = Adjoint(sim)
    with pytest.raises(ic.ICError) as e:
        adj.step(-1, U, lam)
    assert e.value.code == ic.IC_E_ARG
    sim.set_particles(np.array([[3.0, 4.0, 5.0]]), np.array([0.0]), np.array([0.0]))
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_step(sim.ctx, 0, list(U), list(lam))
    assert e.value.code == ic.IC_E_STATE          # particles set: the particle entry point is needed
    hot = Simulation(W.Fluid(16, 16, 16, kT=1e-3, seed=3), prec="fp64")
    hadj = Adjoint(hot)
    with pytest.raises(ic.ICError) as e:
        hadj.step(0, hot.U.clone(), hot.U.clone())
    assert e.value.code == ic.IC_E_STATE          # kT != 0
    with pytest.raises(ic.ICError) as e:
        ic.ic_bind_adjoint(sim.ctx, adj.ws, 16)
    assert e.value.code == ic.IC_E_ARG


def test_workspace_is_unbound_when_the_adjoint_object_goes():
    import gc
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation
    sim = Simulation(W.Fluid(16, 16, 16, kT=0.0, seed=4), prec="fp64")
    U, lam = sim.U.clone(), sim.U.clone()
    adj = Adjoint(sim)
    adj.step(0, U, lam)
    del adj
    gc.collect()
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_step(sim.ctx, 0, list(U), list(lam))
    assert e.value.code == ic.IC_E_STATE and "not bound" in str(e.value)
