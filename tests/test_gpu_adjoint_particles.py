"""Reverse mode of the whole IC step with particles
(ic_adjoint_step_particles), through the C ABI, against the FP64 reverse-mode
oracle (oracle/ic_adjoint.py: step_vjp_particles, run_grad_particles) and
against central differences of the GPU forward step.

Bars: FP64 max|x_gpu - x_oracle| / max|x_oracle| <= 1e-12 per field and per
particle quantity for one reversed step, <= 1e-11 over a checkpointed
multi-step reversal; FP32 (fields in FP32, particle algebra in FP64) <= 1e-5
for one reversed step from FP32-representable inputs.
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
         dict(axis=2, shape="plane", m=1, x0=4.0, amp=2e-3, omega=0.7, phase=0.0)]


def _particles(fl, n, seed):
    """n particles, the first two with overlapping kernel supports; masses
    and energies on both sides of the fluid's."""
    rng = np.random.default_rng(seed)
    L = np.array([fl.nx, fl.ny, fl.nz], dtype=np.float64)
    q = rng.uniform(0.0, 1.0, (n, 3)) * L
    if n > 1:
        q[1] = (q[0] + np.array([1.3, -0.8, 1.1])) % L
    return dict(q=q, u=1e-2 * rng.standard_normal((n, 3)), me=rng.uniform(-4.0, 8.0, n),
                eps=rng.uniform(-0.5, 1.0, n), ks=rng.uniform(0.0, 0.5, n),
                qeq=(q + rng.uniform(-0.5, 0.5, (n, 3))) % L, fext=1e-3 * rng.standard_normal((n, 3)))


def _setup(shape, prec, seed, npart=6):
    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation
    nx, ny, nz = shape
    fl = W.Fluid(nx, ny, nz, kT=0.0, seed=seed)
    drho, g = W.random_fields(fl.shape, seed)
    lr, lg = W.random_fields(fl.shape, seed + 1, 1.0, 1.0)
    if prec == "fp32":
        drho, g = drho.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
        lr, lg = lr.astype(np.float32).astype(np.float64), lg.astype(np.float32).astype(np.float64)
    P = _particles(fl, npart, seed + 2)
    rng = np.random.default_rng(seed + 3)
    seeds = dict(lq=rng.standard_normal((npart, 3)), lu=rng.standard_normal((npart, 3)),
                 lF=rng.standard_normal((npart, 3)))
    sim = Simulation(fl, prec=prec, max_particles=npart)
    sim.set_particles(P["q"], P["me"], P["eps"], u=P["u"], ks=P["ks"], qeq=P["qeq"], fext=P["fext"])
    sim.set_forcing(MODES)
    return fl, sim, Adjoint(sim), drho, g, lr, lg, P, seeds


def _dev(sim, drho, g):
    t = sim.torch
    U = t.empty((4,) + sim.shape, dtype=sim.dtype, device=sim.device)
    U[0].copy_(t.as_tensor(drho))
    for a in range(3):
        U[1 + a].copy_(t.as_tensor(g[a]))
    return U


def _d64(sim, x):
    return sim.torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=sim.device)


def _rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def _state(drho, g, P, n):
    return dict(drho=drho, g=list(g), n=n, q=P["q"], u=P["u"], me=P["me"], eps=P["eps"],
                ks=P["ks"], qeq=P["qeq"], fext=P["fext"])


def _compare(sim, adj, lam, lq, lu, want, nmodes):
    got = lam.detach().cpu().double().numpy()
    e = {"drho": _rel(got[0], want["lr"])}
    for a in range(3):
        e["g%d" % a] = _rel(got[1 + a], want["lg"][a])
    e["q"] = _rel(lq.cpu().numpy(), want["lq"])
    e["u"] = _rel(lu.cpu().numpy(), want["lu"])
    dme, deps, dks = adj.particle_grad(reset=True)
    e["me"] = _rel(dme, want["dme"])
    e["eps"] = _rel(deps, want["deps"])
    e["ks"] = _rel(dks, want["dks"])
    e["A"] = _rel(adj.drive_grad(nmodes, reset=True), want["dA"])
    print("  ", {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    return e


@pytest.mark.parametrize("prec,shape,tol", [
    ("fp64", (37, 21, 11), 1e-12),
    ("fp64", (24, 17, 9), 1e-12),
    ("fp32", (37, 21, 11), 1e-5),
    ("fp32", (64, 32, 40), 1e-5),
])
def test_one_reversed_step_with_particles_matches_oracle(prec, shape, tol):
    from paper_1307_0702_amd import ic
    print(f"particle adjoint step vs oracle {prec} {shape}", flush=True)
    fl, sim, adj, drho, g, lr, lg, P, sd = _setup(shape, prec, 300 + shape[0])
    n = 4
    # the particle state the GPU reverses from is the one it holds (wrapped)
    qd, ud = _d64(sim, P["q"]), _d64(sim, P["u"])
    ic.ic_copy_particles(sim.ctx, qd, ud)
    P = dict(P, q=qd.cpu().numpy(), u=ud.cpu().numpy())
    U = _dev(sim, drho, g)
    lam = _dev(sim, lr, lg)
    lq, lu, lF = _d64(sim, sd["lq"]), _d64(sim, sd["lu"]), _d64(sim, sd["lF"])
    bound_before = sim.U.clone()
    adj.step(n, U, lam, qd, ud, lq, lu, lF)
    sim.synchronize()
    want = OA.step_vjp_particles(_state(drho, g, P, n), fl.as_dict(), MODES, lr, list(lg),
                                 sd["lq"], sd["lu"], sd["lF"])
    errs = _compare(sim, adj, lam, lq, lu, want, len(MODES))
    for k, v in errs.items():
        assert v <= tol, (k, v)
    assert sim.torch.equal(sim.U, bound_before)
    q_after, _ = sim.get_particles()
    assert np.array_equal(q_after, P["q"])


@pytest.mark.parametrize("every", [3, "auto"])
def test_checkpointed_reversal_with_particles_matches_oracle_run_grad(every):
    shape = (30, 20, 16)
    print(f"particle adjoint, 7 steps checkpointed every {every}, {shape}", flush=True)
    fl, sim, adj, drho, g, lr, lg, P, sd = _setup(shape, "fp64", 520, npart=5)
    n0, nsteps = 2, 7
    qd, ud = _d64(sim, P["q"]), _d64(sim, P["u"])
    from paper_1307_0702_amd import ic
    ic.ic_copy_particles(sim.ctx, qd, ud)
    P = dict(P, q=qd.cpu().numpy(), u=ud.cpu().numpy())
    U0 = _dev(sim, drho, g)
    UN, ck = adj.forward(U0, n0, nsteps, every=every, q0=qd, u0=ud)
    # "auto" keeps the whole (small) trajectory: no re-stepping
    assert sorted(ck) == ([2, 5, 8] if every == 3 else list(range(2, 9)))
    lam = _dev(sim, lr, lg)
    lq, lu, lF = _d64(sim, sd["lq"]), _d64(sim, sd["lu"]), _d64(sim, sd["lF"])
    adj.drive_grad(len(MODES), reset=True)
    adj.particle_grad(reset=True)
    adj.backward(lam, n0, nsteps, ck, every=every, lq=lq, lu=lu, lF=lF)
    sim.synchronize()
    want, final = OA.run_grad_particles(_state(drho, g, P, n0), fl.as_dict(), MODES, nsteps,
                                        cr=lr, cg=list(lg), cq=sd["lq"], cu=sd["lu"], cF=sd["lF"])
    errs = _compare(sim, adj, lam, lq, lu, want, len(MODES))
    fwd = UN.cpu().numpy()
    errs["forward"] = max([_rel(fwd[0], final["drho"])] + [_rel(fwd[1 + a], final["g"][a]) for a in range(3)])
    for k, v in errs.items():
        assert v <= 1e-11, (k, v)


def test_rollout_gradients_match_central_differences_of_the_gpu_forward():
    import torch
    from paper_1307_0702_amd.adjoint import rollout_particles
    shape = (24, 20, 16)
    fl, sim, adj, drho, g, lr, lg, P, sd = _setup(shape, "fp64", 640, npart=4)
    n0, nsteps = 1, 6
    U0 = _dev(sim, drho, g)
    q0, u0 = _d64(sim, P["q"]), _d64(sim, P["u"])
    amps = torch.tensor([m["amp"] for m in MODES], dtype=torch.float64)
    me = torch.tensor(P["me"], dtype=torch.float64)
    eps = torch.tensor(P["eps"], dtype=torch.float64)
    C = _dev(sim, lr, lg)
    cq, cu, cF = _d64(sim, sd["lq"]), _d64(sim, sd["lu"]), _d64(sim, sd["lF"])
    fixed = dict(ks=P["ks"], qeq=P["qeq"], fext=P["fext"])

    def run(U0_, q0_, u0_, amps_, me_, eps_):
        return rollout_particles(adj, U0_, q0_, u0_, amps_, me_, eps_, MODES, n0, nsteps, every=4, **fixed)

    def loss(*args):
        UN, qN, uN, F = run(*args)
        return (UN * C).sum() + (qN * cq).sum() + (uN * cu).sum() + (F * cF).sum()

    xs = [U0.clone().requires_grad_(True), q0.clone().requires_grad_(True), u0.clone().requires_grad_(True),
          amps.clone().requires_grad_(True), me.clone().requires_grad_(True), eps.clone().requires_grad_(True)]
    loss(*xs).backward()
    grads = [x.grad for x in xs]
    base = [U0, q0, u0, amps, me, eps]
    rng = np.random.default_rng(641)
    steps = [1e-3, 1e-4, 1e-4, 1e-5, 1e-4, 1e-4]
    for i, name in enumerate(["U0", "q0", "u0", "amps", "me", "eps"]):
        d = torch.as_tensor(rng.standard_normal(tuple(base[i].shape)), dtype=torch.float64,
                            device=base[i].device)
        if i == 0:
            d = 1e-2 * d
        e = steps[i]
        ap = [b if j != i else b + e * d for j, b in enumerate(base)]
        am = [b if j != i else b - e * d for j, b in enumerate(base)]
        fd = (float(loss(*ap)) - float(loss(*am))) / (2 * e)
        an = float((grads[i] * d.to(grads[i].device)).sum())
        print(f"  {name}: fd {fd:.12e} adjoint {an:.12e}", flush=True)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (name, fd, an)


def test_particle_free_context_gives_the_fluid_adjoint_bit_for_bit():
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation
    fl = W.Fluid(24, 17, 9, kT=0.0, seed=9)
    drho, g = W.random_fields(fl.shape, 9)
    lr, lg = W.random_fields(fl.shape, 10, 1.0, 1.0)
    sim = Simulation(fl, prec="fp64", max_particles=2)
    sim.set_forcing(MODES)
    adj = Adjoint(sim)
    U = _dev(sim, drho, g)
    l1, l2 = _dev(sim, lr, lg), _dev(sim, lr, lg)
    ic.ic_adjoint_step(sim.ctx, 3, list(U), list(l1))
    ic.ic_adjoint_step_particles(sim.ctx, 3, list(U), None, None, list(l2), None, None, None)
    sim.synchronize()
    assert sim.torch.equal(l1, l2)


def test_particle_adjoint_error_paths():
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint
    from paper_1307_0702_amd.ic import Simulation
    fl = W.Fluid(16, 16, 16, kT=0.0, seed=3)
    sim = Simulation(fl, prec="fp64", max_particles=2)
    sim.set_particles(np.array([[3.0, 4.0, 5.0]]), np.array([1.0]), np.array([0.2]))
    U, lam = sim.U.clone(), sim.U.clone()
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_step_particles(sim.ctx, 0, list(U), None, None, list(lam), None, None)
    assert e.value.code == ic.IC_E_STATE          # workspace not bound
    adj = Adjoint(sim)                              # bound while the object lives
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_step_particles(sim.ctx, 0, list(U), None, None, list(lam), None, None)
    assert e.value.code == ic.IC_E_ARG            # particles set, arrays missing
    t = sim.torch
    z = t.zeros((1, 3), dtype=t.float64, device=sim.device)
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_step_particles(sim.ctx, -1, list(U), z, z, list(lam), z, z)
    assert e.value.code == ic.IC_E_ARG
    # positions are checked before they index the grid: on the host when
    # loaded, on the device (replaced by 0, reported by the next
    # synchronising call) when handed to a reversed step
    bad = z.clone()
    bad[0, 1] = float("nan")
    with pytest.raises(ic.ICError) as e:
        ic.ic_load_particles(sim.ctx, bad, z)
    assert e.value.code == ic.IC_E_ARG
    ic.ic_load_particles(sim.ctx, z + 20.5, z)                   # wrapped into the box
    q_in, _ = sim.get_particles()
    assert np.allclose(q_in, 4.5)
    ic.ic_adjoint_step_particles(sim.ctx, 0, list(U), bad, z, list(lam), z.clone(), z.clone())
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_particle_grad(sim.ctx, 1)
    assert e.value.code == ic.IC_E_ARG
    ic.ic_adjoint_particle_grad(sim.ctx, 1)                      # the flag was cleared
    hot = Simulation(W.Fluid(16, 16, 16, kT=1e-3, seed=3), prec="fp64", max_particles=1)
    hadj = Adjoint(hot)
    with pytest.raises(ic.ICError) as e:
        ic.ic_adjoint_step_particles(hot.ctx, 0, list(hot.U), None, None, list(hot.U.clone()), None, None)
    assert e.value.code == ic.IC_E_STATE and "kT" in str(e.value)   # kT != 0
    del adj, hadj


def test_force_loss_gradient_on_the_64cube_workload():
    # the reverse-mode benchmark's configuration (64^3, 16 tethered
    # particles, four resonant drives, checkpoints every 64 steps) over one
    # period of the m = 1 drive: dL/dA, dL/dm_e and dL/deps of the mean
    # x-force against central differences of the GPU forward run
    import torch
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint, rollout_particles
    from paper_1307_0702_amd.ic import Simulation
    w = W.adjoint_64()
    fl, p = w.fluid, w.particles
    md = [m.as_dict() for m in w.modes]
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    sim = Simulation(fl, prec="fp64", max_particles=p.n)
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing(md)
    adj = Adjoint(sim)
    q0 = torch.empty((p.n, 3), dtype=torch.float64, device=sim.device)
    u0 = torch.empty_like(q0)
    ic.ic_copy_particles(sim.ctx, q0, u0)
    U0 = torch.zeros((4,) + sim.shape, dtype=sim.dtype, device=sim.device)
    nsteps = w.period_steps

    def loss(a_, me_, eps_):
        _, _, _, F = rollout_particles(adj, U0, q0, u0, a_, me_, eps_, md, 0, nsteps, 64,
                                       ks=p.ks, qeq=p.qeq, fext=p.fext)
        return -F[:, 0].mean()

    base = [torch.tensor([m["amp"] for m in md], dtype=torch.float64),
            torch.tensor(p.me, dtype=torch.float64), torch.tensor(eps, dtype=torch.float64)]
    xs = [b.clone().requires_grad_(True) for b in base]
    loss(*xs).backward()
    # positions near 30 h carry ~4e-15 of rounding per step, which bounds how
    # small a central difference of the mean force can be resolved: the
    # steps keep the signal (2 h dL) far above it
    rng = np.random.default_rng(12)
    for i, (name, h) in enumerate((("amp", 2.3e-8), ("m_e", 1e-3), ("eps", 1e-3))):
        d = torch.as_tensor(rng.standard_normal(tuple(base[i].shape)), dtype=torch.float64)
        ap = [b if j != i else b + h * d for j, b in enumerate(base)]
        am = [b if j != i else b - h * d for j, b in enumerate(base)]
        with torch.no_grad():
            fd = (float(loss(*ap)) - float(loss(*am))) / (2 * h)
        an = float((xs[i].grad * d).sum())
        print(f"  {name}: fd {fd:.10e} adjoint {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-4 * abs(fd), (name, fd, an)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1.2e-4)])
def test_force_loss_gradient_on_the_64cube_workload_matches_oracle(prec, tol):
    # The reverse-mode benchmark's configuration from a developed state (one
    # drive period stepped on the GPU): the gradient of the mean x-force over
    # 12 steps in the drive amplitudes, m_e, eps, the initial positions and
    # the initial fields, against the FP64 oracle's run_grad_particles from
    # the same state.  FP32 bar: the per-step bar 1e-5 over 12 steps.
    import torch
    from paper_1307_0702_amd import ic
    from paper_1307_0702_amd.adjoint import Adjoint, rollout_particles
    from paper_1307_0702_amd.ic import Simulation
    w = W.adjoint_64()
    fl, p = w.fluid, w.particles
    md = [m.as_dict() for m in w.modes]
    eps = np.array([ic.ic_eps_from_kappa_ratio(fl.cf, r) for r in p.kappa_ratio])
    sim = Simulation(fl, prec=prec, max_particles=p.n)
    sim.set_particles(p.q, p.me, eps, ks=p.ks, qeq=p.qeq, fext=p.fext)
    sim.set_forcing(md)
    n0, nsteps = w.period_steps, 12
    print(f"64^3 workload {prec}: {n0} steps to a developed state", flush=True)
    sim.step(n0)
    U0 = sim.U.clone()
    q0 = torch.empty((p.n, 3), dtype=torch.float64, device=sim.device)
    u0 = torch.empty_like(q0)
    ic.ic_get_state(sim.ctx, None, q0, u0)
    adj = Adjoint(sim)
    base = [torch.tensor([m["amp"] for m in md], dtype=torch.float64),
            torch.tensor(p.me, dtype=torch.float64), torch.tensor(eps, dtype=torch.float64)]
    xs = [U0.clone().requires_grad_(True), q0.clone().requires_grad_(True)] + \
         [b.clone().requires_grad_(True) for b in base]
    _, _, _, F = rollout_particles(adj, xs[0], xs[1], u0, xs[2], xs[3], xs[4], md, n0, nsteps, 4,
                                   ks=p.ks, qeq=p.qeq, fext=p.fext)
    (-F[:, 0].mean()).backward()
    U = U0.double().cpu().numpy()
    st = dict(drho=U[0], g=[U[1], U[2], U[3]], n=n0, q=q0.cpu().numpy(), u=u0.cpu().numpy(),
              me=np.asarray(p.me, float), eps=eps, ks=np.asarray(p.ks, float),
              qeq=np.asarray(p.qeq, float), fext=np.asarray(p.fext, float))
    cF = np.zeros((p.n, 3))
    cF[:, 0] = -1.0 / (p.n * nsteps)
    print("  oracle gradient", flush=True)
    want, _ = OA.run_grad_particles(st, fl.as_dict(), md, nsteps, cF=cF)
    got_U = xs[0].grad.double().cpu().numpy()
    errs = {"A": _rel(xs[2].grad.numpy(), want["dA"]), "me": _rel(xs[3].grad.numpy(), want["dme"]),
            "eps": _rel(xs[4].grad.numpy(), want["deps"]), "q0": _rel(xs[1].grad.cpu().numpy(), want["lq"]),
            "drho0": _rel(got_U[0], want["lr"])}
    for a in range(3):
        errs["g%d" % a] = _rel(got_U[1 + a], want["lg"][a])
    print("  ", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)


def test_two_rollouts_with_different_parameters_then_one_backward():
    # A loss that sums two rollouts of one context with different excess
    # masses: the backward of each must reverse its own trajectory, not the
    # parameters the shared context holds when backward runs.
    import torch
    from paper_1307_0702_amd.adjoint import rollout_particles
    shape = (24, 20, 16)
    fl, sim, adj, drho, g, lr, lg, P, sd = _setup(shape, "fp64", 650, npart=4)
    n0, nsteps = 1, 5
    U0 = _dev(sim, drho, g)
    q0, u0 = _d64(sim, P["q"]), _d64(sim, P["u"])
    fixed = dict(ks=P["ks"], qeq=P["qeq"], fext=P["fext"])
    C = _dev(sim, lr, lg)
    cF = _d64(sim, sd["lF"])
    me_a = torch.tensor(P["me"], dtype=torch.float64)
    me_b = me_a + 3.0
    eps = torch.tensor(P["eps"], dtype=torch.float64)
    amps = torch.tensor([m["amp"] for m in MODES], dtype=torch.float64)

    def one(me_, x_):
        UN, _, _, F = rollout_particles(adj, x_[0], q0, u0, amps, me_, x_[1], MODES, n0, nsteps,
                                        every=2, **fixed)
        return (UN * C).sum() + (F * cF).sum()

    def leaves():
        return [U0.clone().requires_grad_(True), eps.clone().requires_grad_(True)]

    xa, xb = leaves(), leaves()
    (one(me_a, xa) + one(me_b, xb)).backward()
    ya = leaves()
    one(me_a, ya).backward()
    yb = leaves()
    one(me_b, yb).backward()
    for got, want in ((xa, ya), (xb, yb)):
        for x, y in zip(got, want):
            err = _rel(x.grad.detach().cpu().numpy(), y.grad.detach().cpu().numpy())
            print(f"  summed against separate backward: {err:.2e}", flush=True)
            assert err <= 1e-12
    # and the two trajectories really differ
    assert _rel(xa[1].grad.cpu().numpy(), xb[1].grad.cpu().numpy()) > 1e-6
