"""Builds oracle state dicts from the seeded workloads (test helper)."""
import numpy as np

from oracle import ic_oracle as O


def make_state(w, n0=0):
    fl = w.fluid
    p = w.particles
    eps = O.eps_from_kappa_ratio(fl.cf, p.kappa_ratio) if p.n else np.zeros(0)
    g = [np.array(w.g[a], dtype=np.float64) for a in range(3)]
    drho = np.array(w.drho, dtype=np.float64)
    st = dict(drho=drho, g=g, n=n0, q=np.array(p.q, dtype=np.float64).reshape(-1, 3),
              me=np.array(p.me, dtype=np.float64), eps=eps,
              ks=np.array(p.ks, dtype=np.float64), qeq=np.array(p.qeq, dtype=np.float64).reshape(-1, 3),
              fext=np.array(p.fext, dtype=np.float64).reshape(-1, 3))
    if p.u is None:
        st["u"] = O._velocity_at(g, drho, st["q"], fl.as_dict()) if p.n else np.zeros((0, 3))
    else:
        st["u"] = np.array(p.u, dtype=np.float64).reshape(-1, 3)
    return st


def modes_of(w):
    return [m.as_dict() for m in w.modes]
