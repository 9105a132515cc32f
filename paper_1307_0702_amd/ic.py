"""Thin ctypes binding of libic.so (the C ABI in include/ic.h).

Module-level functions carry the C names (ic_create, ic_step, ...) and only
marshal arguments; `Simulation` bundles them with torch-owned device memory
(fields and workspace) and the current torch stream.  Every step of the path
runs in the HIP kernels of libic.so: if the library is missing this module
raises at import time.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libic.so")

IC_OK, IC_E_ARG, IC_E_UNSTABLE, IC_E_MASS, IC_E_STATE, IC_E_HIP, IC_E_CAPACITY = 0, -1, -2, -3, -4, -5, -6
IC_FP32, IC_FP64 = 1, 2
IC_CELL, IC_FACE_X, IC_FACE_Y, IC_FACE_Z, IC_FACES = 0, 1, 2, 3, 4
IC_MODE_COS, IC_MODE_PLANE = 0, 1
IC_MAX_MODES = 8
IC_NOALLOC_MAX_POINTS = 16384

EXPORTED = [
    "ic_create", "ic_destroy", "ic_workspace_size", "ic_bind", "ic_set_particles",
    "ic_get_particles", "ic_set_forcing", "ic_set_step", "ic_get_step", "ic_step",
    "ic_step_prepare",
    "ic_interpolate", "ic_interpolate_noalloc", "ic_spread", "ic_avg_force", "ic_conserved",
    "ic_eps_from_kappa_ratio", "ic_strerror", "ic_last_error", "ic_profile", "ic_profile_read",
    "ic_set_tile", "ic_get_tile", "ic_graph_create", "ic_graph_launch", "ic_graph_destroy",
    "ic_adjoint_workspace_size", "ic_bind_adjoint", "ic_adjoint_step", "ic_adjoint_drive",
    "ic_adjoint_step_particles", "ic_adjoint_particle_grad", "ic_copy_particles", "ic_load_particles",
    "ic_get_state", "ic_set_state",
]


class ic_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("h", ctypes.c_double), ("rho0", ctypes.c_double),
                ("cf", ctypes.c_double), ("eta", ctypes.c_double), ("zeta", ctypes.c_double),
                ("kT", ctypes.c_double), ("dt", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("max_particles", ctypes.c_int32)]


class ic_mode(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int32), ("shape", ctypes.c_int32), ("m", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("x0", ctypes.c_double), ("amp", ctypes.c_double),
                ("omega", ctypes.c_double), ("phase", ctypes.c_double)]


class ICError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libic.so not built: {path} is missing (run __graft_entry__.build())")
    # torch first: libic.so then binds to the HIP runtime torch has loaded,
    # so the streams and memory torch hands over belong to the same runtime
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ic_create": ([ctypes.POINTER(ic_params), P, ctypes.POINTER(P)], ctypes.c_int),
        "ic_destroy": ([P], ctypes.c_int),
        "ic_workspace_size": ([ctypes.POINTER(ic_params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "ic_bind": ([P, P, P, P, P, P, ctypes.c_size_t], ctypes.c_int),
        "ic_set_particles": ([P, ctypes.c_int32, P, P, P, P, P, P, P], ctypes.c_int),
        "ic_get_particles": ([P, P, P], ctypes.c_int),
        "ic_set_forcing": ([P, ctypes.c_int32, ctypes.POINTER(ic_mode)], ctypes.c_int),
        "ic_set_step": ([P, ctypes.c_int64], ctypes.c_int),
        "ic_get_step": ([P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "ic_step": ([P, ctypes.c_int64], ctypes.c_int),
        "ic_step_prepare": ([P], ctypes.c_int),
        "ic_interpolate": ([P, ctypes.c_int32, P, ctypes.c_int32, P, P], ctypes.c_int),
        "ic_interpolate_noalloc": ([P, ctypes.c_int32, P, ctypes.c_int32, P, P], ctypes.c_int),
        "ic_spread": ([P, ctypes.c_int32, P, P, ctypes.c_int32, P], ctypes.c_int),
        "ic_avg_force": ([P, P, P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32], ctypes.c_int),
        "ic_conserved": ([P, dp], ctypes.c_int),
        "ic_eps_from_kappa_ratio": ([ctypes.c_double, ctypes.c_double], ctypes.c_double),
        "ic_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "ic_profile": ([P, ctypes.c_int32], ctypes.c_int),
        "ic_profile_read": ([P, dp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "ic_last_error": ([P], ctypes.c_char_p),
        "ic_set_tile": ([P, ctypes.c_int32], ctypes.c_int),
        "ic_get_tile": ([P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "ic_graph_create": ([ctypes.POINTER(P), ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(P)],
                            ctypes.c_int),
        "ic_graph_launch": ([P, P], ctypes.c_int),
        "ic_graph_destroy": ([P], ctypes.c_int),
        "ic_adjoint_workspace_size": ([ctypes.POINTER(ic_params), ctypes.POINTER(ctypes.c_size_t)],
                                      ctypes.c_int),
        "ic_bind_adjoint": ([P, P, ctypes.c_size_t], ctypes.c_int),
        "ic_adjoint_step": ([P, ctypes.c_int64, P, P, P, P, P, P, P, P], ctypes.c_int),
        "ic_adjoint_drive": ([P, dp, ctypes.c_int32], ctypes.c_int),
        "ic_adjoint_step_particles": ([P, ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, P, P, P],
                                      ctypes.c_int),
        "ic_adjoint_particle_grad": ([P, P, P, P, ctypes.c_int32], ctypes.c_int),
        "ic_copy_particles": ([P, P, P], ctypes.c_int),
        "ic_get_state": ([P, P, P, P, P, P, P], ctypes.c_int),
        "ic_set_state": ([P, P, P, P, P, P, P], ctypes.c_int),
        "ic_load_particles": ([P, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = load_library()


def _check(rc, ctx=None):
    if rc != IC_OK:
        msg = _lib.ic_last_error(ctx).decode() if ctx else _lib.ic_strerror(rc).decode()
        raise ICError(rc, msg or _lib.ic_strerror(rc).decode())


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


# --- C names, marshalling only ----------------------------------------------

def ic_create(params: ic_params, stream: int = 0):
    ctx = ctypes.c_void_p()
    _check(_lib.ic_create(ctypes.byref(params), ctypes.c_void_p(stream), ctypes.byref(ctx)))
    return ctx


def ic_destroy(ctx):
    _check(_lib.ic_destroy(ctx))


def ic_workspace_size(params: ic_params) -> int:
    n = ctypes.c_size_t()
    _check(_lib.ic_workspace_size(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def ic_bind(ctx, drho, gx, gy, gz, ws, nbytes):
    _check(_lib.ic_bind(ctx, _ptr(drho), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(ws), nbytes), ctx)


def ic_set_particles(ctx, q, u, me, eps, ks=None, qeq=None, fext=None):
    n = 0 if q is None else len(q)
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
            for a in (q, u, me, eps, ks, qeq, fext)]
    _check(_lib.ic_set_particles(ctx, n, *[_ptr(a) for a in arrs]), ctx)


def ic_get_particles(ctx, n):
    q = np.zeros((n, 3))
    u = np.zeros((n, 3))
    _check(_lib.ic_get_particles(ctx, _ptr(q), _ptr(u)), ctx)
    return q, u


def ic_set_forcing(ctx, modes):
    arr = (ic_mode * max(1, len(modes)))()
    for i, m in enumerate(modes):
        shape = IC_MODE_PLANE if m["shape"] == "plane" else IC_MODE_COS
        arr[i] = ic_mode(int(m["axis"]), shape, int(m.get("m", 1)), 0, float(m["x0"]),
                         float(m["amp"]), float(m["omega"]), float(m.get("phase", 0.0)))
    _check(_lib.ic_set_forcing(ctx, len(modes), arr), ctx)


def ic_set_step(ctx, n):
    _check(_lib.ic_set_step(ctx, int(n)), ctx)


def ic_get_step(ctx):
    n = ctypes.c_int64()
    _check(_lib.ic_get_step(ctx, ctypes.byref(n)), ctx)
    return n.value


def ic_step(ctx, nsteps):
    _check(_lib.ic_step(ctx, int(nsteps)), ctx)


def ic_step_prepare(ctx):
    _check(_lib.ic_step_prepare(ctx), ctx)


def ic_set_tile(ctx, tz):
    _check(_lib.ic_set_tile(ctx, int(tz)), ctx)


def ic_get_tile(ctx):
    tz = ctypes.c_int32()
    _check(_lib.ic_get_tile(ctx, ctypes.byref(tz)), ctx)
    return tz.value


def ic_graph_create(ctxs, nsteps):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    g = ctypes.c_void_p()
    rc = _lib.ic_graph_create(arr, len(ctxs), int(nsteps), ctypes.byref(g))
    _check(rc, ctxs[0] if ctxs else None)
    return g


def ic_graph_launch(graph, stream=0):
    _check(_lib.ic_graph_launch(graph, ctypes.c_void_p(stream)))


def ic_graph_destroy(graph):
    _check(_lib.ic_graph_destroy(graph))


def ic_adjoint_workspace_size(params):
    n = ctypes.c_size_t()
    _check(_lib.ic_adjoint_workspace_size(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def ic_bind_adjoint(ctx, ws, nbytes):
    _check(_lib.ic_bind_adjoint(ctx, _ptr(ws), int(nbytes)), ctx)


def ic_adjoint_step(ctx, n, U, lam):
    """U: the four state fields of step n (device); lam: the four adjoint
    fields (device), dL/dU^{n+1} in, dL/dU^n out."""
    _check(_lib.ic_adjoint_step(ctx, int(n), *[_ptr(x) for x in U], *[_ptr(x) for x in lam]), ctx)


def ic_adjoint_drive(ctx, nmodes, reset=False):
    """dL/dA_m of the context's first nmodes drives (it holds at most
    IC_MAX_MODES)."""
    out = (ctypes.c_double * IC_MAX_MODES)()
    _check(_lib.ic_adjoint_drive(ctx, out, int(bool(reset))), ctx)
    return np.array(list(out)[:int(nmodes)])


def ic_adjoint_step_particles(ctx, n, U, q, u, lam, lq, lu, lF=None):
    """U: the four state fields of step n; q, u: the particle state of step
    n ([np][3] float64); lam, lq, lu: adjoints after the step in, before
    the step out; lF: dL/dF^{n+1/2} or None.  All device tensors."""
    _check(_lib.ic_adjoint_step_particles(ctx, int(n), *[_ptr(x) for x in U], _ptr(q), _ptr(u),
                                          *[_ptr(x) for x in lam], _ptr(lq), _ptr(lu), _ptr(lF)), ctx)


def ic_adjoint_particle_grad(ctx, n, reset=False):
    """Accumulated (dL/dm_e, dL/deps_pf, dL/dk_s), host float64 [n] each."""
    out = [np.zeros(n) for _ in range(3)]
    _check(_lib.ic_adjoint_particle_grad(ctx, *[_ptr(x) for x in out], int(bool(reset))), ctx)
    return tuple(out)


def ic_get_state(ctx, fields, q_dev=None, u_dev=None):
    """fields: four device tensors (or None) receiving (drho, gx, gy, gz)."""
    f = list(fields) if fields is not None else [None] * 4
    _check(_lib.ic_get_state(ctx, *[_ptr(x) for x in f], _ptr(q_dev), _ptr(u_dev)), ctx)


def ic_set_state(ctx, fields, q_dev=None, u_dev=None):
    f = list(fields) if fields is not None else [None] * 4
    _check(_lib.ic_set_state(ctx, *[_ptr(x) for x in f], _ptr(q_dev), _ptr(u_dev)), ctx)


def ic_copy_particles(ctx, q_dev, u_dev):
    _check(_lib.ic_copy_particles(ctx, _ptr(q_dev), _ptr(u_dev)), ctx)


def ic_load_particles(ctx, q_dev, u_dev):
    _check(_lib.ic_load_particles(ctx, _ptr(q_dev), _ptr(u_dev)), ctx)


def ic_interpolate(ctx, n, q_dev, kind, field_dev, out_dev):
    _check(_lib.ic_interpolate(ctx, int(n), _ptr(q_dev), int(kind), _ptr(field_dev), _ptr(out_dev)), ctx)


def ic_interpolate_noalloc(ctx, n, q, kind, field_dev, out):
    """q ([n][3] float64) and out (float64 [n], or [n][3] for IC_FACES):
    host numpy arrays or device tensors; field_dev: a device tensor."""
    _check(_lib.ic_interpolate_noalloc(ctx, int(n), _ptr(q), int(kind), _ptr(field_dev), _ptr(out)),
           ctx)


def ic_spread(ctx, n, q_dev, f_dev, kind, field_dev):
    _check(_lib.ic_spread(ctx, int(n), _ptr(q_dev), _ptr(f_dev), int(kind), _ptr(field_dev)), ctx)


def ic_avg_force(ctx, n, reset=False):
    f = np.zeros((n, 3))
    lam = np.zeros((n, 3))
    ns = ctypes.c_int64()
    _check(_lib.ic_avg_force(ctx, _ptr(f), _ptr(lam), ctypes.byref(ns), int(bool(reset))), ctx)
    return f, lam, ns.value


def ic_conserved(ctx):
    out = (ctypes.c_double * 4)()
    _check(_lib.ic_conserved(ctx, out), ctx)
    return np.array(list(out))


def ic_profile(ctx, enable):
    _check(_lib.ic_profile(ctx, int(bool(enable))), ctx)


def ic_profile_read(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.ic_profile_read(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def ic_eps_from_kappa_ratio(cf, kappa_ratio):
    return _lib.ic_eps_from_kappa_ratio(float(cf), float(kappa_ratio))


# --- convenience wrapper with torch-owned memory ------------------------------

class Simulation:
    """One context with its fields and workspace allocated by torch on the
    current device and its work enqueued on the current torch stream."""

    def __init__(self, fluid, prec="fp64", max_particles=0, device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.dtype = torch.float64 if prec == "fp64" else torch.float32
        fl = fluid if isinstance(fluid, dict) else fluid.as_dict()
        self.fluid = fl
        self.params = ic_params(int(fl["nx"]), int(fl["ny"]), int(fl["nz"]),
                                IC_FP64 if prec == "fp64" else IC_FP32,
                                float(fl["h"]), float(fl["rho0"]), float(fl["cf"]),
                                float(fl["eta"]), float(fl["zeta"]), float(fl["kT"]),
                                float(fl["dt"]), int(fl.get("seed", 0)),
                                int(fl.get("replica", 0)), int(max_particles))
        self.shape = (int(fl["nz"]), int(fl["ny"]), int(fl["nx"]))
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ctx = ic_create(self.params, self.stream.cuda_stream)
            self.U = torch.zeros((4,) + self.shape, dtype=self.dtype, device=self.device)
            nbytes = ic_workspace_size(self.params)
            self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws_raw.data_ptr()) % 256
            self.ws = self._ws_raw[off:off + nbytes]
            ic_bind(self.ctx, self.U[0], self.U[1], self.U[2], self.U[3], self.ws, nbytes)
        self.np = 0

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        # at interpreter shutdown the module's globals may already be gone;
        # the process is ending then, and its device memory goes with it
        lib = globals().get("_lib")
        if ctx is None or lib is None:
            return
        try:
            self.synchronize()
        except Exception:
            pass
        lib.ic_destroy(ctx)
        self.ctx = None

    def synchronize(self):
        self.stream.synchronize()

    def set_state(self, drho, g):
        t = self.torch
        self.U[0].copy_(t.as_tensor(np.asarray(drho)).to(self.dtype))
        for a in range(3):
            self.U[1 + a].copy_(t.as_tensor(np.asarray(g[a])).to(self.dtype))
        self.synchronize()

    def get_state(self):
        self.synchronize()
        U = self.U.detach().to("cpu").to(self.torch.float64).numpy()
        return U[0].copy(), [U[1].copy(), U[2].copy(), U[3].copy()]

    def set_particles(self, q, me, eps, u=None, ks=None, qeq=None, fext=None):
        q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
        self.np = len(q)
        ic_set_particles(self.ctx, q, u, me, eps, ks, qeq, fext)

    def get_particles(self):
        return ic_get_particles(self.ctx, self.np)

    def set_forcing(self, modes):
        ic_set_forcing(self.ctx, modes)

    def set_step(self, n):
        ic_set_step(self.ctx, n)

    def step(self, n=1):
        ic_step(self.ctx, n)

    def prepare(self):
        """Captures the step graph of long ic_step calls now (ic_step_prepare)."""
        ic_step_prepare(self.ctx)

    def set_tile(self, tz):
        ic_set_tile(self.ctx, tz)

    def tile(self):
        return ic_get_tile(self.ctx)

    def avg_force(self, reset=False):
        return ic_avg_force(self.ctx, self.np, reset)

    def conserved(self):
        return ic_conserved(self.ctx)

    def interpolate(self, q, kind, field):
        t = self.torch
        qd = t.as_tensor(np.ascontiguousarray(q, dtype=np.float64)).to(self.device)
        out = t.zeros((len(q), 3) if kind == IC_FACES else len(q), dtype=t.float64, device=self.device)
        fd = field if isinstance(field, t.Tensor) else t.as_tensor(np.asarray(field)).to(self.dtype).to(self.device)
        fd = fd.contiguous()
        ic_interpolate(self.ctx, len(q), qd, kind, fd, out)
        self.synchronize()
        return out.cpu().numpy()

    def spread(self, q, f, kind, field):
        t = self.torch
        qd = t.as_tensor(np.ascontiguousarray(q, dtype=np.float64)).to(self.device)
        fv = t.as_tensor(np.ascontiguousarray(f, dtype=np.float64)).to(self.device)
        ic_spread(self.ctx, len(q), qd, fv, kind, field)
        self.synchronize()
        return field
