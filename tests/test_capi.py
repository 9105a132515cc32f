"""Host-side checks of libic.so: every symbol include/ic.h declares is
exported, and argument checks that run before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ic.h")).read()
    return sorted(set(re.findall(r"\b(ic_[a-z_]+)\s*\(", txt)))


def test_header_is_plain_c(tmp_path):
    # the boundary header compiles as C99 (no C++ types in any signature)
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_ic.c"
    src.write_text('#include "ic.h"\nint main(void) { return 0; }\n')
    res = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                          "-fsyntax-only", "-I" + os.path.join(ROOT, "include"), str(src)],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr


def test_header_and_binding_agree():
    from paper_1307_0702_amd import ic
    assert _declared() == sorted(ic.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_1307_0702_amd import ic
    lib = ctypes.CDLL(ic.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def _params(**kw):
    from paper_1307_0702_amd import ic
    d = dict(nx=8, ny=8, nz=8, prec=ic.IC_FP64, h=1.0, rho0=1.0, cf=1.0, eta=0.5, zeta=0.5,
             kT=0.0, dt=0.1, seed=1, replica=0, max_particles=4)
    d.update(kw)
    return ic.ic_params(*[d[k] for k, _ in ic.ic_params._fields_])


@pytest.mark.parametrize("kw,code", [
    (dict(nx=3), -1), (dict(h=0.0), -1), (dict(eta=-1.0), -1), (dict(prec=7), -1),
    (dict(kT=float("nan")), -1), (dict(max_particles=-1), -1),
    (dict(nx=1024, ny=1024, nz=1024, prec=1), -1), (dict(nx=1024, ny=1024, nz=512, prec=2), -1),
    (dict(dt=0.6), -2), (dict(eta=3.0, dt=0.1), -2),
])
def test_create_rejects_bad_params(kw, code):
    from paper_1307_0702_amd import ic
    ctx = ctypes.c_void_p()
    rc = ic._lib.ic_create(ctypes.byref(_params(**kw)), None, ctypes.byref(ctx))
    assert rc == code
    assert not ctx.value


def test_create_destroy_and_workspace_size():
    from paper_1307_0702_amd import ic
    p = _params()
    ctx = ic.ic_create(p, 0)
    n = ic.ic_workspace_size(p)
    # two stage copies of the four fields at least
    assert n >= 2 * 4 * 8 ** 3 * 8
    assert ic.ic_get_step(ctx) == 0
    ic.ic_set_step(ctx, 12)
    assert ic.ic_get_step(ctx) == 12
    with pytest.raises(ic.ICError) as e:
        ic.ic_step(ctx, 1)             # nothing bound yet
    assert e.value.code == ic.IC_E_STATE
    ic.ic_destroy(ctx)


def test_eps_from_kappa_ratio():
    from paper_1307_0702_amd import ic
    assert ic.ic_eps_from_kappa_ratio(1.0, 0.5) == pytest.approx(1.0)
    assert ic.ic_eps_from_kappa_ratio(4.0, 0.25) == pytest.approx(48.0)
    assert ic._lib.ic_strerror(-3).decode().startswith("non-positive mass")


def test_unbound_and_null_contexts_are_refused_before_device_work():
    # every entry point that needs bound buffers refuses an unbound context
    # with IC_E_STATE, and a NULL context with IC_E_ARG, without touching
    # the device
    from paper_1307_0702_amd import ic
    L = ic._lib
    ctx = ic.ic_create(_params(), 0)
    null = ctypes.c_void_p()
    buf = (ctypes.c_double * 12)()
    i64 = ctypes.c_int64()
    calls = {
        "ic_step": lambda c: L.ic_step(c, 1),
        "ic_step_prepare": lambda c: L.ic_step_prepare(c),
        "ic_set_particles": lambda c: L.ic_set_particles(c, 1, buf, None, buf, buf, None, None, None),
        "ic_get_particles": lambda c: L.ic_get_particles(c, buf, buf),
        "ic_get_state": lambda c: L.ic_get_state(c, None, None, None, None, buf, buf),
        "ic_set_state": lambda c: L.ic_set_state(c, None, None, None, None, buf, buf),
        "ic_copy_particles": lambda c: L.ic_copy_particles(c, buf, buf),
        "ic_load_particles": lambda c: L.ic_load_particles(c, buf, buf),
        "ic_adjoint_step": lambda c: L.ic_adjoint_step(c, 0, buf, buf, buf, buf, buf, buf, buf, buf),
        "ic_adjoint_step_particles": lambda c: L.ic_adjoint_step_particles(
            c, 0, buf, buf, buf, buf, buf, buf, buf, buf, buf, buf, buf, buf, None),
        "ic_spread": lambda c: L.ic_spread(c, 1, buf, buf, 0, buf),
        "ic_avg_force": lambda c: L.ic_avg_force(c, buf, buf, ctypes.byref(i64), 0),
    }
    for name, call in calls.items():
        assert call(ctx) == ic.IC_E_STATE, name
        assert call(null) == ic.IC_E_ARG, name
    # the adjoint accumulators need a bound adjoint workspace
    assert L.ic_adjoint_particle_grad(ctx, buf, buf, buf, 0) == ic.IC_E_STATE
    assert L.ic_adjoint_drive(ctx, buf, 0) == ic.IC_E_STATE
    assert L.ic_adjoint_particle_grad(null, buf, buf, buf, 0) == ic.IC_E_ARG
    # bad interpolation kinds are refused before any launch
    assert L.ic_interpolate(ctx, 1, buf, 5, buf, buf) == ic.IC_E_ARG
    assert L.ic_interpolate(ctx, 1, buf, -1, buf, buf) == ic.IC_E_ARG
    ic.ic_destroy(ctx)
