"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/segpart.h, and rejects invalid meshes and parameters
before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_1408_2355_amd import segpart as sp
from workloads import icosphere

HEADER = os.path.join(ROOT, "include", "segpart.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp_[a-z_]+)\s*\(", text)))


def test_header_declares_and_library_exports_every_entry_point():
    names = _declared()
    assert len(names) >= 25
    lib = sp.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(sp.EXPORTED)


def test_binding_has_a_function_per_entry_point():
    # the Python binding mirrors the C names one to one (marshalling only)
    missing = [n for n in sp.EXPORTED if not callable(getattr(sp, n, None))]
    assert missing == []


def test_version_and_defaults():
    assert sp.sp_version() == (1, 3)
    p = sp.params(5e-5)
    assert p.tau == 5e-5 and p.energy_every == 2000 and p.precision == sp.SP_MIXED
    assert p.cg_rtol == 1e-10 and p.check_every == 8 and p.precond == sp.SP_PRECOND_CHEB1
    p = sp.params(1e-3, precision="fp64", n_steps=7)
    assert p.precision == sp.SP_FP64 and p.n_steps == 7


def _expect(code, fn, *a):
    with pytest.raises(sp.SegpartError) as e:
        fn(*a)
    assert e.value.code == code, str(e.value)
    return str(e.value)


def test_mesh_validation_errors():
    v, f = icosphere(1)
    bad = f.copy()
    bad[3, 1] = v.shape[0]          # index out of range
    assert "out of range" in _expect(sp.SP_EMESH, sp.sp_mesh_create, v, bad)
    _expect(sp.SP_EMESH, sp.sp_mesh_create, v, f[1:])    # open surface
    deg = f.copy()
    deg[0] = [deg[0, 0], deg[0, 0], deg[0, 2]]           # repeated corner
    _expect(sp.SP_EMESH, sp.sp_mesh_create, v, deg)
    flat = v.copy()
    a, b, c = f[5]
    flat[c] = 0.5 * (flat[a] + flat[b])                  # zero-area triangle
    _expect(sp.SP_EMESH, sp.sp_mesh_create, flat, f)
    nanv = v.copy()
    nanv[2, 0] = np.nan
    _expect(sp.SP_EINVAL, sp.sp_mesh_create, nanv, f)
    _expect(sp.SP_EINVAL, sp.sp_mesh_create, v[:2], f[:1])


# --- parameter and batch validation before any device work (NULL mesh: the
# library reports the parameter error first, so these run without a GPU) ---

def _arr(a, t):
    a = np.ascontiguousarray(a, t)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32 if t == np.int32 else C.c_double))


def _rejects(call, what):
    rc = call()
    msg = sp.sp_last_error()
    assert rc == sp.SP_EINVAL, (rc, msg)
    assert what in msg, msg


def _entry_points(prm, m, eps):
    """Every entry point that takes parameters and a batch, called with a NULL
    mesh; each must reject the arguments before looking at the mesh."""
    lib = sp.lib()
    (mm, mp), (ee, ep) = _arr(m, np.int32), _arr(eps, np.float64)
    u0, up = _arr(np.ones(64), np.float64)
    h = C.c_void_p()
    srv = sp.Server(1 << 30)  # no device work until a request is placed
    ticket = C.c_int64()
    try:
        yield lambda: lib.sp_solve(None, C.byref(prm), mm.size, mp, ep, up, None, None, None,
                                   None, None, None, None)
        yield lambda: lib.sp_solve_async(None, C.byref(prm), mm.size, mp, ep, None, None, None,
                                         None, None, None, None, None)
        yield lambda: lib.sp_state_create(None, C.byref(prm), mm.size, mp, ep, up, None,
                                          C.byref(h))
        yield lambda: lib.sp_server_submit(srv.h, None, C.byref(prm), mm.size, mp, ep, up,
                                           C.byref(ticket))
    finally:
        srv.close()


@pytest.mark.parametrize("tau", [0.0, -1e-3, float("nan"), float("inf")])
def test_rejects_nonpositive_or_nonfinite_tau(tau):
    prm = sp.params(1e-3, n_steps=3)
    prm.tau = tau
    for call in _entry_points(prm, [3], [0.1]):
        _rejects(call, "tau must be > 0")


@pytest.mark.parametrize("eps", [0.0, -0.1, float("nan")])
def test_rejects_nonpositive_or_nonfinite_eps(eps):
    prm = sp.params(1e-3, n_steps=3)
    for call in _entry_points(prm, [3, 4], [0.1, eps]):
        _rejects(call, "eps must be > 0 (restart 1)")


@pytest.mark.parametrize("m", [0, -2])
def test_rejects_m_below_one(m):
    prm = sp.params(1e-3, n_steps=3)
    for call in _entry_points(prm, [3, m], [0.1, 0.1]):
        _rejects(call, "m must be >= 1 (restart 1)")


def test_rejects_bad_solver_settings():
    for field, value, what in [("cg_rtol", 0.0, "cg_rtol"), ("cg_rtol", 1.0, "cg_rtol"),
                               ("cg_max_iter", 0, "cg_max_iter"),
                               ("extrapolate", 9, "extrapolate"),
                               ("precond", 2, "precond"), ("precond", -1, "precond"),
                               ("inner_rtol", 0.0, "inner_rtol")]:
        prm = sp.params(1e-3, n_steps=3)
        setattr(prm, field, value)
        for call in _entry_points(prm, [3], [0.1]):
            _rejects(call, what)


def test_null_mesh_is_reported_after_valid_arguments():
    prm = sp.params(1e-3, n_steps=3)
    for call in _entry_points(prm, [3], [0.1]):
        _rejects(call, "NULL mesh")


def test_stats_struct_matches_header():
    # sp_stats grew a double (hbm_bytes) in 1.2; the binding's layout follows
    assert C.sizeof(sp.sp_stats) == 56
    assert [f for f, _ in sp.sp_stats._fields_][-1] == "hbm_bytes"
