"""Python binding of libsegpart (ctypes, argument marshalling only).

Each ``sp_*`` function here mirrors the C entry point of the same name in
include/segpart.h: it converts numpy arrays (or torch tensors for the
device-pointer calls) to pointers, calls the library, and raises
``SegpartError`` on a negative status.  All computation happens in the HIP
library; nothing here falls back to the CPU.  ``Mesh``, ``State`` and
``Server`` are small owners of the opaque handles.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsegpart.so")

SP_OK, SP_EINVAL, SP_EMESH, SP_ENOMEM, SP_EDEVICE, SP_ENOCONV, SP_EAGAIN, SP_ENOTFOUND = \
    0, -1, -2, -3, -4, -5, -6, -7
SP_FP64, SP_MIXED = 0, 1
SP_PRECOND_JACOBI, SP_PRECOND_CHEB1 = 0, 1
SP_MAT_M, SP_MAT_A = 0, 1
SP_STAGE_HEAT, SP_STAGE_NODE, SP_STAGE_NORM = 1, 2, 3
SP_KERNEL_MATVEC, SP_KERNEL_UPDATE, SP_KERNEL_DIRECTION, SP_KERNEL_PRECOND = 0, 1, 2, 3

_NAMES = {SP_EINVAL: "SP_EINVAL", SP_EMESH: "SP_EMESH", SP_ENOMEM: "SP_ENOMEM",
          SP_EDEVICE: "SP_EDEVICE", SP_ENOCONV: "SP_ENOCONV", SP_EAGAIN: "SP_EAGAIN",
          SP_ENOTFOUND: "SP_ENOTFOUND"}


class SegpartError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class sp_params(C.Structure):
    _fields_ = [("tau", C.c_double), ("n_steps", C.c_int64), ("stop_tol", C.c_double),
                ("max_steps", C.c_int64), ("energy_every", C.c_int64),
                ("precision", C.c_int32), ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int32),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int32),
                ("check_every", C.c_int32), ("extrapolate", C.c_int32),
                ("precond", C.c_int32)]


class sp_stats(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("cg_iters", C.c_int64),
                ("outer_sweeps", C.c_int64), ("col_iters_max", C.c_int64),
                ("seconds", C.c_double), ("converged", C.c_int32), ("reserved", C.c_int32),
                ("hbm_bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class sp_level(C.Structure):
    _fields_ = [("eps", C.c_double), ("tau", C.c_double), ("refine", C.c_int32),
                ("reserved", C.c_int32)]


class sp_level_result(C.Structure):
    _fields_ = [("n_vert", C.c_int64), ("steps", C.c_int64), ("energy", C.c_double),
                ("s_eps", C.c_double), ("seconds", C.c_double), ("converged", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


# void (*)(double* xyz, int64_t n, void* ctx)
PROJECT_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int64, C.c_void_p)
# void (*)(int32_t level, const sp_level_result* results, void* ctx)
LEVEL_FN = C.CFUNCTYPE(None, C.c_int32, C.POINTER(sp_level_result), C.c_void_p)

_lib = None

P = C.c_void_p
PP = C.POINTER(C.c_void_p)
D = C.POINTER(C.c_double)
I32 = C.POINTER(C.c_int32)
I64 = C.POINTER(C.c_int64)

_SIGS = {
    "sp_last_error": (C.c_char_p, []),
    "sp_version": (C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "sp_params_default": (None, [C.POINTER(sp_params), C.c_double]),
    "sp_mesh_create": (C.c_int, [C.c_int64, D, C.c_int64, I32, PP]),
    "sp_mesh_info": (C.c_int, [P, I64, I64, I64, D]),
    "sp_mesh_export": (C.c_int, [P, C.c_int32, I64, I32, D]),
    "sp_mesh_destroy": (None, [P]),
    "sp_solve": (C.c_int, [P, C.POINTER(sp_params), C.c_int32, I32, D, D, D, I32, I32, D, D,
                           D, C.POINTER(sp_stats)]),
    "sp_solve_async": (C.c_int, [P, C.POINTER(sp_params), C.c_int32, I32, D, P, P, P, P, P,
                                 P, P, P]),
    "sp_solve_async_noalloc": (C.c_int, [P, C.POINTER(sp_params), C.c_int32, I32, D, P, P, P,
                                         P, P, P, P, P]),
    "sp_state_create": (C.c_int, [P, C.POINTER(sp_params), C.c_int32, I32, D, D, P, PP]),
    "sp_state_step": (C.c_int, [P, C.c_int64]),
    "sp_state_stage": (C.c_int, [P, C.c_int32]),
    "sp_state_energy": (C.c_int, [P, D, D, D]),
    "sp_state_read": (C.c_int, [P, D, I64]),
    "sp_state_multipliers": (C.c_int, [P, D]),
    "sp_state_write": (C.c_int, [P, D, C.c_int64, C.c_int32]),
    "sp_state_labels": (C.c_int, [P, I32, I32]),
    "sp_state_checkpoint_size": (C.c_int, [P, I64]),
    "sp_state_checkpoint": (C.c_int, [P, P, C.c_int64]),
    "sp_state_restore": (C.c_int, [P, P, C.c_int64]),
    "sp_state_history": (C.c_int, [P, C.c_int32, C.c_int64, I64, D, I64]),
    "sp_state_stats": (C.c_int, [P, C.POINTER(sp_stats)]),
    "sp_state_profile": (C.c_int, [P, C.c_int32]),
    "sp_state_kernel_time": (C.c_int, [P, C.c_int32, I64, D, D]),
    "sp_state_tiling": (C.c_int, [P, I32, I32, I32, D]),
    "sp_state_destroy": (None, [P]),
    "sp_server_create": (C.c_int, [C.c_int64, C.c_int32, PP]),
    "sp_server_submit": (C.c_int, [P, P, C.POINTER(sp_params), C.c_int32, I32, D, D, I64]),
    "sp_server_poll": (C.c_int, [P, C.c_int64, I32]),
    "sp_server_wait": (C.c_int, [P, C.c_int64, C.c_double]),
    "sp_server_fetch": (C.c_int, [P, C.c_int64, D, I32, D, D, D, D]),
    "sp_server_stats": (C.c_int, [P, D, D, D, I64]),
    "sp_server_request_stats": (C.c_int, [P, C.c_int64, I64, I64]),
    "sp_server_destroy": (None, [P]),
    "sp_mesh_refine": (C.c_int, [P, PROJECT_FN, P, PP]),
    "sp_mesh_parents": (C.c_int, [P, I32, I64]),
    "sp_prolong": (C.c_int, [P, C.c_int32, D, D]),
    "sp_continue": (C.c_int, [P, C.POINTER(sp_params), C.c_int32, C.c_int32, D, C.c_int32,
                              C.POINTER(sp_level), PROJECT_FN, P, C.POINTER(sp_level_result),
                              D, PP, D, LEVEL_FN, P]),
    "sp_region_eigen": (C.c_int, [P, C.c_int32, I32, I32, C.c_int32, D, C.c_double, C.c_double,
                                  C.c_int32, D, D, I32]),
    "sp_region_graph": (C.c_int, [P, C.c_int32, I32, I32, C.POINTER(C.c_uint8), I32]),
}
EXPORTED = tuple(_SIGS)


def lib():
    """Load libsegpart.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1408_2355_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _check(rc, allow=()):
    if rc < 0 and rc not in allow:
        raise SegpartError(rc, lib().sp_last_error().decode())
    return rc


def _dp(a):
    return None if a is None else a.ctypes.data_as(D)


def _ip(a, t=I32):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def params(tau, **kw):
    """sp_params with the library defaults for tau, overridden by keywords
    (precision may be given as "fp64" / "mixed")."""
    p = sp_params()
    lib().sp_params_default(C.byref(p), float(tau))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": SP_FP64, "mixed": SP_MIXED}[v]
        if k == "precond" and isinstance(v, str):
            v = {"jacobi": SP_PRECOND_JACOBI, "cheb1": SP_PRECOND_CHEB1}[v]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def sp_version():
    a, b = C.c_int(), C.c_int()
    _check(lib().sp_version(C.byref(a), C.byref(b)))
    return a.value, b.value


def sp_mesh_create(xyz, tri):
    xyz = _f64(xyz)
    tri = _i32(tri)
    h = C.c_void_p()
    _check(lib().sp_mesh_create(xyz.shape[0], _dp(xyz), tri.shape[0], _ip(tri), C.byref(h)))
    return h


def sp_mesh_info(h):
    n, t, z, a = C.c_int64(), C.c_int64(), C.c_int64(), C.c_double()
    _check(lib().sp_mesh_info(h, C.byref(n), C.byref(t), C.byref(z), C.byref(a)))
    return n.value, t.value, z.value, a.value


def sp_mesh_export(h, which):
    n, _, nnz, _ = sp_mesh_info(h)
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    _check(lib().sp_mesh_export(h, which, _ip(rp, I64), _ip(col), _dp(val)))
    return rp, col, val


def _batch(m, eps, u0=None, n=None):
    m = _i32(np.atleast_1d(m))
    eps = _f64(np.broadcast_to(np.asarray(eps, np.float64), m.shape))
    if u0 is not None:
        u0 = _f64(u0)
        if u0.shape != (int(m.sum()), n):
            raise ValueError(f"u0 must have shape ({int(m.sum())}, {n}), got {u0.shape}")
    return m, eps, u0


def sp_solve(mesh_h, prm, m, eps, u0, want_u=True, want_labels=True):
    """Returns (status, dict of outputs).  status is SP_OK or SP_ENOCONV."""
    n = sp_mesh_info(mesh_h)[0]
    m, eps, u0 = _batch(m, eps, u0, n)
    nres, R = m.size, int(m.sum())
    out = dict(lam=np.empty(R), s_eps=np.empty(nres), energy=np.empty(nres))
    if want_u:
        out["u"] = np.empty((R, n))
    if want_labels:
        out["labels"] = np.empty((nres, n), np.int32)
        out["labels_argmax"] = np.empty((nres, n), np.int32)
    st = sp_stats()
    rc = _check(lib().sp_solve(mesh_h, C.byref(prm), nres, _ip(m), _dp(eps), _dp(u0),
                               _dp(out.get("u")), _ip(out.get("labels")),
                               _ip(out.get("labels_argmax")), _dp(out["lam"]),
                               _dp(out["s_eps"]), _dp(out["energy"]), C.byref(st)),
                allow=(SP_ENOCONV,))
    out["stats"] = st.as_dict()
    return rc, out


def _tptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def sp_solve_async(mesh_h, prm, m, eps, d_u0, d_u_out=None, d_labels=None,
                   d_labels_argmax=None, d_lambda=None, d_s_eps=None, d_energy=None,
                   stream=None):
    """Device-pointer form; tensors are torch CUDA (HIP) tensors, stream a
    torch.cuda.Stream (None = the current stream)."""
    import torch
    m, eps, _ = _batch(m, eps)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().sp_solve_async(mesh_h, C.byref(prm), m.size, _ip(m), _dp(eps), _tptr(d_u0),
                                _tptr(d_u_out), _tptr(d_labels), _tptr(d_labels_argmax),
                                _tptr(d_lambda), _tptr(d_s_eps), _tptr(d_energy),
                                C.c_void_p(stream.cuda_stream)))


def sp_solve_async_noalloc(mesh_h, prm, m, eps, d_u0, d_u_out=None, d_labels=None,
                           d_labels_argmax=None, d_lambda=None, d_s_eps=None, d_energy=None,
                           stream=None):
    """Allocation-free form of sp_solve_async (the library's static scratch
    holds every work buffer; same arguments)."""
    import torch
    m, eps, _ = _batch(m, eps)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().sp_solve_async_noalloc(mesh_h, C.byref(prm), m.size, _ip(m), _dp(eps),
                                        _tptr(d_u0), _tptr(d_u_out), _tptr(d_labels),
                                        _tptr(d_labels_argmax), _tptr(d_lambda), _tptr(d_s_eps),
                                        _tptr(d_energy), C.c_void_p(stream.cuda_stream)))


def _project_cb(project):
    """C callback around project(points [k, 3]) -> projected points [k, 3]."""
    if project is None:
        return PROJECT_FN()

    def cb(ptr, n, _ctx):
        a = np.ctypeslib.as_array(ptr, shape=(int(n) * 3,)).reshape(int(n), 3)
        a[:] = project(a.copy())

    return PROJECT_FN(cb)


def sp_mesh_refine(h, project=None):
    cb = _project_cb(project)
    out = C.c_void_p()
    _check(lib().sp_mesh_refine(h, cb, None, C.byref(out)))
    return out


def sp_mesh_parents(h):
    n, _, _, _ = sp_mesh_info(h)
    nc = C.c_int64()
    _check(lib().sp_mesh_parents(h, None, C.byref(nc)))
    par = np.empty((n - nc.value, 2), np.int32)
    _check(lib().sp_mesh_parents(h, _ip(par), None))
    return par, nc.value


def sp_prolong(fine_h, u_coarse):
    u = _f64(np.atleast_2d(u_coarse))
    n, _, _, _ = sp_mesh_info(fine_h)
    out = np.empty((u.shape[0], n))
    _check(lib().sp_prolong(fine_h, u.shape[0], _dp(u), _dp(out)))
    return out


def sp_continue(mesh_h, prm, m, u0, levels, project=None, want_u=True, n_restarts=1,
                on_level=None):
    """levels: sequence of (eps, tau, refine); u0 [n_restarts * m, n];
    on_level(level, [n_restarts result dicts]) is called after each level.
    Returns (status, results [n_levels][n_restarts] dicts, lambda
    [n_levels, n_restarts * m], final mesh handle or None, u_final)."""
    n0, t0, _, _ = sp_mesh_info(mesh_h)
    u0 = _f64(u0)
    R = n_restarts * m
    if u0.shape != (R, n0):
        raise ValueError(f"u0 must have shape ({R}, {n0}), got {u0.shape}")
    lv = (sp_level * len(levels))()
    n, t = n0, t0
    for i, (eps, tau, ref) in enumerate(levels):
        lv[i].eps, lv[i].tau, lv[i].refine = float(eps), float(tau), int(bool(ref))
        if ref:  # closed surface: one new vertex per edge, 3 t / 2 edges
            n, t = n + 3 * t // 2, 4 * t
    res = (sp_level_result * (len(levels) * n_restarts))()
    lam = np.empty((len(levels), R))
    u = np.empty((R, n)) if want_u else None
    fin = C.c_void_p()
    cb = _project_cb(project)
    if on_level is None:
        lcb = LEVEL_FN()
    else:
        def _lcb(level, ptr, _ctx):
            on_level(int(level), [ptr[r].as_dict() for r in range(n_restarts)])
        lcb = LEVEL_FN(_lcb)
    rc = _check(lib().sp_continue(mesh_h, C.byref(prm), n_restarts, m, _dp(u0), len(levels), lv,
                                  cb, None, res, _dp(lam), C.byref(fin), _dp(u), lcb, None),
                allow=(SP_ENOCONV,))
    out = [[res[l * n_restarts + r].as_dict() for r in range(n_restarts)]
           for l in range(len(levels))]
    return rc, out, lam, (fin if fin.value else None), u


def sp_region_eigen(mesh_h, m, labels, u0=None, shift=1e3, tol=1e-12, max_iter=500,
                    want_u=False, interior=False):
    """Returns (status, lambda [sum m], u [sum m, n] or None, iterations)."""
    n = sp_mesh_info(mesh_h)[0]
    m = _i32(np.atleast_1d(m))
    lab = _i32(np.atleast_2d(labels))
    if lab.shape != (m.size, n):
        raise ValueError(f"labels must have shape ({m.size}, {n}), got {lab.shape}")
    R = int(m.sum())
    if u0 is not None:
        u0 = _f64(u0)
        if u0.shape != (R, n):
            raise ValueError(f"u0 must have shape ({R}, {n}), got {u0.shape}")
    lam = np.empty(R)
    u = np.empty((R, n)) if want_u else None
    it = C.c_int32()
    rc = _check(lib().sp_region_eigen(mesh_h, m.size, _ip(m), _ip(lab), int(bool(interior)),
                                      _dp(u0), float(shift),
                                      float(tol), int(max_iter), _dp(lam), _dp(u), C.byref(it)),
                allow=(SP_ENOCONV,))
    return rc, lam, u, it.value


def sp_region_graph(mesh_h, m, labels):
    """Returns (list of adjacency matrices [m_r, m_r] bool, sides [sum m])."""
    n = sp_mesh_info(mesh_h)[0]
    m = _i32(np.atleast_1d(m))
    lab = _i32(np.atleast_2d(labels))
    if lab.shape != (m.size, n):
        raise ValueError(f"labels must have shape ({m.size}, {n}), got {lab.shape}")
    adj = np.zeros(int((m.astype(np.int64) ** 2).sum()), np.uint8)
    sides = np.empty(int(m.sum()), np.int32)
    _check(lib().sp_region_graph(mesh_h, m.size, _ip(m), _ip(lab),
                                 adj.ctypes.data_as(C.POINTER(C.c_uint8)), _ip(sides)))
    out, o = [], 0
    for k in m:
        out.append(adj[o:o + k * k].reshape(k, k).astype(bool))
        o += k * k
    return out, sides


class Mesh:
    """Owner of an sp_mesh handle."""

    def __init__(self, xyz=None, tri=None, handle=None):
        self.h = sp_mesh_create(xyz, tri) if handle is None else handle
        self.n_vert, self.n_tri, self.nnz, self.area = sp_mesh_info(self.h)

    def refine(self, project=None):
        """4-fold midpoint refinement; project(points [k, 3]) moves the new
        vertices onto the surface."""
        return Mesh(handle=sp_mesh_refine(self.h, project))

    def parents(self):
        """(parents [n_new, 2], n_coarse) of a refined mesh."""
        return sp_mesh_parents(self.h)

    def prolong(self, u_coarse):
        """u_coarse [cols, n_coarse] -> [cols, n_vert] on this refined mesh."""
        return sp_prolong(self.h, u_coarse)

    def export(self, which):
        """(row_ptr, col, val) CSR of M (SP_MAT_M) or A (SP_MAT_A)."""
        return sp_mesh_export(self.h, which)

    def close(self):
        if getattr(self, "h", None):
            sp_mesh_destroy(self.h)
            self.h = None

    __del__ = close


def solve(mesh, prm, m, eps, u0, **kw):
    return sp_solve(mesh.h, prm, m, eps, u0, **kw)


def continue_levels(mesh, prm, m, u0, levels, project=None, want_u=True, n_restarts=1,
                    on_level=None):
    """sp_continue on a Mesh; the final mesh comes back as a Mesh (or None)."""
    rc, res, lam, fin, u = sp_continue(mesh.h, prm, m, u0, levels, project, want_u, n_restarts,
                                       on_level)
    return rc, res, lam, (Mesh(handle=fin) if fin is not None else None), u


# ------------------------------------------------------------------------
# Entry points that the State and Server owners below use: one function per
# C entry point, same name, handles passed as the first argument.

def sp_last_error():
    return lib().sp_last_error().decode()


def sp_params_default(tau):
    p = sp_params()
    lib().sp_params_default(C.byref(p), float(tau))
    return p


def sp_mesh_destroy(h):
    lib().sp_mesh_destroy(h)


def sp_state_create(mesh_h, prm, m, eps, u0, stream=None):
    n = sp_mesh_info(mesh_h)[0]
    m, eps, u0 = _batch(m, eps, u0, n)
    h = C.c_void_p()
    s = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(lib().sp_state_create(mesh_h, C.byref(prm), m.size, _ip(m), _dp(eps), _dp(u0), s,
                                 C.byref(h)))
    return h


def sp_state_step(h, k=1):
    return _check(lib().sp_state_step(h, int(k)), allow=(SP_ENOCONV,))


def sp_state_stage(h, which):
    _check(lib().sp_state_stage(h, int(which)))


def sp_state_energy(h, R, nres):
    lam, s, e = np.empty(R), np.empty(nres), np.empty(nres)
    _check(lib().sp_state_energy(h, _dp(lam), _dp(s), _dp(e)))
    return lam, s, e


def sp_state_read(h, R, n):
    u = np.empty((R, n))
    k = C.c_int64()
    _check(lib().sp_state_read(h, _dp(u), C.byref(k)))
    return u, k.value


def sp_state_write(h, u, step=0, normalise=False):
    u = _f64(u)
    _check(lib().sp_state_write(h, _dp(u), int(step), int(bool(normalise))))


def sp_state_multipliers(h, R):
    out = np.empty(R)
    _check(lib().sp_state_multipliers(h, _dp(out)))
    return out


def sp_state_checkpoint_size(h):
    b = C.c_int64()
    _check(lib().sp_state_checkpoint_size(h, C.byref(b)))
    return b.value


def sp_state_checkpoint(h):
    """The state's checkpoint image as a numpy uint8 array."""
    buf = np.empty(sp_state_checkpoint_size(h), np.uint8)
    _check(lib().sp_state_checkpoint(h, buf.ctypes.data_as(P), buf.size))
    return buf


def sp_state_restore(h, image):
    image = np.ascontiguousarray(image, np.uint8)
    _check(lib().sp_state_restore(h, image.ctypes.data_as(P), image.size))


def sp_state_labels(h, nres, n):
    a = np.empty((nres, n), np.int32)
    b = np.empty_like(a)
    _check(lib().sp_state_labels(h, _ip(a), _ip(b)))
    return a, b


def sp_state_history(h, r):
    cnt = C.c_int64()
    _check(lib().sp_state_history(h, r, 0, None, None, C.byref(cnt)))
    k = np.empty(cnt.value, np.int64)
    e = np.empty(cnt.value)
    _check(lib().sp_state_history(h, r, cnt.value, _ip(k, I64), _dp(e), C.byref(cnt)))
    return k, e


def sp_state_stats(h):
    st = sp_stats()
    _check(lib().sp_state_stats(h, C.byref(st)))
    return st.as_dict()


def sp_state_profile(h, on=True):
    _check(lib().sp_state_profile(h, int(bool(on))))


def sp_state_kernel_time(h, which=SP_KERNEL_MATVEC):
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    _check(lib().sp_state_kernel_time(h, int(which), C.byref(n), C.byref(ms), C.byref(b)))
    return n.value, ms.value, b.value


def sp_state_tiling(h):
    a, b, c, us = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().sp_state_tiling(h, C.byref(a), C.byref(b), C.byref(c), C.byref(us)))
    return dict(lanes_per_row=a.value, rows_per_chunk=b.value, groups_per_xcd=c.value,
                matvec_us=us.value)


def sp_state_destroy(h):
    lib().sp_state_destroy(h)


def sp_server_create(hbm_budget_bytes, max_batch_columns=0):
    h = C.c_void_p()
    _check(lib().sp_server_create(int(hbm_budget_bytes), int(max_batch_columns), C.byref(h)))
    return h


def sp_server_submit(h, mesh_h, prm, m, eps, u0):
    n = sp_mesh_info(mesh_h)[0]
    m, eps, u0 = _batch(m, eps, u0, n)
    t = C.c_int64()
    _check(lib().sp_server_submit(h, mesh_h, C.byref(prm), m.size, _ip(m), _dp(eps), _dp(u0),
                                  C.byref(t)))
    return t.value


def sp_server_poll(h, ticket):
    d = C.c_int32()
    _check(lib().sp_server_poll(h, int(ticket), C.byref(d)))
    return bool(d.value)


def sp_server_wait(h, ticket, timeout_s=600.0):
    return _check(lib().sp_server_wait(h, int(ticket), float(timeout_s)),
                  allow=(SP_EAGAIN,)) == SP_OK


def sp_server_fetch(h, ticket, R, nres, n):
    out = dict(u=np.empty((R, n)), labels=np.empty((nres, n), np.int32), lam=np.empty(R),
               s_eps=np.empty(nres), energy=np.empty(nres))
    lat = C.c_double()
    _check(lib().sp_server_fetch(h, int(ticket), _dp(out["u"]), _ip(out["labels"]),
                                 _dp(out["lam"]), _dp(out["s_eps"]), _dp(out["energy"]),
                                 C.byref(lat)))
    out["latency_s"] = lat.value
    return out


def sp_server_request_stats(h, ticket):
    it, st = C.c_int64(), C.c_int64()
    _check(lib().sp_server_request_stats(h, int(ticket), C.byref(it), C.byref(st)))
    return dict(col_iters=it.value, steps=st.value)


def sp_server_stats(h):
    p50, p99, cd, n = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
    _check(lib().sp_server_stats(h, C.byref(p50), C.byref(p99), C.byref(cd), C.byref(n)))
    return dict(p50_s=p50.value, p99_s=p99.value, cdof_per_s=cd.value, completed=n.value)


def sp_server_destroy(h):
    lib().sp_server_destroy(h)


class State:
    """Owner of an sp_state handle (a batch kept on the GPU)."""

    def __init__(self, mesh, prm, m, eps, u0, stream=None):
        self.mesh = mesh
        self.m, self.eps, _ = _batch(m, eps)
        self.R = int(self.m.sum())
        self.h = sp_state_create(mesh.h, prm, m, eps, u0, stream)

    def step(self, k=1):
        return sp_state_step(self.h, k)

    def stage(self, which):
        sp_state_stage(self.h, which)

    def energy(self):
        return sp_state_energy(self.h, self.R, self.m.size)

    def read(self):
        return sp_state_read(self.h, self.R, self.mesh.n_vert)

    def write(self, u, step=0, normalise=False):
        sp_state_write(self.h, u, step, normalise)

    def checkpoint(self):
        """Checkpoint image (numpy uint8) of the whole device state."""
        return sp_state_checkpoint(self.h)

    def restore(self, image):
        """Continue exactly from an image of sp_state_checkpoint (same batch)."""
        sp_state_restore(self.h, image)

    def multipliers(self):
        """lambda_i^eps [sum m] of the current state."""
        return sp_state_multipliers(self.h, self.R)

    def labels(self):
        return sp_state_labels(self.h, self.m.size, self.mesh.n_vert)

    def history(self, r):
        return sp_state_history(self.h, r)

    def stats(self):
        return sp_state_stats(self.h)

    def profile(self, on=True):
        sp_state_profile(self.h, on)

    def kernel_time(self, which=SP_KERNEL_MATVEC):
        """(launches, total ms, algorithmic bytes per launch) of a kernel class."""
        return sp_state_kernel_time(self.h, which)

    def tiling(self):
        """Tiling of the row-parallel kernels (see sp_state_tiling)."""
        return sp_state_tiling(self.h)

    def close(self):
        if getattr(self, "h", None):
            sp_state_destroy(self.h)
            self.h = None

    __del__ = close


class Server:
    """Owner of an sp_server handle (continuous-batching request loop).

    Each request runs on its mesh's device buffers until it is fetched, so
    the Mesh object is kept referenced per ticket until then (and until the
    server is closed)."""

    def __init__(self, hbm_budget_bytes, max_batch_columns=0):
        self.h = sp_server_create(hbm_budget_bytes, max_batch_columns)
        self._shape = {}
        self._mesh = {}

    def submit(self, mesh, prm, m, eps, u0):
        mm, _, _ = _batch(m, eps)
        t = sp_server_submit(self.h, mesh.h, prm, m, eps, u0)
        self._shape[t] = (int(mm.sum()), mm.size, mesh.n_vert)
        self._mesh[t] = mesh
        return t

    def poll(self, ticket):
        return sp_server_poll(self.h, ticket)

    def wait(self, ticket, timeout_s=600.0):
        return sp_server_wait(self.h, ticket, timeout_s)

    def request_stats(self, ticket):
        """CG column-iterations and steps of a finished, not yet fetched request."""
        return sp_server_request_stats(self.h, ticket)

    def fetch(self, ticket):
        R, nres, n = self._shape[ticket]
        try:
            out = sp_server_fetch(self.h, ticket, R, nres, n)
        except SegpartError as e:
            if e.code != SP_EAGAIN:  # the request is gone (failed): release it
                self._shape.pop(ticket, None)
                self._mesh.pop(ticket, None)
            raise
        del self._shape[ticket]
        del self._mesh[ticket]
        return out

    def stats(self):
        return sp_server_stats(self.h)

    def close(self):
        if getattr(self, "h", None):
            sp_server_destroy(self.h)  # stops every batch before the meshes go
            self.h = None
        if getattr(self, "_mesh", None):
            self._mesh.clear()

    __del__ = close
