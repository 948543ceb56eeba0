"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/segpart.h, and rejects invalid meshes and parameters
before touching the GPU."""
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
    assert sp.sp_version() == (1, 1)
    p = sp.params(5e-5)
    assert p.tau == 5e-5 and p.energy_every == 2000 and p.precision == sp.SP_MIXED
    assert p.cg_rtol == 1e-10 and p.check_every == 8
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
