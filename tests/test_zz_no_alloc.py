"""The allocation-free entry point sp_solve_async_noalloc against the
allocating sp_solve_async, through the C ABI.

Same inputs on the same stream, two calls in a row, the second with a smaller
batch on a smaller mesh (so it runs over what the first left in the shared
scratch): every output agrees within 1e-12 (the same kernels and tilings; in
practice bit for bit, since neither path searches tilings at these sizes).  The
first call runs the multi-kernel mixed-precision path, the second the
one-workgroup float64 path.  A batch whose buffers exceed the scratch is
rejected with SP_ENOMEM before any work, leaving the outputs untouched.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import icosphere, batch_u0  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _outputs(R, nres, n, dev):
    nan = float("nan")
    return dict(u=torch.full((R, n), nan, dtype=torch.float64, device=dev),
                lab=torch.full((nres, n), -7, dtype=torch.int32, device=dev),
                lab_am=torch.full((nres, n), -7, dtype=torch.int32, device=dev),
                lam=torch.full((R,), nan, dtype=torch.float64, device=dev),
                s_eps=torch.full((nres,), nan, dtype=torch.float64, device=dev),
                energy=torch.full((nres,), nan, dtype=torch.float64, device=dev))


def _call(fn, mesh, prm, ms, eps, d_u0, out, stream):
    fn(mesh.h, prm, ms, eps, d_u0, d_u_out=out["u"], d_labels=out["lab"],
       d_labels_argmax=out["lab_am"], d_lambda=out["lam"], d_s_eps=out["s_eps"],
       d_energy=out["energy"], stream=stream)


def _rel(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [
    # (icosphere level, groups (seed, restarts, m), eps, tau, steps, precision)
    (4, [(9101, 2, 4), (9102, 1, 5)], 0.08, 1e-3, 12, "mixed"),   # 13 columns, multi-kernel
    (3, [(9103, 2, 3)], 0.1, 1e-3, 9, "fp64"),                    # 6 columns, one workgroup
]


def test_noalloc_matches_the_allocating_call_twice():
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    for level, groups, eps, tau, steps, precision in CASES:
        v, f = icosphere(level)
        n = v.shape[0]
        u0, ms = batch_u0(n, groups)
        R, nres = int(ms.sum()), ms.size
        epsv = np.full(nres, eps)
        mesh = sp.Mesh(v, f)
        prm = sp.params(tau, precision=precision, n_steps=steps, energy_every=0)
        d_u0 = torch.from_numpy(u0).to(dev)
        print(f"no-alloc call: level {level}, {R} columns, {precision}", flush=True)
        ref, got = _outputs(R, nres, n, dev), _outputs(R, nres, n, dev)
        with torch.cuda.stream(s):
            _call(sp.sp_solve_async, mesh, prm, ms, epsv, d_u0, ref, s)
            _call(sp.sp_solve_async_noalloc, mesh, prm, ms, epsv, d_u0, got, s)
        s.synchronize()
        for key in ("u", "lam", "s_eps", "energy"):
            assert torch.isfinite(got[key]).all(), key
            assert _rel(got[key], ref[key]) <= 1e-12, key
        assert torch.equal(got["lab"], ref["lab"])
        assert torch.equal(got["lab_am"], ref["lab_am"])
        mesh.close()


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    dev = torch.device("cuda:0")
    v, f = icosphere(6)                     # 40962 vertices x 192 columns: ~0.7 GB of buffers
    n = v.shape[0]
    u0, ms = batch_u0(n, [(9104, 16, 12)])
    R, nres = int(ms.sum()), ms.size
    mesh = sp.Mesh(v, f)
    prm = sp.params(1e-4, precision="mixed", n_steps=2, energy_every=0)
    d_u0 = torch.from_numpy(u0).to(dev)
    out = _outputs(R, nres, n, dev)
    s = torch.cuda.Stream()
    with pytest.raises(sp.SegpartError) as e:
        _call(sp.sp_solve_async_noalloc, mesh, prm, ms, np.full(nres, 0.02), d_u0, out, s)
    s.synchronize()
    assert e.value.code == sp.SP_ENOMEM and "128 MiB" in str(e.value)
    assert torch.isnan(out["energy"]).all() and (out["lab"] == -7).all()
    mesh.close()
