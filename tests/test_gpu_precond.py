"""The CG's degree-1 Chebyshev polynomial preconditioner (sp_params.precond).

Preconditioning changes only how each heat solve (M + tau A) u~ = M u of
Algorithm 2.2 converges, never what it converges to: with either
preconditioner the flow matches the oracle (exact sparse LU solves) to the
solver tolerance, the two runs match each other, and the polynomial form
needs fewer iterations.  Checked in float64 and in mixed precision, on
surfaces and time steps whose spectra of D^-1 (M + tau A) differ (condition
numbers of about 2, 10 and 90), and on region-restricted solves.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import flow  # noqa: E402
from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import icosphere, torus, batch_u0  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [  # surface, tau, steps
    ("sphere5", 5e-5, 12),
    ("sphere5", 2e-3, 8),
    ("torus", 2e-2, 6),
]


def _surface(name):
    return icosphere(5) if name == "sphere5" else torus(96, 64)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("surface,tau,steps", CASES)
def test_cheb1_matches_jacobi_and_oracle_in_fewer_iterations(precision, surface, tau, steps):
    v, f = _surface(surface)
    u0, ms = batch_u0(v.shape[0], [(61, 2, 4), (62, 1, 7)])   # 15 columns, ragged m
    eps = np.array([0.06, 0.06, 0.09])
    print(f"precond {precision} {surface} tau {tau}: n={v.shape[0]}", flush=True)
    mesh = sp.Mesh(v, f)
    out = {}
    for pc in ("jacobi", "cheb1"):
        prm = sp.params(tau, precision=precision, n_steps=steps, energy_every=0,
                        cg_rtol=1e-12, precond=pc)
        rc, o = sp.solve(mesh, prm, ms, eps, u0)
        assert rc == sp.SP_OK and o["stats"]["converged"] == 1
        out[pc] = o
    mesh.close()
    ref = flow.run(flow.Problem(v, f, tau), u0[:4], [4], [0.06], steps)
    bar = 1e-9 if precision == "fp64" else 1e-7
    a, b = out["cheb1"], out["jacobi"]
    assert rel(a["u"], b["u"]) < bar
    assert rel(a["lam"], b["lam"]) < bar
    assert rel(a["u"][:4], ref["u"]) < bar
    assert rel(a["lam"][:4], ref["lam"]) < bar
    assert rel(a["s_eps"][:1], ref["s_eps"]) < bar
    # about half the iterations (each costs one more gather pass)
    assert a["stats"]["cg_iters"] < 0.8 * b["stats"]["cg_iters"], (
        a["stats"]["cg_iters"], b["stats"]["cg_iters"])


def test_cheb1_state_stepping_matches_one_call():
    """Stepping a state one step per call (the preconditioner pass's start
    and partial sums set up afresh each heat solve) gives the bits of one
    call over all steps."""
    v, f = icosphere(5)
    u0, ms = batch_u0(v.shape[0], [(63, 3, 3)])
    eps = np.full(ms.size, 0.08)
    mesh = sp.Mesh(v, f)
    prm = sp.params(5e-4, precision="mixed", n_steps=1, energy_every=0, precond="cheb1")
    a = sp.State(mesh, prm, ms, eps, u0)
    b = sp.State(mesh, prm, ms, eps, u0)
    a.step(9)
    for _ in range(9):
        b.step(1)
    ua, ub = a.read()[0], b.read()[0]
    a.close()
    b.close()
    mesh.close()
    assert np.array_equal(ua, ub)


@pytest.mark.parametrize("pc", ["jacobi", "cheb1"])
def test_kernel_profile_classes(pc):
    """sp_state_kernel_time: the preconditioner pass is a class of its own
    (launched once per iteration with the polynomial preconditioner, never
    with Jacobi), every class reports positive algorithmic bytes."""
    v, f = icosphere(5)
    u0, ms = batch_u0(v.shape[0], [(64, 2, 5)])
    mesh = sp.Mesh(v, f)
    prm = sp.params(5e-4, precision="mixed", n_steps=1, energy_every=0, precond=pc)
    st = sp.State(mesh, prm, ms, np.full(ms.size, 0.08), u0)
    st.step(2)
    st.profile(True)
    st.step(3)
    kt = [st.kernel_time(k) for k in range(4)]
    st.profile(False)
    st.close()
    mesh.close()
    n_iter = kt[sp.SP_KERNEL_MATVEC][0]
    assert n_iter > 0
    for k in range(3):
        assert kt[k][0] == n_iter and kt[k][1] > 0 and kt[k][2] > 0
    if pc == "cheb1":
        assert kt[sp.SP_KERNEL_PRECOND][0] == n_iter and kt[sp.SP_KERNEL_PRECOND][2] > 0
    else:
        assert kt[sp.SP_KERNEL_PRECOND][0] == 0


def test_deferred_iterate_when_the_solve_ends_early():
    """A refinement sweep 0 predicted to be followed by another keeps its
    correction and leaves the iterate to the next sweep; when the step then
    converges after sweep 0 after all (a step with one sweep right after one
    with two), a last update forms the iterate.  The run passes through such
    steps and still matches the oracle."""
    v, f = icosphere(5)
    u0, ms = batch_u0(v.shape[0], [(65, 2, 4)])
    eps = np.full(ms.size, 0.05)
    tau = 2e-4
    mesh = sp.Mesh(v, f)
    prm = sp.params(tau, precision="mixed", n_steps=1, energy_every=0, cg_rtol=1e-10)
    st = sp.State(mesh, prm, ms, eps, u0)
    sweeps, steps, seen = [], 0, -1
    while steps < 120 and (seen < 0 or steps < seen + 5):
        s0 = st.stats()["outer_sweeps"]
        st.step(1)
        steps += 1
        sweeps.append(st.stats()["outer_sweeps"] - s0)
        if seen < 0 and len(sweeps) >= 2 and sweeps[-2] >= 2 and sweeps[-1] == 1:
            seen = steps
    u, k = st.read()
    st.close()
    mesh.close()
    assert seen > 0, sweeps
    ref = flow.run(flow.Problem(v, f, tau), u0[:4], [4], [0.05], k)
    assert rel(u[:4], ref["u"]) < 1e-5
