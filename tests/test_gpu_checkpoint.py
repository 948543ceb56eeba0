"""Checkpoint and resume through the C ABI (sp_state_checkpoint / _restore).

A run interrupted after k steps, checkpointed, restored into a fresh state
and continued must give exactly (bit for bit) the state, energies and energy
history of the uninterrupted run, in float64 and in mixed precision (where
the heat solves start from an extrapolation of each column's previous heat
increments and the last normalisation may still be pending).  A restore into
a different batch is rejected and leaves the state untouched.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import flow  # noqa: E402
from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import icosphere, batch_u0  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def sphere5():
    v, f = icosphere(5)
    mesh = sp.Mesh(v, f)
    yield v, f, mesh
    mesh.close()


GROUPS = [(5101, 3, 4), (5102, 2, 7), (5103, 2, 3)]   # 6 + 14 + 6 = 26 columns, unaligned m


def _run(mesh, prm, ms, eps, u0, k1, k2, checkpoint_at=None):
    st = sp.State(mesh, prm, ms, eps, u0)
    st.step(k1)
    img = st.checkpoint() if checkpoint_at else None
    st.step(k2)
    u, step = st.read()
    lam, s, e = st.energy()
    hist = [st.history(r) for r in range(len(ms))]
    stats = st.stats()
    st.close()
    return dict(u=u, step=step, lam=lam, s=s, e=e, hist=hist, stats=stats), img


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_from_checkpoint_is_exact(sphere5, precision):
    v, f, mesh = sphere5
    u0, ms = batch_u0(v.shape[0], GROUPS)
    eps = np.array([0.08] * 3 + [0.1] * 2 + [0.12] * 2)
    prm = sp.params(5e-4, precision=precision, n_steps=1, energy_every=3, cg_rtol=1e-10)
    print(f"checkpoint {precision}: uninterrupted run", flush=True)
    full, img = _run(mesh, prm, ms, eps, u0, 7, 8, checkpoint_at=7)
    assert img.size > 0
    print(f"checkpoint {precision}: resumed run", flush=True)
    st = sp.State(mesh, prm, ms, eps, u0)
    st.step(2)                       # a different state and history, then replaced
    st.restore(img)
    assert st.read()[1] == 7
    st.step(8)
    u, step = st.read()
    lam, s, e = st.energy()
    hist = [st.history(r) for r in range(len(ms))]
    st.close()
    assert step == full["step"] == 15
    assert np.array_equal(u, full["u"])
    assert np.array_equal(lam, full["lam"])
    assert np.array_equal(s, full["s"]) and np.array_equal(e, full["e"])
    for (k0, e0), (k1, e1) in zip(full["hist"], hist):
        assert np.array_equal(k0, k1) and np.array_equal(e0, e1)
    # and the uninterrupted run itself is right (oracle, restart 0 of each group)
    ref = flow.run(flow.Problem(v, f, 5e-4), u0[:4], [4], [0.08], 15)
    tol = 1e-8 if precision == "fp64" else 1e-5   # cg_rtol 1e-10 over 15 steps
    assert np.abs(full["u"][:4] - ref["u"]).max() < tol * np.abs(ref["u"]).max()


def test_write_restarts_the_extrapolation_but_stays_within_tolerance(sphere5):
    """sp_state_write forgets the kept increments: the continued mixed run
    agrees with the uninterrupted one to the solver tolerance only."""
    v, f, mesh = sphere5
    u0, ms = batch_u0(v.shape[0], GROUPS)
    eps = np.full(ms.size, 0.1)
    prm = sp.params(5e-4, precision="mixed", n_steps=1, energy_every=0, cg_rtol=1e-10)
    full, _ = _run(mesh, prm, ms, eps, u0, 6, 6)
    st = sp.State(mesh, prm, ms, eps, u0)
    st.step(6)
    u6, k = st.read()
    st2 = sp.State(mesh, prm, ms, eps, u0)
    st2.write(u6, step=k)
    st2.step(6)
    u, _ = st2.read()
    st.close()
    st2.close()
    assert np.abs(u - full["u"]).max() < 1e-7 * np.abs(full["u"]).max()


def test_restore_rejects_another_batch(sphere5):
    v, f, mesh = sphere5
    u0, ms = batch_u0(v.shape[0], GROUPS)
    eps = np.full(ms.size, 0.1)
    prm = sp.params(5e-4, precision="mixed", n_steps=1, energy_every=0)
    a = sp.State(mesh, prm, ms, eps, u0)
    a.step(3)
    img = a.checkpoint()
    u_before = a.read()[0]
    # other eps for one restart
    eps2 = eps.copy()
    eps2[-1] = 0.2
    b = sp.State(mesh, prm, ms, eps2, u0)
    with pytest.raises(sp.SegpartError) as e:
        b.restore(img)
    assert e.value.code == sp.SP_EINVAL
    # other precision
    c = sp.State(mesh, sp.params(5e-4, precision="fp64", n_steps=1, energy_every=0), ms, eps, u0)
    with pytest.raises(sp.SegpartError) as e:
        c.restore(img)
    assert e.value.code == sp.SP_EINVAL
    # truncated and corrupted images
    with pytest.raises(sp.SegpartError) as e:
        a.restore(img[: img.size // 2])
    assert e.value.code == sp.SP_EINVAL
    bad = img.copy()
    bad[:8] = 0
    with pytest.raises(sp.SegpartError) as e:
        a.restore(bad)
    assert e.value.code == sp.SP_EINVAL
    assert np.array_equal(a.read()[0], u_before)     # state untouched
    for s in (a, b, c):
        s.close()


def test_reading_the_state_does_not_perturb_the_run(sphere5):
    """A mixed step may leave its normalisation pending (applied as the next
    step reads the state); reading the state in between applies it to the
    stored copy instead.  Both routes give the same bits."""
    v, f, mesh = sphere5
    u0, ms = batch_u0(v.shape[0], GROUPS)
    eps = np.full(ms.size, 0.1)
    prm = sp.params(5e-4, precision="mixed", n_steps=1, energy_every=4)
    a = sp.State(mesh, prm, ms, eps, u0)
    b = sp.State(mesh, prm, ms, eps, u0)
    a.step(9)
    for k in range(9):
        b.step(1)
        b.read()                      # every step: flushes the pending factor
        b.labels()
    ua, ub = a.read()[0], b.read()[0]
    assert np.array_equal(ua, ub)
    assert np.array_equal(a.energy()[2], b.energy()[2])
    a.close()
    b.close()
