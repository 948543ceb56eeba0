"""Edge cases of the time step through the C ABI, against the oracle.

* m = 1: S_eps = 0 and the node step is the identity, so the flow is the
  normalised heat flow; float64 and mixed;
* the smallest mesh (the icosahedron, 12 vertices) with m = 2, 3 and 33 in
  one batch (33 crosses the 8-component blocks of the S_eps kernels and the
  4-column groups), on the one-workgroup path and the multi-kernel path;
* step(0) is rejected (SP_EINVAL) and changes nothing; a ragged batch of
  130 restarts of m = 2 (more restarts than one S_eps tile holds) against
  the oracle on sampled restarts.
Float64 bar 1e-10 (CG rtol 1e-13), mixed 1e-5.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import flow  # noqa: E402
from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import icosahedron, icosphere, uniform_u0  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def run_gpu(v, f, ms, eps, u0, tau, steps, precision):
    mesh = sp.Mesh(v, f)
    prm = sp.params(tau, n_steps=steps, precision=precision, energy_every=0,
                    cg_rtol=1e-13 if precision == "fp64" else 1e-10)
    rc, out = sp.solve(mesh, prm, ms, eps, u0)
    mesh.close()
    assert rc == sp.SP_OK
    return out


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_single_component_is_the_normalised_heat_flow(gpu, precision, bar):
    v, f = icosphere(3)
    u0 = uniform_u0(41, 1, 1, v.shape[0])
    print(f"m = 1, 40 steps, {precision}", flush=True)
    out = run_gpu(v, f, [1], [0.05], u0, 1e-3, 40, precision)
    ref = flow.run(flow.Problem(v, f, 1e-3), u0, [1], [0.05], 40)
    assert out["s_eps"][0] == 0.0
    assert rel(out["u"], ref["u"]) < bar
    assert abs(out["lam"][0] - ref["lam"][0]) < bar * ref["lam"][0]
    assert abs(out["energy"][0] - out["lam"][0]) == 0.0


@pytest.mark.parametrize("small", ["1", "0"])
def test_icosahedron_with_odd_m(gpu, monkeypatch, small):
    monkeypatch.setenv("SEGPART_SMALL", small)
    v, f = icosahedron()
    ms, eps = [2, 3, 33], [0.3, 0.2, 0.5]
    u0 = uniform_u0(42, 1, sum(ms), v.shape[0])
    print(f"icosahedron, m = 2, 3, 33, one-workgroup path {small}", flush=True)
    out = run_gpu(v, f, ms, eps, u0, 2e-3, 25, "fp64")
    ref = flow.run(flow.Problem(v, f, 2e-3), u0, ms, eps, 25)
    assert rel(out["u"], ref["u"]) < 1e-10
    assert rel(out["lam"], ref["lam"]) < 1e-10
    assert rel(out["s_eps"], ref["s_eps"]) < 1e-10
    assert rel(out["energy"], ref["energy"]) < 1e-10


def test_zero_steps_and_many_restarts(gpu):
    v, f = icosphere(2)
    n = v.shape[0]
    R = 130
    ms = [2] * R
    eps = list(np.linspace(0.1, 0.3, R))
    u0 = uniform_u0(43, R, 2, n).reshape(2 * R, n)
    mesh = sp.Mesh(v, f)
    prm = sp.params(1e-3, precision="fp64", n_steps=1, energy_every=0, cg_rtol=1e-13)
    st = sp.State(mesh, prm, ms, eps, u0)
    try:
        u_before, k0 = st.read()
        with pytest.raises(sp.SegpartError) as err:  # k >= 1 (header); the state is untouched
            st.step(0)
        assert err.value.code == sp.SP_EINVAL
        u_after, k1 = st.read()
        assert k0 == k1 == 0 and np.array_equal(u_before, u_after)
        print("130 restarts of m = 2, 10 steps", flush=True)
        assert st.step(10) == sp.SP_OK
        lam, s_eps, e = st.energy()
        u, _ = st.read()
    finally:
        st.close()
        mesh.close()
    prob = flow.Problem(v, f, 1e-3)
    for r in (0, 63, 64, 129):
        ref = flow.run(prob, u0[2 * r:2 * r + 2], [2], [eps[r]], 10)
        assert rel(u[2 * r:2 * r + 2], ref["u"]) < 1e-10
        assert abs(s_eps[r] - ref["s_eps"][0]) < 1e-10 * ref["s_eps"][0]
        assert abs(e[r] - ref["energy"][0]) < 1e-10 * ref["energy"][0]


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_wide_batch_node_step_paths(gpu, precision, bar):
    """A batch wider than one 256-column tile (one row per wavefront): 64
    restarts of m = 4 fill tile 0 (the node step's cross-lane sums), then m =
    12 restarts straddle the next tile edges (the general path) and m = 3 ones
    break the 4-column alignment; sampled restarts against the oracle."""
    v, f = icosphere(3)
    n = v.shape[0]
    ms = [4] * 64 + [12] * 24 + [3] * 5
    eps = [0.1] * len(ms)
    u0 = uniform_u0(44, 1, sum(ms), n)
    print(f"wide batch ({sum(ms)} columns), 15 steps, {precision}", flush=True)
    out = run_gpu(v, f, ms, eps, u0, 1e-3, 15, precision)
    prob = flow.Problem(v, f, 1e-3)
    col0 = np.concatenate([[0], np.cumsum(ms)])
    for r in (0, 63, 64, 70, 87, 88, 92):
        ref = flow.run(prob, u0[col0[r]:col0[r + 1]], [ms[r]], [0.1], 15)
        assert rel(out["u"][col0[r]:col0[r + 1]], ref["u"]) < bar
        assert abs(out["energy"][r] - ref["energy"][0]) < bar * ref["energy"][0]


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_node_step_restarts_of_any_length_across_tile_edges(gpu, precision, bar):
    """Restarts of unaligned length that cross both 256-column tile edges
    (m = 7 from column 255, m = 60 from column 496), a 250-column restart
    starting on column 5 and short odd ones, on the multi-kernel path: every
    restart's state after 10 steps against the oracle's steps (the state only:
    the oracle's pair sum for S_eps is quadratic in m)."""
    v, f = icosphere(2)
    n = v.shape[0]
    ms = [5, 250, 7, 31, 3, 200, 60]
    eps = [0.2] * len(ms)
    u0 = uniform_u0(45, 1, sum(ms), n)
    print(f"restarts {ms} ({sum(ms)} columns), 10 steps, {precision}", flush=True)
    out = run_gpu(v, f, ms, eps, u0, 1e-3, 10, precision)
    prob = flow.Problem(v, f, 1e-3)
    col0 = np.concatenate([[0], np.cumsum(ms)])
    for r in range(len(ms)):
        u = flow.normalise(prob.M, u0[col0[r]:col0[r + 1]])
        for _ in range(10):
            u = flow.step(prob, u, eps[r])
        assert rel(out["u"][col0[r]:col0[r + 1]], u) < bar, r


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_initial_state_is_rejected(gpu, bad):
    """A NaN or infinite value anywhere in u0 is SP_EINVAL from every entry
    point that takes a host u0 (validated before the upload)."""
    v, f = icosphere(2)
    mesh = sp.Mesh(v, f)
    u0 = uniform_u0(43, 2, 3, v.shape[0])
    u0[4, 17] = bad
    prm = sp.params(1e-3, n_steps=2, precision="mixed", energy_every=0)
    with pytest.raises(sp.SegpartError) as e:
        sp.solve(mesh, prm, [3, 3], [0.1, 0.1], u0)
    assert e.value.code == sp.SP_EINVAL and "non-finite" in str(e.value)
    with pytest.raises(sp.SegpartError) as e:
        sp.State(mesh, prm, [3, 3], [0.1, 0.1], u0)
    assert e.value.code == sp.SP_EINVAL and "non-finite" in str(e.value)
    srv = sp.Server(1 << 30, 64)
    with pytest.raises(sp.SegpartError) as e:
        srv.submit(mesh, prm, [3, 3], [0.1, 0.1], u0)
    assert e.value.code == sp.SP_EINVAL and "non-finite" in str(e.value)
    srv.close()
    mesh.close()


def test_hbm_bytes_model_is_plausible(gpu):
    """sp_stats.hbm_bytes: the modelled algorithmic bytes per component-DOF
    update of a mixed run lie between one CG iteration's worth and the float64
    form's per-step bound (32 B per inner iteration per element plus the fixed
    passes)."""
    v, f = icosphere(5)
    mesh = sp.Mesh(v, f)
    u0 = uniform_u0(44, 4, 8, v.shape[0])
    prm = sp.params(5e-4, n_steps=5, precision="mixed", energy_every=1)
    st = sp.State(mesh, prm, [8] * 4, [0.1] * 4, u0)
    st.step(5)
    s = st.stats()
    st.close()
    mesh.close()
    per_cdof = s["hbm_bytes"] / (32 * v.shape[0] * 5)
    iters = s["cg_iters"] / 5
    print(f"hbm_bytes {s['hbm_bytes']:.3e}, {per_cdof:.0f} B per cdof update, "
          f"{iters:.1f} iterations per step", flush=True)
    assert 32 * 1 < per_cdof < 32 * iters + 400
