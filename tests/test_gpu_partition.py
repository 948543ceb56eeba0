"""Partition post-processing through the C ABI against the oracle.

* sp_region_graph: adjacency and side counts equal the oracle's (exactly) on
  the polyhedral partitions of the level-5 sphere (tetrahedral, cubic,
  dodecahedral: 3, 4 and 5 sides, Gauss-Bonnet 12 = 6 chi) and cubic labels
  with voids, four restarts in one call; an adjacency of 2^31 entries or more
  is rejected (SP_EINVAL) before any allocation;
* sp_region_eigen: the first Dirichlet eigenvalue of every region equals the
  oracle's shift-invert value (1e-9 relative; inverse iteration to 1e-13
  relative change) for the Y-partition lunes of a longitude-latitude sphere
  (near 15/4), the polyhedral partitions of the level-4 sphere, and the
  argmax partition of a short m = 4 flow; the eigenvectors vanish outside
  their regions and have unit M-norm; an empty region gives NaN; the default
  start (1 on the region) reaches the same values; the interior reading
  (boundary vertices left out) against the oracle's, above the plain one;
* sp_state_multipliers: lambda_i^eps against the oracle on the state read
  back (1e-11), float64 and mixed (a pending normalisation applied first),
  and sum lambda^eps = sum lambda + 2 S_eps.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fem  # noqa: E402
from oracle import flow  # noqa: E402
from oracle.partition import (gauss_bonnet_sides, interior_labels, region_eigen,  # noqa: E402
                              region_graph)
from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import icosahedron, icosphere, uniform_u0  # noqa: E402

pytestmark = pytest.mark.gpu

DIRS = {
    "tetra": np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]) / np.sqrt(3),
    "cube": np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
                     dtype=np.float64),
    "dodeca": icosahedron()[0],
}


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def nearest(v, dirs):
    return np.argmax(v @ dirs.T, axis=1).astype(np.int32)


def test_region_graph_matches_oracle(gpu):
    v, f = icosphere(5)
    mesh = sp.Mesh(v, f)
    labs, ms = [], []
    for name in ("tetra", "cube", "dodeca"):
        labs.append(nearest(v, DIRS[name]))
        ms.append(DIRS[name].shape[0])
    # the cubic labels again with voids
    lab_void = labs[1].copy()
    lab_void[::5] = -1
    labs.append(lab_void)
    ms.append(6)
    print("region graph, 4 restarts on the level-5 sphere", flush=True)
    adjs, sides = sp.sp_region_graph(mesh.h, ms, np.stack(labs))
    off = 0
    for lab, m, adj in zip(labs, ms, adjs):
        ref_adj, ref_sides, n_k = region_graph(f, lab, m)
        assert np.array_equal(adj, ref_adj)
        assert np.array_equal(sides[off:off + m], ref_sides)
        assert gauss_bonnet_sides(n_k, 2) == (12, 12)
        off += m
    mesh.close()


def test_region_graph_rejects_oversized_adjacency(gpu):
    # sum of m^2 over the restarts must stay below 2^31 (int offsets)
    v, f = icosphere(1)
    mesh = sp.Mesh(v, f)
    try:
        ms = [4096] * 129
        with pytest.raises(sp.SegpartError) as e:
            sp.sp_region_graph(mesh.h, ms, np.zeros((len(ms), v.shape[0]), np.int32))
        assert e.value.code == sp.SP_EINVAL and "2^31" in str(e.value)
    finally:
        mesh.close()


def uv_sphere(nlat, nlon):
    pts = [(0.0, 0.0, 1.0)]
    for i in range(1, nlat):
        th = np.pi * i / nlat
        for j in range(nlon):
            ph = 2 * np.pi * j / nlon
            pts.append((np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)))
    pts.append((0.0, 0.0, -1.0))
    ring = lambda i, j: 1 + (i - 1) * nlon + (j % nlon)  # noqa: E731
    south = len(pts) - 1
    tri = []
    for j in range(nlon):
        tri.append((0, ring(1, j), ring(1, j + 1)))
        tri.append((south, ring(nlat - 1, j + 1), ring(nlat - 1, j)))
    for i in range(1, nlat - 1):
        for j in range(nlon):
            a, b, c, d = ring(i, j), ring(i + 1, j), ring(i + 1, j + 1), ring(i, j + 1)
            tri += [(a, b, c), (a, c, d)]
    return np.array(pts), np.array(tri, dtype=np.int32)


def lune_labels(v, m):
    ph = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi)
    k = ph / (2 * np.pi / m)
    on = (np.abs(k - np.round(k)) < 1e-9) | (np.hypot(v[:, 0], v[:, 1]) < 1e-12)
    lab = (np.floor(k).astype(np.int32) % m)
    lab[on] = -1
    return lab


def check_eigen(v, f, labels, ms, u0=None, interior=False):
    mesh = sp.Mesh(v, f)
    M, A = fem.assemble(v, f)
    rc, lam, u, its = sp.sp_region_eigen(mesh.h, ms, labels, u0=u0, shift=1e3, tol=1e-13,
                                         max_iter=400, want_u=True, interior=interior)
    assert rc == sp.SP_OK, its
    off = 0
    for r, m in enumerate(ms):
        ref = region_eigen(M, A, labels[r], m, interior=interior)
        keep = interior_labels(M, labels[r]) if interior else labels[r]
        got = lam[off:off + m]
        fin = np.isfinite(ref)
        assert np.array_equal(fin, np.isfinite(got))
        assert np.max(np.abs(got[fin] - ref[fin]) / ref[fin]) < 1e-9
        for i in range(m):
            if not fin[i]:
                continue
            x = u[off + i]
            assert np.all(x[keep != i] == 0.0)
            assert abs(x @ (M @ x) - 1.0) < 1e-10
        off += m
    mesh.close()
    return lam, its


def test_region_eigen_lunes(gpu):
    v, f = uv_sphere(32, 48)
    lab = lune_labels(v, 3)
    print("region eigenvalues, Y-partition lunes", flush=True)
    lam, its = check_eigen(v, f, lab[None, :], [3])
    assert np.all(np.abs(lam - 15.0 / 4.0) < 0.03)  # 3.771 on this mesh (second order in h)


def test_region_eigen_polyhedral_and_empty(gpu):
    v, f = icosphere(4)
    labs = [nearest(v, DIRS["tetra"]), nearest(v, DIRS["cube"])]
    # a restart of 5 components whose last region is empty
    labs.append(nearest(v, DIRS["tetra"]))
    print("region eigenvalues, polyhedral partitions of the level-4 sphere", flush=True)
    lam, _ = check_eigen(v, f, np.stack(labs), [4, 6, 5])
    assert np.isnan(lam[-1]) and np.all(np.isfinite(lam[:-1]))


def test_region_eigen_of_a_flow_partition(gpu):
    v, f = icosphere(4)
    m = 4
    u0 = uniform_u0(21, 1, m, v.shape[0])
    prob = flow.Problem(v, f, 2e-3)
    res = flow.run(prob, u0, [m], [0.05], 300)
    lab = res["labels_argmax"]
    print("region eigenvalues of an m = 4 flow partition (start: its components)", flush=True)
    lam_u, _ = check_eigen(v, f, lab, [m], u0=res["u"])
    lam_1, _ = check_eigen(v, f, lab, [m])
    assert np.max(np.abs(lam_u - lam_1) / lam_1) < 1e-9
    print("  interior reading", flush=True)
    lam_in, _ = check_eigen(v, f, lab, [m], u0=res["u"], interior=True)
    assert np.all(lam_in > lam_u)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_multipliers_match_oracle(gpu, precision):
    """lambda^eps of a state stepped on the GPU (mixed: its last normalisation
    still pending) against the oracle on the state read back; m = 3, 5, 11
    (one, and more than one, block of 8 components)."""
    from oracle import energy as oen
    v, f = icosphere(4)
    n = v.shape[0]
    ms = [3, 5, 11]
    eps = [0.05, 0.1, 0.08]
    u0 = uniform_u0(33, 1, sum(ms), n)
    mesh = sp.Mesh(v, f)
    prm = sp.params(2e-3, precision=precision, n_steps=1, energy_every=1, cg_rtol=1e-12,
                    extrapolate=3)
    print(f"multipliers after 12 steps, {precision}", flush=True)
    st = sp.State(mesh, prm, ms, eps, u0)
    try:
        st.step(12)
        lm = st.multipliers()
        lam, s_eps, _ = st.energy()
        u, _ = st.read()
    finally:
        st.close()
    M, A = fem.assemble(v, f)
    lo = 0
    for r, m in enumerate(ms):
        ref = oen.multipliers(v, f, M, A, u[lo:lo + m], eps[r])
        assert np.max(np.abs(lm[lo:lo + m] - ref) / np.abs(ref)) < 1e-11
        assert abs(lm[lo:lo + m].sum() - (lam[lo:lo + m].sum() + 2 * s_eps[r])) <= \
            1e-12 * lm[lo:lo + m].sum()
        lo += m
    mesh.close()
