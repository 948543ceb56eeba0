"""Synthetic input generators: mesh counts, topology, geometry, seeding."""
import numpy as np
import pytest

from workloads import (icosphere, torus, ellipsoid, surface_mesh, uniform_u0,
                       one_hot_u0, batch_u0, poisson_trace, surface_d, surface_d_phi,
                       project_surface_d, project_ellipsoid, project_sphere)


def _edge_counts(tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], 0)
    e = np.sort(e, axis=1)
    _, counts = np.unique(e[:, 0].astype(np.int64) * (tri.max() + 1) + e[:, 1],
                          return_counts=True)
    return counts


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts_and_closed(level):
    v, f = icosphere(level)
    assert v.shape == (10 * 4**level + 2, 3)
    assert f.shape == (20 * 4**level, 3)
    assert f.dtype == np.int32
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    counts = _edge_counts(f)
    assert (counts == 2).all()                       # closed 2-manifold
    assert v.shape[0] - counts.size + f.shape[0] == 2  # Euler characteristic
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert (np.einsum("ij,ij->i", n, v[f].mean(1)) > 0).all()  # outward


def test_icosphere_degrees():
    v, f = icosphere(3)
    deg = np.bincount(f.ravel(), minlength=v.shape[0])   # triangles per vertex
    assert (deg == 5).sum() == 12 and (deg == 6).sum() == v.shape[0] - 12


def test_torus_topology_and_surface():
    v, f = torus(24, 16, 1.0, 0.4)
    assert v.shape == (384, 3) and f.shape == (768, 3)
    counts = _edge_counts(f)
    assert (counts == 2).all()
    assert v.shape[0] - counts.size + f.shape[0] == 0    # genus one
    rho = np.hypot(v[:, 0], v[:, 1])
    np.testing.assert_allclose((rho - 1.0) ** 2 + v[:, 2] ** 2, 0.16, atol=1e-14)
    c = v[f].mean(1)
    ph = np.arctan2(c[:, 1], c[:, 0])
    ctr = np.stack([np.cos(ph), np.sin(ph), 0 * ph], 1)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert (np.einsum("ij,ij->i", n, c - ctr) > 0).all()


def test_ellipsoid_on_surface():
    v, f = ellipsoid(2, (1.0, 0.8, 0.6))
    q = (v[:, 0] / 1.0) ** 2 + (v[:, 1] / 0.8) ** 2 + (v[:, 2] / 0.6) ** 2
    np.testing.assert_allclose(q, 1.0, atol=1e-14)
    assert f.shape == (320, 3)


def test_surface_mesh_names():
    v, f = surface_mesh("sphere3")
    assert v.shape[0] == 642
    v, f = surface_mesh("torus32")
    assert v.shape[0] == 1024


def test_seeded_states_reproducible():
    a = uniform_u0(1003, 2, 3, 50)
    b = uniform_u0(1003, 2, 3, 50)
    assert a.shape == (6, 50) and np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() < 1.0
    c = uniform_u0(1004, 2, 3, 50)
    assert not np.array_equal(a, c)
    oh = one_hot_u0(7, 1, 4, 100)
    assert np.array_equal(oh.sum(0), np.ones(100))
    u, ms = batch_u0(30, [(1, 2, 3), (2, 1, 5)])
    assert u.shape == (11, 30) and list(ms) == [3, 3, 5]
    np.testing.assert_array_equal(u[:6], uniform_u0(1, 2, 3, 30))


def test_poisson_trace():
    tr = poisson_trace(5000, 50, 50.0, ["sphere3", "torus512"], (3, 32),
                       (0.02, 0.01), (1, 32))
    assert len(tr) == 50
    t = [r["t_arrive"] for r in tr]
    assert t[0] == 0.0 and all(np.diff(t) >= 0)
    assert all(3 <= r["m"] <= 32 and 1 <= r["restarts"] <= 32 for r in tr)
    assert tr == poisson_trace(5000, 50, 50.0, ["sphere3", "torus512"], (3, 32),
                               (0.02, 0.01), (1, 32))


@pytest.mark.parametrize("level", [1, 3])
def test_surface_d_on_surface_closed_outward(level):
    v, f = surface_d(level)
    assert np.abs(surface_d_phi(v)).max() < 1e-14
    counts = _edge_counts(f)
    assert (counts == 2).all() and v.shape[0] - counts.size + f.shape[0] == 2
    # outward: the face normal agrees with grad Phi at the face centroid
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    c = v[f].mean(1)
    g = np.stack([2 * (c[:, 0] - c[:, 2] ** 2), 2 * c[:, 1],
                  -4 * c[:, 2] * (c[:, 0] - c[:, 2] ** 2) + 2 * c[:, 2]], 1)
    assert (np.einsum("ij,ij->i", n, g) > 0).all()
    assert np.array_equal(surface_mesh(f"surfaceD{level}")[0], v)


def test_projections_land_on_their_surfaces():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((200, 3)) * 0.7 + 0.1
    assert np.abs(np.linalg.norm(project_sphere(x), axis=1) - 1).max() < 1e-15
    a = np.array([1.0, 0.8, 0.6])
    y = project_ellipsoid(x, a)
    assert np.abs(((y / a) ** 2).sum(1) - 1).max() < 1e-14
    assert np.abs(surface_d_phi(project_surface_d(x))).max() < 1e-13
    # points already on a surface stay (to rounding)
    v, _ = surface_d(2)
    assert np.abs(project_surface_d(v) - v).max() < 1e-15

