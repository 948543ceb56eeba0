"""Pins of the oracle's partition post-processing, CPU only.

* region_eigen against closed forms: the first Dirichlet eigenvalue of a
  disk sector of angle alpha is j_{pi/alpha,1}^2 (Bessel zero), 20.1907 for
  alpha = 2 pi / 3 and 26.3746 for a quadrant (the reduced problem of
  Section 3.2); a lune of angle 2 pi / 3 on the unit sphere has 15/4
  (Section 3.1); the whole sphere has 0.  Meshes whose boundaries follow the
  regions (structured sector meshes, a longitude-latitude sphere) make the
  discrete values converge at second order, checked by halving h;
* the two readings of a label partition bracket the region's eigenvalue: for
  the Y-partition labelled by longitude on icosphere meshes (boundaries that
  cut through triangles) the plain value lies below 15/4 and the interior
  one above, both within O(h), the bracket shrinking as h halves;
* region_graph and the Gauss-Bonnet identity on partitions whose cell
  structure is known: the Y-partition (three 2-gons), the tetrahedral (four
  triangles), cubic (six quadrilaterals) and dodecahedral (twelve pentagons)
  partitions of the sphere, each labelled by nearest direction.
"""
import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import jv

from oracle import fem
from oracle.partition import gauss_bonnet_sides, interior_labels, region_eigen, region_graph
from workloads import icosahedron, icosphere


def bessel_zero(nu):
    """First positive zero of J_nu (bracketed root of the Bessel function)."""
    xs = np.linspace(0.5, 20.0, 4000)
    f = jv(nu, xs)
    k = np.flatnonzero(np.sign(f[:-1]) != np.sign(f[1:]))[0]
    return brentq(lambda x: jv(nu, x), xs[k], xs[k + 1], xtol=1e-14)


def sector_mesh(alpha, K):
    """Flat sector {r <= 1, 0 <= theta <= alpha}: the structured mesh of the
    triangle {0 <= t <= s <= 1} (K steps) mapped by (s, t) -> s (cos, sin)(alpha t / s).
    Returns xyz, tri, and labels (0 inside, -1 on the boundary)."""
    idx = {}
    pts, lab = [], []
    for i in range(K + 1):
        for j in range(i + 1):
            s = i / K
            th = alpha * (j / i) if i > 0 else 0.0
            idx[(i, j)] = len(pts)
            pts.append((s * np.cos(th), s * np.sin(th), 0.0))
            lab.append(0 if (0 < j < i < K) else -1)
    tri = []
    for i in range(K):
        for j in range(i + 1):
            tri.append((idx[(i, j)], idx[(i + 1, j)], idx[(i + 1, j + 1)]))
            if j < i:
                tri.append((idx[(i, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]))
    return np.array(pts), np.array(tri), np.array(lab)


@pytest.mark.parametrize("alpha,paper", [(2 * np.pi / 3, 20.19), (np.pi / 2, 26.37)])
def test_disk_sector_first_eigenvalue(alpha, paper):
    exact = bessel_zero(np.pi / alpha) ** 2
    assert abs(exact - paper) < 0.01
    errs = []
    for K in (24, 48):
        v, f, lab = sector_mesh(alpha, K)
        M, A = fem.assemble(v, f)
        lam = region_eigen(M, A, lab, 1)[0]
        errs.append(lam - exact)
    assert errs[1] > 0 and errs[0] > errs[1]        # from above (conforming subspace)
    assert 3.0 < errs[0] / errs[1] < 5.0            # second order in h
    assert abs(errs[1]) < 0.01 * exact


def uv_sphere(nlat, nlon):
    """Unit sphere from latitude rings (nlat - 1 rings) and nlon meridians
    (longitude 0 is a meridian), plus the two poles."""
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
    return np.array(pts), np.array(tri)


def lune_labels(v, m):
    """Open lunes 0 < phi < 2 pi/m, ... ; vertices on the meridians phi = 2 pi k/m
    and the poles get -1 (the Dirichlet boundary)."""
    ph = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi)
    k = ph / (2 * np.pi / m)
    on = (np.abs(k - np.round(k)) < 1e-9) | (np.hypot(v[:, 0], v[:, 1]) < 1e-12)
    lab = np.floor(k).astype(int) % m
    lab[on] = -1
    return lab


def test_y_partition_lunes_have_15_over_4():
    errs = []
    for nlat, nlon in ((24, 36), (48, 72)):
        v, f = uv_sphere(nlat, nlon)
        M, A = fem.assemble(v, f)
        lam = region_eigen(M, A, lune_labels(v, 3), 3)
        assert np.ptp(lam) < 1e-9 * lam.mean()   # the three lunes are congruent
        errs.append(lam.mean() - 15.0 / 4.0)
    assert errs[1] > 0 and 3.0 < errs[0] / errs[1] < 5.0
    assert errs[1] < 0.01 * 15.0 / 4.0


def test_whole_sphere_has_zero():
    v, f = icosphere(2)
    M, A = fem.assemble(v, f)
    assert abs(region_eigen(M, A, np.zeros(v.shape[0], int), 1)[0]) < 1e-10


def nearest_labels(v, dirs):
    return np.argmax(v @ np.asarray(dirs, np.float64).T, axis=1)


def polyhedron_dirs(name):
    if name == "tetra":
        return np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]) / np.sqrt(3)
    if name == "cube":
        return np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])
    if name == "dodeca":
        return icosahedron()[0]  # the dodecahedron's faces face the icosahedron's vertices
    raise ValueError(name)


@pytest.mark.parametrize("name,m,k", [("tetra", 4, 3), ("cube", 6, 4), ("dodeca", 12, 5)])
def test_polyhedral_partitions_side_counts(name, m, k):
    v, f = icosphere(5)
    lab = nearest_labels(v, polyhedron_dirs(name))
    adj, sides, n_k = region_graph(f, lab, m)
    assert np.array_equal(adj, adj.T) and not adj.diagonal().any()
    assert np.all(sides == k) and n_k[k] == m
    lhs, rhs = gauss_bonnet_sides(n_k, 2)
    assert lhs == rhs == 12


def test_y_partition_side_counts():
    v, f = icosphere(5)
    ph = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi)
    lab = np.minimum((ph / (2 * np.pi / 3)).astype(int), 2)
    adj, sides, n_k = region_graph(f, lab, 3)
    assert np.all(sides == 2) and n_k[2] == 3
    assert gauss_bonnet_sides(n_k, 2) == (12, 12)
    # a void vertex (label -1) separates nothing by itself
    lab2 = lab.copy()
    lab2[::7] = -1
    assert np.array_equal(region_graph(f, lab2, 3)[0], adj)


def test_label_partition_brackets_the_lune():
    widths = []
    for level in (4, 5):
        v, f = icosphere(level)
        M, A = fem.assemble(v, f)
        ph = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi)
        lab = np.minimum((ph / (2 * np.pi / 3)).astype(int), 2)
        lo = region_eigen(M, A, lab, 3)
        hi = region_eigen(M, A, lab, 3, interior=True)
        assert np.all(lo < 15.0 / 4.0) and np.all(hi > 15.0 / 4.0)
        widths.append(float(np.max(hi - lo)))
    assert widths[1] < 0.6 * widths[0]
    inner = interior_labels(M, lab)
    assert np.all(inner[lab == -1] == -1) and (inner == -1).sum() > 0



def test_gauss_bonnet_sides_counts_every_term():
    # one heptagon needs one extra pentagon on the sphere: 13 pentagons + 1 heptagon
    n_k = np.zeros(9, int)
    n_k[5], n_k[6], n_k[7] = 13, 10, 1
    assert gauss_bonnet_sides(n_k, 2) == (13, 13)
    # an octagon on the torus (chi = 0) balanced by two pentagons
    n_k = np.zeros(9, int)
    n_k[5], n_k[8] = 2, 1
    assert gauss_bonnet_sides(n_k, 0) == (2, 2)
