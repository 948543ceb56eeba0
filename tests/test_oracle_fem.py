"""Pins of the oracle's P1 matrices against closed forms and the mathematics.

Mass and stiffness (Section 2.1 of the paper, the spaces S_h) are checked
against: exact areas, exact integrals of linear functions on single flat
triangles, the kernel of the Laplacian, symmetry/definiteness, and the
spectrum of the Laplace-Beltrami operator on the unit sphere, l(l+1) with
multiplicity 2l+1, which the discrete generalised eigenvalues must approach
at second order in h.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from scipy.special import ellipeinc, ellipkinc

from oracle import fem
from workloads import icosphere, torus, ellipsoid


def test_level0_area_closed_form():
    # regular icosahedron inscribed in the unit sphere: edge 4/sqrt(10+2 sqrt5),
    # area 5 sqrt3 a^2
    v, f = icosphere(0)
    M, _ = fem.assemble(v, f)
    a = 4.0 / np.sqrt(10.0 + 2.0 * np.sqrt(5.0))
    one = np.ones(12)
    assert abs(one @ M @ one - 5.0 * np.sqrt(3.0) * a * a) < 1e-13


def test_sphere_area_second_order():
    err = []
    for level in range(1, 7):
        v, f = icosphere(level)
        M, _ = fem.assemble(v, f)
        one = np.ones(v.shape[0])
        err.append(4.0 * np.pi - one @ M @ one)
    err = np.array(err)
    assert (err > 0).all()                     # inscribed polyhedra, from below
    ratios = err[:-1] / err[1:]
    assert np.all(np.diff(ratios) > 0)          # ratios increase towards 4
    assert np.all(np.abs(ratios[2:] - 4.0) < 0.02)  # O(h^2)


def test_torus_and_ellipsoid_area():
    v, f = torus(256, 256, 1.0, 0.4)
    assert abs(fem.surface_area(v, f) - 4 * np.pi**2 * 0.4) < 2e-3
    # triaxial ellipsoid area via Legendre incomplete elliptic integrals
    a, b, c = 1.0, 0.8, 0.6
    phi = np.arccos(c / a)
    k2 = a * a * (b * b - c * c) / (b * b * (a * a - c * c))
    exact = 2 * np.pi * c * c + 2 * np.pi * a * b / np.sin(phi) * (
        ellipeinc(phi, k2) * np.sin(phi) ** 2 + ellipkinc(phi, k2) * np.cos(phi) ** 2)
    v, f = ellipsoid(6)
    assert 0 < exact - fem.surface_area(v, f) < 1e-3


def test_mass_exact_on_unit_right_triangle():
    xyz = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]])
    tri = np.array([[0, 1, 2]])
    M, _ = fem.assemble(xyz, tri)
    x = xyz[:, 0]
    one = np.ones(3)
    assert abs(x @ M @ x - 1.0 / 12.0) < 1e-15      # int x^2
    assert abs(x @ M @ one - 1.0 / 6.0) < 1e-15     # int x
    assert abs(one @ M @ one - 0.5) < 1e-15         # area
    y = xyz[:, 1]
    assert abs(x @ M @ y - 1.0 / 24.0) < 1e-15      # int x y


def test_stiffness_linear_function_on_tilted_triangle():
    rng = np.random.default_rng(4)
    for _ in range(5):
        xyz = rng.normal(size=(3, 3))
        tri = np.array([[0, 1, 2]])
        _, A = fem.assemble(xyz, tri)
        c = rng.normal(size=3)
        u = xyz @ c                                   # nodal values of c.x
        nrm = np.cross(xyz[1] - xyz[0], xyz[2] - xyz[0])
        area = 0.5 * np.linalg.norm(nrm)
        nhat = nrm / np.linalg.norm(nrm)
        ctan = c - (c @ nhat) * nhat                  # tangential gradient
        assert abs(u @ A @ u - area * ctan @ ctan) < 1e-12 * (1 + area * ctan @ ctan)
        # the normal direction of c carries no energy
        un = xyz @ nhat
        assert abs(un @ A @ un) < 1e-12


def test_symmetry_kernel_definiteness():
    v, f = icosphere(2)
    M, A = fem.assemble(v, f)
    assert abs(M - M.T).max() < 1e-16 * abs(M).max()
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    one = np.ones(v.shape[0])
    assert np.abs(A @ one).max() < 1e-14 * abs(A).max()
    wm = np.linalg.eigvalsh(M.toarray())
    assert wm.min() > 0
    wa = np.linalg.eigvalsh(A.toarray())
    assert abs(wa[0]) < 1e-12 and wa[1] > 1e-3       # one-dimensional kernel
    # consistent mass row sums are one third of the incident triangle areas
    _, _, area = fem.triangle_geometry(v, f.astype(np.int64))
    lumped = np.bincount(f.ravel(), weights=np.repeat(area, 3), minlength=v.shape[0]) / 3
    np.testing.assert_allclose(M @ one, lumped, rtol=1e-14)


def _sphere_spectrum(level, k=16):
    v, f = icosphere(level)
    M, A = fem.assemble(v, f)
    if level <= 2:
        return sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)[:k]
    w = spla.eigsh(A.tocsc(), k=k, M=M.tocsc(), sigma=-0.5, which="LM",
                   return_eigenvectors=False)
    return np.sort(w)


def test_sphere_spectrum_converges_to_l_l_plus_1():
    exact = np.concatenate([[0.0], np.full(3, 2.0), np.full(5, 6.0), np.full(7, 12.0)])
    errs = []
    for level in (2, 3, 4):
        w = _sphere_spectrum(level)
        assert abs(w[0]) < 1e-10
        errs.append(np.abs(w - exact)[1:9].max())
        # multiplicities: l = 1 triple is exactly degenerate by symmetry
        assert np.ptp(w[1:4]) < 1e-10
    errs = np.array(errs)
    assert np.all(errs[:-1] / errs[1:] > 3.5)   # second order in h
    assert errs[-1] < 0.02


def test_dense_brute_force_level1():
    # tiny mesh: every eigenpair of (A, M) satisfies A v = mu M v with
    # v^T M v = 1, and the Rayleigh quotient of v is mu
    v, f = icosphere(1)
    M, A = fem.assemble(v, f)
    w, V = sla.eigh(A.toarray(), M.toarray())
    Md, Ad = M.toarray(), A.toarray()
    np.testing.assert_allclose(V.T @ Md @ V, np.eye(42), atol=1e-12)
    np.testing.assert_allclose(Ad @ V, Md @ V * w[None, :], atol=1e-11)
    assert abs(w[0]) < 1e-12 and np.all(w[1:] > 1.0)


@pytest.mark.parametrize("level", [1, 3])
def test_interpolated_coordinates_rayleigh(level):
    # x, y, z restricted to the sphere are l = 1 eigenfunctions (eigenvalue 2)
    v, f = icosphere(level)
    M, A = fem.assemble(v, f)
    for k in range(3):
        x = v[:, k]
        rq = (x @ A @ x) / (x @ M @ x)
        assert abs(rq - 2.0) < (0.5 if level == 1 else 0.05)
