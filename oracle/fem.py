"""P1 surface finite element matrices (oracle; test infrastructure only).

Section 2.1 of the paper: S_h is the space of continuous functions on the
triangulated surface Gamma_h that are affine on each flat triangle.  With the
nodal basis {phi_z}, the heat step of Algorithm 2.2 needs

    M[z, w] = int_{Gamma_h} phi_z phi_w          (consistent mass)
    A[z, w] = int_{Gamma_h} grad phi_z . grad phi_w   (stiffness)

Both are written here straight from their definitions:

* On a triangle T the basis functions are the barycentric coordinates
  b_0, b_1, b_2, and the exact monomial rule
      int_T b_0^n0 b_1^n1 b_2^n2 = 2 |T| n0! n1! n2! / (n0 + n1 + n2 + 2)!
  gives the mass entries.
* The tangential gradient of b_a on the flat triangle is J g^{-1} dhat_a,
  where J = [x1 - x0, x2 - x0] (3 x 2), g = J^T J is the metric and dhat_a
  the gradient of b_a on the reference triangle (-1,-1), (1,0), (0,1).  So
  int_T grad b_a . grad b_b = |T| dhat_a^T g^{-1} dhat_b, with
  |T| = sqrt(det g) / 2.

Element contributions are summed into scipy CSR matrices (duplicates add).
"""
from __future__ import annotations

from math import factorial

import numpy as np
import scipy.sparse as sp

__all__ = ["simplex_monomial", "triangle_geometry", "mass_matrix",
           "stiffness_matrix", "assemble", "surface_area"]

_DHAT = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])


def simplex_monomial(counts, area):
    """int_T b_0^n0 b_1^n1 b_2^n2 dsigma on a flat triangle of the given area."""
    n = sum(counts)
    num = 1
    for c in counts:
        num *= factorial(c)
    return 2.0 * area * num / factorial(n + 2)


def triangle_geometry(xyz, tri):
    """Per-triangle Jacobian J [T,3,2], metric g [T,2,2] and area [T]."""
    x0 = xyz[tri[:, 0]]
    J = np.stack([xyz[tri[:, 1]] - x0, xyz[tri[:, 2]] - x0], axis=2)
    g = np.einsum("tki,tkj->tij", J, J)
    det = g[:, 0, 0] * g[:, 1, 1] - g[:, 0, 1] * g[:, 1, 0]
    area = 0.5 * np.sqrt(det)
    return J, g, area


def _scatter(tri, local, n):
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    return sp.coo_matrix((local.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()


def mass_matrix(xyz, tri):
    _, _, area = triangle_geometry(xyz, tri)
    local = np.empty((tri.shape[0], 3, 3))
    for a in range(3):
        for b in range(3):
            counts = [0, 0, 0]
            counts[a] += 1
            counts[b] += 1
            local[:, a, b] = simplex_monomial(counts, 1.0) * area
    return _scatter(tri, local, xyz.shape[0])


def stiffness_matrix(xyz, tri):
    _, g, area = triangle_geometry(xyz, tri)
    ginv = np.linalg.inv(g)
    local = area[:, None, None] * np.einsum("ai,tij,bj->tab", _DHAT, ginv, _DHAT)
    return _scatter(tri, local, xyz.shape[0])


def assemble(xyz, tri):
    """(M, A) as scipy CSR float64 matrices, in the caller's vertex order."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    return mass_matrix(xyz, tri), stiffness_matrix(xyz, tri)


def surface_area(xyz, tri):
    """|Gamma_h| = sum of triangle areas."""
    return float(triangle_geometry(np.asarray(xyz, np.float64),
                                   np.asarray(tri, np.int64))[2].sum())
