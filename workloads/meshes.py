"""Synthetic closed triangulated surfaces.

These generators build inputs only: vertex coordinates (float64, shape
[n_vert, 3]) and triangle connectivity (int32, shape [n_tri, 3], outward
orientation).  Every vertex lies on the smooth surface it approximates, as the
discretisation section of the paper assumes for the triangulated surface.
None of the partition method's arithmetic lives here; both the CPU oracle and
the GPU library consume these arrays unchanged.

Surfaces:
  * ``icosphere(level)``  unit sphere by repeated 4-fold midpoint subdivision of
    the regular icosahedron, new vertices pushed radially onto the sphere;
    n_vert = 10*4**level + 2, n_tri = 20*4**level.
  * ``torus(nu, nv, R, r)``  ring torus, structured (phi, theta) grid with each
    quad split on a fixed diagonal; n_vert = nu*nv, n_tri = 2*nu*nv.
  * ``ellipsoid(level, axes)``  icosphere vertices scaled by the axes, so they
    lie exactly on the ellipsoid.
  * ``surface_d(level)``  surface (D) of Section 3.3, the zero set of
    (x1 - x3^2)^2 + x2^2 + x3^2 - 1: the image of the unit sphere under
    (y1, y2, y3) -> (y1 + y3^2, y2, y3), so icosphere vertices mapped this
    way lie exactly on it (same genus as the sphere, strongly varying
    curvature).
"""
from __future__ import annotations

import numpy as np

__all__ = ["icosahedron", "icosphere", "torus", "ellipsoid", "surface_d", "surface_mesh",
           "MESH_KINDS", "project_sphere", "project_ellipsoid", "project_surface_d",
           "surface_d_phi"]


def icosahedron():
    """Regular icosahedron inscribed in the unit sphere (12 vertices, 20 faces)."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        (-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
        (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
        (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1),
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
        (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
        (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
        (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
    ], dtype=np.int64)
    return v, f


def _subdivide(v, f):
    """One 4-fold split: a new vertex at each edge midpoint, projected radially."""
    n = v.shape[0]
    a, b, c = f[:, 0], f[:, 1], f[:, 2]
    e = np.concatenate([np.stack([a, b], 1), np.stack([b, c], 1),
                        np.stack([c, a], 1)], 0)
    e.sort(axis=1)
    key = e[:, 0] * n + e[:, 1]
    uniq, inv = np.unique(key, return_inverse=True)
    i0, i1 = uniq // n, uniq % n
    mid = 0.5 * (v[i0] + v[i1])
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    nf = f.shape[0]
    ab = n + inv[0:nf]
    bc = n + inv[nf:2 * nf]
    ca = n + inv[2 * nf:3 * nf]
    nfaces = np.concatenate([
        np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
        np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)], 0)
    return np.concatenate([v, mid], 0), nfaces


def icosphere(level: int):
    """Unit-sphere mesh at subdivision ``level`` (level 0 is the icosahedron)."""
    if level < 0:
        raise ValueError("level must be >= 0")
    v, f = icosahedron()
    for _ in range(level):
        v, f = _subdivide(v, f)
    return np.ascontiguousarray(v), np.ascontiguousarray(f.astype(np.int32))


def torus(nu: int, nv: int, R: float = 1.0, r: float = 0.4):
    """Ring torus x = ((R + r cos t) cos p, (R + r cos t) sin p, r sin t).

    ``nu`` samples of p around the central circle, ``nv`` samples of t around
    the tube.  The quad (i, j), (i+1, j), (i+1, j+1), (i, j+1) is split along
    its (i, j)-(i+1, j+1) diagonal; indices wrap periodically.
    """
    if nu < 3 or nv < 3:
        raise ValueError("torus needs nu, nv >= 3")
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    p = 2.0 * np.pi * i / nu
    t = 2.0 * np.pi * j / nv
    rho = R + r * np.cos(t)
    xyz = np.stack([rho * np.cos(p), rho * np.sin(p), r * np.sin(t)], -1)
    xyz = xyz.reshape(-1, 3)
    vid = lambda a, b: (a % nu) * nv + (b % nv)  # noqa: E731
    q00 = vid(i, j).ravel()
    q10 = vid(i + 1, j).ravel()
    q11 = vid(i + 1, j + 1).ravel()
    q01 = vid(i, j + 1).ravel()
    tri = np.concatenate([np.stack([q00, q10, q11], 1),
                          np.stack([q00, q11, q01], 1)], 0)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(tri.astype(np.int32))


def ellipsoid(level: int, axes=(1.0, 0.8, 0.6)):
    """Icosphere vertices scaled by ``axes``: they lie exactly on the ellipsoid."""
    v, f = icosphere(level)
    return np.ascontiguousarray(v * np.asarray(axes, dtype=np.float64)[None, :]), f


def surface_d(level: int):
    """Surface (D) from the level-``level`` icosphere: x = (y1 + y3^2, y2, y3).
    The map has Jacobian determinant 1, so the outward orientation is kept."""
    v, f = icosphere(level)
    x = v.copy()
    x[:, 0] += v[:, 2] * v[:, 2]
    return np.ascontiguousarray(x), f


def surface_d_phi(x):
    """Level-set function of surface (D): (x1 - x3^2)^2 + x2^2 + x3^2 - 1."""
    x = np.asarray(x, dtype=np.float64)
    return (x[:, 0] - x[:, 2] ** 2) ** 2 + x[:, 1] ** 2 + x[:, 2] ** 2 - 1.0


MESH_KINDS = ("sphere3", "sphere4", "sphere5", "sphere6", "sphere7", "sphere8",
              "torus512", "ellipsoid7")


def surface_mesh(kind: str):
    """Named workload meshes: ``sphereL`` (icosphere level L), ``torusN`` (N x N
    ring torus, R=1, r=0.4), ``ellipsoidL`` (axes 1, 0.8, 0.6), ``surfaceDL``
    (surface (D) from icosphere level L).  MESH_KINDS lists the kinds of the
    serving request stream."""
    if kind.startswith("sphere"):
        return icosphere(int(kind[6:]))
    if kind.startswith("torus"):
        n = int(kind[5:])
        return torus(n, n, 1.0, 0.4)
    if kind.startswith("ellipsoid"):
        return ellipsoid(int(kind[9:]))
    if kind.startswith("surfaceD"):
        return surface_d(int(kind[8:]))
    raise ValueError(f"unknown mesh kind {kind!r}")


def project_sphere(x):
    """Points x [k, 3] moved radially onto the unit sphere (how the icosphere
    places its edge midpoints; the surface map for refining sphere meshes)."""
    x = np.asarray(x, dtype=np.float64)
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def project_ellipsoid(x, axes=(1.0, 0.8, 0.6)):
    """Points x [k, 3] moved along the ray from the centre onto the ellipsoid
    with semi-axes ``axes`` (the lift the ellipsoid meshes are built with)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.asarray(axes, dtype=np.float64)[None, :]
    return x / np.sqrt(((x / a) ** 2).sum(axis=1, keepdims=True))


def project_surface_d(x):
    """Points x [k, 3] moved onto surface (D) through the sphere it is the image
    of: y = (x1 - x3^2, x2, x3) scaled to unit length, then mapped back."""
    x = np.asarray(x, dtype=np.float64)
    y = x.copy()
    y[:, 0] -= x[:, 2] * x[:, 2]
    y /= np.linalg.norm(y, axis=1, keepdims=True)
    out = y.copy()
    out[:, 0] += y[:, 2] * y[:, 2]
    return out

