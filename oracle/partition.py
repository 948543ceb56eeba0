"""Post-processing of a computed partition (oracle; test infrastructure only).

Two readings of a partition {Gamma_i} given as vertex labels:

* ``region_eigen``  the first Dirichlet eigenvalue of every region: the
  partition problem's energy is sum_i lambda_1(Gamma_i) (Problem 1.1), which
  does not depend on eps.  Discretely, region i gets the P1 functions that
  vanish at every vertex not labelled i, and lambda_1 is the smallest
  eigenvalue of the pencil (A_II, M_II) restricted to the vertices I labelled
  i.  Such functions live on every triangle that touches the region, half an
  element beyond it, so on a partition that covers the surface the value
  lies below the region's own (O(h)); with ``interior`` the region's
  boundary vertices (those with a neighbour labelled otherwise) are left out
  too, which keeps the functions inside it, and the value lies above.  The
  two bracket the eigenvalue of the region the labels describe.  On the
  sphere the three lunes of the Y-partition give 15/4 each (Section 3.1);
  the reduced problem on the unit disk gives 20.19 for a sector of angle
  2 pi / 3 and 26.37 for a quadrant (Section 3.2).
* ``region_graph``  which regions touch (share a mesh edge), the number of
  sides of each region (its number of neighbours, one arc per neighbour) and
  the counts n_k of regions with k sides.  For a partition whose junctions
  are all triple points these satisfy the identity the paper derives from
  Euler's formula (equation gauss-bonnet):
      4 n_2 + 3 n_3 + 2 n_4 + n_5 = 6 chi + sum_{k >= 7} (k - 6) n_k.

The eigenvalues come from a direct sparse factorisation (scipy's shift-invert
Lanczos at sigma = 0), not from the iteration the GPU uses.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

__all__ = ["region_eigen", "interior_labels", "region_graph", "gauss_bonnet_sides"]


def interior_labels(M, labels):
    """labels with every vertex that has a neighbour (a mesh edge: an
    off-diagonal entry of the mass matrix, all of which are positive) of
    another label set to -1."""
    labels = np.asarray(labels)
    C = M.tocoo()
    off = C.row != C.col
    bad = np.zeros(labels.shape[0], dtype=bool)
    diff = labels[C.row[off]] != labels[C.col[off]]
    bad[C.row[off][diff]] = True
    out = labels.copy()
    out[bad] = -1
    return out


def region_eigen(M, A, labels, m, interior=False):
    """lambda_1 of regions 0..m-1 (labels [N] int); NaN for an empty region."""
    labels = np.asarray(labels)
    M = M.tocsr()
    A = A.tocsr()
    if interior:
        labels = interior_labels(M, labels)
    out = np.full(m, np.nan)
    for i in range(m):
        idx = np.flatnonzero(labels == i)
        if idx.size == 0:
            continue
        Mi = M[idx][:, idx].tocsc()
        Ai = A[idx][:, idx].tocsc()
        if idx.size <= 3:
            w = np.linalg.eigvalsh(np.linalg.solve(Mi.toarray(), Ai.toarray()))
            out[i] = float(np.min(w))
            continue
        w = spla.eigsh(Ai, k=1, M=Mi, sigma=0.0, which="LM", return_eigenvectors=False)
        out[i] = float(w[0])
    return out


def region_graph(tri, labels, m):
    """Adjacency [m, m] (bool) of regions 0..m-1 across mesh edges (vertices
    with other labels, e.g. -1, are ignored), sides [m] and the counts n_k
    (array indexed by k)."""
    tri = np.asarray(tri)
    labels = np.asarray(labels)
    adj = np.zeros((m, m), dtype=bool)
    for a, b in ((0, 1), (1, 2), (2, 0)):
        la, lb = labels[tri[:, a]], labels[tri[:, b]]
        ok = (la != lb) & (la >= 0) & (lb >= 0) & (la < m) & (lb < m)
        adj[la[ok], lb[ok]] = True
        adj[lb[ok], la[ok]] = True
    sides = adj.sum(axis=1)
    n_k = np.bincount(sides, minlength=8)
    return adj, sides, n_k


def gauss_bonnet_sides(n_k, chi):
    """Both sides of the paper's identity for side counts n_k."""
    n_k = np.asarray(n_k)
    get = lambda k: int(n_k[k]) if k < n_k.size else 0  # noqa: E731
    lhs = 4 * get(2) + 3 * get(3) + 2 * get(4) + get(5)
    rhs = 6 * chi + sum((k - 6) * int(n_k[k]) for k in range(7, n_k.size))
    return lhs, rhs
