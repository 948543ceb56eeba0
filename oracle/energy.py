"""Energies of a discrete state (oracle; test infrastructure only).

* Eigenvalue estimates (Section 3.2 of the paper; and the Caffarelli-Lin
  identity lambda_1(Gamma_i) = int |grad u_i|^2 for unit-L2 eigenfunctions in
  Section 1): lambda_i = u_i^T A u_i / u_i^T M u_i, the Rayleigh quotient of
  component i.
* Regularisation energy, equation (Seps-u):
      S_eps = (1/eps^2) int_{Gamma_h} sum_i sum_{j != i} u_i^2 u_j^2.
  Each u_i is affine on a triangle T, u_i = sum_p a_ip b_p, so u_i^2 u_j^2 is a
  quartic in the barycentric coordinates and its integral is exact:
      int_T u_i^2 u_j^2 = sum_{p,q,r,s} a_ip a_iq a_jr a_js int_T b_p b_q b_r b_s,
  with the monomial rule of ``fem.simplex_monomial``.  The double sum over
  ordered pairs i != j is evaluated pair by pair (no expansion identity).
* Total energy E = sum_i lambda_i + S_eps.  The paper writes a factor 1/2 on
  the Dirichlet term of E^eps, but the totals it tabulates (tables of
  Section 3.2-3.3) equal sum_i lambda_i + S_eps; that reading is used here.
"""
from __future__ import annotations

import itertools

import numpy as np

from .fem import simplex_monomial, triangle_geometry

__all__ = ["quartic_table", "rayleigh", "pair_integrals", "s_eps", "energy", "multipliers"]


def quartic_table():
    """I[p,q,r,s] = int_T b_p b_q b_r b_s / |T| for p,q,r,s in {0,1,2}."""
    table = np.empty((3, 3, 3, 3))
    for idx in itertools.product(range(3), repeat=4):
        counts = [idx.count(k) for k in range(3)]
        table[idx] = simplex_monomial(counts, 1.0)
    return table


_I4 = quartic_table()


def rayleigh(M, A, u):
    """lambda_i = u_i^T A u_i / u_i^T M u_i for each row u_i of u [m, N]."""
    num = np.einsum("in,in->i", u, (A @ u.T).T)
    den = np.einsum("in,in->i", u, (M @ u.T).T)
    return num / den


def pair_integrals(xyz, tri, u, chunk=8192):
    """P[i, j] = int_{Gamma_h} u_i^2 u_j^2 for all ordered pairs (i, j)."""
    tri = np.asarray(tri, np.int64)
    _, _, area = triangle_geometry(np.asarray(xyz, np.float64), tri)
    m = u.shape[0]
    out = np.zeros((m, m))
    for t0 in range(0, tri.shape[0], chunk):
        t = tri[t0:t0 + chunk]
        a = u[:, t]                                   # [m, T, 3]
        H = np.einsum("itp,itq->itpq", a, a)          # a_ip a_iq
        B = np.einsum("pqrs,jtrs->jtpq", _I4, H)      # sum_rs I a_jr a_js
        out += np.einsum("itpq,jtpq,t->ij", H, B, area[t0:t0 + chunk])
    return out


def s_eps(xyz, tri, u, eps):
    """Equation (Seps-u): (1/eps^2) sum over ordered pairs i != j of the pair
    integrals."""
    P = pair_integrals(xyz, tri, u)
    off = P.sum() - np.trace(P)
    return off / (eps * eps)


def energy(xyz, tri, M, A, u, eps):
    """(lambda [m], S_eps, E = sum lambda + S_eps) for one restart u [m, N]."""
    lam = rayleigh(M, A, u)
    s = s_eps(xyz, tri, u, eps)
    return lam, s, float(lam.sum() + s)


def multipliers(xyz, tri, M, A, u, eps):
    """The Lagrange multipliers of the gradient flow (Section 2.2, after
    Caffarelli & Lin): lambda_i^eps = int |grad u_i|^2 + (2/eps^2) int
    (sum_{j != i} u_j^2) u_i^2 for each row u_i of a unit-norm state u [m, N].
    The Dirichlet term is u_i^T A u_i / u_i^T M u_i (equal to u_i^T A u_i at
    unit norm); the coupling is the off-diagonal row sum of the pair
    integrals."""
    lam = rayleigh(M, A, u)
    P = pair_integrals(xyz, tri, u)
    return lam + (2.0 / (eps * eps)) * (P.sum(axis=1) - np.diag(P))

