"""The convergence study in eps of Section 3.1 (oracle; test infrastructure only).

The paper computes a minimiser on a coarse mesh at a large eps, then
repeatedly refines the mesh, shrinks tau, takes the previous minimiser as the
new initial condition and runs again with a smaller eps, each level until
the stopping rule of Section 2.2 holds (energy change below 1e-6 between two
checks M_tau steps apart, M_tau * tau = 0.1).  Table tab:u-eps lists the
energy and S_eps at each level's minimiser.

Pieces, each in the paper's terms:

* ``refine``   every triangle split into four at its edge midpoints (two
               bisections of the paper's refinement, which halve h); the
               new vertices are moved onto the surface by ``project`` (a
               map of points [k, 3] supplied with the surface; None leaves
               them at the midpoints).
               New vertex j is the midpoint of the j-th edge (a, b), a < b,
               in lexicographic order of (a, b), numbered after the coarse
               vertices; coarse triangle (a, b, c) with midpoints ab, bc, ca
               becomes (a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca).
* ``prolong``  the coarse minimiser carried to the fine mesh as the P1
               function it is: a coarse vertex keeps its value, a new
               vertex takes the mean of its edge's end values (the value of
               the coarse P1 function at the edge midpoint, before the
               vertex is moved onto the surface).
* ``run``      the level loop.  Each level runs ``flow.run`` in stop mode
               (or a fixed step count), with energy_every = M_tau =
               round(0.1 / tau).

The schedule's reading (the paper halves eps per row of tab:u-eps, divides
tau by sqrt(2) per level and bisects once per level) is left to the caller:
the levels are given as (eps, tau, refine) triples.
"""
from __future__ import annotations

import numpy as np

from . import flow

__all__ = ["refine", "prolong", "m_tau", "run"]


def refine(xyz, tri, project=None):
    """4-fold midpoint split.  Returns (xyz_fine, tri_fine, parents [E, 2])."""
    xyz = np.asarray(xyz, np.float64)
    tri = np.asarray(tri, np.int64)
    n = xyz.shape[0]
    # the three edges of every triangle, (min, max) ordered
    edges = {}
    for t in range(tri.shape[0]):
        a, b, c = (int(x) for x in tri[t])
        for p, q in ((a, b), (b, c), (c, a)):
            edges[(min(p, q), max(p, q))] = None
    keys = sorted(edges)
    for j, k in enumerate(keys):
        edges[k] = n + j
    parents = np.array(keys, dtype=np.int64).reshape(-1, 2)
    mid = 0.5 * (xyz[parents[:, 0]] + xyz[parents[:, 1]])
    if project is not None:
        mid = project(mid)
    fine_xyz = np.concatenate([xyz, mid], 0)
    out = []
    for t in range(tri.shape[0]):
        a, b, c = (int(x) for x in tri[t])
        ab = edges[(min(a, b), max(a, b))]
        bc = edges[(min(b, c), max(b, c))]
        ca = edges[(min(c, a), max(c, a))]
        out += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
    return fine_xyz, np.array(out, dtype=np.int64), parents


def prolong(u, parents):
    """u [m, n_coarse] -> [m, n_coarse + E]: new vertex = mean of its parents."""
    u = np.asarray(u, np.float64)
    return np.concatenate([u, 0.5 * (u[:, parents[:, 0]] + u[:, parents[:, 1]])], 1)


def m_tau(tau):
    """Energy cadence of the stopping rule: M_tau with M_tau * tau = 0.1,
    rounded to the nearest integer (halves up), at least 1."""
    return max(1, int(np.floor(0.1 / tau + 0.5)))


def run(xyz, tri, u0, m, levels, project=None, stop_tol=1e-6, n_steps=0,
        max_steps=10**7):
    """Level loop.  levels: sequence of (eps, tau, refine) (level 0 cannot
    refine).  u0 [m, n] on the first mesh (normalised by flow.run).  n_steps
    > 0 runs that many steps per level instead of the stopping rule.

    Returns a list of dicts (one per level): eps, tau, n_vert, steps, energy,
    s_eps, lam [m], and the final xyz, tri, u.
    """
    xyz = np.asarray(xyz, np.float64)
    tri = np.asarray(tri, np.int64)
    u = np.asarray(u0, np.float64)
    rows = []
    if levels and levels[0][2]:
        raise ValueError("level 0 cannot refine")
    for lvl, (eps, tau, ref) in enumerate(levels):
        if ref:
            xyz, tri, parents = refine(xyz, tri, project)
            u = prolong(u, parents)
        prob = flow.Problem(xyz, tri, tau)
        res = flow.run(prob, u, [m], [eps], n_steps, energy_every=m_tau(tau),
                       stop_tol=stop_tol, max_steps=max_steps)
        u = res["u"]
        rows.append(dict(eps=float(eps), tau=float(tau), n_vert=int(xyz.shape[0]),
                         steps=int(res["steps"][0]), energy=float(res["energy"][0]),
                         s_eps=float(res["s_eps"][0]), lam=res["lam"].copy()))
    return rows, xyz, tri, u
