"""Seeded initial states and request traces.

Only random numbers are drawn here; normalisation and everything else the
method does to an initial state happens on either side of the comparison.

Layout of an initial state for a batch of restarts: a float64 array of shape
[sum_r m_r, n_vert]; restart r owns the m_r consecutive rows starting at
sum_{s<r} m_s, one row per component (component values contiguous).
"""
from __future__ import annotations

import numpy as np

__all__ = ["uniform_u0", "one_hot_u0", "batch_u0", "poisson_trace", "eps_study_levels"]


def _rng(seed: int):
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_u0(seed: int, n_restarts: int, m: int, n_vert: int):
    """iid U[0,1) values, shape [n_restarts * m, n_vert] (restart-major)."""
    u = _rng(seed).random((n_restarts, m, n_vert))
    return np.ascontiguousarray(u.reshape(n_restarts * m, n_vert))


def one_hot_u0(seed: int, n_restarts: int, m: int, n_vert: int):
    """The paper's random start (Section 2.2, after Algorithm 2.2): at every
    node one component, drawn uniformly from 1..m, is set to one and the others
    to zero.  Shape [n_restarts * m, n_vert].  A component that no node picked
    is left all zero; callers reject such a draw (it cannot be normalised)."""
    pick = _rng(seed).integers(0, m, size=(n_restarts, n_vert))
    u = np.zeros((n_restarts, m, n_vert))
    r_idx = np.arange(n_restarts)[:, None]
    v_idx = np.arange(n_vert)[None, :]
    u[r_idx, pick, v_idx] = 1.0
    return np.ascontiguousarray(u.reshape(n_restarts * m, n_vert))


def batch_u0(n_vert: int, groups):
    """Concatenate uniform draws for several (seed, n_restarts, m) groups.

    Returns (u0 [sum m_r, n_vert], m_per_restart int32 array)."""
    blocks, ms = [], []
    for seed, n_restarts, m in groups:
        blocks.append(uniform_u0(seed, n_restarts, m, n_vert))
        ms.extend([m] * n_restarts)
    return (np.ascontiguousarray(np.concatenate(blocks, 0)),
            np.asarray(ms, dtype=np.int32))


def poisson_trace(seed: int, n_requests: int, rate: float, kinds, m_range,
                  eps_choices, restart_range):
    """A finite seeded trace of partition requests arriving as a Poisson
    process of the given rate (requests per second).

    Returns a list of dicts with keys t_arrive, kind, m, eps, restarts, seed."""
    g = _rng(seed)
    gaps = g.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n_requests):
        out.append(dict(
            t_arrive=float(t[k]),
            kind=str(kinds[int(g.integers(0, len(kinds)))]),
            m=int(g.integers(m_range[0], m_range[1] + 1)),
            eps=float(eps_choices[int(g.integers(0, len(eps_choices)))]),
            restarts=int(g.integers(restart_range[0], restart_range[1] + 1)),
            seed=int(g.integers(0, 2**31 - 1)),
        ))
    return out


def eps_study_levels(n_levels: int, eps0: float = 0.5, tau0: float = 8e-4):
    """Level schedule of the convergence study in eps (Section 3.1, table
    tab:u-eps): eps halves from level to level (the table's rows), tau shrinks
    by 1/sqrt(2) per level, and the mesh is refined (4-fold midpoint split =
    two of the paper's bisections) before every second level (levels 2, 4,
    ...), so h shrinks by 1/sqrt(2) per level on average as with one bisection
    per level.  Returns [(eps, tau, refine)] for levels 0 .. n_levels - 1."""
    out = []
    eps, tau = float(eps0), float(tau0)
    for lvl in range(n_levels):
        out.append((eps, tau, lvl >= 2 and lvl % 2 == 0))
        eps *= 0.5
        tau /= 2.0 ** 0.5
    return out

