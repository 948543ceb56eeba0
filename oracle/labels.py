"""Partition labels of a state (oracle; test infrastructure only).

Equation (vi) of the paper: Gamma_i^{eps,h} = { v_i > 0 } with
v_i = u_i - sum_{j != i} u_j.  These sets leave a void between regions; a
vertex where no v_i is positive gets label -1.  Should more than one v_i be
positive (possible only where P1 values undershoot below zero) the largest
wins.  The second labelling is the plain argmax of u_i (lowest index on ties).
"""
from __future__ import annotations

import numpy as np

__all__ = ["labels"]


def labels(u):
    """u [m, N] -> (v_label [N] int32, argmax_label [N] int32)."""
    m = u.shape[0]
    v = np.empty_like(u)
    for i in range(m):
        others = [j for j in range(m) if j != i]
        v[i] = u[i] - u[others].sum(axis=0)
    best = np.argmax(v, axis=0)
    vmax = v[best, np.arange(u.shape[1])]
    vlab = np.where(vmax > 0.0, best, -1).astype(np.int32)
    return vlab, np.argmax(u, axis=0).astype(np.int32)
