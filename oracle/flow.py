"""Algorithm 2.2 of the paper, step by step (oracle; test infrastructure only).

Given eps > 0, m, a time step tau > 0 and an initial state, each time step
k -> k+1 does, for every component i = 1..m of a restart:

  1. heat step, implicit Euler: find u~_i in S_h with
         (1/tau) (u~_i - u_i, chi) + (grad u~_i, grad chi) = 0   for all chi,
     i.e. (M + tau A) u~_i = M u_i.  Solved here exactly (sparse LU).
  2. nonlinear step, the per-node ODE with the other components frozen at
     their step-1 values (the Jacobi form the paper chooses), solved exactly:
         u^_i(z) = u~_i(z) exp( -(2 tau / eps^2) sum_{j != i} u~_j(z)^2 ).
     The paper's text prints tau/eps^2 once and 2 tau/eps^2 in the ODE and in
     its practical form; the ODE's coefficient 2/eps^2 integrated over one
     step of length tau gives 2 tau / eps^2, which is used.
  3. normalisation in L2(Gamma_h):  u_i <- u^_i / sqrt(u^_i^T M u^_i).

The initial state is normalised the same way before the first step (the
random start of Section 2.2 normalises each component).  Energies are taken
every ``energy_every`` steps (the paper's M_tau with M_tau * tau = 0.1) and
the run stops, when asked to, once |E_k - E_{k - M_tau}| < stop_tol (the
paper uses 1e-6).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import assemble
from .energy import energy as _energy
from .labels import labels as _labels

__all__ = ["Problem", "normalise", "heat_step", "nodal_step", "step",
           "split_restarts", "run"]


class Problem:
    """Matrices of one mesh and one time step: M, A and the LU of M + tau A."""

    def __init__(self, xyz, tri, tau):
        self.xyz = np.asarray(xyz, np.float64)
        self.tri = np.asarray(tri, np.int64)
        self.tau = float(tau)
        self.M, self.A = assemble(self.xyz, self.tri)
        self.K = (self.M + self.tau * self.A).tocsc()
        self._lu = None

    @property
    def lu(self):
        if self._lu is None:
            self._lu = spla.splu(self.K)
        return self._lu

    @property
    def n(self):
        return self.xyz.shape[0]


def normalise(M, u):
    """Scale every row u_i of u [m, N] to unit M-norm (unit L2(Gamma_h) norm)."""
    nrm2 = np.einsum("in,in->i", u, (M @ u.T).T)
    if np.any(~(nrm2 > 0.0)):
        raise ValueError("a component has zero (or non-finite) L2 norm")
    return u / np.sqrt(nrm2)[:, None]


def heat_step(prob, u):
    """Step 1: solve (M + tau A) u~_i = M u_i for every row of u [m, N]."""
    rhs = prob.M @ u.T
    return np.ascontiguousarray(prob.lu.solve(rhs).T)


def nodal_step(ut, tau, eps):
    """Step 2: u^_i = u~_i exp(-(2 tau/eps^2) sum_{j != i} u~_j^2), per node."""
    m = ut.shape[0]
    sq = ut * ut
    out = np.empty_like(ut)
    for i in range(m):
        others = np.zeros(ut.shape[1])
        for j in range(m):
            if j != i:
                others += sq[j]
        out[i] = ut[i] * np.exp(-(2.0 * tau / (eps * eps)) * others)
    return out


def step(prob, u, eps):
    """One full time step (steps 1-3) of one restart u [m, N]."""
    return normalise(prob.M, nodal_step(heat_step(prob, u), prob.tau, eps))


def split_restarts(u, m_per_restart):
    """Row blocks of a batch state [sum m_r, N], one per restart."""
    offs = np.concatenate([[0], np.cumsum(m_per_restart)])
    return [u[offs[r]:offs[r + 1]] for r in range(len(m_per_restart))]


def run(prob, u0, m_per_restart, eps_per_restart, n_steps, energy_every=0,
        stop_tol=1e-6, max_steps=10**7):
    """Run a batch of independent restarts.

    u0 [sum m_r, N] (not yet normalised); restart r has m_r components and
    parameter eps_r.  n_steps > 0 runs that many steps; n_steps == 0 runs until
    the energy changes by less than stop_tol between two checks
    ``energy_every`` steps apart (per restart), or max_steps.

    Returns a dict with the final state u [sum m_r, N], lambda [sum m_r],
    s_eps [R], energy [R], steps [R], labels [R, N], labels_argmax [R, N],
    history (list per restart of (step, E) pairs).
    """
    m_per_restart = [int(x) for x in m_per_restart]
    eps_per_restart = [float(x) for x in eps_per_restart]
    blocks = [normalise(prob.M, b) for b in split_restarts(np.asarray(u0, np.float64),
                                                         m_per_restart)]
    out_u, lam, s, e, steps, hist, lab, lab_am = [], [], [], [], [], [], [], []
    for r, u in enumerate(blocks):
        eps = eps_per_restart[r]
        h = []
        if n_steps > 0:
            for k in range(1, n_steps + 1):
                u = step(prob, u, eps)
                if energy_every and k % energy_every == 0:
                    h.append((k, _energy(prob.xyz, prob.tri, prob.M, prob.A, u, eps)[2]))
            k_done = n_steps
        else:
            if energy_every <= 0:
                raise ValueError("stop mode needs energy_every > 0")
            e_prev = _energy(prob.xyz, prob.tri, prob.M, prob.A, u, eps)[2]
            h.append((0, e_prev))
            k_done = 0
            while k_done < max_steps:
                for _ in range(energy_every):
                    u = step(prob, u, eps)
                k_done += energy_every
                e_now = _energy(prob.xyz, prob.tri, prob.M, prob.A, u, eps)[2]
                h.append((k_done, e_now))
                if abs(e_now - e_prev) < stop_tol:
                    break
                e_prev = e_now
        l_r, s_r, e_r = _energy(prob.xyz, prob.tri, prob.M, prob.A, u, eps)
        v, am = _labels(u)
        out_u.append(u)
        lam.append(l_r)
        s.append(s_r)
        e.append(e_r)
        steps.append(k_done)
        hist.append(h)
        lab.append(v)
        lab_am.append(am)
    return dict(u=np.concatenate(out_u, 0), lam=np.concatenate(lam), s_eps=np.array(s),
                energy=np.array(e), steps=np.array(steps), history=hist,
                labels=np.stack(lab), labels_argmax=np.stack(lab_am))
