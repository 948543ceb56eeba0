"""Pins of the oracle's energies: the quartic element integrals of S_eps
(equation Seps-u), the Rayleigh-quotient eigenvalue estimates (Section 3.2),
the Y-partition value 45/4 (Section 3.1, Bishop's conjecture) and the
energy identity of the paper's tables (E = sum lambda_i + S_eps)."""
import os

import numpy as np
import pytest
from scipy.integrate import dblquad

from oracle import energy, fem
from workloads import icosphere


def test_quartic_table_sums_and_values():
    t = energy.quartic_table()
    # sum_p b_p = 1 on the triangle, so the 81 entries sum to int 1 / |T| = 1
    assert abs(t.sum() - 1.0) < 1e-15
    # fully symmetric in its four indices
    for perm in [(1, 0, 2, 3), (0, 2, 1, 3), (3, 1, 2, 0)]:
        assert np.array_equal(t, t.transpose(perm))
    assert abs(t[0, 0, 0, 0] - 1 / 15) < 1e-16
    assert abs(t[0, 0, 0, 1] - 1 / 60) < 1e-16
    assert abs(t[0, 0, 1, 1] - 1 / 90) < 1e-16
    assert abs(t[0, 0, 1, 2] - 1 / 180) < 1e-16


def _brute_pair(xyz, ui, uj):
    """int_T ui^2 uj^2 by adaptive quadrature over the reference triangle."""
    area = 0.5 * np.linalg.norm(np.cross(xyz[1] - xyz[0], xyz[2] - xyz[0]))

    def f(s, r):  # b1 = r, b2 = s, b0 = 1 - r - s
        b = np.array([1.0 - r - s, r, s])
        return (ui @ b) ** 2 * (uj @ b) ** 2

    val, _ = dblquad(f, 0.0, 1.0, 0.0, lambda r: 1.0 - r, epsabs=1e-14, epsrel=1e-13)
    return 2.0 * area * val


def test_pair_integrals_vs_adaptive_quadrature():
    rng = np.random.default_rng(11)
    xyz = rng.normal(size=(3, 3))
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    u = rng.normal(size=(3, 3))          # 3 components, nodal values
    P = energy.pair_integrals(xyz, tri, u)
    for i in range(3):
        for j in range(3):
            ref = _brute_pair(xyz, u[i], u[j])
            assert abs(P[i, j] - ref) < 1e-11 * max(1.0, abs(ref))
    eps = 0.3
    s = energy.s_eps(xyz, tri, u, eps)
    ref = sum(_brute_pair(xyz, u[i], u[j]) for i in range(3) for j in range(3) if i != j)
    assert abs(s - ref / eps**2) < 1e-10 * abs(ref / eps**2)


def test_s_eps_segregated_and_constant():
    v, f = icosphere(2)
    n = v.shape[0]
    # supports with no common triangle: S_eps vanishes identically
    u = np.zeros((2, n))
    u[0, v[:, 2] > 0.5] = 1.0
    u[1, v[:, 2] < -0.5] = 1.0
    shared = (u[0][f].max(1) > 0) & (u[1][f].max(1) > 0)
    assert not shared.any()
    assert energy.s_eps(v, f, u, 0.1) == 0.0
    # constants c_i: S_eps = (1/eps^2) sum_{i != j} c_i^2 c_j^2 |Gamma_h|
    c = np.array([0.3, 0.7, 1.1])
    u = np.repeat(c[:, None], n, axis=1)
    area = fem.surface_area(v, f)
    ref = ((c**2).sum() ** 2 - (c**4).sum()) * area / 0.04
    assert abs(energy.s_eps(v, f, u, 0.2) - ref) < 1e-13 * ref


def test_rayleigh_scale_invariant_and_constant():
    v, f = icosphere(2)
    M, A = fem.assemble(v, f)
    rng = np.random.default_rng(3)
    u = rng.random((4, v.shape[0]))
    lam = energy.rayleigh(M, A, u)
    np.testing.assert_allclose(energy.rayleigh(M, A, 3.7 * u), lam, rtol=1e-14)
    assert np.all(lam > 0)
    assert abs(energy.rayleigh(M, A, np.ones((1, v.shape[0])))[0]) < 1e-14


def _lune_state(v):
    th = np.arccos(np.clip(v[:, 2], -1, 1))
    ph = np.arctan2(v[:, 1], v[:, 0])
    s = np.sin(th) ** 1.5
    u1 = np.where((ph > 0) & (ph < 2 * np.pi / 3), np.sin(1.5 * ph) * s, 0.0)
    u2 = np.where((ph < 0) & (ph > -2 * np.pi / 3), -np.sin(1.5 * ph) * s, 0.0)
    u3 = np.where(np.abs(ph) > 2 * np.pi / 3, np.sin(1.5 * np.abs(ph) - np.pi) * s, 0.0)
    return np.stack([u1, u2, u3])


def test_y_partition_lune_energy_45_over_4():
    """Section 3.1: the Y-partition eigenfunctions sin(3 phi/2) sin(theta)^(3/2)
    have eigenvalue 15/4 each (nu(nu+1), nu = 3/2), total 45/4.  The P1
    interpolant's Rayleigh quotient approaches it from below at first order
    (the lune functions are only Lipschitz across the partition boundary);
    Richardson extrapolation of two levels recovers 45/4."""
    tot = []
    for level in (4, 5, 6):
        v, f = icosphere(level)
        M, A = fem.assemble(v, f)
        u = _lune_state(v)
        lam = energy.rayleigh(M, A, u)
        assert np.all(lam < 3.75) and np.all(lam > 3.6)
        tot.append(lam.sum())
    tot = np.array(tot)
    err = 11.25 - tot
    assert np.all(err > 0) and np.all(np.diff(err) < 0)
    assert np.all(np.abs(err[:-1] / err[1:] - 2.0) < 0.3)      # first order
    assert abs(2 * tot[-1] - tot[-2] - 11.25) < 3e-3
    # the lune functions have disjoint supports; their interpolants overlap
    # only on triangles cut by the boundary, so S_eps shrinks fast with h
    s = [energy.s_eps(*icosphere(level), _lune_state(icosphere(level)[0]), 0.1)
         for level in (3, 4, 5)]
    assert s[0] > s[1] > s[2] > 0 and s[1] / s[2] > 8


def _read_table(path):
    rows = []
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_paper_totals_equal_sum_lambda_plus_s_eps(golden_dir):
    """The totals of the paper's sphere table equal sum_i lambda_i + S_eps
    (not (1/2) sum lambda_i + S_eps): the energy the oracle reports."""
    for row in _read_table(os.path.join(golden_dir, "tab_many_m_sphere.txt")):
        m, s, total = int(row[0]), float(row[1]), float(row[2])
        classes = [tuple(map(float, c.split(":"))) for c in row[3:]]
        assert sum(int(c) for c, _ in classes) == m
        lam_sum = sum(c * lam for c, lam in classes)
        assert abs(lam_sum + s - total) < 0.015 + 1e-5 * total
        assert abs(0.5 * lam_sum + s - total) > 1.0


def test_paper_eps_table_consistency(golden_dir):
    """tab:u-eps: error = 45/4 - E and eoc_i = log(err_i/err_{i-1}) / log(1/2);
    at eps = 1/2 the flow sits at the constant state, whose S_eps is
    m(m-1)/(eps^2 |Gamma|) = 6/(0.25 * 4 pi) on the unit sphere."""
    rows = np.array([[float(x) for x in r]
                     for r in _read_table(os.path.join(golden_dir, "tab_u_eps.txt"))])
    eps, E, err, eoc, S = rows[:, 0], rows[:, 1], rows[:, 2], rows[:, 3], rows[:, 4]
    np.testing.assert_allclose(11.25 - E, err, atol=1e-4)
    eoc_ref = np.log(err[1:] / err[:-1]) / np.log(0.5)
    np.testing.assert_allclose(eoc_ref, eoc[1:], atol=2e-3)
    np.testing.assert_allclose(eps[1:] / eps[:-1], 0.5, rtol=1e-5)
    assert abs(S[0] - 6.0 / (0.25 * 4 * np.pi)) < 2e-4


def test_multipliers_closed_forms():
    v, f = icosphere(2)
    n = v.shape[0]
    M, A = fem.assemble(v, f)
    area = fem.surface_area(v, f)
    # unit-norm constants: lambda_i = 0, lambda_i^eps = (2/eps^2)(m-1)/|Gamma_h|
    m, eps = 3, 0.3
    u = np.full((m, n), 1.0 / np.sqrt(area))
    lm = energy.multipliers(v, f, M, A, u, eps)
    ref = 2.0 / eps**2 * (m - 1) / area
    assert np.all(np.abs(lm - ref) < 1e-12 * ref)
    # constants of different size c_i: (2/eps^2) c_i^2 (sum_{j != i} c_j^2) |Gamma_h|
    c = np.array([0.3, 0.7, 1.1])
    u = np.repeat(c[:, None], n, axis=1)
    lm = energy.multipliers(v, f, M, A, u, eps)
    ref = 2.0 / eps**2 * c**2 * ((c**2).sum() - c**2) * area
    assert np.max(np.abs(lm - ref) / ref) < 1e-12
    # supports without a common triangle: lambda^eps = lambda
    u = np.zeros((2, n))
    u[0, v[:, 2] > 0.5] = 1.0
    u[1, v[:, 2] < -0.5] = 1.0
    assert np.array_equal(energy.multipliers(v, f, M, A, u, 0.1), energy.rayleigh(M, A, u))
    # the paper's identity: sum_i lambda_i^eps = sum_i lambda_i + 2 S_eps
    rng = np.random.default_rng(5)
    u = rng.random((4, n))
    lm = energy.multipliers(v, f, M, A, u, 0.2)
    lam, s, _ = energy.energy(v, f, M, A, u, 0.2)
    assert abs(lm.sum() - (lam.sum() + 2 * s)) < 1e-12 * lm.sum()
