"""Pins of the oracle's whole flow against the sphere partitions the paper
reports (Sections 3.1 and 3.2), CPU only.

From iid uniform data the gradient flow on the unit sphere settles, for
m = 3, into the Y-partition (three lunes of angle 2 pi / 3 meeting at two
antipodal triple points) and, for m = 6, into the cubic partition (six
spherical quadrilaterals centred on +-e_k up to a rotation).  Neither
partition is built into the oracle: these are properties of the whole
flow (heat solve, node step, normalisation, in sequence), which the
stage-by-stage pins do not cover.  Checked on the argmax partition of one seeded run (level-4 icosphere,
eps = 0.05, tau = eps / 200, 4000 steps, so t = 1):

* region areas (the mass-matrix row sums over each region) equal |Gamma_h| / m
  within 4 %;
* region centroids: for m = 3 pairwise at 120 degrees (cosines -1/2 within
  0.06); for m = 6 three antipodal pairs (cosine below -0.95) whose other
  cosines are near 0 (within 0.15);
* the region graph: three 2-gons (m = 3), six quadrilaterals (m = 6);
* for m = 3 the two readings of the regions' first Dirichlet eigenvalue
  bracket the lune value: their sums lie below and above 45/4.
"""
import numpy as np
import pytest

from oracle import flow
from oracle.partition import region_eigen, region_graph
from workloads import icosphere, uniform_u0

LEVEL, EPS, STEPS, SEED = 4, 0.05, 4000, 1


def partition_geometry(xyz, M, labels, m):
    """Areas [m], unit centroid directions [m, 3] and their cosines [m, m]."""
    w = np.asarray(M.sum(axis=1)).ravel()
    area = np.array([w[labels == i].sum() for i in range(m)])
    cen = np.array([(w[labels == i, None] * xyz[labels == i]).sum(axis=0) for i in range(m)])
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    return area, cen, cen @ cen.T


@pytest.fixture(scope="module")
def runs():
    xyz, tri = icosphere(LEVEL)
    prob = flow.Problem(xyz, tri, EPS / 200.0)
    out = {}
    for m in (3, 6):
        u0 = uniform_u0(SEED, 1, m, xyz.shape[0])
        r = flow.run(prob, u0, [m], [EPS], STEPS)
        out[m] = r["labels_argmax"][0]
    return xyz, tri, prob, out


def test_m3_flow_reaches_the_y_partition(runs):
    xyz, tri, prob, lab = runs
    area, _, cos = partition_geometry(xyz, prob.M, lab[3], 3)
    total = area.sum()
    assert np.all(np.abs(area / (total / 3) - 1) < 0.04), area
    off = cos[~np.eye(3, dtype=bool)]
    assert np.all(np.abs(off + 0.5) < 0.06), cos
    _, sides, n_k = region_graph(tri, lab[3], 3)
    assert list(sides) == [2, 2, 2]
    lp = region_eigen(prob.M, prob.A, lab[3], 3)
    li = region_eigen(prob.M, prob.A, lab[3], 3, interior=True)
    assert lp.sum() < 45 / 4 < li.sum(), (lp, li)


def test_m6_flow_reaches_the_cubic_partition(runs):
    xyz, tri, prob, lab = runs
    area, _, cos = partition_geometry(xyz, prob.M, lab[6], 6)
    total = area.sum()
    assert np.all(np.abs(area / (total / 6) - 1) < 0.04), area
    # every region has exactly one antipode; all other pairs are orthogonal
    anti = cos < -0.95
    assert np.all(anti.sum(axis=1) == 1), cos
    rest = cos[~anti & ~np.eye(6, dtype=bool)]
    assert np.all(np.abs(rest) < 0.15), cos
    _, sides, n_k = region_graph(tri, lab[6], 6)
    assert list(sides) == [4] * 6
