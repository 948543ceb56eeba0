"""The sphere partitions of the level-6 workload through the C ABI.

The level-6 sphere workload (eps = 0.02, tau = 1e-4) is where the lune
energy (m = 3) and the face-centred partition (m = 6) are expected; 2000
steps from iid uniform data do not get there (the oracle's energy is still
16.1 for m = 3).  Here the GPU takes the route the paper takes to small eps
(Section 3.1): a continuation.  Four restarts of iid U[0,1) data (seed 1, so
restart 0 is the oracle run pinned on the level-4 sphere) run 4000 steps on
the level-4 sphere at eps = 0.05, tau = 2.5e-4; the state is refined to level
5 (same eps, 4000 steps) and then to level 6 at the workload's eps = 0.02,
tau = 1e-4 (4000 steps); mixed precision.  On the lowest-energy restart's
argmax partition (computed here from the state read back):

* region areas equal |Gamma_h| / m within 4 % (M row sums, exported);
* m = 3: the energy lies within 1 % of the paper's eps table (Section 3.1)
  interpolated to eps = 0.02: the error 45/4 - E taken as a power of eps
  through the rows eps = 1/32 and 1/64 (9.2732; the mesh is not the paper's);
  region centroids pairwise at 120 degrees (cosines -1/2 within 0.05);
  three 2-gons (sp_region_graph); the two readings of the regions' first
  Dirichlet eigenvalue (sp_region_eigen) bracket the lunes: their sums lie
  below and above 45/4 = 11.25;
* m = 6: three antipodal pairs of centroids (cosine below -0.95), every other
  pair within 0.12 of orthogonal; six quadrilaterals (sp_region_graph); the
  six regions' first Dirichlet eigenvalues (plain reading) within 2 % of their
  mean, as the six congruent faces of the cube partition require.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import icosphere, project_sphere, uniform_u0  # noqa: E402

pytestmark = pytest.mark.gpu

LEVELS = [(0.05, 2.5e-4, 0), (0.05, 2.5e-4, 1), (0.02, 1e-4, 1)]
STEPS, RESTARTS, SEED = 4000, 4, 1
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tab_u_eps.txt")


def table_energy(eps):
    """E at eps from the eps table: 45/4 - E = a eps^p through the two rows
    whose eps bracket it."""
    rows = np.loadtxt(TABLE)
    k = int(np.flatnonzero(rows[:, 0] >= eps)[-1])
    (e0, E0), (e1, E1) = rows[k, :2], rows[k + 1, :2]
    p = np.log((45 / 4 - E0) / (45 / 4 - E1)) / np.log(e0 / e1)
    return 45 / 4 - (45 / 4 - E1) * (eps / e1) ** p


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run(m):
    v, f = icosphere(4)
    mesh = sp.Mesh(v, f)
    u0 = uniform_u0(SEED, RESTARTS, m, v.shape[0])
    prm = sp.params(LEVELS[0][1], n_steps=STEPS, precision="mixed")
    print(f"[geometry] m={m}: continuation level 4 -> 6, {RESTARTS} restarts", flush=True)
    rc, res, lam, fin, u = sp.continue_levels(mesh, prm, m, u0, LEVELS, project_sphere,
                                              n_restarts=RESTARTS)
    assert rc == sp.SP_OK
    assert fin is not None
    e = np.array([r["energy"] for r in res[-1]])
    print(f"[geometry] m={m}: final energies {np.round(e, 5)}", flush=True)
    best = int(np.argmin(e))
    ub = u[best * m:(best + 1) * m]
    return fin, ub, e[best]


def geometry(fin, ub, m):
    xyz, _ = icosphere(6)
    rp, col, val = fin.export(sp.SP_MAT_M)
    w = np.add.reduceat(val, rp[:-1])  # M row sums (lumped vertex areas)
    assert w.shape[0] == xyz.shape[0]
    lab = np.argmax(ub, axis=0).astype(np.int32)
    area = np.array([w[lab == i].sum() for i in range(m)])
    cen = np.array([(w[lab == i, None] * xyz[lab == i]).sum(axis=0) for i in range(m)])
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    return lab, area, cen @ cen.T


def test_level6_m3_lunes(gpu):
    fin, ub, e = run(3)
    lab, area, cos = geometry(fin, ub, 3)
    et = table_energy(LEVELS[-1][0])
    print(f"[geometry] m=3: E {e:.5f} (table {et:.5f}), areas {np.round(area, 4)}", flush=True)
    assert abs(e - et) < 0.01 * et
    assert np.all(np.abs(area / (area.sum() / 3) - 1) < 0.04), area
    off = cos[~np.eye(3, dtype=bool)]
    assert np.all(np.abs(off + 0.5) < 0.05), cos
    _, sides = sp.sp_region_graph(fin.h, [3], lab[None])
    assert list(sides) == [2, 2, 2]
    rc, lp, _, _ = sp.sp_region_eigen(fin.h, [3], lab[None])
    rc2, li, _, _ = sp.sp_region_eigen(fin.h, [3], lab[None], interior=True)
    print(f"[geometry] m=3: region lambda_1 plain {lp}, interior {li}", flush=True)
    assert rc == sp.SP_OK and rc2 == sp.SP_OK
    assert lp.sum() < 45 / 4 < li.sum()
    fin.close()


def test_level6_m6_cube(gpu):
    fin, ub, e = run(6)
    lab, area, cos = geometry(fin, ub, 6)
    print(f"[geometry] m=6: E {e:.5f}, areas {np.round(area, 4)}", flush=True)
    assert np.all(np.abs(area / (area.sum() / 6) - 1) < 0.04), area
    anti = cos < -0.95
    assert np.all(anti.sum(axis=1) == 1), cos
    rest = cos[~anti & ~np.eye(6, dtype=bool)]
    assert np.all(np.abs(rest) < 0.12), cos
    _, sides = sp.sp_region_graph(fin.h, [6], lab[None])
    assert list(sides) == [4] * 6
    rc, lp, _, _ = sp.sp_region_eigen(fin.h, [6], lab[None])
    print(f"[geometry] m=6: region lambda_1 plain {lp}", flush=True)
    assert rc == sp.SP_OK
    assert np.all(np.abs(lp / lp.mean() - 1) < 0.02), lp
    fin.close()
