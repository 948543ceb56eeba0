"""The continuation study (Section 3.1) through the C ABI against the oracle.

* sp_mesh_refine: the parents table equals the oracle's refinement (bit for
  bit), and the refined mesh's M and A equal the oracle's matrices on the
  oracle-refined mesh (1e-13 relative); refining twice works; a mesh that
  was not refined has no parents (SP_EINVAL);
* sp_prolong: bit-exact against the oracle's prolongation on random data
  (the mean of two float64 values, same operation order);
* sp_continue with a fixed step count per level (so the comparison does not
  depend on where the stopping rule lands): level 4 sphere, two restarts of
  m = 3 in one batch, each against the oracle run alone, three levels of the
  eps study (the third refines to level 5, which runs on the
  multi-kernel path; levels 0-1 on the one-workgroup path), float64 (bar
  1e-10 on u, lambda, S_eps, E, CG rtol 1e-13) and mixed precision (bar 1e-5);
* sp_continue with the stopping rule: the same two restarts and three levels
  against the oracle run to the rule, each restart stopping on its own: per
  level the same step count and E, S_eps within 1e-7 relative (float64).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import continuation as cont  # noqa: E402
from oracle import fem  # noqa: E402
from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import eps_study_levels, icosphere, project_sphere, uniform_u0  # noqa: E402

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def csr_dense(rp, col, val, n):
    d = np.zeros((n, n))
    for i in range(n):
        d[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    return d


def test_refine_matches_oracle(gpu):
    v, f = icosphere(2)
    print("refine level 2 sphere twice", flush=True)
    mesh = sp.Mesh(v, f)
    fine = mesh.refine(project_sphere)
    vf, ff, parents = cont.refine(v, f, project_sphere)
    par, nc = fine.parents()
    assert nc == v.shape[0] and np.array_equal(par, parents)
    assert (fine.n_vert, fine.n_tri) == (vf.shape[0], ff.shape[0])
    M, A = fem.assemble(vf, ff)
    for which, ref in ((sp.SP_MAT_M, M), (sp.SP_MAT_A, A)):
        got = csr_dense(*fine.export(which), fine.n_vert)
        assert rel(got, ref.toarray()) < 1e-13
    fine2 = fine.refine(project_sphere)
    vf2, ff2, parents2 = cont.refine(vf, ff, project_sphere)
    assert np.array_equal(fine2.parents()[0], parents2)
    assert fine2.n_vert == icosphere(4)[0].shape[0]
    with pytest.raises(sp.SegpartError) as e:
        mesh.parents()
    assert e.value.code == sp.SP_EINVAL
    fine2.close()
    fine.close()
    mesh.close()


def test_prolong_bit_exact(gpu):
    v, f = icosphere(3)
    mesh = sp.Mesh(v, f)
    fine = mesh.refine(project_sphere)
    _, _, parents = cont.refine(v, f, project_sphere)
    rng = np.random.default_rng(11)
    for cols in (1, 3, 7):
        print(f"prolong level 3 -> 4, {cols} columns", flush=True)
        u = rng.standard_normal((cols, v.shape[0]))
        got = fine.prolong(u)
        assert np.array_equal(got, cont.prolong(u, parents))
    fine.close()
    mesh.close()


def _levels():
    return eps_study_levels(3)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_continue_fixed_steps_matches_oracle(gpu, precision, bar):
    v, f = icosphere(4)
    m, steps, nres = 3, 150, 2
    u0 = uniform_u0(7, nres, m, v.shape[0])
    print(f"continue, {nres} restarts, 3 levels x {steps} steps, {precision}", flush=True)
    mesh = sp.Mesh(v, f)
    prm = sp.params(8e-4, n_steps=steps, precision=precision,
                    cg_rtol=1e-13 if precision == "fp64" else 1e-10)
    rc, res, lam, fin, u = sp.continue_levels(mesh, prm, m, u0, _levels(), project_sphere,
                                              n_restarts=nres)
    assert rc == sp.SP_OK
    for r in range(nres):
        rows, xyz, tri, uref = cont.run(v, f, u0[r * m:(r + 1) * m], m, _levels(), project_sphere,
                                        n_steps=steps)
        assert fin is not None and fin.n_vert == xyz.shape[0]
        for lvl, ref in enumerate(rows):
            g = res[lvl][r]
            assert g["n_vert"] == ref["n_vert"] and g["steps"] == steps and g["converged"] == 1
            assert abs(g["energy"] - ref["energy"]) <= bar * abs(ref["energy"])
            assert abs(g["s_eps"] - ref["s_eps"]) <= bar * abs(ref["s_eps"])
            assert rel(lam[lvl, r * m:(r + 1) * m], ref["lam"]) < bar
        assert rel(u[r * m:(r + 1) * m], uref) < bar
    fin.close()
    mesh.close()


def test_continue_stop_rule_matches_oracle(gpu):
    """Two restarts to the stopping rule in one batch: each stops on its own
    (its own step count per level) and matches the oracle run alone."""
    v, f = icosphere(4)
    m, nres = 3, 2
    u0 = uniform_u0(7, nres, m, v.shape[0])
    print("continue, 2 restarts, 3 levels to the stopping rule, fp64", flush=True)
    mesh = sp.Mesh(v, f)
    prm = sp.params(8e-4, n_steps=0, precision="fp64", cg_rtol=1e-13, stop_tol=1e-6)
    rc, res, lam, fin, u = sp.continue_levels(mesh, prm, m, u0, _levels(), project_sphere,
                                              n_restarts=nres)
    assert rc == sp.SP_OK
    for r in range(nres):
        rows, *_ = cont.run(v, f, u0[r * m:(r + 1) * m], m, _levels(), project_sphere,
                            stop_tol=1e-6)
        for lvl, ref in enumerate(rows):
            g = res[lvl][r]
            print(f"  restart {r} eps {ref['eps']}: steps {g['steps']} (oracle {ref['steps']}), "
                  f"E {g['energy']:.6f} ({ref['energy']:.6f})", flush=True)
            assert g["steps"] == ref["steps"]
            assert abs(g["energy"] - ref["energy"]) <= 1e-7 * ref["energy"]
            assert abs(g["s_eps"] - ref["s_eps"]) <= 1e-7 * ref["s_eps"]
    fin.close()
    mesh.close()
