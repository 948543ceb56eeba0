"""Serving loop: continuous batching on one GPU through the C ABI.

A request's result must not depend on which other requests share its batch:
it is compared with the same request served alone (1e-10 relative in float64
batches, 1e-5 in mixed) and with the CPU oracle.  In mixed precision the heat
solves start from an extrapolation of each column's own previous increments;
requests admitted into a running batch must not disturb the residents'
extrapolation, which shows in the residents' CG iteration counts.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import flow  # noqa: E402
from paper_1408_2355_amd import segpart as sp  # noqa: E402
from workloads import icosphere, uniform_u0, batch_u0  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def rel(a, b):
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def meshes():
    out = {}
    for lvl in (3, 4):
        v, f = icosphere(lvl)
        out[lvl] = (v, f, sp.Mesh(v, f))
    return out


def _req(level, seed, nres, m, eps, steps, precision, tau=1e-3):
    return dict(level=level, seed=seed, nres=nres, m=m, eps=eps, steps=steps,
                precision=precision, tau=tau)


def _submit(srv, meshes, q):
    v, f, mesh = meshes[q["level"]]
    u0 = uniform_u0(q["seed"], q["nres"], q["m"], v.shape[0])
    prm = sp.params(q["tau"], precision=q["precision"], n_steps=q["steps"], cg_rtol=1e-12,
                    energy_every=0)
    return srv.submit(mesh, prm, [q["m"]] * q["nres"], [q["eps"]] * q["nres"], u0), u0


def test_result_alone_equals_result_in_mix(meshes):
    a = _req(3, 101, 2, 3, 0.1, 40, "fp64")
    others = [_req(3, 102, 3, 5, 0.08, 60, "fp64"), _req(3, 103, 1, 4, 0.12, 25, "fp64"),
              _req(4, 104, 2, 3, 0.1, 30, "fp64"), _req(3, 105, 2, 6, 0.1, 50, "mixed")]
    print("server alone", flush=True)
    srv = sp.Server(8 << 30, 256)
    t, u0 = _submit(srv, meshes, a)
    assert srv.wait(t, 120)
    alone = srv.fetch(t)
    print("server mix", flush=True)
    tickets = [_submit(srv, meshes, q)[0] for q in others[:2]]
    time.sleep(0.05)                       # a joins batches that are already running
    ta, _ = _submit(srv, meshes, a)
    tickets += [_submit(srv, meshes, q)[0] for q in others[2:]]
    for tk in tickets + [ta]:
        assert srv.wait(tk, 300)
    mix = srv.fetch(ta)
    for k in ("u", "lam", "s_eps", "energy"):
        assert rel(mix[k], alone[k]) < 1e-10, k
    np.testing.assert_array_equal(mix["labels"], alone["labels"])
    # and both agree with the oracle
    v, f, _ = meshes[3]
    ref = flow.run(flow.Problem(v, f, a["tau"]), u0, [3, 3], [0.1, 0.1], a["steps"])
    assert rel(alone["u"], ref["u"]) < 1e-10
    assert rel(alone["lam"], ref["lam"]) < 1e-10
    assert rel(alone["s_eps"], ref["s_eps"]) < 1e-10
    st = srv.stats()
    assert st["completed"] == 6
    assert st["p99_s"] >= st["p50_s"] > 0 and st["cdof_per_s"] > 0
    for tk in tickets:
        out = srv.fetch(tk)
        assert np.isfinite(out["u"]).all() and out["latency_s"] > 0
    srv.close()


def test_mixed_request_matches_oracle_in_mix(meshes):
    srv = sp.Server(8 << 30, 128)
    q = _req(3, 201, 2, 4, 0.08, 30, "mixed")
    t0, _ = _submit(srv, meshes, _req(3, 202, 4, 4, 0.08, 60, "mixed"))
    t1, u0 = _submit(srv, meshes, q)
    assert srv.wait(t1, 120) and srv.wait(t0, 120)
    out = srv.fetch(t1)
    v, f, _ = meshes[3]
    ref = flow.run(flow.Problem(v, f, q["tau"]), u0, [4, 4], [0.08, 0.08], q["steps"])
    assert rel(out["lam"], ref["lam"]) < 1e-5
    assert rel(out["energy"], ref["energy"]) < 1e-5
    srv.close()


def test_mixed_request_alone_equals_result_in_mix(meshes):
    """A mixed-precision request (extrapolated starts, 5 increments) served
    alone, then again while other requests are admitted into its running batch
    one after another: same u, lambda, S_eps and E within 1e-5 (the mixed
    bar), both against the oracle too, and no extra CG iterations for it (each
    admission used to drop every resident's extrapolation history)."""
    v, f, mesh = meshes[4]
    steps, m, nres, eps, tau = 400, 4, 2, 0.1, 1e-3

    def prm(n_steps):
        return sp.params(tau, precision="mixed", n_steps=n_steps, energy_every=0)

    u0 = uniform_u0(301, nres, m, v.shape[0])
    print("server mixed alone", flush=True)
    srv = sp.Server(8 << 30, 128)
    t = srv.submit(mesh, prm(steps), [m] * nres, [eps] * nres, u0)
    assert srv.wait(t, 300)
    st_alone = srv.request_stats(t)
    alone = srv.fetch(t)
    assert st_alone["steps"] == steps and st_alone["col_iters"] > 0
    print("server mixed mix", flush=True)
    ta = srv.submit(mesh, prm(steps), [m] * nres, [eps] * nres, u0)
    during, k = 0, 0
    while not srv.poll(ta) and k < 12:
        ub = uniform_u0(310 + k, 1, 3, v.shape[0])
        tb = srv.submit(mesh, prm(10), [3], [0.08], ub)    # joins the running batch
        assert srv.wait(tb, 120)
        if not srv.poll(ta):
            during += 1
        out_b = srv.fetch(tb)
        assert np.isfinite(out_b["energy"]).all()
        k += 1
    assert srv.wait(ta, 300)
    st_mix = srv.request_stats(ta)
    mix = srv.fetch(ta)
    srv.close()
    print(f"admissions during the run {during}; column CG iterations alone "
          f"{st_alone['col_iters']}, in the mix {st_mix['col_iters']}", flush=True)
    assert during >= 2, "the other requests did not overlap the resident one"
    for key in ("u", "lam", "s_eps", "energy"):
        assert rel(mix[key], alone[key]) < 1e-5, key
    ref = flow.run(flow.Problem(v, f, tau), u0, [m] * nres, [eps] * nres, steps)
    for key in ("u", "lam", "s_eps", "energy"):
        assert rel(alone[key], ref[key]) < 1e-5, key
        assert rel(mix[key], ref[key]) < 1e-5, key
    # the resident kept its start guesses: its iteration count does not grow
    # with the admissions (a lost history costs ~10 iterations per column each)
    assert st_mix["col_iters"] <= 1.02 * st_alone["col_iters"] + 2 * m * nres


def test_budget_and_ticket_errors(meshes):
    v, f, mesh = meshes[3]
    srv = sp.Server(1 << 20, 64)          # 1 MiB: nothing fits
    u0 = uniform_u0(1, 1, 3, v.shape[0])
    with pytest.raises(sp.SegpartError) as e:
        srv.submit(mesh, sp.params(1e-3, n_steps=2), [3], [0.1], u0)
    assert e.value.code == sp.SP_ENOMEM
    with pytest.raises(sp.SegpartError) as e:
        srv.poll(12345)
    assert e.value.code == sp.SP_ENOTFOUND
    srv.close()


def test_queue_waits_for_memory_then_runs(meshes):
    """A budget that holds one batch at a time: the second request waits in
    the queue until the first batch drains, then runs (admission by HBM)."""
    v, f, mesh = meshes[4]
    prm = sp.params(1e-3, precision="fp64", n_steps=20, cg_rtol=1e-12, energy_every=0)
    u0 = uniform_u0(7, 2, 3, v.shape[0])
    srv = sp.Server(12 << 20, 64)           # room for one 64-column batch
    t1 = srv.submit(mesh, prm, [3, 3], [0.1, 0.1], u0)
    prm2 = sp.params(2e-3, precision="fp64", n_steps=20, cg_rtol=1e-12, energy_every=0)
    t2 = srv.submit(mesh, prm2, [3, 3], [0.1, 0.1], u0)   # other tau: needs its own batch
    assert srv.wait(t1, 120) and srv.wait(t2, 120)
    r1, r2 = srv.fetch(t1), srv.fetch(t2)
    ref = flow.run(flow.Problem(v, f, 2e-3), u0, [3, 3], [0.1, 0.1], 20)
    assert rel(r2["u"], ref["u"]) < 1e-10
    assert r2["latency_s"] >= r1["latency_s"] * 0.5
    srv.close()
