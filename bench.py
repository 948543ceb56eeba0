#!/usr/bin/env python3
"""Throughput benchmark of the segregation time step on one MI355X.

Default workload (the batched-restart configuration): unit sphere,
icosahedral level 7 (163842 vertices), m in {4, 8, 12, 16} with 64 seeded
U[0,1) initial states each (2560 columns in one batch), eps = 0.01,
tau = 5e-5, float32 CG inside float64 refinement (outer rtol 1e-10).

One timed "step" is one full time step of every restart (heat solve, node
step, normalisation) plus the energy evaluation and its read-back (the stop
test's input), i.e. every per-step part of the hot path; mesh set-up and the
initial normalisation happen before timing, labels after.  The timed steps
follow --warmup steps of the same run (default 5: steps 6-25 are timed, in
the transient after the random start, where the heat solves need about 20
inner iterations and two refinement sweeps); the warm-up steps are timed on
their own and reported too.

Printed: ONE JSON line with the throughput in component-DOF updates per
second (restart x component x vertex values advanced one step); the plain
float64 form (one restart at a time) on a sample of the same restarts over
the same steps, polled every CG iteration and every 8; the relative energy
error of the batched mixed form against that float64 run; the roofline of
the dominant kernel (HIP events on the library's stream over a second,
profiled pass of the same steps on a fresh state of the batch: the run is
deterministic, and recording the events turns the graph-replayed CG blocks
into launch-by-launch iterations, so the throughput is timed without them);
the serving loop on a seeded Poisson request stream (p50/p99
latency, served cdof/s against the plain form); and the CPU oracle on all
host cores (at most 16) on a bounded sample, run before the GPU is touched.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
KERNEL_NAMES = ("matvec q=(M+tau A)p", "update r", "direction p", "precond z=P r")

WORKLOADS = {
    # name: (mesh kind, [(seed, restarts, m)], eps, tau)
    "sphere7-batched": ("sphere7", [(3004, 64, 4), (3008, 64, 8), (3012, 64, 12),
                                    (3016, 64, 16)], 0.01, 5e-5),
    "torus512-batched": ("torus512", [(4008, 16, 8), (4016, 16, 16), (4032, 16, 32)],
                         0.01, 5e-5),
    "ellipsoid7-batched": ("ellipsoid7", [(4108, 16, 8), (4116, 16, 16), (4132, 16, 32)],
                           0.01, 5e-5),
    "surfaceD7-batched": ("surfaceD7", [(4208, 16, 8), (4216, 16, 16), (4232, 16, 32)],
                          0.01, 5e-5),
    "sphere3": ("sphere3", [(1003, 1, 3)], 0.1, 1e-3),
}
MESH_TEXT = {"sphere": "unit sphere, icosahedral level {}", "torus": "ring torus {0}x{0} (R 1, r 0.4)",
             "ellipsoid": "ellipsoid (1, 0.8, 0.6), icosahedral level {}",
             "surfaceD": "surface (D) (x1 - x3^2)^2 + x2^2 + x3^2 = 1, from icosahedral level {}"}

# request stream of the serving benchmark: every mesh kind, m in 3..32,
# eps in {0.02, 0.01, 0.005}, tau = eps / 200, 1..32 restarts, 200 steps
SERVE = dict(seed=5000, m_range=(3, 32), eps=(0.02, 0.01, 0.005), restarts=(1, 32), steps=200)


def traffic_record(kernel):
    """Measured HBM bytes per launch of `kernel` from the counter summaries in
    profiles/ (FETCH_SIZE and WRITE_SIZE runs scaled by a copy calibration),
    used only while the kernel source is the one that was measured."""
    import glob
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1408_2355_amd", "csrc", "kernels.hip")
    with open(src, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic-record "):
                    continue
                kv = dict(re.findall(r'(\w+)=("[^"]*"|\S+)', line))
                if kv.get("kernel", "").strip('"') == kernel and kv.get("source_sha256") == sha:
                    fetch = float(kv["fetch_bytes_per_launch"])
                    write = float(kv["write_bytes_per_launch"])
                    return fetch + write, (fetch + write) / float(kv["algorithmic_bytes_per_launch"]), \
                        os.path.relpath(path, ROOT)
    return None, None, None


def mesh_text(kind):
    for k, fmt in MESH_TEXT.items():
        if kind.startswith(k):
            return fmt.format(kind[len(k):])
    return kind


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_worker(prob, v, f, groups, eps, w, steps, barrier, out):
    """Restart w of every m group, `steps` time steps each with its energy."""
    from threadpoolctl import threadpool_limits
    from oracle import energy, flow
    from workloads import uniform_u0
    n = v.shape[0]
    with threadpool_limits(limits=1):
        us = [(flow.normalise(prob.M, uniform_u0(seed, w + 1, m, n)[w * m:(w + 1) * m]), m)
              for seed, _, m in groups]
        barrier.wait()
        t0 = time.time()
        cols = 0
        for u, m in us:
            for _ in range(steps):
                u = flow.step(prob, u, eps)
                energy.energy(v, f, prob.M, prob.A, u, eps)
            cols += m
        out.put((cols * n * steps, t0, time.time()))


def cpu_baseline(v, f, groups, eps, tau, steps=1):
    """The oracle on all host cores (at most 16, the GPU machine's CPU share): one
    process per core, each running restart w (its index) of every m group for
    `steps` steps with the energy, single-threaded BLAS; the factorisation of
    M + tau A is set-up, made once before the processes fork and not timed.
    cdof/s = all processes' updates / (last end - common start)."""
    import multiprocessing as mp
    from oracle import flow
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    prob = flow.Problem(v, f, tau)
    _ = prob.lu
    ctx = mp.get_context("fork")        # before any GPU work in this process
    barrier, out = ctx.Barrier(cores), ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker,
                         args=(prob, v, f, groups, eps, w, steps, barrier, out))
             for w in range(cores)]
    for p in procs:
        p.start()
    res = [out.get() for _ in procs]
    for p in procs:
        p.join()
    work = sum(r[0] for r in res)
    dt = max(r[2] for r in res) - min(r[1] for r in res)
    cols = sum(m for _, _, m in groups)
    return dict(value=work / dt, unit="cdof/s", cores=cores, kind="oracle",
                sample=f"{cores} processes, one per core, each restart w = 0..{cores - 1} of "
                       f"every m group ({cols} columns) for {steps} step(s) with the energy "
                       f"(exact sparse-LU heat solve, single-threaded BLAS): "
                       f"{cores * cols} of the workload's columns, {dt:.1f} s wall")


def serve_leg(sp, n_requests, rate, budget_gb=200.0, inner_rtol=1e-6, with_plain=True):
    """Serving: the first ``n_requests`` requests of the seeded Poisson stream
    (every mesh kind, m 3..32, eps in {0.02, 0.01, 0.005}, tau = eps/200,
    1..32 restarts, 200 steps, mixed precision) submitted at their arrival
    times (``rate`` per second) to one server.  Inputs are generated before the
    clock starts.  Latency = finish - submit per request (server clock).  The
    plain float64 form runs the first request of each mesh kind, its first
    restart alone, 200 steps, polled every CG iteration and every 8."""
    from workloads import MESH_KINDS, poisson_trace, surface_mesh, uniform_u0
    trace = poisson_trace(SERVE["seed"], n_requests, rate, MESH_KINDS,
                          SERVE["m_range"], SERVE["eps"], SERVE["restarts"])
    meshes = {}
    for kind in sorted({r["kind"] for r in trace}):
        meshes[kind] = sp.Mesh(*surface_mesh(kind))
        log(f"[serve] mesh {kind}: {meshes[kind].n_vert} vertices")
    reqs, work = [], 0.0
    for r in trace:
        n = meshes[r["kind"]].n_vert
        u0 = uniform_u0(r["seed"], r["restarts"], r["m"], n)
        prm = sp.params(r["eps"] / 200.0, precision="mixed", n_steps=SERVE["steps"],
                        cg_rtol=1e-10, inner_rtol=inner_rtol)
        reqs.append((r, prm, u0))
        work += r["restarts"] * r["m"] * n * SERVE["steps"]
    span = trace[-1]["t_arrive"]
    log(f"[serve] {len(trace)} requests at {rate} req/s over {span:.2f} s, {work:.3e} cdof offered")
    srv = sp.Server(int(budget_gb * 2**30))
    tickets = []
    t0 = time.perf_counter()
    for r, prm, u0 in reqs:
        dt = t0 + r["t_arrive"] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(meshes[r["kind"]], prm, [r["m"]] * r["restarts"],
                                  [r["eps"]] * r["restarts"], u0))
    del reqs
    sample = sorted({r["kind"]: i for i, r in reversed(list(enumerate(trace)))}.values())
    lat, ok, served_e, its = [], 0, {}, 0
    for i, t in enumerate(tickets):
        done = srv.wait(t, timeout_s=600.0)
        assert done, f"request {i} did not finish"
        its += srv.request_stats(t)["col_iters"]
        out = srv.fetch(t)
        lat.append(out["latency_s"])
        ok += int(np.isfinite(out["energy"]).all())
        if i in sample:
            served_e[i] = float(out["energy"][0])
        log(f"[serve] request {i} ({trace[i]['kind']}, m {trace[i]['m']}, "
            f"{trace[i]['restarts']} restarts) done, latency {out['latency_s']:.2f} s")
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    res = {
        "requests": len(trace), "rate_per_s": rate, "cdof_per_s": work / wall,
        "latency_p50_s": st["p50_s"], "latency_p99_s": st["p99_s"], "latency_max_s": max(lat),
        "completed": st["completed"], "finite_results": ok,
        "offered_cdof_per_s": work / max(span, 1e-9), "wall_s": wall,
        "server_cdof_per_s": st["cdof_per_s"],
        "column_cg_iters_per_step": its / sum(r["restarts"] * r["m"] * SERVE["steps"]
                                              for r in trace),
    }
    if with_plain:
        for poll in (1, 8):
            cd, tt, errs = 0.0, 0.0, []
            for i in sample:
                r = trace[i]
                mesh = meshes[r["kind"]]
                n = mesh.n_vert
                u1 = uniform_u0(r["seed"], r["restarts"], r["m"], n)[:r["m"]]
                pprm = sp.params(r["eps"] / 200.0, precision="fp64", n_steps=SERVE["steps"],
                                 cg_rtol=1e-10, cg_max_iter=2000, check_every=poll)
                ps = sp.State(mesh, pprm, [r["m"]], [r["eps"]], u1)
                t1 = time.perf_counter()
                ps.step(SERVE["steps"])
                tt += time.perf_counter() - t1
                cd += r["m"] * n * SERVE["steps"]
                e64 = ps.energy()[2][0]
                ps.close()
                errs.append(abs(served_e[i] - e64) / abs(e64))
            key = "plain_fp64" if poll == 8 else "plain_fp64_poll1"
            res[key] = {"value": cd / tt, "unit": "cdof/s",
                        "sample": f"first request of each mesh kind ({len(sample)} requests), "
                                  f"its first restart alone, float64, host convergence poll "
                                  f"every {'CG iteration' if poll == 1 else '8 CG iterations'}, "
                                  "200 steps",
                        "served_energy_rel_err_vs_fp64": max(errs)}
            res["speedup_vs_" + key] = res["cdof_per_s"] / (cd / tt)
            log(f"[serve] plain float64 (poll {poll}): {cd / tt:.3e} cdof/s, served "
                f"{res['cdof_per_s'] / (cd / tt):.2f}x, energy err {max(errs):.1e}")
    for m in meshes.values():
        m.close()
    return res


def serve(args, sp):
    """--serve: the serving leg alone, as its own JSON line."""
    r = serve_leg(sp, args.serve_requests, args.serve_rate, args.serve_budget_gb,
                  args.inner_rtol, with_plain=not args.no_plain)
    result = {
        "metric": "serving latency and throughput (Poisson request stream, continuous batching)",
        "value": r["cdof_per_s"], "unit": "cdof/s", "n_gpus": 1, "steps": SERVE["steps"],
        "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"serve: first {r['requests']} requests of the seeded stream "
                               f"(seed {SERVE['seed']}, {args.serve_rate} req/s), all mesh "
                               "kinds, m 3..32, eps {0.02,0.01,0.005}, tau eps/200, "
                               "1..32 restarts, 200 steps, mixed precision"},
    }
    result.update({k: v for k, v in r.items() if k != "cdof_per_s"})
    print(json.dumps(result), flush=True)


def eps_study(args, sp):
    """The convergence study in eps (Section 3.1): sp_continue over the
    schedule of workloads.eps_study_levels, m = 3, random U[0,1) start (seed
    7), mixed precision, stopping rule |dE| < 1e-6 every M_tau steps."""
    from workloads import eps_study_levels, icosphere, project_sphere, uniform_u0
    levels = eps_study_levels(args.eps_study)
    v, f = icosphere(args.eps_study_mesh)
    m, nres = 3, args.eps_study_restarts
    u0 = uniform_u0(7, nres, m, v.shape[0])
    mesh = sp.Mesh(v, f)
    prm = sp.params(levels[0][1], n_steps=0, stop_tol=1e-6, max_steps=200000,
                    precision="mixed", cg_rtol=1e-10, inner_rtol=args.inner_rtol,
                    check_every=args.check_every, extrapolate=args.extrapolate)
    log(f"[bench] eps study: {len(levels)} levels from icosphere level {args.eps_study_mesh} "
        f"({v.shape[0]} vertices)")
    t0 = time.perf_counter()
    def progress(level, rs):
        e = [r["energy"] for r in rs]
        log(f"[bench]   level {level} done: n {rs[0]['n_vert']}, {rs[0]['seconds']:.1f} s, "
            f"steps {min(r['steps'] for r in rs)}..{max(r['steps'] for r in rs)}, "
            f"E {min(e):.4f}..{max(e):.4f}")

    rc, res_all, lam_all, fin, u_all = sp.continue_levels(mesh, prm, m, u0, levels, project_sphere,
                                                          n_restarts=nres, on_level=progress)
    wall = time.perf_counter() - t0
    # the restart with the lowest final energy is the study's answer
    best = int(np.argmin([res_all[-1][r]["energy"] for r in range(nres)]))
    res = [lvl[best] for lvl in res_all]
    lam = lam_all[:, best * m:(best + 1) * m]
    u_fin = u_all[best * m:(best + 1) * m]
    total_steps = sum(x["steps"] for lvl in res_all for x in lvl)
    cdof_all = sum(float(x["steps"]) * x["n_vert"] * m for lvl in res_all for x in lvl)
    # the final partition, read sharply: the first Dirichlet eigenvalue of each
    # region of its argmax labels (Problem 1.1's energy, no eps in it)
    last = fin if fin is not None else mesh
    st = sp.State(last, sp.params(levels[-1][1], precision="fp64"), [m], [levels[-1][0]], u_fin)
    _, lab_am = st.labels()
    st.close()
    t1 = time.perf_counter()
    rc_e, lam_reg, _, its = sp.sp_region_eigen(last.h, [m], lab_am, u0=u_fin, shift=1.0, tol=1e-10,
                                               max_iter=200)
    rc_i, lam_in, _, its_in = sp.sp_region_eigen(last.h, [m], lab_am, u0=u_fin, shift=1.0,
                                                 tol=1e-10, max_iter=200, interior=True)
    t_eig = time.perf_counter() - t1
    log(f"[bench]   regions of the final partition: lambda_1 in [{np.round(lam_reg, 5)}, "
        f"{np.round(lam_in, 5)}], sum in [{lam_reg.sum():.5f}, {lam_in.sum():.5f}] (45/4 = 11.25), "
        f"{its} + {its_in} inverse iterations, {t_eig:.1f} s")
    table = np.loadtxt(os.path.join(ROOT, "tests", "golden", "tab_u_eps.txt"), ndmin=2)
    rows = []
    for i, ((eps, tau, ref), r) in enumerate(zip(levels, res)):
        row = dict(eps=eps, tau=tau, n_vert=r["n_vert"], steps=r["steps"],
                   energy=r["energy"], s_eps=r["s_eps"], seconds=round(r["seconds"], 3),
                   lam=[float(x) for x in lam[i]])
        if i < table.shape[0] and abs(table[i, 0] - eps) < 1e-5 * eps:  # table rounds eps
            row["paper_energy"], row["paper_s_eps"] = float(table[i, 1]), float(table[i, 4])
        rows.append(row)
        log(f"[bench]   eps {eps:.5g} tau {tau:.4g} n {r['n_vert']}: {r['steps']} steps, "
            f"E {r['energy']:.4f} S {r['s_eps']:.4f} ({r['seconds']:.1f} s)"
            + (f"  paper E {row['paper_energy']:.4f} S {row['paper_s_eps']:.4f}"
               if "paper_energy" in row else ""))
    for i in range(1, len(rows)):  # eoc of the energy error against 45/4 and of S_eps
        e0, e1 = 11.25 - rows[i - 1]["energy"], 11.25 - rows[i]["energy"]
        if e0 > 0 and e1 > 0:
            rows[i]["eoc_energy"] = float(np.log(e1 / e0) / np.log(0.5))
        rows[i]["eoc_s_eps"] = float(np.log(rows[i]["s_eps"] / rows[i - 1]["s_eps"]) / np.log(0.5))
    if fin is not None:
        fin.close()
    mesh.close()
    print(json.dumps({
        "metric": "eps study (continuation to the stopping rule): component-DOF updates/s",
        "value": cdof_all / wall, "unit": "cdof/s", "n_gpus": 1, "steps": int(total_steps),
        "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"eps study: unit sphere from icosahedral level {args.eps_study_mesh}, "
                               f"{nres} random restart(s) of m 3 in one batch, {len(levels)} levels "
                               "(eps 0.5 halving, tau 8e-4 / sqrt(2) per level, 4-fold refinement "
                               "before levels 2, 4, ...), stop |dE| < 1e-6 every M_tau = 0.1 / tau "
                               "steps per restart, mixed precision; levels reported for the restart "
                               "with the lowest final energy"},
        "best_restart": best,
        "final_energy_per_restart": [float(res_all[-1][r]["energy"]) for r in range(nres)],
        "wall_s": wall, "status": int(rc), "levels": rows,
        "final_partition": {"region_lambda_1_plain": [float(x) for x in lam_reg],
                            "region_lambda_1_interior": [float(x) for x in lam_in],
                            "sum_plain": float(lam_reg.sum()), "sum_interior": float(lam_in.sum()),
                            "y_partition_value": 11.25,
                            "inverse_iterations": [int(its), int(its_in)], "seconds": t_eig,
                            "status": [int(rc_e), int(rc_i)]}}))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed steps first (also timed on their own and reported as "
                         "warmup_window)")
    ap.add_argument("--workload", default="sphere7-batched", choices=sorted(WORKLOADS))
    ap.add_argument("--no-plain", action="store_true", help="skip the plain float64 legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving legs")
    ap.add_argument("--inner-rtol", type=float, default=1e-6,
                    help="relative reduction of each float32 inner solve")
    ap.add_argument("--check-every", type=int, default=8,
                    help="CG iterations between host convergence polls")
    ap.add_argument("--precond", default="cheb1", choices=("cheb1", "jacobi"),
                    help="CG preconditioner of the batched run (degree-1 Chebyshev "
                         "polynomial in D^-1 K, or Jacobi)")
    ap.add_argument("--extrapolate", type=int, default=5, choices=range(9),
                    help="previous heat increments used for each solve's start "
                         "(0: start from u)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark only: a seeded Poisson request stream over every "
                         "mesh kind through the continuous-batching server; prints latency "
                         "p50/p99 and throughput")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-rate", type=float, default=50.0, help="arrivals per second")
    ap.add_argument("--serve-sub-requests", type=int, default=8,
                    help="requests of the below-capacity stream in the default line")
    ap.add_argument("--serve-sub-rate", type=float, default=0.25)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--eps-study", type=int, default=0, metavar="LEVELS",
                    help="continuation benchmark instead: the convergence study in eps of "
                         "Section 3.1 (table tab:u-eps) for LEVELS levels from icosphere level "
                         "--eps-study-mesh, m = 3, each level to the stopping rule; prints the "
                         "per-level energies beside the paper's and the whole study's throughput")
    ap.add_argument("--eps-study-mesh", type=int, default=5)
    ap.add_argument("--eps-study-restarts", type=int, default=1,
                    help="random restarts run together through the study (the best is reported)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(restarts would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe * 2**20 // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 4, "copies": 5}))
        return

    from workloads import surface_mesh, batch_u0, uniform_u0
    if not (args.serve or args.eps_study):
        kind, groups, eps, tau = WORKLOADS[args.workload]
        v, f = surface_mesh(kind)
        cpu = None
        if not args.no_cpu:
            # first, while no GPU work has happened in this process (the oracle's
            # worker processes are forked from it)
            log("[bench] cpu oracle sample")
            cpu = cpu_baseline(v, f, groups, eps, tau, steps=1)
            log(f"[bench] cpu oracle {cpu['value']:.3e} cdof/s on {cpu['cores']} cores")

    import torch
    from paper_1408_2355_amd import segpart as sp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.serve:
        return serve(args, sp)
    if args.eps_study:
        return eps_study(args, sp)
    n = v.shape[0]
    u0, ms = batch_u0(n, groups)
    R, nres = int(ms.sum()), ms.size
    log(f"[bench] workload {args.workload}: n={n} restarts={nres} columns={R}")

    mesh = sp.Mesh(v, f)
    prm = sp.params(tau, precision="mixed", n_steps=1, energy_every=1, cg_rtol=1e-10,
                    inner_rtol=args.inner_rtol, max_outer=8, cg_max_iter=500,
                    check_every=args.check_every, extrapolate=args.extrapolate,
                    precond=args.precond)
    st = sp.State(mesh, prm, ms, np.full(nres, eps), u0)
    del u0
    log(f"[bench] warmup {args.warmup} steps")
    w0 = st.stats()
    tw = time.perf_counter()
    st.step(args.warmup)
    torch.cuda.synchronize()
    tw = time.perf_counter() - tw
    s0 = st.stats()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    rc = st.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s1 = st.stats()
    lam_b, seps_b, e_b = st.energy()
    tiling = st.tiling()
    st.close()
    value = R * n * args.steps / dt
    log(f"[bench] {value:.3e} cdof/s, {1e3 * dt / args.steps:.2f} ms/step, rc={rc}")

    # kernel times: the same warm-up and timed steps again, on a fresh state of
    # the same batch (the run is deterministic: the same iterations and results,
    # bit for bit), with HIP events recorded on the library's stream around
    # every CG kernel.  Recording them replaces the graph-replayed CG blocks by
    # launch-by-launch iterations, so the throughput above is timed without.
    log(f"[bench] profiled pass over the same {args.warmup} + {args.steps} steps")
    u0, _ = batch_u0(n, groups)
    pst = sp.State(mesh, prm, ms, np.full(nres, eps), u0)
    del u0
    pst.step(args.warmup)
    torch.cuda.synchronize()
    pst.profile(True)
    tp = time.perf_counter()
    pst.step(args.steps)
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    kt = [pst.kernel_time(k) for k in range(len(KERNEL_NAMES))]
    pst.profile(False)
    same = bool(np.array_equal(pst.energy()[2], e_b))
    pst.close()
    log(f"[bench] profiled pass {1e3 * tp / args.steps:.2f} ms/step, energies identical: {same}")

    # dominant kernel class by total time
    k = int(np.argmax([t[1] for t in kt]))
    launches, ms_tot, bytes_launch = kt[k]
    avg_s = ms_tot / max(launches, 1) * 1e-3
    achieved = bytes_launch / avg_s / 1e9 if launches else 0.0
    traffic, traffic_ratio, traffic_src = traffic_record(KERNEL_NAMES[k])
    roofline = dict(bound="hbm", kernel=KERNEL_NAMES[k], achieved=achieved, peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                    traffic_vs_algorithmic=traffic_ratio, traffic_source=traffic_src,
                    launches=launches, avg_us=avg_s * 1e6, bytes_per_launch=bytes_launch,
                    kernel_ms_total={KERNEL_NAMES[i]: kt[i][1]
                                     for i in range(len(KERNEL_NAMES)) if kt[i][0]})
    # the practical HBM rate: a 2 GiB device-to-device copy (read + write bytes),
    # after the timed window
    cx = torch.ones(2**29, dtype=torch.float32, device="cuda:0")
    cy = torch.empty_like(cx)
    cy.copy_(cx)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record()
    for _ in range(5):
        cy.copy_(cx)
    ce1.record()
    ce1.synchronize()
    copy_gbs = 5 * 2 * cx.numel() * 4 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del cx, cy
    roofline["copy_GBps"] = copy_gbs
    roofline["frac_of_copy"] = achieved / copy_gbs

    out = {
        "metric": "component-DOF updates/s (batched mixed-precision vs plain FP64 GPU, "
                  "<=1e-5 rel energy err)",
        "value": value, "unit": "cdof/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {mesh_text(kind)} ({n} vertices), "
                               f"m in {sorted(set(int(x) for x in ms))} x "
                               f"{groups[0][1]} restarts ({R} columns), eps {eps}, tau {tau}, "
                               f"float32 CG ({args.precond} preconditioner) in float64 "
                               "refinement, outer rtol 1e-10, "
                               f"energy every step; timed steps {args.warmup + 1}.."
                               f"{args.warmup + args.steps} of the run",
                   "columns": R, "n_vert": n},
        "warmup_window": {"steps": args.warmup,
                          "cdof_per_s": R * n * args.warmup / tw if args.warmup else None,
                          "iters_per_step": (s0["cg_iters"] - w0["cg_iters"]) / max(args.warmup, 1)},
        "cg": {"iters_per_step": (s1["cg_iters"] - s0["cg_iters"]) / args.steps,
               "outer_sweeps_per_step": (s1["outer_sweeps"] - s0["outer_sweeps"]) / args.steps,
               "converged": s1["converged"],
               "model_hbm_bytes_per_cdof": (s1["hbm_bytes"] - s0["hbm_bytes"]) / (R * n * args.steps)},
        "roofline": roofline,
        "tiling": tiling,
        "profiled_pass": {"ms_per_step": 1e3 * tp / args.steps, "energies_identical": same},
    }

    if not args.no_plain:
        # plain float64 form: restart 0 of each m group alone over the same
        # steps as the batch (warmup, then the timed window), with the
        # library's defaults (host poll every 8 CG iterations, the degree-1
        # Chebyshev preconditioner: the reference point of the speed-up),
        # polled every iteration, and, polled every iteration, with Jacobi
        for poll, pc, key in ((8, "cheb1", "plain_fp64"), (1, "cheb1", "plain_fp64_poll1"),
                              (1, "jacobi", "plain_fp64_jacobi")):
            pprm = sp.params(tau, precision="fp64", n_steps=1, energy_every=1, cg_rtol=1e-10,
                             cg_max_iter=2000, check_every=poll, precond=pc)
            cd, tt, errs, lerrs, serrs = 0.0, 0.0, [], [], []
            r0 = 0                      # index of the group's first restart in the batch
            c0 = 0                      # its first column
            for seed, nr, m in groups:
                u1 = uniform_u0(seed, 1, m, n)
                ps = sp.State(mesh, pprm, [m], [eps], u1)
                ps.step(args.warmup)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ps.step(args.steps)
                torch.cuda.synchronize()
                tt += time.perf_counter() - t0
                cd += m * n * args.steps
                l64, _, e64 = ps.energy()
                errs.append(abs(e_b[r0] - e64[0]) / abs(e64[0]))
                lerrs.append(float(np.max(np.abs(lam_b[c0:c0 + m] - l64) / np.abs(l64))))
                serrs.append(abs(lam_b[c0:c0 + m].sum() - l64.sum()) / abs(l64.sum()))
                ps.close()
                r0 += nr
                c0 += nr * m
            plain = cd / tt
            out[key] = {"value": plain, "unit": "cdof/s",
                        "sample": "restart 0 of each m group, one restart per solve, float64, "
                                  f"{pc} preconditioner, host convergence poll every "
                                  + ("CG iteration" if poll == 1 else "8 CG iterations")}
            out["speedup_vs_" + key] = value / plain
            log(f"[bench] plain fp64 ({pc}, poll {poll}) {plain:.3e} cdof/s, "
                f"speedup {value / plain:.2f}")
        out["energy_rel_err_vs_fp64"] = max(errs)
        out["lambda_rel_err_vs_fp64"] = max(lerrs)        # every lambda_i of the sampled restarts
        out["sum_lambda_rel_err_vs_fp64"] = max(serrs)
        log(f"[bench] energy err vs fp64 {max(errs):.2e}")

    mesh.close()

    if not args.no_serve:
        # the serving loop: the overloaded stream (50 requests/s) and a short
        # stream below capacity
        out["serving"] = {}
        for name, nreq, rate, plain_too in (("overloaded", args.serve_requests, args.serve_rate,
                                             not args.no_plain),
                                            ("below_capacity", args.serve_sub_requests,
                                             args.serve_sub_rate, False)):
            if nreq > 0:
                log(f"[bench] serving, {name}: {nreq} requests at {rate} req/s")
                out["serving"][name] = serve_leg(sp, nreq, rate, args.serve_budget_gb,
                                                 args.inner_rtol, with_plain=plain_too)

    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
