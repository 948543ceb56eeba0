#!/usr/bin/env python3
"""Throughput benchmark of the segregation time step on one MI355X.

Default workload (the batched-restart configuration): unit sphere,
icosahedral level 7 (163842 vertices), m in {4, 8, 12, 16} with 64 seeded
U[0,1) initial states each (2560 columns in one batch), eps = 0.01,
tau = 5e-5, float32 CG inside float64 refinement (outer rtol 1e-10).

One timed "step" is one full time step of every restart (heat solve, node
step, normalisation) plus the energy evaluation and its read-back (the stop
test's input), i.e. every per-step part of the hot path; mesh set-up and the
initial normalisation happen before timing, labels after.

Printed: ONE JSON line with the throughput in component-DOF updates per
second (restart x component x vertex values advanced one step), the plain
float64 form (one restart at a time, host convergence check every CG
iteration) measured on a sample of the same restarts, the relative energy
error of the batched mixed form against that float64 run, the roofline of the
dominant kernel (HIP events on the library's stream), and the CPU oracle on
a bounded sample.
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
KERNEL_NAMES = ("matvec q=(M+tau A)p", "update x,r", "direction p")

WORKLOADS = {
    # name: (mesh level, [(seed, restarts, m)], eps, tau)
    "sphere7-batched": (7, [(3004, 64, 4), (3008, 64, 8), (3012, 64, 12), (3016, 64, 16)],
                        0.01, 5e-5),
    "sphere3": (3, [(1003, 1, 3)], 0.1, 1e-3),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(v, f, groups, eps, tau, steps=1):
    """The oracle on restart 0 of every m group, `steps` time steps each with
    its energy (BLAS limited to one thread: the oracle's solve is serial)."""
    from threadpoolctl import threadpool_limits
    from oracle import energy, flow
    from workloads import uniform_u0
    with threadpool_limits(limits=1):
        prob = flow.Problem(v, f, tau)
        _ = prob.lu                       # factorisation = set-up, not timed
        cols = 0
        t0 = time.perf_counter()
        for seed, _, m in groups:
            u = flow.normalise(prob.M, uniform_u0(seed, 1, m, v.shape[0]))
            for _ in range(steps):
                u = flow.step(prob, u, eps)
                energy.energy(v, f, prob.M, prob.A, u, eps)
            cols += m
        dt = time.perf_counter() - t0
    return dict(value=cols * v.shape[0] * steps / dt, unit="cdof/s", cores=1, kind="oracle",
                sample=f"restart 0 of each m group ({cols} of the workload's columns), "
                       f"{steps} step(s) with energy, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sphere7-batched", choices=sorted(WORKLOADS))
    ap.add_argument("--no-plain", action="store_true", help="skip the plain float64 leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--inner-rtol", type=float, default=1e-6,
                    help="relative reduction of each float32 inner solve")
    ap.add_argument("--check-every", type=int, default=8,
                    help="CG iterations between host convergence polls")
    ap.add_argument("--no-extrapolate", action="store_true",
                    help="start every heat solve from u (not u + previous increment)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe * 2**20 // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 4, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(restarts would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1408_2355_amd import segpart as sp
    from workloads import icosphere, batch_u0, uniform_u0

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    level, groups, eps, tau = WORKLOADS[args.workload]
    v, f = icosphere(level)
    n = v.shape[0]
    u0, ms = batch_u0(n, groups)
    R, nres = int(ms.sum()), ms.size
    log(f"[bench] workload {args.workload}: n={n} restarts={nres} columns={R}")

    mesh = sp.Mesh(v, f)
    prm = sp.params(tau, precision="mixed", n_steps=1, energy_every=1, cg_rtol=1e-10,
                    inner_rtol=args.inner_rtol, max_outer=8, cg_max_iter=500,
                    check_every=args.check_every, extrapolate=int(not args.no_extrapolate))
    st = sp.State(mesh, prm, ms, np.full(nres, eps), u0)
    del u0
    log("[bench] warmup")
    st.step(args.warmup)
    torch.cuda.synchronize()
    st.profile(True)
    s0 = st.stats()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    rc = st.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s1 = st.stats()
    kt = [st.kernel_time(k) for k in range(3)]
    st.profile(False)
    lam_b, seps_b, e_b = st.energy()
    value = R * n * args.steps / dt
    log(f"[bench] {value:.3e} cdof/s, {1e3 * dt / args.steps:.2f} ms/step, rc={rc}")

    # dominant kernel class by total time
    k = int(np.argmax([t[1] for t in kt]))
    launches, ms_tot, bytes_launch = kt[k]
    avg_s = ms_tot / max(launches, 1) * 1e-3
    achieved = bytes_launch / avg_s / 1e9 if launches else 0.0
    roofline = dict(bound="hbm", kernel=KERNEL_NAMES[k], achieved=achieved, peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=None,
                    launches=launches, avg_us=avg_s * 1e6, bytes_per_launch=bytes_launch,
                    kernel_ms_total={KERNEL_NAMES[i]: kt[i][1] for i in range(3)})

    out = {
        "metric": "component-DOF updates/s (batched mixed-precision vs plain FP64 GPU, "
                  "<=1e-5 rel energy err)",
        "value": value, "unit": "cdof/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: icosphere level {level} ({n} vertices), "
                               f"m in {sorted(set(int(x) for x in ms))} x "
                               f"{groups[0][1]} restarts ({R} columns), eps {eps}, tau {tau}, "
                               "float32 CG in float64 refinement, outer rtol 1e-10, "
                               "energy every step",
                   "columns": R, "n_vert": n},
        "cg": {"iters_per_step": (s1["cg_iters"] - s0["cg_iters"]) / args.steps,
               "outer_sweeps_per_step": (s1["outer_sweeps"] - s0["outer_sweeps"]) / args.steps,
               "converged": s1["converged"]},
        "roofline": roofline,
        "tiling": st.tiling(),
    }

    if not args.no_plain:
        # plain float64 form: restart 0 of each m group alone, host poll every
        # CG iteration, same step count as the batch (warmup + timed)
        pprm = sp.params(tau, precision="fp64", n_steps=1, energy_every=1, cg_rtol=1e-10,
                         cg_max_iter=2000, check_every=1)
        cd, tt, errs = 0.0, 0.0, []
        r0 = 0                      # index of the group's first restart in the batch
        for seed, nr, m in groups:
            u1 = uniform_u0(seed, 1, m, n)
            ps = sp.State(mesh, pprm, [m], [eps], u1)
            ps.step(args.warmup)
            t0 = time.perf_counter()
            ps.step(args.steps)
            tt += time.perf_counter() - t0
            cd += m * n * args.steps
            _, _, e64 = ps.energy()
            errs.append(abs(e_b[r0] - e64[0]) / abs(e64[0]))
            ps.close()
            r0 += nr
        plain = cd / tt
        out["plain_fp64"] = {"value": plain, "unit": "cdof/s",
                             "sample": "restart 0 of each m group, one restart per solve, "
                                       "float64, host convergence poll every CG iteration"}
        out["speedup_vs_plain_fp64"] = value / plain
        out["energy_rel_err_vs_fp64"] = max(errs)
        log(f"[bench] plain fp64 {plain:.3e} cdof/s, speedup {value / plain:.2f}, "
            f"energy err {max(errs):.2e}")

    if not args.no_cpu:
        log("[bench] cpu oracle sample")
        out["cpu_baseline"] = cpu_baseline(v, f, groups, eps, tau)

    st.close()
    mesh.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
