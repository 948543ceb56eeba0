"""Write the oracle's reference results for the level-6 sphere workload.

Unit sphere, icosahedral level 6 (40962 vertices), eps = 0.02, tau = 1e-4,
2000 steps, energy every 100 steps; two runs: m = 3 (u0 seed 2003) and m = 6
(u0 seed 2006), iid U[0,1) initial values.  Calls only oracle/ and workloads/.

Stored per run (config2_oracle.npz): lambda, S_eps, E, the energy history,
the final state at 512 seeded sample vertices, the labels at those vertices,
the per-label vertex counts, and the oracle's own noise floor: the largest
relative change of those quantities when u0 is perturbed by 1e-14 relative.

    python tests/golden/make_config2.py      (a few minutes on one core)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import flow  # noqa: E402
from workloads import icosphere, uniform_u0  # noqa: E402

LEVEL, EPS, TAU, STEPS, EVERY = 6, 0.02, 1e-4, 2000, 100
RUNS = {"m3": (3, 2003), "m6": (6, 2006)}


def rel(a, b):
    return float(np.abs(np.asarray(a) - b).max() / np.abs(b).max())


def main(out=os.path.join(HERE, "config2_oracle.npz")):
    v, f = icosphere(LEVEL)
    prob = flow.Problem(v, f, TAU)
    sample = np.sort(np.random.Generator(np.random.PCG64(62)).choice(v.shape[0], 512,
                                                                      replace=False))
    data = {"sample": sample}
    for name, (m, seed) in RUNS.items():
        u0 = uniform_u0(seed, 1, m, v.shape[0])
        res = flow.run(prob, u0, [m], [EPS], STEPS, energy_every=EVERY)
        rng = np.random.default_rng(7)
        up = u0 * (1.0 + 1e-14 * rng.standard_normal(u0.shape))
        alt = flow.run(prob, up, [m], [EPS], STEPS, energy_every=EVERY)
        floor = max(rel(alt["u"], res["u"]), rel(alt["lam"], res["lam"]),
                    rel(alt["s_eps"], res["s_eps"]))
        data[f"{name}_lam"] = res["lam"]
        data[f"{name}_s_eps"] = res["s_eps"]
        data[f"{name}_energy"] = res["energy"]
        data[f"{name}_history"] = np.array(res["history"][0])
        data[f"{name}_u_sample"] = res["u"][:, sample]
        data[f"{name}_labels_sample"] = res["labels"][0][sample]
        data[f"{name}_label_counts"] = np.bincount(res["labels"][0] + 1, minlength=m + 1)
        data[f"{name}_noise_floor"] = floor
        print(name, "lambda", res["lam"], "S_eps", res["s_eps"], "E", res["energy"],
              "floor", floor, flush=True)
    np.savez(out, **data)
    print("wrote", out)


if __name__ == "__main__":
    main()
