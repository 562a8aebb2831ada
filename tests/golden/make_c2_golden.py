"""Writes scheme_comparison_thermalised.json: a thermalised configuration of the plain FP64
32 x 32 scheme comparison (beta 2, m0 0.1), made by the oracle alone.

From the seeded Philox hot start (seed 3232, chain 0) the oracle runs N_THERM trajectories of
the 5-stage scheme (Eq. (4)), tau = 1, 10 steps, CG tolerance 1e-12, trajectory counters
0 .. N_THERM - 1, and stores the links (lexicographic layout: x fastest, then t, then mu
innermost), the mean plaquette and the acceptance of the last 100 of them.  The GPU test
loads these links and runs the next trajectory of every scheme of the comparison against the
oracle's trajectory from the same links and random numbers.

    python tests/golden/make_c2_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

OUT = os.path.join(HERE, "scheme_comparison_thermalised.json")
L, BETA, M0, SEED, N_THERM, TOL = 32, 2.0, 0.1, 3232, 200, 1e-12


def main():
    q = oracle.random_links(L, L, SEED, 0)
    acc = []
    t0 = time.time()
    for t in range(N_THERM):
        q, info = oracle.hmc_trajectory(q, BETA, M0, SEED, 0, t, "omelyan", 1.0, 10, 1, tol=TOL)
        assert info["rc"] == 0
        acc.append(bool(info["accepted"]))
        if t % 20 == 19:
            print(f"trajectory {t + 1}: plaquette {info['plaquette']:.6f} ({time.time() - t0:.0f} s)",
                  flush=True)
    rec = {"L": L, "beta": BETA, "m0": M0, "seed": SEED, "chain": 0, "n_therm": N_THERM,
           "scheme": "omelyan", "tau": 1.0, "n_steps": 10, "tol": TOL,
           "plaquette": oracle.mean_plaquette(q), "acceptance_last_100": sum(acc[-100:]) / 100,
           "links": [float(v) for v in q.ravel()]}
    with open(OUT, "w") as fh:
        json.dump(rec, fh)
        fh.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
