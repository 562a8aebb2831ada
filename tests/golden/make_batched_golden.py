"""Writes batched_workload_trajectories.json and batched_workload_thermalised.json: FP64
oracle trajectories of sampled chains of the batched benchmark workload.

The workload is 512 chains, L in {16, 32, 64, 128} with weights 4:3:2:1, beta U[1, 4],
m0 U[0.02, 0.2] (the recipe of bench.workload, seed 1512), hot start, adapted nested
force-gradient scheme (Eq. (11)) with tau = 1, 8 outer and 4 inner steps.  Sampled chains:
the first chain of each lattice size, and the L = 128 chain with the smallest mass (the
slowest solves).  Every value comes from the oracle alone (CG tolerance 1e-12), for the first
trajectory of each chain; the GPU test runs the whole 512-chain batch in mixed precision and
compares these chains.

batched_workload_thermalised.json holds, for two L = 16, two L = 32 and one L = 64 chain of the same
workload, the links after N_THERM oracle trajectories from the hot start (tolerance 1e-12,
trajectory counters 0 .. N_THERM - 1) in the lexicographic layout (x fastest, then t, then mu
innermost), and the oracle's trajectory with counter N_THERM from those links at CG tolerance
1e-14: the benchmark loads these links into the batch after its timed steps, runs one
trajectory of the whole batch at the timed settings and reports the Delta H error against
this record.

    python tests/golden/make_batched_golden.py [first] [thermalised]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from bench import workload  # noqa: E402  (the input recipe only: seeded numpy draws)

OUT = os.path.join(HERE, "batched_workload_trajectories.json")
OUT_THERM = os.path.join(HERE, "batched_workload_thermalised.json")
SEED, N_CHAINS, TAU, N_OUTER, N_INNER, TOL = 1512, 512, 1.0, 8, 4, 1e-12
N_THERM, TOL_CHECK = 20, 1e-14


def sampled_chains(L, m0):
    picks = [L.index(size) for size in (16, 32, 64, 128)]
    big = [c for c in range(len(L)) if L[c] == 128]
    slowest = min(big, key=lambda c: m0[c])
    if slowest not in picks:
        picks.append(slowest)
    return picks


def thermalised_chains(L):
    picks = []
    for size, n in ((16, 2), (32, 2), (64, 1)):
        picks += [c for c in range(len(L)) if L[c] == size][:n]
    return picks


def record(info):
    return {k: (bool(v) if k == "accepted" else
                int(v) if k in ("n_solves", "n_cg_iters", "n_dinv") else float(v))
            for k, v in info.items() if k != "rc"}


def thermalised(L, beta, m0):
    out = {"seed": SEED, "n_chains": N_CHAINS, "scheme": "adapted_nested_fg", "tau": TAU,
           "n_outer": N_OUTER, "n_inner": N_INNER, "n_therm": N_THERM, "tol_therm": TOL,
           "tol": TOL_CHECK, "chains": []}
    for c in thermalised_chains(L):
        t0 = time.time()
        q = oracle.random_links(L[c], L[c], SEED, c)
        for t in range(N_THERM):
            q, info = oracle.hmc_trajectory(q, beta[c], m0[c], SEED, c, t, "adapted_nested_fg",
                                            TAU, N_OUTER, N_INNER, tol=TOL)
            assert info["rc"] == 0
        start = q.copy()
        _, info = oracle.hmc_trajectory(start, beta[c], m0[c], SEED, c, N_THERM,
                                        "adapted_nested_fg", TAU, N_OUTER, N_INNER, tol=TOL_CHECK)
        assert info["rc"] == 0
        rec = {"chain": c, "L": L[c], "beta": beta[c], "m0": m0[c], "traj": N_THERM,
               "links": [float(v) for v in start.ravel()]}
        rec.update(record(info))
        out["chains"].append(rec)
        print(f"thermalised chain {c} (L={L[c]}): dH={info['dH']:.12g} "
              f"accepted={info['accepted']} ({time.time() - t0:.0f} s)", flush=True)
    return out


def main():
    parts = sys.argv[1:] or ["first", "thermalised"]
    L, beta, m0 = workload(SEED, N_CHAINS)
    if "thermalised" in parts:
        with open(OUT_THERM, "w") as fh:
            json.dump(thermalised(L, beta, m0), fh, sort_keys=True)
            fh.write("\n")
    if "first" not in parts:
        return
    out = {"seed": SEED, "n_chains": N_CHAINS, "scheme": "adapted_nested_fg", "tau": TAU,
           "n_outer": N_OUTER, "n_inner": N_INNER, "tol": TOL, "chains": []}
    for c in sampled_chains(L, m0):
        t0 = time.time()
        q = oracle.random_links(L[c], L[c], SEED, c)
        _, info = oracle.hmc_trajectory(q, beta[c], m0[c], SEED, c, 0, "adapted_nested_fg", TAU,
                                        N_OUTER, N_INNER, tol=TOL)
        assert info["rc"] == 0
        rec = {"chain": c, "L": L[c], "beta": beta[c], "m0": m0[c]}
        rec.update(record(info))
        out["chains"].append(rec)
        print(f"chain {c} (L={L[c]}, m0={m0[c]:.4f}): dH={info['dH']:.12g} "
              f"accepted={info['accepted']} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
