"""Writes batched_workload_trajectories.json: FP64 oracle trajectories of sampled chains of
the batched benchmark workload.

The workload is 512 chains, L in {16, 32, 64, 128} with weights 4:3:2:1, beta U[1, 4],
m0 U[0.02, 0.2] (the recipe of bench.workload, seed 1512), hot start, adapted nested
force-gradient scheme (Eq. (11)) with tau = 1, 8 outer and 4 inner steps.  Sampled chains:
the first chain of each lattice size, and the L = 128 chain with the smallest mass (the
slowest solves).  Every value comes from the oracle alone (CG tolerance 1e-12), for the first
trajectory of each chain; the GPU test runs the whole 512-chain batch in mixed precision and
compares these chains.

    python tests/golden/make_batched_golden.py
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
SEED, N_CHAINS, TAU, N_OUTER, N_INNER, TOL = 1512, 512, 1.0, 8, 4, 1e-12


def sampled_chains(L, m0):
    picks = [L.index(size) for size in (16, 32, 64, 128)]
    big = [c for c in range(len(L)) if L[c] == 128]
    slowest = min(big, key=lambda c: m0[c])
    if slowest not in picks:
        picks.append(slowest)
    return picks


def main():
    L, beta, m0 = workload(SEED, N_CHAINS)
    out = {"seed": SEED, "n_chains": N_CHAINS, "scheme": "adapted_nested_fg", "tau": TAU,
           "n_outer": N_OUTER, "n_inner": N_INNER, "tol": TOL, "chains": []}
    for c in sampled_chains(L, m0):
        t0 = time.time()
        q = oracle.random_links(L[c], L[c], SEED, c)
        _, info = oracle.hmc_trajectory(q, beta[c], m0[c], SEED, c, 0, "adapted_nested_fg", TAU,
                                        N_OUTER, N_INNER, tol=TOL)
        assert info["rc"] == 0
        rec = {"chain": c, "L": L[c], "beta": beta[c], "m0": m0[c]}
        rec.update({k: (bool(v) if k == "accepted" else
                        int(v) if k in ("n_solves", "n_cg_iters", "n_dinv") else float(v))
                    for k, v in info.items() if k != "rc"})
        out["chains"].append(rec)
        print(f"chain {c} (L={L[c]}, m0={m0[c]:.4f}): dH={info['dH']:.12g} "
              f"accepted={info['accepted']} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
