"""Writes precision_trajectories.json: FP64 oracle trajectories of the precision workload.

The workload is the adapted nested force-gradient scheme (Eq. (11)) with tau = 1,
8 outer and 4 inner steps, beta = 4, m0 = 0.05, on 128 x 128 and 256 x 256 lattices,
started from the seeded Philox hot start.  Every value in the file comes from the
oracle alone (CG tolerance 1e-12); the GPU tests replay the same seeded trajectories in
mixed precision and compare Delta H and the accept decisions.

    python tests/golden/make_precision_golden.py [L ...]

Each lattice size is written under its own key, so sizes can be produced separately
and merged into the existing file.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

OUT = os.path.join(HERE, "precision_trajectories.json")
BETA, M0, TAU, N_OUTER, N_INNER, TOL = 4.0, 0.05, 1.0, 8, 4, 1e-12
RUNS = {128: (1283, 4), 256: (2563, 2)}  # L -> (seed, trajectories)


def run(L):
    seed, n_traj = RUNS[L]
    q = oracle.random_links(L, L, seed, 0)
    trajs = []
    for t in range(n_traj):
        t0 = time.time()
        q, info = oracle.hmc_trajectory(q, BETA, M0, seed, 0, t, "adapted_nested_fg", TAU,
                                        N_OUTER, N_INNER, tol=TOL)
        assert info["rc"] == 0
        trajs.append({k: (bool(v) if k == "accepted" else
                          int(v) if k in ("n_solves", "n_cg_iters", "n_dinv") else float(v))
                      for k, v in info.items() if k != "rc"})
        print(f"L={L} trajectory {t}: dH={info['dH']:.12g} accepted={info['accepted']} "
              f"({time.time() - t0:.0f} s)", flush=True)
    return {"seed": seed, "beta": BETA, "m0": M0, "scheme": "adapted_nested_fg", "tau": TAU,
            "n_outer": N_OUTER, "n_inner": N_INNER, "tol": TOL, "trajectories": trajs}


def main():
    sizes = [int(a) for a in sys.argv[1:]] or sorted(RUNS)
    for L in sizes:
        result = run(L)
        data = {}
        if os.path.exists(OUT):
            with open(OUT) as fh:
                data = json.load(fh)
        data[str(L)] = result
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main()
