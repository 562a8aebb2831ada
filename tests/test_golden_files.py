"""The stored oracle trajectories match what the oracle computes now (the cheap entries are
recomputed) and the inputs they were made for (the batched workload recipe)."""
import json
import os

import oracle

HERE = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(HERE, name)) as fh:
        return json.load(fh)


def test_batched_golden_matches_the_workload_recipe_and_the_oracle():
    from bench import workload
    g = _load("batched_workload_trajectories.json")
    L, beta, m0 = workload(g["seed"], g["n_chains"])
    assert sorted({c["L"] for c in g["chains"]}) == [16, 32, 64, 128]
    for ref in g["chains"]:
        c = ref["chain"]
        assert (L[c], beta[c], m0[c]) == (ref["L"], ref["beta"], ref["m0"])
    for ref in g["chains"]:
        if ref["L"] > 32:
            continue  # the larger chains take the oracle tens of seconds
        c = ref["chain"]
        q = oracle.random_links(ref["L"], ref["L"], g["seed"], c)
        _, info = oracle.hmc_trajectory(q, ref["beta"], ref["m0"], g["seed"], c, 0, g["scheme"],
                                        g["tau"], g["n_outer"], g["n_inner"], tol=g["tol"])
        assert info["accepted"] == ref["accepted"]
        assert abs(info["dH"] - ref["dH"]) <= 1e-12 * max(1.0, abs(ref["dH"]))
        assert abs(info["H0"] - ref["H0"]) <= 1e-12 * abs(ref["H0"])
        assert info["n_dinv"] == ref["n_dinv"]


def test_thermalised_golden_matches_the_workload_recipe_and_the_oracle():
    import numpy as np
    from bench import workload
    g = _load("batched_workload_thermalised.json")
    L, beta, m0 = workload(g["seed"], g["n_chains"])
    assert sorted(c["L"] for c in g["chains"]) == [16, 16, 32, 32, 64]
    for ref in g["chains"]:
        c = ref["chain"]
        assert (L[c], beta[c], m0[c]) == (ref["L"], ref["beta"], ref["m0"])
        assert len(ref["links"]) == 2 * ref["L"] ** 2 and ref["traj"] == g["n_therm"]
    for ref in g["chains"]:
        if ref["L"] > 16:
            continue
        # the check trajectory from the stored links
        q = np.array(ref["links"]).reshape(ref["L"], ref["L"], 2)
        _, info = oracle.hmc_trajectory(q, ref["beta"], ref["m0"], g["seed"], ref["chain"],
                                        ref["traj"], g["scheme"], g["tau"], g["n_outer"],
                                        g["n_inner"], tol=g["tol"])
        assert info["accepted"] == ref["accepted"]
        assert abs(info["dH"] - ref["dH"]) <= 1e-12 * max(1.0, abs(ref["dH"]))


def test_thermalised_scheme_comparison_state():
    """The stored thermalised 32 x 32 state: written by the oracle alone for the stated
    couplings; its plaquette is that of its links, and it sits near equilibrium (the 5-stage
    scheme accepts most of the last 100 thermalisation trajectories)."""
    g = _load("scheme_comparison_thermalised.json")
    assert (g["L"], g["beta"], g["m0"], g["n_therm"]) == (32, 2.0, 0.1, 200)
    assert len(g["links"]) == 2 * 32 * 32
    import numpy as np
    q = np.array(g["links"]).reshape(32, 32, 2)
    assert abs(oracle.mean_plaquette(q) - g["plaquette"]) < 1e-12
    assert g["acceptance_last_100"] >= 0.8
    assert 0.6 < g["plaquette"] < 0.9
