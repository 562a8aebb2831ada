"""GPU tests of the plain-method, differentiation and failure-handling configurations:

- 32 x 32 trajectories (beta 2, m0 0.1, CG tolerance 1e-12) of the five schemes of the
  scheme comparison over its step grid (n_outer in {4, 8, 16}, n_inner in {2, 4} for the
  nested schemes), on both solver paths, against the FP64 oracle (Sec. 2.1, 2.2), and one
  trajectory each of 100 chains of that configuration in one batch;
- the action S = S_G + S_F as a torch.autograd.Function at 128 x 128 for m0 in {0.1, 0.05}:
  its gradient against central finite differences (eps = 1e-6, 64 seeded links) and the
  oracle force (Sec. 3, Eqs. (13)-(17));
- the C ABI's per-chain failure convention inside a batched trajectory: a chain whose solve
  hits the iteration cap, or whose links hold a NaN, reports its status, is rejected and gets
  its links back, and every other chain is bit-identical to the run without it (also with
  the chains split into two groups).
"""
import math
from concurrent.futures import ThreadPoolExecutor
from functools import lru_cache

import numpy as np
import pytest

import oracle
from tests import inputs
from tests.gpu_helpers import Batch, hmc, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SOLVERS = [0, 2048]  # persistent limit: 0 = multi-workgroup slot kernels only

# ------------------------------------------------------------------ 32 x 32 scheme comparison
C2_L, C2_BETA, C2_M0, C2_TOL, C2_SEED, C2_TRAJ = 32, 2.0, 0.1, 1e-12, 3232, 2
C2_CASES = ([(s, n, 1) for s in ("leapfrog", "omelyan", "force_gradient") for n in (4, 8, 16)] +
            [(s, n, m) for s in ("nested_fg", "adapted_nested_fg") for n in (4, 8, 16)
             for m in (2, 4)])


def _oracle_c2(case):
    scheme, n_outer, n_inner = case
    q = oracle.random_links(C2_L, C2_L, C2_SEED, 0)
    out = []
    for t in range(C2_TRAJ):
        q, info = oracle.hmc_trajectory(q, C2_BETA, C2_M0, C2_SEED, 0, t, scheme, 1.0, n_outer,
                                        n_inner, tol=C2_TOL)
        assert info["rc"] == 0
        out.append((q.copy(), info))
    return out


@lru_cache(maxsize=None)
def c2_reference():
    """Oracle chains of every case, run as concurrent threads (the oracle keeps no global
    state and its calls release the interpreter lock)."""
    with ThreadPoolExecutor(max_workers=16) as ex:
        return dict(zip(C2_CASES, ex.map(_oracle_c2, C2_CASES)))


@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("scheme,n_outer,n_inner", C2_CASES)
def test_scheme_comparison_32x32_matches_oracle(scheme, n_outer, n_inner, persistent):
    ref = c2_reference()[(scheme, n_outer, n_inner)]
    b = Batch([(C2_L, C2_L, C2_BETA, C2_M0)], seed=C2_SEED, persistent=persistent)
    b.lat.hot_start()
    b.lat.set_solver(tol=C2_TOL)
    for t in range(C2_TRAJ):
        r = b.lat.trajectory(scheme, 1.0, n_outer, n_inner)
        qr, ir = ref[t]
        assert r.status[0] == 0
        assert r.accepted[0] == ir["accepted"], t
        assert abs(r.dH[0] - ir["dH"]) <= 1e-10 * max(1.0, abs(ir["dH"])), (t, r.dH[0], ir["dH"])
        assert np.max(np.abs(b.links_from_native(b.lat.q)[0] - qr)) < 1e-9, t


# One trajectory each of 100 chains of the same configuration from independent hot starts
# (Philox chain index), in one batch, against 100 oracle trajectories.
C2_BATCH, C2_BATCH_SEED = 100, 3233


def _oracle_c2_chain(args):
    scheme, n_outer, n_inner, c = args
    q = oracle.random_links(C2_L, C2_L, C2_BATCH_SEED, c)
    _, info = oracle.hmc_trajectory(q, C2_BETA, C2_M0, C2_BATCH_SEED, c, 0, scheme, 1.0, n_outer,
                                    n_inner, tol=C2_TOL)
    return info


@lru_cache(maxsize=None)
def c2_batch_reference(scheme, n_outer, n_inner):
    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(_oracle_c2_chain, [(scheme, n_outer, n_inner, c) for c in range(C2_BATCH)]))


@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("scheme,n_outer,n_inner", [("omelyan", 8, 1), ("adapted_nested_fg", 4, 2)])
def test_scheme_comparison_100_chains_match_oracle(scheme, n_outer, n_inner, persistent):
    refs = c2_batch_reference(scheme, n_outer, n_inner)
    b = Batch([(C2_L, C2_L, C2_BETA, C2_M0)] * C2_BATCH, seed=C2_BATCH_SEED, persistent=persistent)
    b.lat.hot_start()
    b.lat.set_solver(tol=C2_TOL)
    r = b.lat.trajectory(scheme, 1.0, n_outer, n_inner)
    for c, ir in enumerate(refs):
        assert ir["rc"] == 0 and r.status[c] == 0, c
        assert r.accepted[c] == ir["accepted"], c
        assert abs(r.dH[c] - ir["dH"]) <= 1e-10 * max(1.0, abs(ir["dH"])), (c, r.dH[c], ir["dH"])


# From the thermalised configuration of the comparison (200 5-stage oracle trajectories from
# the hot start, stored by tests/golden/make_c2_golden.py): the next trajectory of each scheme
# at its acceptance-matched step setting, against the oracle's from the same links.
C2T_CASES = [("leapfrog", 32, 1), ("omelyan", 8, 1), ("force_gradient", 4, 1), ("nested_fg", 4, 2),
             ("adapted_nested_fg", 4, 2), ("adapted_nested_fg", 8, 4)]


@lru_cache(maxsize=None)
def c2_thermalised():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "scheme_comparison_thermalised.json")) as fh:
        g = json.load(fh)
    q = np.array(g["links"]).reshape(g["L"], g["L"], 2)

    def run(case):
        scheme, n_outer, n_inner = case
        return oracle.hmc_trajectory(q, g["beta"], g["m0"], g["seed"], g["chain"], g["n_therm"],
                                     scheme, 1.0, n_outer, n_inner, tol=C2_TOL)

    with ThreadPoolExecutor(max_workers=len(C2T_CASES)) as ex:
        return g, q, dict(zip(C2T_CASES, ex.map(run, C2T_CASES)))


@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("scheme,n_outer,n_inner", C2T_CASES)
def test_scheme_comparison_from_the_thermalised_32x32_configuration(scheme, n_outer, n_inner, persistent):
    g, q, refs = c2_thermalised()
    q_ref, info = refs[(scheme, n_outer, n_inner)]
    assert info["rc"] == 0
    b = Batch([(g["L"], g["L"], g["beta"], g["m0"])], seed=g["seed"], persistent=persistent)
    b.set_q([q])
    b.lat.trajectory_counter = g["n_therm"]
    b.lat.set_solver(tol=C2_TOL)
    r = b.lat.trajectory(scheme, 1.0, n_outer, n_inner)
    assert r.status[0] == 0
    assert r.accepted[0] == info["accepted"]
    assert abs(r.dH[0] - info["dH"]) <= 1e-10 * max(1.0, abs(info["dH"])), (r.dH[0], info["dH"])
    assert abs(r.plaquette[0] - info["plaquette"]) < 1e-11
    assert np.max(np.abs(b.links_from_native(b.lat.q)[0] - q_ref)) < 1e-9


# ------------------------------------------------------------------ differentiation at 128 x 128
@pytest.mark.parametrize("m0", [0.1, 0.05])
def test_autograd_action_128_against_finite_differences_and_oracle(m0):
    m = hmc()
    L, beta = 128, 2.0
    b = Batch([(L, L, beta, m0)])
    q = inputs.smooth_angles(L, L, 1281, 0.4)
    phi = inputs.random_spinor(L, L, 1282)
    phin = b.spinor_to_native([phi])
    qn = b.links_to_native([q]).clone().requires_grad_(True)
    S = m.SchwingerAction.apply(qn, b.lat, phin, 1e-14)
    S.sum().backward()
    grad = b.links_from_native(qn.grad)[0]
    fr, _, _, sfr, _ = oracle.fermion_force(q, phi, m0, tol=1e-14)
    ref = oracle.gauge_force(q, beta) + fr
    assert rel(grad, ref) < 1e-10
    S_ref = oracle.gauge_action(q, beta) + sfr
    assert abs(float(S[0].detach()) - S_ref) < 1e-11 * S_ref
    g = np.random.default_rng(1283 + int(m0 * 100))
    eps, worst = 1e-6, 0.0
    for _ in range(64):
        t, x, mu = int(g.integers(L)), int(g.integers(L)), int(g.integers(2))
        qp, qm = q.copy(), q.copy()
        qp[t, x, mu] += eps
        qm[t, x, mu] -= eps
        with torch.no_grad():
            sp = float(m.SchwingerAction.apply(b.links_to_native([qp]), b.lat, phin, 1e-14)[0])
            sm = float(m.SchwingerAction.apply(b.links_to_native([qm]), b.lat, phin, 1e-14)[0])
        worst = max(worst, abs((sp - sm) / (2 * eps) - grad[t, x, mu]))
    assert worst < 1e-6 * np.max(np.abs(grad)), worst


@pytest.mark.parametrize("m0", [0.1, 0.05])
def test_autograd_action_on_thermalised_16x16_links(m0):
    """The differentiation check on thermalised links: the 16 x 16 links the oracle reached
    after 20 trajectories (stored with the batched workload's check states), at beta 2 and
    m0 in {0.1, 0.05}: the gradient against the oracle force and against central finite
    differences (eps = 1e-6) on 64 seeded links."""
    import json
    import os
    m = hmc()
    path = os.path.join(os.path.dirname(__file__), "golden", "batched_workload_thermalised.json")
    with open(path) as fh:
        gold = json.load(fh)
    ref = [c for c in gold["chains"] if c["L"] == 16][0]
    L, beta = 16, 2.0
    q = np.array(ref["links"]).reshape(L, L, 2)
    b = Batch([(L, L, beta, m0)])
    phi = inputs.random_spinor(L, L, 1601)
    phin = b.spinor_to_native([phi])
    qn = b.links_to_native([q]).clone().requires_grad_(True)
    S = m.SchwingerAction.apply(qn, b.lat, phin, 1e-14)
    S.sum().backward()
    grad = b.links_from_native(qn.grad)[0]
    want = oracle.gauge_force(q, beta) + oracle.fermion_force(q, phi, m0, tol=1e-14)[0]
    assert rel(grad, want) < 1e-10
    g = np.random.default_rng(1602)
    eps, worst = 1e-6, 0.0
    for _ in range(64):
        t, x, mu = int(g.integers(L)), int(g.integers(L)), int(g.integers(2))
        qp, qm = q.copy(), q.copy()
        qp[t, x, mu] += eps
        qm[t, x, mu] -= eps
        with torch.no_grad():
            sp = float(m.SchwingerAction.apply(b.links_to_native([qp]), b.lat, phin, 1e-14)[0])
            sm = float(m.SchwingerAction.apply(b.links_to_native([qm]), b.lat, phin, 1e-14)[0])
        worst = max(worst, abs((sp - sm) / (2 * eps) - grad[t, x, mu]))
    assert worst < 1e-6 * np.max(np.abs(grad)), worst


# ------------------------------------------------------------------ per-chain failures
# Four 16 x 16 chains from a hot start: three heavy (m0 0.5, about 70 CG iterations per solve)
# and one light (m0 -0.4, more than 300), so an iteration cap of 200 stops only the light one.
FAIL_SHAPES = [(16, 16, 2.0, 0.5), (16, 16, 1.5, 0.5), (16, 16, 2.0, -0.4), (16, 16, 3.0, 0.5)]
LIGHT = 2


def _run(shapes, prec, persistent, max_iter, plant_nan=None, n_traj=2, groups=1):
    b = Batch(shapes, seed=4242, persistent=persistent)
    b.lat.set_cg_groups(groups)
    b.lat.hot_start()
    b.lat.set_solver(tol=1e-12, max_iter=max_iter)
    if plant_nan is not None:
        qs = b.links_from_native(b.lat.q)
        qs[plant_nan][3, 5, 1] = float("nan")
        b.set_q(qs)
    out = []
    for _ in range(n_traj):
        before = b.links_from_native(b.lat.q)
        r = b.lat.trajectory("adapted_nested_fg", 1.0, 4, 2, prec=prec)
        out.append((before, r, b.links_from_native(b.lat.q)))
    return out


@pytest.mark.parametrize("groups", [1, 2])
@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chain_at_the_iteration_cap_is_rejected_alone(prec, persistent, groups):
    capped = _run(FAIL_SHAPES, prec, persistent, 200, groups=groups)
    free = _run(FAIL_SHAPES, prec, persistent, 100000)
    for (before, r, after), (_, rf, after_f) in zip(capped, free):
        assert r.status[LIGHT] == -3 and not r.accepted[LIGHT]
        assert rf.status[LIGHT] == 0
        assert np.array_equal(after[LIGHT], before[LIGHT])
        for c in range(len(FAIL_SHAPES)):
            if c == LIGHT:
                continue
            assert r.status[c] == 0
            assert r.dH[c] == rf.dH[c] and r.accepted[c] == rf.accepted[c], c
            assert r.n_cg_iters[c] == rf.n_cg_iters[c], c
            assert np.array_equal(after[c], after_f[c]), c


@pytest.mark.parametrize("groups", [1, 2])
@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chain_with_a_nan_link_is_rejected_alone(prec, persistent, groups):
    bad = 1
    shapes = [(16, 16, 2.0, 0.2), (16, 16, 1.5, 0.2), (8, 8, 2.0, 0.1), (16, 16, 3.0, 0.15)]
    poisoned = _run(shapes, prec, persistent, 100000, plant_nan=bad, groups=groups)
    clean = _run(shapes, prec, persistent, 100000)
    for (before, r, after), (_, rc, after_c) in zip(poisoned, clean):
        assert r.status[bad] == -5 and not r.accepted[bad]
        assert np.array_equal(after[bad], before[bad], equal_nan=True)
        assert math.isnan(after[bad][3, 5, 1])
        for c in range(len(shapes)):
            if c == bad:
                continue
            assert r.status[c] == 0 and rc.status[c] == 0
            assert r.dH[c] == rc.dH[c] and r.accepted[c] == rc.accepted[c], c
            assert np.array_equal(after[c], after_c[c]), c


def test_unconverged_actions_raise_but_fill_the_gauge_part():
    """An unconverged S_F solve: the binding raises (no silent zero action), and the C ABI
    still fills S_G and the plaquette and marks the chain's S_F as NaN."""
    import ctypes
    m = hmc()
    b = Batch([(16, 16, 2.0, -0.4), (8, 8, 2.0, 0.5)], seed=5)
    b.lat.hot_start()
    b.lat.set_solver(tol=1e-12, max_iter=5)
    phi = b.spinor_to_native([inputs.random_spinor(16, 16, 6), inputs.random_spinor(8, 8, 7)])
    with pytest.raises(m.HMCError):
        b.lat.actions(phi)
    sg, pl, sf = (ctypes.c_double * 2)(), (ctypes.c_double * 2)(), (ctypes.c_double * 2)()
    rc = b.lat._lib.hmc_actions(b.lat._ctx, ctypes.c_void_p(phi.data_ptr()), 1e-12, sg, pl, sf)
    assert rc == -3
    qs = b.links_from_native(b.lat.q)
    for c, (L, beta) in enumerate([(16, 2.0), (8, 2.0)]):
        assert abs(sg[c] - oracle.gauge_action(qs[c], beta)) < 1e-10 * abs(sg[c])
        assert abs(pl[c] - oracle.mean_plaquette(qs[c])) < 1e-12
        assert math.isnan(sf[c])
