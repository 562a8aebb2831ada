"""GPU tests of the method's degenerate cases, against the oracle:

- a zero-length trajectory (tau = 0): the links come back unchanged, and Delta H is only the
  difference between the pseudofermion action of the heat bath, zeta^dagger zeta (Sec. 2.1),
  and its value from the solve at the same links;
- strong coupling (beta = 0), where the gauge action and the gauge force vanish and only the
  fermion force moves the links;
- reversibility of the molecular dynamics on the GPU (Sec. 2.1): integrating, reversing the
  momenta and integrating again returns to the start, for every scheme and both forms of the
  force-gradient kick;
- 2 x 2 chains, whose forward and backward neighbours coincide, in batches with larger ones.
"""
import numpy as np
import pytest

import oracle
from tests import inputs
from tests.gpu_helpers import Batch, run_oracle_chain

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("persistent", [0, 2048])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_zero_length_trajectory_keeps_the_links(prec, persistent):
    shapes = [(8, 8, 2.0, 0.1), (2, 2, 1.0, 0.15), (6, 4, 3.0, 0.05), (32, 16, 1.5, 0.2)]
    seed = 404
    b = Batch(shapes, seed=seed, persistent=persistent)
    b.lat.hot_start()
    b.lat.set_solver(tol=1e-12)
    q0 = b.links_from_native(b.lat.q)
    r = b.lat.trajectory("adapted_nested_fg", 0.0, 4, 2, prec=prec)
    q1 = b.links_from_native(b.lat.q)
    for c, (Lx, Lt, beta, m0) in enumerate(shapes):
        assert r.status[c] == 0
        assert np.array_equal(q1[c], q0[c]), c
        qo, io = oracle.hmc_trajectory(q0[c], beta, m0, seed, c, 0, "adapted_nested_fg", 0.0, 4, 2,
                                       tol=1e-12)
        assert io["rc"] == 0 and np.array_equal(qo, q0[c])
        # both sides: only the solver's residual separates the two pseudofermion actions
        assert abs(io["dH"]) < 1e-8 and abs(r.dH[c]) < 1e-8, (c, io["dH"], r.dH[c])
        assert r.accepted[c] == io["accepted"]


@pytest.mark.parametrize("scheme,n_outer,n_inner", [("omelyan", 8, 1), ("force_gradient", 4, 1),
                                                    ("adapted_nested_fg", 4, 2)])
def test_strong_coupling_matches_oracle(scheme, n_outer, n_inner):
    shapes = [(8, 8, 0.0, 0.1), (4, 6, 0.0, 0.3), (2, 2, 0.0, 0.2)]
    seed = 505
    b = Batch(shapes, seed=seed, persistent=0)
    b.lat.hot_start()
    b.lat.set_solver(tol=1e-13)
    for f in b.links_from_native(b.lat.gauge_force()):
        assert np.all(f == 0.0)
    sg, _, _ = b.lat.actions()
    assert all(s == 0.0 for s in sg)
    refs = [run_oracle_chain(s[0], s[1], s[2], s[3], seed, c, 2, scheme, 1.0, n_outer, n_inner, 1e-13)
            for c, s in enumerate(shapes)]
    for t in range(2):
        r = b.lat.trajectory(scheme, 1.0, n_outer, n_inner)
        qs = b.links_from_native(b.lat.q)
        for c in range(len(shapes)):
            qr, ir = refs[c][t]
            assert r.accepted[c] == ir["accepted"], (t, c)
            assert abs(r.dH[c] - ir["dH"]) < 1e-10 * max(1.0, abs(ir["dH"])), (t, c)
            assert np.max(np.abs(qs[c] - qr)) < 1e-9


SCHEMES = ["leapfrog", "omelyan", "force_gradient", "omelyan_11stage", "nested_leapfrog",
           "nested_omelyan", "nested_fg", "adapted_nested_fg"]
FG_SCHEMES = {"force_gradient", "nested_fg", "adapted_nested_fg"}


@pytest.mark.parametrize("scheme,fg", [(s, "shift") for s in SCHEMES] +
                         [(s, "exact") for s in SCHEMES if s in FG_SCHEMES])
def test_md_is_reversible(scheme, fg):
    shapes = [(8, 8, 2.0, 0.1), (6, 4, 1.5, 0.2), (2, 2, 1.0, 0.3)]
    b = Batch(shapes, persistent=0)
    b.lat.set_fg_mode(fg)
    q0 = [inputs.random_angles(s[0], s[1], 71 + c) for c, s in enumerate(shapes)]
    p0 = [inputs.random_momenta(s[0], s[1], 81 + c) for c, s in enumerate(shapes)]
    phi = [inputs.random_spinor(s[0], s[1], 91 + c) for c, s in enumerate(shapes)]
    b.set_q(q0)
    b.links_to_native(p0, out=b.lat.p)
    b.spinor_to_native(phi, out=b.lat.phi)
    b.lat.set_solver(tol=1e-14)
    b.lat.integrate(scheme, 1.0, 4, 3)
    moved = b.links_from_native(b.lat.q)
    assert max(np.max(np.abs(m - q)) for m, q in zip(moved, q0)) > 1e-2
    b.lat.p.neg_()
    b.lat.integrate(scheme, 1.0, 4, 3)
    q2, p2 = b.links_from_native(b.lat.q), b.links_from_native(b.lat.p)
    for c in range(len(shapes)):
        assert np.max(np.abs(q2[c] - q0[c])) < 1e-10, c
        assert np.max(np.abs(p2[c] + p0[c])) < 1e-10, c
