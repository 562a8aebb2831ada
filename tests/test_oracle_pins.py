"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each checks the oracle against a closed
form (free-field Fourier transform, exact quenched plaquette), a library routine
(numpy dense solve/eig), an invariant (adjointness, gamma5-hermiticity, gauge
invariance, reversibility), finite differences of the actions the forces derive
from, published known-answer vectors (Philox4x32-10), or values typed from the
paper (stage sequences of Eqs. (3)-(5), (10), (11); inversion counts of Sec. 3 /
Table 1).  A plausible mistake in the oracle (a dropped term, a wrong sign or
index, a transposed operand, a wrong coefficient) fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def dense_dirac(q, m0, dagger=False):
    """Dense 2V x 2V matrix of the oracle's D (or D^dagger), column by column."""
    Lt, Lx, _ = q.shape
    n = 2 * Lx * Lt
    Dm = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        f = oracle.dirac_dagger if dagger else oracle.dirac
        Dm[:, j] = f(q, e.reshape(Lt, Lx, 2), m0).ravel()
    return Dm


SIG1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIG2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIG3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def momentum_space_dirac(kx, kt, m0):
    """D(k) = m0 + sum_mu (1 - cos k_mu) + i sum_mu sigma_mu sin k_mu (Fourier transform of D)."""
    return ((m0 + (1 - math.cos(kx)) + (1 - math.cos(kt))) * np.eye(2)
            + 1j * (SIG1 * math.sin(kx) + SIG2 * math.sin(kt)))


def multiset_distance(a, b):
    """Largest distance after greedily pairing each element of b with its nearest unused a."""
    a = list(a)
    worst = 0.0
    for v in b:
        j = int(np.argmin([abs(v - w) for w in a]))
        worst = max(worst, abs(v - a.pop(j)))
    return worst


# ------------------------------------------------------------------ random numbers
def test_philox_known_answers():
    kat = load_golden("philox4x32_10_kat.json")
    for v in kat["vectors"]:
        ctr = [int(c, 16) for c in v["ctr"]]
        key = [int(k, 16) for k in v["key"]]
        out = oracle.philox4x32_10(ctr, key)
        assert [int(o) for o in out] == [int(o, 16) for o in v["out"]]


def test_uniforms_are_the_top_53_bits():
    seed = 0x123456789ABCDEF
    for idx in (0, 1, 77, 2**31 + 5):
        w = oracle.philox4x32_10([idx, 1, 3, 2], [seed & 0xFFFFFFFF, seed >> 32])
        u = oracle.uniform_pair(seed, 2, 3, 1, idx)
        a = (int(w[0]) | (int(w[1]) << 32)) >> 11
        b = (int(w[2]) | (int(w[3]) << 32)) >> 11
        assert u[0] == a / 2.0**53 and u[1] == b / 2.0**53


def test_gaussian_moments():
    g = np.array([oracle.gaussian_pair(7, 0, 0, 1, i) for i in range(40000)]).ravel()
    n = g.size
    assert abs(g.mean()) < 5 / math.sqrt(n)
    assert abs(g.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(np.mean(g**4) - 3) < 5 * math.sqrt(96 / n)
    # Box-Muller pair against numpy's log/cos/sin on the same uniforms
    for i in range(50):
        u = oracle.uniform_pair(7, 0, 0, 1, i)
        r = math.sqrt(-2 * math.log(1 - u[0]))
        gp = oracle.gaussian_pair(7, 0, 0, 1, i)
        assert abs(gp[0] - r * math.cos(2 * math.pi * u[1])) < 1e-14 * max(1, r)
        assert abs(gp[1] - r * math.sin(2 * math.pi * u[1])) < 1e-14 * max(1, r)


def test_box_muller_log_against_high_precision():
    """The written ln of the Box-Muller step against mpmath at 40 digits: within 2 ulp over
    random 53-bit arguments, exact at powers of two times ln 2's split, 0 at 1."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    rng = np.random.default_rng(3)
    args = [float(k) * 2.0**-53 for k in rng.integers(1, 2**53, size=4000)]
    args += [2.0**-53, 0.5, 0.70710678118654752, 0.7071067811865476, 0.999999, 1.0 - 2.0**-53]
    for y in args:
        got = oracle.ln_unit(y)
        want = mpmath.log(mpmath.mpf(y))
        assert abs(mpmath.mpf(got) - want) <= 2 * 2.0**-52 * abs(want) + 1e-300, y
    assert oracle.ln_unit(1.0) == 0.0
    for e in (1, 2, 17, 53):
        assert abs(oracle.ln_unit(2.0**-e) + e * math.log(2)) <= 2.0**-52 * e * math.log(2)


def test_box_muller_sincos_against_high_precision():
    """The written sin/cos of 2 pi u against mpmath within 1 ulp of 1 over random arguments,
    and exact on the quadrant points (a wrong quadrant rotation or series sign fails)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    rng = np.random.default_rng(4)
    us = [float(k) * 2.0**-53 for k in rng.integers(0, 2**53, size=4000)]
    us += [0.125, 0.375, 0.625, 0.875, 1.0 - 2.0**-53, 2.0**-53]
    for u in us:
        sn, cs = oracle.sincos_turn(u)
        x = 2 * mpmath.pi * mpmath.mpf(u)
        assert abs(mpmath.mpf(sn) - mpmath.sin(x)) <= 2.0**-52, u
        assert abs(mpmath.mpf(cs) - mpmath.cos(x)) <= 2.0**-52, u
    assert oracle.sincos_turn(0.0) == (0.0, 1.0)
    assert oracle.sincos_turn(0.25) == (1.0, 0.0)
    assert oracle.sincos_turn(0.5) == (0.0, -1.0)
    assert oracle.sincos_turn(0.75) == (-1.0, 0.0)


def test_pseudofermion_and_momentum_normalisation():
    # <zeta^dagger zeta> = 2V for density exp(-zeta^dagger zeta); <p^2/2> = 1/2 per link
    Lx = Lt = 16
    z = np.array([oracle.random_zeta(Lx, Lt, 11, 0, t) for t in range(40)])
    v = np.sum(np.abs(z) ** 2, axis=(1, 2, 3))
    assert abs(v.mean() / (2 * Lx * Lt) - 1) < 5 * v.std() / (2 * Lx * Lt) / math.sqrt(40) + 1e-3
    p = np.array([oracle.random_momenta(Lx, Lt, 11, 0, t) for t in range(40)])
    assert abs(np.mean(p**2) - 1) < 0.02


def test_streams_are_distinct_and_reproducible():
    a = oracle.random_momenta(8, 8, 5, chain=0, traj=0)
    assert np.array_equal(a, oracle.random_momenta(8, 8, 5, chain=0, traj=0))
    assert not np.allclose(a, oracle.random_momenta(8, 8, 5, chain=1, traj=0))
    assert not np.allclose(a, oracle.random_momenta(8, 8, 5, chain=0, traj=1))
    q = oracle.random_links(8, 8, 5)
    assert q.min() >= -math.pi and q.max() < math.pi


# ------------------------------------------------------------------ Wilson-Dirac operator
@pytest.mark.parametrize("Lx,Lt", [(4, 4), (6, 4), (8, 8)])
def test_plane_waves_constant_background(Lx, Lt):
    """Plane waves diagonalise D in a constant U(1) background: D psi_k = D(k + a) psi_k.
    Fixes the hopping projectors, the sigma matrices, the link placement and the
    antiperiodic time boundary (k_t = (2j+1) pi / Lt)."""
    g = np.random.default_rng(3)
    m0 = 0.1
    for trial in range(6):
        ax, at = g.uniform(-1, 1, size=2)
        q = np.zeros((Lt, Lx, 2))
        q[..., 0] = ax
        q[..., 1] = at
        jx, jt = g.integers(0, Lx), g.integers(0, Lt)
        kx, kt = 2 * math.pi * jx / Lx, (2 * jt + 1) * math.pi / Lt
        u = g.normal(size=2) + 1j * g.normal(size=2)
        t, x = np.meshgrid(np.arange(Lt), np.arange(Lx), indexing="ij")
        phase = np.exp(1j * (kx * x + kt * t))
        psi = phase[..., None] * u[None, None, :]
        out = oracle.dirac(q, psi, m0)
        expect = phase[..., None] * (momentum_space_dirac(kx + ax, kt + at, m0) @ u)[None, None, :]
        assert np.max(np.abs(out - expect)) < 1e-12


def test_free_field_spectrum():
    Lx, Lt, m0 = 4, 6, 0.1
    q = np.zeros((Lt, Lx, 2))
    ev = np.linalg.eigvals(dense_dirac(q, m0))
    expect = []
    for jx in range(Lx):
        for jt in range(Lt):
            kx, kt = 2 * math.pi * jx / Lx, (2 * jt + 1) * math.pi / Lt
            M = m0 + (1 - math.cos(kx)) + (1 - math.cos(kt))
            w = math.sqrt(math.sin(kx) ** 2 + math.sin(kt) ** 2)
            expect += [M + 1j * w, M - 1j * w]
    assert multiset_distance(ev, np.array(expect)) < 1e-12


@pytest.mark.parametrize("Lx,Lt", [(2, 2), (6, 10), (34, 18)])
def test_dirac_at_listed_sites_is_the_full_operator(Lx, Lt):
    """The per-site evaluation of D (used for sampled sites of large lattices) gives the bits
    of the whole-lattice D at every site, in any order and with repeats, so it inherits the
    pins of D (plane waves, free-field spectrum, adjointness, gauge invariance)."""
    q = inputs.random_angles(Lx, Lt, 71)
    psi = inputs.random_spinor(Lx, Lt, 72)
    full = oracle.dirac(q, psi, 0.13).reshape(Lx * Lt, 2)
    sites = np.arange(Lx * Lt)
    assert np.array_equal(oracle.dirac_sites(q, psi, 0.13, sites), full)
    picks = np.random.default_rng(73).integers(0, Lx * Lt, size=3 * Lx * Lt)
    assert np.array_equal(oracle.dirac_sites(q, psi, 0.13, picks), full[picks])


def test_adjointness_and_gamma5_hermiticity():
    Lx, Lt, m0 = 8, 6, 0.1
    q = inputs.random_angles(Lx, Lt, 1)
    a = inputs.random_spinor(Lx, Lt, 2)
    b = inputs.random_spinor(Lx, Lt, 3)
    lhs = np.vdot(a, oracle.dirac(q, b, m0))
    rhs = np.vdot(oracle.dirac_dagger(q, a, m0), b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # D^dagger = sigma_3 D sigma_3 (gamma5 = sigma_3 anticommutes with sigma_1, sigma_2)
    s3b = b * np.array([1, -1])
    lhs = oracle.dirac_dagger(q, b, m0)
    rhs = oracle.dirac(q, s3b, m0) * np.array([1, -1])
    assert np.max(np.abs(lhs - rhs)) < 1e-12
    # dense: D^dagger is the conjugate transpose of D
    q4 = inputs.random_angles(4, 4, 9)
    assert np.max(np.abs(dense_dirac(q4, m0, dagger=True) - dense_dirac(q4, m0).conj().T)) < 1e-14


def gauge_transform(q, alpha):
    """q_mu(n) -> q_mu(n) + alpha(n) - alpha(n + mu)."""
    qt = q.copy()
    qt[..., 0] += alpha - np.roll(alpha, -1, axis=1)
    qt[..., 1] += alpha - np.roll(alpha, -1, axis=0)
    return qt


def test_gauge_invariance():
    Lx, Lt, beta, m0 = 8, 8, 2.0, 0.1
    q = inputs.random_angles(Lx, Lt, 4)
    phi = inputs.random_spinor(Lx, Lt, 5)
    alpha = inputs.random_gauge_transform(Lx, Lt, 6)
    qt = gauge_transform(q, alpha)
    phit = np.exp(1j * alpha)[..., None] * phi
    psi = inputs.random_spinor(Lx, Lt, 7)
    psit = np.exp(1j * alpha)[..., None] * psi
    # covariance of D
    assert np.max(np.abs(oracle.dirac(qt, psit, m0) - np.exp(1j * alpha)[..., None] * oracle.dirac(q, psi, m0))) < 1e-12
    assert abs(oracle.gauge_action(qt, beta) - oracle.gauge_action(q, beta)) < 1e-12 * oracle.gauge_action(q, beta)
    sf = oracle.fermion_action(q, phi, m0, tol=1e-14)
    assert abs(oracle.fermion_action(qt, phit, m0, tol=1e-14) - sf) < 1e-12 * sf
    assert np.max(np.abs(oracle.gauge_force(qt, beta) - oracle.gauge_force(q, beta))) < 1e-12
    f0 = oracle.fermion_force(q, phi, m0, tol=1e-14)[0]
    f1 = oracle.fermion_force(qt, phit, m0, tol=1e-14)[0]
    assert np.max(np.abs(f1 - f0)) < 1e-10 * np.max(np.abs(f0))


# ------------------------------------------------------------------ solver and fermion action
def test_cg_matches_dense_solve():
    Lx, Lt, m0 = 4, 4, 0.1
    q = inputs.random_angles(Lx, Lt, 8)
    phi = inputs.random_spinor(Lx, Lt, 9)
    Dm = dense_dirac(q, m0)
    A = Dm.conj().T @ Dm
    x_ref = np.linalg.solve(A, phi.ravel())
    x, it, res = oracle.cg(q, phi, m0, tol=1e-14)
    assert it > 0 and res < 1e-12
    assert np.max(np.abs(x.ravel() - x_ref)) < 1e-11 * np.max(np.abs(x_ref))
    # S_F of Eq. (14) against the dense quadratic form
    sf = oracle.fermion_action(q, phi, m0, tol=1e-14)
    assert abs(sf - np.vdot(phi.ravel(), x_ref).real) < 1e-11 * sf


def test_cg_reports_nonconvergence():
    q = inputs.random_angles(8, 8, 8)
    phi = inputs.random_spinor(8, 8, 9)
    x, it, res = oracle.cg(q, phi, 0.1, tol=1e-14, max_iter=3)
    assert it == -1 and res > 1e-6


def test_pseudofermion_heatbath_identity():
    """phi = D^dagger zeta gives S_F = phi^dagger (D^dagger D)^{-1} phi = zeta^dagger zeta."""
    Lx, Lt, m0 = 8, 8, 0.1
    q = inputs.random_angles(Lx, Lt, 10)
    zeta = oracle.random_zeta(Lx, Lt, 3)
    phi = oracle.dirac_dagger(q, zeta, m0)
    sf = oracle.fermion_action(q, phi, m0, tol=1e-14)
    assert abs(sf - np.vdot(zeta, zeta).real) < 1e-11 * sf


def test_chi_is_inverse_dagger_of_phi():
    """chi = D xi satisfies D^dagger chi = phi (Eq. (18))."""
    Lx, Lt, m0 = 8, 8, 0.1
    q = inputs.random_angles(Lx, Lt, 12)
    phi = inputs.random_spinor(Lx, Lt, 13)
    f, chi, xi, sf, it = oracle.fermion_force(q, phi, m0, tol=1e-14)
    assert np.max(np.abs(oracle.dirac_dagger(q, chi, m0) - phi)) < 1e-10 * np.max(np.abs(phi))


# ------------------------------------------------------------------ actions and forces
def test_cold_start():
    q = np.zeros((8, 8, 2))
    assert oracle.gauge_action(q, 2.0) == 0.0
    assert np.all(oracle.gauge_force(q, 2.0) == 0.0)
    assert oracle.mean_plaquette(q) == 1.0


def test_uniform_flux_closed_form():
    """q_t(x, t) = theta x with theta = 2 pi k / Lx: every plaquette angle is theta."""
    Lx, Lt, beta = 8, 6, 1.7
    theta = 2 * math.pi * 3 / Lx
    q = np.zeros((Lt, Lx, 2))
    q[..., 1] = theta * np.arange(Lx)[None, :]
    assert abs(oracle.gauge_action(q, beta) - beta * Lx * Lt * (1 - math.cos(theta))) < 1e-12
    assert np.max(np.abs(oracle.gauge_force(q, beta))) < 1e-12


def central_fd(fun, q, links, eps):
    out = []
    for (t, x, mu) in links:
        qp, qm = q.copy(), q.copy()
        qp[t, x, mu] += eps
        qm[t, x, mu] -= eps
        out.append((fun(qp) - fun(qm)) / (2 * eps))
    return np.array(out)


def sample_links(Lx, Lt, n, seed):
    g = np.random.default_rng(seed)
    return [(int(g.integers(Lt)), int(g.integers(Lx)), int(g.integers(2))) for _ in range(n)]


@pytest.mark.parametrize("eps", [1e-6, 1e-4])
def test_gauge_force_finite_differences(eps):
    Lx, Lt, beta = 8, 8, 2.0
    q = inputs.random_angles(Lx, Lt, 14)
    F = oracle.gauge_force(q, beta)
    links = [(t, x, mu) for t in range(Lt) for x in range(Lx) for mu in range(2)]
    fd = central_fd(lambda qq: oracle.gauge_action(qq, beta), q, links, eps)
    an = np.array([F[l] for l in links])
    assert np.max(np.abs(fd - an)) < 1e-6 * np.max(np.abs(F))


@pytest.mark.parametrize("m0", [0.1, 0.05])
def test_fermion_force_finite_differences(m0):
    Lx, Lt = 8, 8
    q = inputs.random_angles(Lx, Lt, 15)
    phi = inputs.random_spinor(Lx, Lt, 16)
    f = oracle.fermion_force(q, phi, m0, tol=1e-14)[0]
    links = sample_links(Lx, Lt, 64, 17)
    fd = central_fd(lambda qq: oracle.fermion_action(qq, phi, m0, tol=1e-14), q, links, 1e-6)
    an = np.array([f[l] for l in links])
    assert np.max(np.abs(fd - an)) < 1e-6 * np.max(np.abs(f))
    fd4 = central_fd(lambda qq: oracle.fermion_action(qq, phi, m0, tol=1e-14), q, links[:8], 1e-4)
    assert np.max(np.abs(fd4 - an[:8])) < 1e-6 * np.max(np.abs(f))


def test_fermion_force_against_log_det():
    """With phi = 0 the action is gone, but d/dq log det(D^dagger D) = 2 Re tr(D^{-1} dD/dq) ties
    the force kernel to the determinant: for a unit-normalised heat-bath average,
    <f> over phi distributed as exp(-S_F) equals -d/dq log det(D^dagger D).  Checked exactly
    with the dense trace: sum over a basis of phi = D^dagger e_j of f equals -d log det."""
    Lx, Lt, m0 = 4, 4, 0.2
    q = inputs.random_angles(Lx, Lt, 18)
    n = 2 * Lx * Lt
    # E[f] with zeta ~ exp(-zeta^dagger zeta) and phi = D^dagger zeta equals the sum over
    # unit vectors zeta = e_j of f(phi_j) (the covariance of zeta is the identity).
    acc = np.zeros_like(q)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        phi = oracle.dirac_dagger(q, e.reshape(Lt, Lx, 2), m0)
        acc += oracle.fermion_force(q, phi, m0, tol=1e-14)[0]

    def logdet(qq):
        return np.linalg.slogdet(dense_dirac(qq, m0))[1] * 2.0

    links = sample_links(Lx, Lt, 6, 19)
    fd = central_fd(logdet, q, links, 1e-5)
    # dS_eff/dq with S_eff = -log det(D^dagger D): the force of the integrated-out fermions
    for (l, d) in zip(links, fd):
        assert abs(acc[l] - (-d)) < 1e-6 * max(1.0, abs(d))


# ------------------------------------------------------------------ integrators
def fractions_of(seq):
    return [(k, float(Fraction(c))) for k, c in seq]


@pytest.mark.parametrize("scheme", list(oracle.SCHEMES))
def test_stage_sequences(scheme):
    gold = load_golden("stage_sequences.json")
    q = inputs.smooth_angles(4, 4, 20)
    p = inputs.random_momenta(4, 4, 21)
    phi = inputs.random_spinor(4, 4, 22)
    _, _, info = oracle.md_integrate(q, p, phi, 2.0, 0.1, scheme, gold["h"], 1, gold["M"],
                                     trace_cap=200)
    got = info["trace"]
    want = fractions_of(gold["schemes"][scheme])
    assert [k for k, _ in got] == [k for k, _ in want]
    assert np.allclose([e for _, e in got], [e for _, e in want], rtol=0, atol=1e-15)


def test_eleven_stage_coefficients_are_fourth_order():
    """The oracle's 11-stage sequence (Eq. (6)) composed as matrix exponentials of two random
    non-commuting matrices A, B against exp(h (A + B)): the local error falls as h^5 (a
    fourth-order scheme), as the published coefficients require; one wrong digit in sigma,
    eta, lambda or theta leaves h^3."""
    from scipy.linalg import expm
    q = inputs.smooth_angles(4, 4, 20)
    p = inputs.random_momenta(4, 4, 21)
    phi = inputs.random_spinor(4, 4, 22)
    _, _, info = oracle.md_integrate(q, p, phi, 2.0, 0.1, "omelyan_11stage", 1.0, 1, 1,
                                     trace_cap=200)
    seq = info["trace"]
    assert [k for k, _ in seq] == ["B", "A"] * 5 + ["B"]
    g = np.random.default_rng(5)
    A, B = g.normal(size=(6, 6)), g.normal(size=(6, 6))

    def local_error(h):
        U = np.eye(6)
        for kind, c in seq:
            U = expm(c * h * (A if kind == "A" else B)) @ U
        return np.linalg.norm(U - expm(h * (A + B)))

    hs = [0.08, 0.04, 0.02]
    errs = [local_error(h) for h in hs]
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(2)]
    assert all(abs(s - 5.0) < 0.3 for s in slopes), slopes


@pytest.mark.parametrize("scheme", list(oracle.SCHEMES))
def test_inversions_per_step(scheme):
    gold = load_golden("inversions_per_step.json")
    q = inputs.smooth_angles(4, 4, 23)
    p = inputs.random_momenta(4, 4, 24)
    phi = inputs.random_spinor(4, 4, 25)
    n_outer = 3
    _, _, info = oracle.md_integrate(q, p, phi, 2.0, 0.1, scheme, 1.0, n_outer, 2)
    assert 2 * info["n_solves"] == gold[scheme] * n_outer


@pytest.mark.parametrize("scheme", list(oracle.SCHEMES))
def test_reversibility(scheme):
    Lx, Lt, beta, m0 = 4, 4, 2.0, 0.1
    q = inputs.random_angles(Lx, Lt, 26)
    p = inputs.random_momenta(Lx, Lt, 27)
    phi = inputs.random_spinor(Lx, Lt, 28)
    q1, p1, _ = oracle.md_integrate(q, p, phi, beta, m0, scheme, 1.0, 5, 3, tol=1e-14)
    q2, p2, _ = oracle.md_integrate(q1, -p1, phi, beta, m0, scheme, 1.0, 5, 3, tol=1e-14)
    assert np.max(np.abs(q2 - q)) < 1e-10
    assert np.max(np.abs(-p2 - p)) < 1e-10


def energy_error(scheme, n, M, seed=30, Lx=4, Lt=4, beta=1.0, m0=0.3, tau=1.0):
    q = inputs.smooth_angles(Lx, Lt, seed, 0.5)
    p = inputs.random_momenta(Lx, Lt, seed + 1)
    phi = inputs.random_spinor(Lx, Lt, seed + 2)
    H0 = oracle.hamiltonian(q, p, phi, beta, m0)
    q1, p1, _ = oracle.md_integrate(q, p, phi, beta, m0, scheme, tau, n, M, tol=1e-14)
    return oracle.hamiltonian(q1, p1, phi, beta, m0) - H0


def phase_error(scheme, n, M, ref, seed=30, Lx=4, Lt=4, beta=1.0, m0=0.3, tau=1.0):
    q = inputs.smooth_angles(Lx, Lt, seed, 0.5)
    p = inputs.random_momenta(Lx, Lt, seed + 1)
    phi = inputs.random_spinor(Lx, Lt, seed + 2)
    q1, p1, _ = oracle.md_integrate(q, p, phi, beta, m0, scheme, tau, n, M, tol=1e-14)
    return math.sqrt(np.sum((q1 - ref[0]) ** 2) + np.sum((p1 - ref[1]) ** 2))


def slope(ns, errs):
    return np.polyfit(np.log(ns), np.log(np.abs(errs)), 1)[0]


@pytest.fixture(scope="module")
def fine_reference():
    q = inputs.smooth_angles(4, 4, 30, 0.5)
    p = inputs.random_momenta(4, 4, 31)
    phi = inputs.random_spinor(4, 4, 32)
    q1, p1, _ = oracle.md_integrate(q, p, phi, 1.0, 0.3, "force_gradient", 1.0, 256, 1, tol=1e-14)
    return q1, p1


@pytest.mark.parametrize("scheme,order,nested", [
    ("leapfrog", 2, False), ("omelyan", 2, False), ("force_gradient", 4, False),
    ("nested_fg", 4, True), ("adapted_nested_fg", 4, True), ("nested_leapfrog", 2, True),
    ("nested_omelyan", 2, True), ("omelyan_11stage", 4, False)])
def test_order_of_convergence(scheme, order, nested, fine_reference):
    """Global phase-space error and energy error scale as h^order; the nested
    force-gradient schemes reach order four effectively with M proportional to 1/h, the
    nested leap-frog and 5-stage schemes stay second order (Sec. 2.2)."""
    ns = [4, 8, 16] if order == 4 else [8, 16, 32]
    Ms = [2 * n if nested else 1 for n in ns]
    errs = [phase_error(scheme, n, M, fine_reference) for n, M in zip(ns, Ms)]
    assert abs(slope(ns, errs) + order) < 0.25, errs
    dH = [energy_error(scheme, n, M) for n, M in zip(ns, Ms)]
    assert abs(slope(ns, dH) + order) < 0.35, dH


def test_nested_fixed_M_is_second_order():
    """With M fixed the inner leap-frog error (h/M)^2 dominates as h -> 0 (Sec. 2.2)."""
    ns = [16, 32, 64]
    dH = [energy_error("adapted_nested_fg", n, 1, m0=0.3, beta=3.0) for n in ns]
    assert abs(slope(ns, dH) + 2) < 0.35, dH


def test_force_gradient_sign_matters():
    """The force-gradient kick must use the shift q - (h^2/24) F: the energy error of
    the force-gradient scheme is far below the 5-stage scheme's at equal h."""
    e5 = abs(energy_error("omelyan", 8, 1))
    efg = abs(energy_error("force_gradient", 8, 1))
    assert efg < 0.1 * e5


# ------------------------------------------------------------------ HMC
def test_hmc_initial_hamiltonian_uses_exact_pseudofermion_action():
    Lx, Lt, beta, m0, seed = 4, 4, 2.0, 0.1, 99
    q = oracle.random_links(Lx, Lt, seed)
    _, info = oracle.hmc_trajectory(q, beta, m0, seed, 0, 0, "omelyan", 1.0, 10, tol=1e-14)
    p = oracle.random_momenta(Lx, Lt, seed, 0, 0)
    zeta = oracle.random_zeta(Lx, Lt, seed, 0, 0)
    phi = oracle.dirac_dagger(q, zeta, m0)
    H0 = oracle.hamiltonian(q, p, phi, beta, m0, tol=1e-14)
    assert abs(info["H0"] - H0) < 1e-11 * abs(H0)
    assert abs(info["H1"] - info["H0"] - info["dH"]) < 1e-10 * abs(H0)


def test_hmc_is_deterministic():
    q = oracle.random_links(8, 8, 5)
    qa, ia = oracle.hmc_trajectory(q, 2.0, 0.1, 5, 0, 3, "adapted_nested_fg", 1.0, 4, 2)
    qb, ib = oracle.hmc_trajectory(q, 2.0, 0.1, 5, 0, 3, "adapted_nested_fg", 1.0, 4, 2)
    assert np.array_equal(qa, qb) and ia["dH"] == ib["dH"]


def test_hmc_rejection_restores_links():
    q = oracle.random_links(4, 4, 6)
    # a huge step makes Delta H large and the update is rejected
    q1, info = oracle.hmc_trajectory(q, 2.0, 0.1, 6, 0, 0, "leapfrog", 4.0, 1)
    if not info["accepted"]:
        assert np.array_equal(q1, q)
    assert info["dH"] > 1.0


def exact_mean_plaquette(beta, V):
    """Quenched U(1) in 2-D on a torus of V plaquettes: Z = sum_k I_k(beta)^V (character
    expansion), so <Re P> = sum_k I_k^(V-1) I_k' / sum_k I_k^V with I_k' = (I_{k-1}+I_{k+1})/2."""
    from scipy.special import ive
    ks = np.arange(-30, 31)
    # scaled Bessel functions: the common factor e^{beta V} cancels in the ratio
    Ik = ive(ks, beta)
    dI = 0.5 * (ive(ks - 1, beta) + ive(ks + 1, beta))
    w = Ik ** (V - 1)
    return float(np.sum(w * dI) / np.sum(w * Ik))


@pytest.mark.slow
def test_quenched_plaquette_is_exact():
    Lx = Lt = 4
    beta = 2.0
    q = oracle.random_links(Lx, Lt, 1234)
    plaq = []
    for traj in range(3200):
        q, info = oracle.hmc_trajectory(q, beta, 0.0, 1234, 0, traj, "omelyan", 1.0, 5,
                                        quenched=True)
        if traj >= 200:
            plaq.append(info["plaquette"])
    plaq = np.array(plaq)
    blocks = plaq.reshape(30, -1).mean(axis=1)
    err = blocks.std(ddof=1) / math.sqrt(len(blocks))
    exact = exact_mean_plaquette(beta, Lx * Lt)
    assert abs(plaq.mean() - exact) < 4 * err + 1e-4, (plaq.mean(), exact, err)


@pytest.mark.slow
def test_creutz_equality():
    """<exp(-Delta H)> = 1 over an equilibrium chain."""
    Lx = Lt = 4
    q = oracle.random_links(Lx, Lt, 77)
    vals = []
    for traj in range(700):
        q, info = oracle.hmc_trajectory(q, 2.0, 0.2, 77, 0, traj, "omelyan", 1.0, 3)
        if traj >= 100:
            vals.append(math.exp(-info["dH"]))
    vals = np.array(vals)
    blocks = vals.reshape(20, -1).mean(axis=1)
    err = blocks.std(ddof=1) / math.sqrt(len(blocks))
    assert abs(vals.mean() - 1) < 4 * err + 1e-3, (vals.mean(), err)
