"""Pins of the oracle's force-gradient term C (Sec. 3, Eqs. (19)-(23)).

The closed forms the paper prints for C_GG and C_FG, and the Z_1/Z_2 construction of
C_FF and C_GF, are checked against what they must equal by definition: C is the gradient
of |F|^2 (Eq. (19)), and each part is twice a Hessian of S_G or S_F applied to a force,
so central finite differences of the (already pinned) forces and of |F|^2 fix every
term.  Symmetry of the Hessian and gauge invariance catch a transposed operand or a
wrong link; the Taylor-shift residual and the inversion counts tie C to Sec. 2.2 and to
the closing paragraph of Sec. 3.
"""
import json
import os

import numpy as np
import pytest

import oracle
from tests import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-14


def grad_fd(fun, q, eps=1e-5):
    """Central-difference gradient of a scalar function of the links."""
    g = np.zeros_like(q)
    for idx in np.ndindex(q.shape):
        e = np.zeros_like(q)
        e[idx] = eps
        g[idx] = (fun(q + e) - fun(q - e)) / (2 * eps)
    return g


def dir_fd(force, q, v, eps=1e-5):
    """Central difference of a force along v: the Hessian of its action applied to v."""
    return (force(q + eps * v) - force(q - eps * v)) / (2 * eps)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def setup(Lx, Lt, seed):
    q = inputs.random_angles(Lx, Lt, seed)
    phi = inputs.random_spinor(Lx, Lt, seed + 1)
    return q, phi


LATS = [(4, 4, 1.3, 0.2), (6, 4, 2.0, 0.1), (2, 2, 1.0, 0.3)]


@pytest.mark.parametrize("Lx,Lt,beta,m0", LATS)
def test_c_gg_is_gradient_of_gauge_force_norm(Lx, Lt, beta, m0):
    q, _ = setup(Lx, Lt, 3)
    C = oracle.fg_term_gg(q, beta)
    ref = grad_fd(lambda qq: np.sum(oracle.gauge_force(qq, beta) ** 2), q)
    assert rel(C, ref) < 1e-8


@pytest.mark.parametrize("Lx,Lt,beta,m0", LATS)
def test_gauge_parts_are_gauge_hessian_products(Lx, Lt, beta, m0):
    """C_GG = 2 Hess(S_G) beta g and C_FG = 2 Hess(S_G) f; the C_FG closed form is linear
    in its force argument, so any v gives 2 Hess(S_G) v."""
    q, phi = setup(Lx, Lt, 5)
    FG = lambda qq: oracle.gauge_force(qq, beta)
    g = FG(q)
    assert rel(oracle.fg_term_gg(q, beta), 2 * dir_fd(FG, q, g)) < 1e-8
    f = oracle.fermion_force(q, phi, m0, tol=TOL)[0]
    assert rel(oracle.fg_term_fg(q, f, beta), 2 * dir_fd(FG, q, f)) < 1e-8
    v = inputs.random_momenta(Lx, Lt, 7)
    assert rel(oracle.fg_term_fg(q, v, beta), 2 * dir_fd(FG, q, v)) < 1e-8


@pytest.mark.parametrize("Lx,Lt,beta,m0", LATS)
def test_fermion_parts_are_fermion_hessian_products(Lx, Lt, beta, m0):
    """Eqs. (22)-(23): v = f gives C_FF = 2 Hess(S_F) f, v = beta g gives C_GF."""
    q, phi = setup(Lx, Lt, 9)
    FF = lambda qq: oracle.fermion_force(qq, phi, m0, tol=TOL)[0]
    f, chi, xi, _, _ = oracle.fermion_force(q, phi, m0, tol=TOL)
    for v in (f, oracle.gauge_force(q, beta), inputs.random_momenta(Lx, Lt, 11)):
        C, it = oracle.fg_term_fermion(q, chi, xi, v, m0, tol=TOL)
        assert it > 0
        assert rel(C, 2 * dir_fd(FF, q, v)) < 1e-7


def test_fermion_hessian_is_symmetric():
    Lx, Lt, m0 = 6, 4, 0.1
    q, phi = setup(Lx, Lt, 13)
    _, chi, xi, _, _ = oracle.fermion_force(q, phi, m0, tol=TOL)
    u = inputs.random_momenta(Lx, Lt, 14)
    v = inputs.random_momenta(Lx, Lt, 15)
    Cu, _ = oracle.fg_term_fermion(q, chi, xi, u, m0, tol=TOL)
    Cv, _ = oracle.fg_term_fermion(q, chi, xi, v, m0, tol=TOL)
    a, b = float(np.sum(v * Cu)), float(np.sum(u * Cv))
    assert abs(a - b) < 1e-11 * max(abs(a), 1.0)


@pytest.mark.parametrize("which", ["gauge", "fermion", "total"])
def test_force_gradient_term_is_gradient_of_force_norm(which):
    """Eq. (19): C = grad |F|^2 for the chosen force set (Eq. (20) parts summed)."""
    Lx, Lt, beta, m0 = 4, 4, 1.5, 0.2
    q, phi = setup(Lx, Lt, 17)

    def F(qq):
        if which == "gauge":
            return oracle.gauge_force(qq, beta)
        if which == "fermion":
            return oracle.fermion_force(qq, phi, m0, tol=TOL)[0]
        return oracle.total_force(qq, phi, beta, m0, tol=TOL)

    C, info = oracle.force_gradient_term(q, phi, beta, m0, which, tol=TOL)
    assert info["rc"] == 0
    assert rel(C, grad_fd(lambda qq: np.sum(F(qq) ** 2), q)) < 1e-7
    # inversions as counted in Sec. 3: two for chi/xi, two (Z_1, Z_2) per fermion part
    assert info["n_dinv"] == {"gauge": 0, "fermion": 4, "total": 6}[which]


def test_force_gradient_term_is_gauge_invariant():
    Lx, Lt, beta, m0 = 6, 4, 1.5, 0.1
    q, phi = setup(Lx, Lt, 19)
    alpha = inputs.random_angles(Lx, Lt, 20)[:, :, 0]
    qg = q.copy()
    qg[:, :, 0] += alpha - np.roll(alpha, -1, axis=1)
    qg[:, :, 1] += alpha - np.roll(alpha, -1, axis=0)
    phig = phi * np.exp(1j * alpha)[:, :, None]
    C, _ = oracle.force_gradient_term(q, phi, beta, m0, "total", tol=TOL)
    Cg, _ = oracle.force_gradient_term(qg, phig, beta, m0, "total", tol=TOL)
    assert rel(Cg, C) < 1e-10


def test_taylor_shift_residual_is_fourth_order():
    """Sec. 2.2: F(q - (h^2/24) F) = F - (h^2/48) C + O(h^4)."""
    Lx, Lt, beta, m0 = 4, 4, 1.5, 0.2
    q, phi = setup(Lx, Lt, 21)
    F0 = oracle.total_force(q, phi, beta, m0, tol=TOL)
    C, _ = oracle.force_gradient_term(q, phi, beta, m0, "total", tol=TOL)
    hs = [0.8, 0.4, 0.2]
    res = []
    for h in hs:
        Fs = oracle.fg_shifted_force(q, phi, beta, m0, h, "total", tol=TOL)
        res.append(np.max(np.abs(Fs - (F0 - (h * h / 48.0) * C))))
    s = np.polyfit(np.log(hs), np.log(res), 1)[0]
    assert abs(s - 4) < 0.2, res


@pytest.mark.parametrize("scheme", ["force_gradient", "nested_fg", "adapted_nested_fg"])
def test_exact_inversions_per_step(scheme):
    """Sec. 3, closing paragraph: 10 inversions per step for Eq. (5) with the exact C,
    8 for Eqs. (10) and (11)."""
    with open(os.path.join(GOLDEN, "inversions_per_step.json")) as fh:
        gold = json.load(fh)["exact_c"]
    q = inputs.smooth_angles(4, 4, 23)
    p = inputs.random_momenta(4, 4, 24)
    phi = inputs.random_spinor(4, 4, 25)
    n_outer = 3
    _, _, info = oracle.md_integrate(q, p, phi, 2.0, 0.1, scheme, 1.0, n_outer, 2, fg_exact=True)
    assert info["n_dinv"] == gold[scheme] * n_outer


@pytest.mark.parametrize("scheme", ["force_gradient", "nested_fg", "adapted_nested_fg"])
def test_exact_reversibility(scheme):
    Lx, Lt, beta, m0 = 4, 4, 2.0, 0.1
    q = inputs.random_angles(Lx, Lt, 26)
    p = inputs.random_momenta(Lx, Lt, 27)
    phi = inputs.random_spinor(Lx, Lt, 28)
    q1, p1, _ = oracle.md_integrate(q, p, phi, beta, m0, scheme, 1.0, 4, 2, tol=TOL, fg_exact=True)
    q2, p2, _ = oracle.md_integrate(q1, -p1, phi, beta, m0, scheme, 1.0, 4, 2, tol=TOL,
                                    fg_exact=True)
    assert np.max(np.abs(q2 - q)) < 1e-10
    assert np.max(np.abs(-p2 - p)) < 1e-10


def energy_error(scheme, n, M, exact, Lx=4, Lt=4, beta=1.0, m0=0.3, tau=1.0, seed=30):
    q = inputs.smooth_angles(Lx, Lt, seed, 0.5)
    p = inputs.random_momenta(Lx, Lt, seed + 1)
    phi = inputs.random_spinor(Lx, Lt, seed + 2)
    H0 = oracle.hamiltonian(q, p, phi, beta, m0)
    q1, p1, _ = oracle.md_integrate(q, p, phi, beta, m0, scheme, tau, n, M, tol=TOL,
                                    fg_exact=exact)
    return oracle.hamiltonian(q1, p1, phi, beta, m0) - H0


@pytest.mark.parametrize("scheme,nested", [("force_gradient", False), ("nested_fg", True),
                                           ("adapted_nested_fg", True)])
def test_exact_schemes_are_fourth_order(scheme, nested):
    ns = [4, 8, 16]
    Ms = [2 * n if nested else 1 for n in ns]
    dH = [energy_error(scheme, n, M, True) for n, M in zip(ns, Ms)]
    s = np.polyfit(np.log(ns), np.log(np.abs(dH)), 1)[0]
    assert abs(s + 4) < 0.35, dH


def test_exact_and_shifted_kicks_differ_at_fifth_order():
    """One force-gradient step with the exact C and with the shifted force differ by
    O(h^5) in p (the shift reproduces C up to O(h^4) in the force, times eps = 2h/3)."""
    Lx, Lt, beta, m0 = 4, 4, 1.5, 0.2
    q = inputs.smooth_angles(Lx, Lt, 40, 0.5)
    p = inputs.random_momenta(Lx, Lt, 41)
    phi = inputs.random_spinor(Lx, Lt, 42)
    hs = [0.4, 0.2, 0.1]
    d = []
    for h in hs:
        _, pe, _ = oracle.md_integrate(q, p, phi, beta, m0, "force_gradient", h, 1, 1, tol=TOL,
                                       fg_exact=True)
        _, ps, _ = oracle.md_integrate(q, p, phi, beta, m0, "force_gradient", h, 1, 1, tol=TOL)
        d.append(np.max(np.abs(pe - ps)))
    s = np.polyfit(np.log(hs), np.log(d), 1)[0]
    assert abs(s - 5) < 0.3, d


def test_hmc_trajectory_reports_exact_inversions():
    q = oracle.random_links(4, 4, 8)
    _, info = oracle.hmc_trajectory(q, 2.0, 0.1, 8, 0, 0, "force_gradient", 1.0, 3, tol=1e-12,
                                    fg_exact=True)
    assert info["rc"] == 0 and info["n_dinv"] == 30
    _, info = oracle.hmc_trajectory(q, 2.0, 0.1, 8, 0, 0, "force_gradient", 1.0, 3, tol=1e-12)
    assert info["n_dinv"] == 24
