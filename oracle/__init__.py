"""Plain FP64 CPU oracle for the Schwinger-model HMC hot path (TEST INFRASTRUCTURE).

This package is the independent reference that the GPU library is checked against.
Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product path never does.  It shares no code with
the GPU path: the arithmetic lives in ``schwinger_oracle.c`` (plain C, double
precision, lexicographic layout), and this module only marshals numpy arrays.

Layout (lexicographic, as in the C file): site n = x + Lx*t.
  links / momenta / forces : float64 arrays of shape (Lt, Lx, 2)  [t, x, mu], mu=0 x, mu=1 t
  spinors                  : complex128 arrays of shape (Lt, Lx, 2) [t, x, s]

Paper: Shcherbakov et al., "Adapted nested force-gradient integrators: the
Schwinger model case", arXiv:1512.03812.  Each wrapper names the passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "schwinger_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

(LEAPFROG, OMELYAN_5STAGE, FORCE_GRADIENT, NESTED_FG, ADAPTED_NESTED_FG, NESTED_LEAPFROG,
 NESTED_5STAGE, OMELYAN_11STAGE) = range(8)
SCHEMES = {
    "leapfrog": LEAPFROG,
    "omelyan": OMELYAN_5STAGE,
    "force_gradient": FORCE_GRADIENT,
    "nested_fg": NESTED_FG,
    "adapted_nested_fg": ADAPTED_NESTED_FG,
    "nested_leapfrog": NESTED_LEAPFROG,
    "nested_omelyan": NESTED_5STAGE,
    "omelyan_11stage": OMELYAN_11STAGE,
}
FLAG_QUENCHED = 1
FLAG_FG_EXACT = 2
FORCE_SETS = {"gauge": 0, "fermion": 1, "total": 2}
STAGE_NAMES = {0: "A", 1: "B", 2: "BG", 3: "BF", 4: "BT", 5: "BTG", 6: "BTF"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        D, I, U32, U64 = ctypes.c_double, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64
        P = ctypes.c_void_p
        sig = {
            "orc_philox4x32_10": (None, [P, P, P]),
            "orc_uniform_pair": (None, [U64, U32, U32, U32, U32, P]),
            "orc_gaussian_pair": (None, [U64, U32, U32, U32, U32, P]),
            "orc_ln_unit": (D, [D]),
            "orc_sincos_turn": (None, [D, P, P]),
            "orc_random_links": (None, [I, I, U64, U32, P]),
            "orc_random_momenta": (None, [I, I, U64, U32, U32, P]),
            "orc_random_zeta": (None, [I, I, U64, U32, U32, P]),
            "orc_metropolis_uniform": (D, [U64, U32, U32]),
            "orc_gauge_action": (D, [I, I, D, P]),
            "orc_mean_plaquette": (D, [I, I, P]),
            "orc_gauge_force": (None, [I, I, D, P, P]),
            "orc_dirac": (None, [I, I, D, P, P, P]),
            "orc_dirac_dagger": (None, [I, I, D, P, P, P]),
            "orc_dirac_sites": (None, [I, I, D, P, P, I, P, P]),
            "orc_cg": (I, [I, I, D, P, P, P, D, I, P]),
            "orc_fermion_force_chixi": (None, [I, I, P, P, P, P]),
            "orc_fermion_force": (I, [I, I, D, P, P, D, I, P, P, P, P]),
            "orc_fermion_action": (D, [I, I, D, P, P, D, I]),
            "orc_fg_term_gg": (None, [I, I, D, P, P]),
            "orc_fg_term_fg": (None, [I, I, D, P, P, P]),
            "orc_fg_term_fermion": (I, [I, I, D, P, P, P, P, D, I, P]),
            "orc_force_gradient_term": (I, [I, I, D, D, P, P, I, D, I, P, P]),
            "orc_md_integrate": (I, [I, I, D, D, I, D, I, I, D, I, I, P, P, P, P, P, P, I]),
            "orc_hmc_trajectory": (I, [I, I, D, D, U64, U32, U32, I, D, I, I, D, I, I, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _links(q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.ndim == 3 and q.shape[2] == 2
    return q


def _spinor(s) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.complex128)
    assert s.ndim == 3 and s.shape[2] == 2
    return s


# ---------------------------------------------------------------- random numbers
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block (Salmon et al., SC'11): 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniform_pair(seed, chain, traj, stream, index) -> np.ndarray:
    out = np.zeros(2)
    lib().orc_uniform_pair(seed, chain, traj, stream, index, _p(out))
    return out


def ln_unit(y: float) -> float:
    """ln y for 0 < y <= 1 by the written method of the Box-Muller step (Cody-Waite reduction,
    atanh series)."""
    return lib().orc_ln_unit(float(y))


def sincos_turn(u: float):
    """(sin 2 pi u, cos 2 pi u) for 0 <= u < 1 by the written method of the Box-Muller step
    (exact quadrant reduction, Taylor series on [-pi/4, pi/4])."""
    sn, cs = ctypes.c_double(), ctypes.c_double()
    lib().orc_sincos_turn(float(u), ctypes.byref(sn), ctypes.byref(cs))
    return sn.value, cs.value


def gaussian_pair(seed, chain, traj, stream, index) -> np.ndarray:
    out = np.zeros(2)
    lib().orc_gaussian_pair(seed, chain, traj, stream, index, _p(out))
    return out


def random_links(Lx, Lt, seed, chain=0) -> np.ndarray:
    q = np.zeros((Lt, Lx, 2))
    lib().orc_random_links(Lx, Lt, seed, chain, _p(q))
    return q


def random_momenta(Lx, Lt, seed, chain=0, traj=0) -> np.ndarray:
    p = np.zeros((Lt, Lx, 2))
    lib().orc_random_momenta(Lx, Lt, seed, chain, traj, _p(p))
    return p


def random_zeta(Lx, Lt, seed, chain=0, traj=0) -> np.ndarray:
    z = np.zeros((Lt, Lx, 2), dtype=np.complex128)
    lib().orc_random_zeta(Lx, Lt, seed, chain, traj, _p(z))
    return z


def metropolis_uniform(seed, chain, traj) -> float:
    return lib().orc_metropolis_uniform(seed, chain, traj)


# ---------------------------------------------------------------- gauge part (Eqs. (13), (16))
def gauge_action(q, beta) -> float:
    q = _links(q)
    return lib().orc_gauge_action(q.shape[1], q.shape[0], beta, _p(q))


def mean_plaquette(q) -> float:
    q = _links(q)
    return lib().orc_mean_plaquette(q.shape[1], q.shape[0], _p(q))


def gauge_force(q, beta) -> np.ndarray:
    q = _links(q)
    F = np.zeros_like(q)
    lib().orc_gauge_force(q.shape[1], q.shape[0], beta, _p(q), _p(F))
    return F


# ---------------------------------------------------------------- Wilson-Dirac operator (Sec. 3)
def dirac(q, psi, m0) -> np.ndarray:
    q, psi = _links(q), _spinor(psi)
    out = np.zeros_like(psi)
    lib().orc_dirac(q.shape[1], q.shape[0], m0, _p(q), _p(psi), _p(out))
    return out


def dirac_sites(q, psi, m0, sites) -> np.ndarray:
    """(D psi) at the lexicographic sites n = x + Lx t listed in `sites`; shape (len, 2)."""
    q, psi = _links(q), _spinor(psi)
    idx = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((idx.size, 2), dtype=np.complex128)
    lib().orc_dirac_sites(q.shape[1], q.shape[0], m0, _p(q), _p(psi), int(idx.size), _p(idx), _p(out))
    return out


def dirac_dagger(q, psi, m0) -> np.ndarray:
    q, psi = _links(q), _spinor(psi)
    out = np.zeros_like(psi)
    lib().orc_dirac_dagger(q.shape[1], q.shape[0], m0, _p(q), _p(psi), _p(out))
    return out


def cg(q, phi, m0, tol=1e-12, max_iter=100000):
    """CG on D^dagger D x = phi (x0 = 0).  Returns (x, iterations or -1, true relative residual)."""
    q, phi = _links(q), _spinor(phi)
    x = np.zeros_like(phi)
    res = ctypes.c_double(0.0)
    it = lib().orc_cg(q.shape[1], q.shape[0], m0, _p(q), _p(phi), _p(x), tol, max_iter,
                      ctypes.byref(res))
    return x, it, res.value


# ---------------------------------------------------------------- fermion part (Eqs. (14), (17), (18))
def fermion_force_chixi(q, chi, xi) -> np.ndarray:
    q, chi, xi = _links(q), _spinor(chi), _spinor(xi)
    f = np.zeros_like(q)
    lib().orc_fermion_force_chixi(q.shape[1], q.shape[0], _p(q), _p(chi), _p(xi), _p(f))
    return f


def fermion_force(q, phi, m0, tol=1e-12, max_iter=100000):
    """Returns (f, chi, xi, S_F, iterations)."""
    q, phi = _links(q), _spinor(phi)
    f = np.zeros_like(q)
    chi = np.zeros_like(phi)
    xi = np.zeros_like(phi)
    sf = ctypes.c_double(0.0)
    it = lib().orc_fermion_force(q.shape[1], q.shape[0], m0, _p(q), _p(phi), tol, max_iter, _p(f),
                                 _p(chi), _p(xi), ctypes.byref(sf))
    return f, chi, xi, sf.value, it


def fermion_action(q, phi, m0, tol=1e-12, max_iter=100000) -> float:
    q, phi = _links(q), _spinor(phi)
    return lib().orc_fermion_action(q.shape[1], q.shape[0], m0, _p(q), _p(phi), tol, max_iter)


def total_force(q, phi, beta, m0, tol=1e-12, quenched=False) -> np.ndarray:
    F = gauge_force(q, beta)
    if not quenched:
        F = F + fermion_force(q, phi, m0, tol)[0]
    return F


def fg_shifted_force(q, phi, beta, m0, h, which="fermion", tol=1e-12) -> np.ndarray:
    """F(q - (h^2/24) F(q)) for F the gauge, fermion or total force (Sec. 2.2, Taylor variant)."""
    def F(qq):
        if which == "gauge":
            return gauge_force(qq, beta)
        if which == "fermion":
            return fermion_force(qq, phi, m0, tol)[0]
        return total_force(qq, phi, beta, m0, tol)
    return F(np.asarray(q) - (h * h / 24.0) * F(q))


# ---------------------------------------------------------------- force-gradient term (Eqs. (19)-(23))
def fg_term_gg(q, beta) -> np.ndarray:
    """C_GG from the eight-plaquette closed form of Sec. 3."""
    q = _links(q)
    C = np.empty_like(q)
    lib().orc_fg_term_gg(q.shape[1], q.shape[0], beta, _p(q), _p(C))
    return C


def fg_term_fg(q, f, beta) -> np.ndarray:
    """C_FG from the closed form of Sec. 3, given the fermion force f."""
    q, f = _links(q), _links(f)
    C = np.empty_like(q)
    lib().orc_fg_term_fg(q.shape[1], q.shape[0], beta, _p(q), _p(f), _p(C))
    return C


def fg_term_fermion(q, chi, xi, v, m0, tol=1e-12, max_iter=100000):
    """4 Re[Z1^+ w2 + w1^+ Z2 - chi^+ D'' xi v] of Eqs. (22)-(23) with weight v.

    v = f gives C_FF, v = beta g gives C_GF.  Returns (C, CG iterations or -1)."""
    q, chi, xi, v = _links(q), _spinor(chi), _spinor(xi), _links(v)
    C = np.empty_like(q)
    it = lib().orc_fg_term_fermion(q.shape[1], q.shape[0], m0, _p(q), _p(chi), _p(xi), _p(v), tol,
                                   max_iter, _p(C))
    return C, it


def force_gradient_term(q, phi, beta, m0, which="total", tol=1e-12, max_iter=100000):
    """C of Eq. (19) for the gauge, fermion or total force.  Returns (C, info dict)."""
    q = _links(q)
    phi = _spinor(phi if phi is not None else np.zeros(q.shape, dtype=np.complex128))
    C = np.empty_like(q)
    cnt = np.zeros(3, dtype=np.int64)
    rc = lib().orc_force_gradient_term(q.shape[1], q.shape[0], beta, m0, _p(q), _p(phi),
                                       FORCE_SETS[which], tol, max_iter, _p(C), _p(cnt))
    return C, {"rc": rc, "n_solves": int(cnt[0]), "n_cg_iters": int(cnt[1]), "n_dinv": int(cnt[2])}


# ---------------------------------------------------------------- molecular dynamics and HMC (Sec. 2)
def _flags(quenched, fg_exact):
    return (FLAG_QUENCHED if quenched else 0) | (FLAG_FG_EXACT if fg_exact else 0)


def md_integrate(q, p, phi, beta, m0, scheme, tau, n_outer, n_inner=1, tol=1e-12, max_iter=100000,
                 quenched=False, trace_cap=0, fg_exact=False):
    """Integrates one trajectory from (q, p); returns (q', p', info dict[, trace]).

    fg_exact: the force-gradient kicks use the exact C of Eqs. (19)-(23) instead of the
    shifted force."""
    q = _links(q).copy()
    p = _links(p).copy()
    if phi is None:
        phi = np.zeros(q.shape, dtype=np.complex128)
    phi = _spinor(phi)
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    counters = np.zeros(4, dtype=np.int64)
    kinds = np.zeros(max(trace_cap, 1), dtype=np.int32)
    eps = np.zeros(max(trace_cap, 1), dtype=np.float64)
    rc = lib().orc_md_integrate(q.shape[1], q.shape[0], beta, m0, scheme, tau, n_outer, n_inner,
                                tol, max_iter, _flags(quenched, fg_exact), _p(q), _p(p),
                                _p(phi), _p(counters), _p(kinds), _p(eps), trace_cap)
    info = {"rc": rc, "n_solves": int(counters[0]), "n_cg_iters": int(counters[1]),
            "n_stages": int(counters[2]), "n_dinv": int(counters[3])}
    if trace_cap:
        n = min(int(counters[2]), trace_cap)
        info["trace"] = [(STAGE_NAMES[int(k)], float(e)) for k, e in zip(kinds[:n], eps[:n])]
    return q, p, info


def hamiltonian(q, p, phi, beta, m0, tol=1e-14, quenched=False) -> float:
    """H = 1/2 sum p^2 + S_G + S_F, Eq. (12)."""
    h = 0.5 * float(np.sum(np.asarray(p) ** 2)) + gauge_action(q, beta)
    if not quenched:
        h += fermion_action(q, phi, m0, tol)
    return h


def hmc_trajectory(q, beta, m0, seed, chain, traj, scheme, tau, n_outer, n_inner=1, tol=1e-12,
                   max_iter=100000, quenched=False, fg_exact=False):
    """One HMC update (Sec. 2.1).  Returns (q_new, info dict)."""
    q = _links(q).copy()
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    info = np.zeros(9)
    rc = lib().orc_hmc_trajectory(q.shape[1], q.shape[0], beta, m0, seed, chain, traj, scheme, tau,
                                  n_outer, n_inner, tol, max_iter, _flags(quenched, fg_exact),
                                  _p(q), _p(info))
    return q, {"rc": rc, "dH": info[0], "accepted": bool(info[1]), "plaquette": info[2],
               "n_solves": int(info[3]), "n_cg_iters": int(info[4]), "H0": info[5], "H1": info[6],
               "u": info[7], "n_dinv": int(info[8])}
