"""MI355X (gfx950) HMC hot path for the two-flavour lattice Schwinger model.

A thin Python binding of the C ABI in ``include/schwinger_hmc.h``: every step of
the method runs in the hand-written HIP kernels of ``libschwinger_hmc.so``;
PyTorch only provides device memory (the workspace tensor and the caller's
field tensors) and the HIP stream.  There is no CPU fallback: importing the
package without the built library raises.

Method: Shcherbakov et al., "Adapted nested force-gradient integrators: the
Schwinger model case", arXiv:1512.03812 (Secs. 2-3).

Native layouts (torch tensors on the GPU):
  real link field (q, p, forces): float64, shape (2, V_total)
  spinor field                  : complex128, shape (2, V_total)
Lexicographic layouts (per chain, chains concatenated):
  links  : float64, shape (..., Lt, Lx, 2)    spinors: complex128, shape (..., Lt, Lx, 2)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import (ADAPTED_NESTED_FG, FORCE_FERMION, FORCE_GAUGE, FORCE_GRADIENT, FORCE_TOTAL,
                   LEAPFROG, NESTED_FG, OMELYAN_5STAGE, PREC_FP64, PREC_MIXED, PRECISIONS,
                   SCHEMES)

__all__ = ["Lattice", "HMCError", "SCHEMES", "PRECISIONS", "SchwingerAction", "library_path"]


class HMCError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{_lib.ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


def library_path() -> str:
    return _lib.LIB_PATH


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _scheme(s):
    return SCHEMES[s] if isinstance(s, str) else int(s)


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


@dataclass
class CGResult:
    iters: List[int]
    converged: List[bool]
    reliable_updates: List[int]
    rel_resid: List[float]
    rel_resid_true: List[float]


@dataclass
class TrajResult:
    dH: List[float]
    H0: List[float]
    H1: List[float]
    plaquette: List[float]
    u: List[float]
    accepted: List[bool]
    status: List[int]
    n_force_evals: int
    n_solves: int
    n_dinv: int
    n_cg_iters: List[int]


class Lattice:
    """One or many independent Schwinger-model chains on one GPU.

    ``Lattice(L, beta, m0, seed)`` makes one L x L chain; ``Lattice.batch(Lx, Lt, beta, m0,
    seed)`` makes many chains of (possibly) different sizes sharing every launch."""

    def __init__(self, L: int = 8, beta: float = 2.0, m0: float = 0.1, seed: int = 0,
                 Lt: Optional[int] = None, device="cuda", _chains=None):
        self._lib = _lib.load()
        if _chains is None:
            _chains = ([L], [Lt if Lt is not None else L], [beta], [m0])
        Lx, Lts, betas, m0s = (list(v) for v in _chains)
        n = len(Lx)
        self.n_chains = n
        self.Lx, self.Lt, self.beta, self.m0 = Lx, Lts, [float(b) for b in betas], [float(m) for m in m0s]
        self.seed = int(seed)
        ctx = ctypes.c_void_p()
        IA = ctypes.c_int * n
        DA = ctypes.c_double * n
        rc = self._lib.hmc_batch_init(ctypes.byref(ctx), n, IA(*Lx), IA(*Lts), DA(*self.beta),
                                      DA(*self.m0), ctypes.c_uint64(self.seed))
        if rc != 0:
            raise HMCError(rc, "invalid lattice parameters (L even >= 2, finite beta and m0)")
        self._ctx = ctx
        self.device = torch.device(device)
        nbytes = self._lib.hmc_workspace_bytes(ctx)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self._check(self._lib.hmc_bind(ctx, _ptr(self.workspace), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream)))
        nch = ctypes.c_int()
        vt = ctypes.c_longlong()
        offs = IA()
        self._check(self._lib.hmc_geometry(ctx, ctypes.byref(nch), ctypes.byref(vt), offs, None, None))
        self.V_total = int(vt.value)
        self.offsets = list(offs)
        self.V = [a * b for a, b in zip(Lx, Lts)]

    @classmethod
    def batch(cls, Lx: Sequence[int], Lt: Optional[Sequence[int]] = None, beta=2.0, m0=0.1,
              seed: int = 0, device="cuda"):
        n = len(Lx)
        Lt = list(Lt) if Lt is not None else list(Lx)
        betas = list(beta) if hasattr(beta, "__len__") else [beta] * n
        m0s = list(m0) if hasattr(m0, "__len__") else [m0] * n
        return cls(seed=seed, device=device, _chains=(list(Lx), Lt, betas, m0s))

    # ---------------------------------------------------------------- plumbing
    def _check(self, rc):
        """Raises HMCError for every nonzero code, an unconverged solve included."""
        if rc != 0:
            raise HMCError(rc, self._lib.hmc_last_error(self._ctx).decode())
        return rc

    def _check_solve(self, rc):
        """As _check, except for the codes that say some chains stopped unconverged
        (HMC_E_NOCONV, HMC_E_NAN): the caller returns per-chain solver results that say which."""
        if rc not in (0, _lib.HMC_E_NOCONV, _lib.HMC_E_NAN):
            self._check(rc)
        return rc

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self._lib.hmc_destroy(ctx)
            self._ctx = None

    def _field(self, which, dtype, shape):
        p = ctypes.c_void_p()
        nb = ctypes.c_size_t()
        self._check(self._lib.hmc_field(self._ctx, which, ctypes.byref(p), ctypes.byref(nb)))
        off = p.value - self.workspace.data_ptr()
        return self.workspace[off:off + nb.value].view(dtype).view(*shape)

    def mark_links_changed(self):
        """Call after writing q through a tensor obtained from `q` earlier."""
        self._check(self._lib.hmc_mark_links_changed(self._ctx))

    def new_links(self):
        return torch.zeros((2, self.V_total), dtype=torch.float64, device=self.device)

    def new_spinor(self):
        return torch.zeros((2, self.V_total), dtype=torch.complex128, device=self.device)

    @property
    def q(self) -> torch.Tensor:
        """Link angles (native layout view into the workspace; writes are seen by the library)."""
        return self._field(_lib.FIELD_Q, torch.float64, (2, self.V_total))

    @property
    def p(self) -> torch.Tensor:
        return self._field(_lib.FIELD_P, torch.float64, (2, self.V_total))

    @property
    def phi(self) -> torch.Tensor:
        return self._field(_lib.FIELD_PHI, torch.complex128, (2, self.V_total))

    @property
    def chi(self) -> torch.Tensor:
        return self._field(_lib.FIELD_CHI, torch.complex128, (2, self.V_total))

    @property
    def xi(self) -> torch.Tensor:
        return self._field(_lib.FIELD_XI, torch.complex128, (2, self.V_total))

    @property
    def zeta(self) -> torch.Tensor:
        return self._field(_lib.FIELD_ZETA, torch.complex128, (2, self.V_total))

    # ---------------------------------------------------------------- layout
    def pack_links(self, lexico: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        lexico = lexico.to(self.device, torch.float64).contiguous()
        assert lexico.numel() == 2 * self.V_total
        out = self.new_links() if out is None else out
        self._check(self._lib.hmc_pack_links(self._ctx, _ptr(lexico), _ptr(out)))
        return out

    def unpack_links(self, native: torch.Tensor) -> torch.Tensor:
        native = native.contiguous()
        out = torch.empty(2 * self.V_total, dtype=torch.float64, device=self.device)
        self._check(self._lib.hmc_unpack_links(self._ctx, _ptr(native), _ptr(out)))
        return out

    def pack_spinor(self, lexico: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        lexico = lexico.to(self.device, torch.complex128).contiguous()
        assert lexico.numel() == 2 * self.V_total
        out = self.new_spinor() if out is None else out
        self._check(self._lib.hmc_pack_spinor(self._ctx, _ptr(lexico), _ptr(out)))
        return out

    def unpack_spinor(self, native: torch.Tensor) -> torch.Tensor:
        native = native.contiguous()
        out = torch.empty(2 * self.V_total, dtype=torch.complex128, device=self.device)
        self._check(self._lib.hmc_unpack_spinor(self._ctx, _ptr(native), _ptr(out)))
        return out

    def chain_view(self, lexico_flat: torch.Tensor, c: int) -> torch.Tensor:
        """Chain c's (Lt, Lx, 2) block of a flat lexicographic field."""
        o = 2 * self.offsets[c]
        return lexico_flat[o:o + 2 * self.V[c]].view(self.Lt[c], self.Lx[c], 2)

    def set_links(self, lexico: torch.Tensor):
        self.pack_links(lexico, out=self.q)

    def get_links(self) -> torch.Tensor:
        return self.unpack_links(self.q)

    # ---------------------------------------------------------------- set-up
    def cold_start(self):
        self._check(self._lib.hmc_cold_start(self._ctx))

    def hot_start(self):
        self._check(self._lib.hmc_hot_start(self._ctx))

    def set_solver(self, tol=1e-12, max_iter=100000, reliable_delta=1e-4):
        self._check(self._lib.hmc_set_solver(self._ctx, tol, max_iter, reliable_delta))

    def set_quenched(self, quenched: bool):
        self._check(self._lib.hmc_set_quenched(self._ctx, int(bool(quenched))))

    def set_fg_mode(self, mode: str):
        """"shift" (default): force-gradient kicks use the shifted force; "exact": they use
        the force-gradient term C of Eq. (19) through a Hessian-vector product."""
        self._check(self._lib.hmc_set_fg_mode(self._ctx, _lib.FG_MODES[mode]))

    def set_graph(self, on: bool):
        """Run trajectories from HIP graphs: one graph per trajectory schedule when every chain
        fits the persistent solver, otherwise each solve's CG iteration slots as replays of
        captured chunks (the rest of the trajectory eager).  Results are bit-identical to the
        eager path."""
        self._check(self._lib.hmc_set_graph(self._ctx, int(bool(on))))

    def set_persistent_limit(self, vmax: int):
        """Chains of at most vmax sites solve inside one persistent workgroup (0: never)."""
        self._check(self._lib.hmc_set_persistent_limit(self._ctx, int(vmax)))

    def set_cg_groups(self, groups: int):
        """Chain groups (1..4, default 1): trajectories advance the chains as that many
        contiguous groups, each on its own stream and host thread (bit-identical results)."""
        self._check(self._lib.hmc_set_cg_groups(self._ctx, int(groups)))

    def set_fused_cg(self, on: bool):
        """One fused kernel per CG iteration where the chains allow it, or two (default)."""
        self._check(self._lib.hmc_set_fused_cg(self._ctx, 1 if on else 0))

    def set_block_size(self, block: int):
        self._check(self._lib.hmc_set_block_size(self._ctx, int(block)))

    def autotune(self, prec="fp64", tol=1e-10, schedule=None) -> dict:
        """hmc_autotune: workgroup size x persistent limit, step-kernel variant, check interval,
        reliable-update factor (mixed), and, given schedule = (scheme, tau, n_outer, n_inner),
        the chain-group count by whole trajectories.  Overwrites p and phi (q is kept)."""
        t = _lib.TuneInfo()
        sched = None
        if schedule is not None:
            scheme, tau, n_outer, n_inner = schedule
            sched = _lib.TuneSchedule(_scheme(scheme), int(n_outer), int(n_inner), 0, float(tau))
        self._check(self._lib.hmc_autotune(self._ctx, _prec(prec), tol,
                                           ctypes.byref(sched) if sched is not None else None,
                                           ctypes.byref(t)))
        names = {v: k for k, v in _lib.STEP_VARIANTS.items()}
        return {"block": t.block, "persistent_limit": t.persistent_limit,
                "step_variant": names.get(t.step_variant, t.step_variant),
                "check_interval": t.check_interval, "groups": t.groups,
                "reliable_delta": t.reliable_delta, "solve_ms": t.solve_ms, "traj_ms": t.traj_ms,
                "candidates": t.candidates}

    def set_step_variant(self, variant):
        """CG step-kernel variant: "plain", "two_sites", "resident" or "waves8"."""
        v = _lib.STEP_VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self._check(self._lib.hmc_set_step_variant(self._ctx, v))

    def set_check_interval(self, every: int):
        self._check(self._lib.hmc_set_check_interval(self._ctx, int(every)))

    def set_timing(self, on: bool):
        """Bracket every CG iteration slot with HIP events (resets the statistics)."""
        self._check(self._lib.hmc_set_timing(self._ctx, int(bool(on))))

    def kernel_stats(self, which: int) -> dict:
        """Event timing of CG step 1 (which=0) or step 2 (which=1) since set_timing; with
        fused = 1, index 0 is the fused one-kernel iteration."""
        st = _lib.KernelStat()
        self._check(self._lib.hmc_get_kernel_stats(self._ctx, int(which), ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    @property
    def trajectory_counter(self) -> int:
        return int(self._lib.hmc_get_trajectory_counter(self._ctx))

    @trajectory_counter.setter
    def trajectory_counter(self, t: int):
        self._check(self._lib.hmc_set_trajectory_counter(self._ctx, int(t)))

    # ---------------------------------------------------------------- operators (Sec. 3)
    def stream_copy(self, src: torch.Tensor, dst: torch.Tensor):
        """dst = src by the library's streaming copy kernel (a bandwidth reference)."""
        if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
            raise ValueError("stream_copy needs contiguous device tensors")
        n = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() < n:
            raise ValueError("dst is smaller than src")
        self._check(self._lib.hmc_stream_copy(self._ctx, _ptr(src), _ptr(dst), n))
        return dst

    def dslash(self, psi: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_spinor() if out is None else out
        self._check(self._lib.hmc_dslash(self._ctx, _ptr(psi), _ptr(out)))
        return out

    def dslash_dagger(self, psi: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_spinor() if out is None else out
        self._check(self._lib.hmc_dslash_dagger(self._ctx, _ptr(psi), _ptr(out)))
        return out

    def _cg_result(self, arr) -> CGResult:
        return CGResult([a.iters for a in arr], [bool(a.converged) for a in arr],
                        [a.reliable_updates for a in arr], [a.rel_resid for a in arr],
                        [a.rel_resid_true for a in arr])

    def cg_solve(self, phi: torch.Tensor, tol=1e-12, max_iter=100000, prec="fp64",
                 out: Optional[torch.Tensor] = None):
        """x = (D^dagger D)^{-1} phi; returns (x, CGResult)."""
        out = self.new_spinor() if out is None else out
        info = (_lib.CGInfo * self.n_chains)()
        self._check_solve(self._lib.hmc_cg_solve(self._ctx, _ptr(phi), _ptr(out), tol, max_iter,
                                                 _prec(prec), info))
        return out, self._cg_result(info)

    def cg_solve_noalloc(self, phi: torch.Tensor, out: torch.Tensor, tol=1e-12, max_iter=100000):
        """hmc_cg_solve_noalloc: the FP64 solve of cg_solve with the library's static scratch
        (no device allocation; every chain within 2048 sites).  out: a caller-owned spinor
        field.  Returns (out, CGResult)."""
        info = (_lib.CGInfo * self.n_chains)()
        self._check_solve(self._lib.hmc_cg_solve_noalloc(self._ctx, _ptr(phi), _ptr(out), tol,
                                                         max_iter, info))
        return out, self._cg_result(info)

    # ---------------------------------------------------------------- forces (Sec. 3)
    def fermion_force(self, phi: torch.Tensor, tol=1e-12, max_iter=100000, prec="fp64",
                      out: Optional[torch.Tensor] = None):
        """f = dS_F/dq (Eq. (17)); returns (f, S_F per chain, CGResult).  A chain whose solve
        stopped unconverged is flagged in CGResult.converged (its f is not the force)."""
        out = self.new_links() if out is None else out
        info = (_lib.CGInfo * self.n_chains)()
        sf = (ctypes.c_double * self.n_chains)()
        self._check_solve(self._lib.hmc_fermion_force(self._ctx, _ptr(phi), _ptr(out), tol,
                                                      max_iter, _prec(prec), info, sf))
        return out, list(sf), self._cg_result(info)

    def fermion_action(self, phi: torch.Tensor, tol=1e-12, max_iter=100000, prec="fp64"):
        """S_F per chain (Eq. (14)); leaves xi and chi = D xi in the workspace.  Raises
        HMCError if a chain's solve stops unconverged."""
        info = (_lib.CGInfo * self.n_chains)()
        sf = (ctypes.c_double * self.n_chains)()
        self._check(self._lib.hmc_fermion_force(self._ctx, _ptr(phi), None, tol, max_iter,
                                                _prec(prec), info, sf))
        return list(sf), self._cg_result(info)

    def fermion_force_chixi(self, chi, xi, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_links() if out is None else out
        self._check(self._lib.hmc_fermion_force_chixi(self._ctx, _ptr(chi), _ptr(xi), _ptr(out)))
        return out

    def total_force_chixi(self, chi, xi, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """F_G + F_F with the fermion force from given chi, xi (Eqs. (16), (17))."""
        out = self.new_links() if out is None else out
        self._check(self._lib.hmc_total_force_chixi(self._ctx, _ptr(chi), _ptr(xi), _ptr(out)))
        return out

    def gauge_force(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_links() if out is None else out
        self._check(self._lib.hmc_gauge_force(self._ctx, _ptr(out)))
        return out

    def actions(self, phi: Optional[torch.Tensor] = None, tol=1e-12):
        """Returns (S_G, mean plaquette, S_F or None) per chain."""
        C = self.n_chains
        sg, pl, sf = (ctypes.c_double * C)(), (ctypes.c_double * C)(), (ctypes.c_double * C)()
        self._check(self._lib.hmc_actions(self._ctx, _ptr(phi), tol, sg, pl,
                                          sf if phi is not None else None))
        return list(sg), list(pl), (list(sf) if phi is not None else None)

    def fg_shifted_force(self, c_h2: float, which="fermion", phi=None, prec="fp64",
                         out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """F(q + c_h2 F(q)); c_h2 = -h^2/24 is the Taylor form of the force-gradient kick."""
        w = {"gauge": FORCE_GAUGE, "fermion": FORCE_FERMION, "total": FORCE_TOTAL}[which] \
            if isinstance(which, str) else int(which)
        out = self.new_links() if out is None else out
        info = (_lib.CGInfo * self.n_chains)()
        self._check(self._lib.hmc_fg_shifted_force(self._ctx, c_h2, w, _ptr(phi), _ptr(out),
                                                   _prec(prec), info))
        return out

    def hessian_vector(self, v: torch.Tensor, which="total", phi=None, prec="fp64",
                       out: Optional[torch.Tensor] = None):
        """H v, H the second derivatives of S_G, S_F or S_G + S_F at the current links
        (Sec. 3, Eqs. (21)-(23)).  Returns (out, CGResult of the Hessian solve or None)."""
        w = _lib.FORCE_SETS[which] if isinstance(which, str) else int(which)
        out = self.new_links() if out is None else out
        info = (_lib.CGInfo * self.n_chains)()
        self._check_solve(self._lib.hmc_hessian_vector(self._ctx, w, _ptr(phi), _ptr(v), _ptr(out),
                                                       _prec(prec), info))
        return out, (self._cg_result(info) if w != FORCE_GAUGE else None)

    def force_gradient_term(self, which="total", phi=None, prec="fp64",
                            out: Optional[torch.Tensor] = None):
        """C = 2 H F of Eq. (19) for the gauge (C_GG), fermion (C_FF) or total force
        (C_GG + C_FG + C_GF + C_FF).  Returns (C, CGResult of the Hessian solve or None)."""
        w = _lib.FORCE_SETS[which] if isinstance(which, str) else int(which)
        out = self.new_links() if out is None else out
        info = (_lib.CGInfo * self.n_chains)()
        self._check_solve(self._lib.hmc_force_gradient_term(self._ctx, w, _ptr(phi), _ptr(out),
                                                            _prec(prec), info))
        return out, (self._cg_result(info) if w != FORCE_GAUGE else None)

    # ---------------------------------------------------------------- updates (Sec. 2.1)
    def update_links(self, eps: float):
        self._check(self._lib.hmc_update_links(self._ctx, eps))

    def update_momenta(self, eps: float, F: torch.Tensor):
        self._check(self._lib.hmc_update_momenta(self._ctx, eps, _ptr(F)))

    # ---------------------------------------------------------------- HMC (Sec. 2)
    def _traj_result(self, arr) -> TrajResult:
        return TrajResult([a.dH for a in arr], [a.H0 for a in arr], [a.H1 for a in arr],
                          [a.plaquette for a in arr], [a.u for a in arr],
                          [bool(a.accepted) for a in arr], [a.status for a in arr],
                          arr[0].n_force_evals, arr[0].n_solves, arr[0].n_dinv,
                          [a.n_cg_iters for a in arr])

    def trajectory(self, scheme="adapted_nested_fg", tau=1.0, n_outer=8, n_inner=4, prec="fp64"):
        info = (_lib.TrajInfo * self.n_chains)()
        self._check_solve(self._lib.hmc_trajectory(self._ctx, _scheme(scheme), tau, n_outer,
                                                   n_inner, _prec(prec), info))
        return self._traj_result(info)

    def refresh(self):
        """Draws p (stream 1) and zeta (stream 2), sets phi = D^dagger zeta (Sec. 2.1)."""
        self._check(self._lib.hmc_refresh(self._ctx))

    def integrate(self, scheme="adapted_nested_fg", tau=1.0, n_outer=8, n_inner=4, prec="fp64"):
        """Molecular dynamics only from the current q, p, phi (no refresh, no Metropolis)."""
        info = (_lib.TrajInfo * self.n_chains)()
        self._check_solve(self._lib.hmc_integrate(self._ctx, _scheme(scheme), tau, n_outer,
                                                  n_inner, _prec(prec), info))
        return self._traj_result(info)


class _ActionForce(torch.autograd.Function):
    """F(q) = dS/dq = F_G + F_F from the chi, xi of the action's forward (Eqs. (16), (17)).

    Its backward is the Hessian-vector product of Sec. 3 (Eq. (21), plus the gauge part),
    computed by the HIP library, so the action is twice differentiable.  The Hessian solve
    uses the tolerance set by Lattice.set_solver."""

    @staticmethod
    def forward(ctx, q, lat, phi, chi, xi):
        lat.q.copy_(q)
        F = lat.total_force_chixi(chi, xi)
        ctx.lat = lat
        ctx.save_for_backward(q, phi)
        return F

    @staticmethod
    def backward(ctx, grad_F):
        q, phi = ctx.saved_tensors
        lat = ctx.lat
        lat.q.copy_(q.detach())
        hv, res = lat.hessian_vector(grad_F.detach().contiguous(), "total", phi)
        if res is not None and not all(res.converged):
            raise HMCError(_lib.HMC_E_NOCONV, "the Hessian solve of the force's backward did not "
                                              "converge")
        return hv, None, None, None, None


class SchwingerAction(torch.autograd.Function):
    """S(q) = S_G(q) + phi^dagger (D^dagger D)^{-1} phi per chain (Eqs. (13), (14)).

    Forward solves xi and forms chi = D xi in the HIP library; backward is the
    hand-written adjoint kernel (the fermion force of Eq. (17)) plus the gauge force
    of Eq. (16), scaled by the incoming gradient of each chain.  The force is itself a
    differentiable function of q whose backward is the library's Hessian-vector product,
    so second derivatives (create_graph=True, torch.autograd.functional.hvp) work too."""

    @staticmethod
    def forward(ctx, q: torch.Tensor, lat: Lattice, phi: torch.Tensor, tol: float = 1e-12,
                prec: str = "fp64"):
        lat.q.copy_(q)
        sf, _ = lat.fermion_action(phi, tol=tol, prec=prec)
        sg, _, _ = lat.actions(None)
        ctx.lat = lat
        ctx.save_for_backward(q, lat.chi.clone(), lat.xi.clone(), phi)
        return torch.tensor([a + b for a, b in zip(sg, sf)], dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, grad_s):
        q, chi, xi, phi = ctx.saved_tensors
        lat = ctx.lat
        F = _ActionForce.apply(q, lat, phi, chi, xi)
        if lat.n_chains == 1:
            grad = grad_s[0] * F
        else:
            scale = torch.repeat_interleave(grad_s, torch.tensor(lat.V, device=grad_s.device))
            grad = F * scale[None, :]
        return grad, None, None, None, None


def trajectories_concurrent(lattices, scheme="adapted_nested_fg", tau=1.0, n_outer=8, n_inner=4,
                            prec="fp64"):
    """One HMC trajectory on each of several Lattice objects at once (hmc_trajectories_concurrent:
    one host thread per context; each must have been created on a stream of its own).
    Returns one TrajResult per lattice, each what lattice.trajectory would have returned."""
    lats = list(lattices)
    if not lats:
        return []
    lib = lats[0]._lib
    n = len(lats)
    infos = [(_lib.TrajInfo * lat.n_chains)() for lat in lats]
    ctxs = (ctypes.c_void_p * n)(*[lat._ctx.value for lat in lats])
    iptr = (ctypes.c_void_p * n)(*[ctypes.cast(i, ctypes.c_void_p).value for i in infos])
    rcs = (ctypes.c_int * n)()
    rc = lib.hmc_trajectories_concurrent(ctxs, n, _scheme(scheme), tau, n_outer, n_inner,
                                         _prec(prec), iptr, rcs)
    if rc == _lib.HMC_E_INVAL and all(r == 0 for r in rcs):
        raise HMCError(rc, "trajectories_concurrent needs distinct bound lattices on distinct streams")
    for lat, r in zip(lats, rcs):
        lat._check_solve(r)
    return [lat._traj_result(i) for lat, i in zip(lats, infos)]
