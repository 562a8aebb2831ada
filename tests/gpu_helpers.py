"""Helpers of the GPU tests: a Lattice with numpy <-> native layout conversion, the relative
error, and oracle reference chains.  The oracle is the checker here; nothing in this module
feeds the HIP path anything that came from it."""
import numpy as np

import oracle

try:
    import torch
except ImportError:  # the CPU-only suite never builds a Batch
    torch = None


def hmc():
    import paper_1512_03812_amd as m
    return m


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


class Batch:
    """A Lattice plus numpy<->native helpers for a list of (Lx, Lt, beta, m0)."""

    def __init__(self, shapes, seed=0, persistent=None):
        m = hmc()
        Lx = [s[0] for s in shapes]
        Lt = [s[1] for s in shapes]
        beta = [s[2] if len(s) > 2 else 2.0 for s in shapes]
        m0 = [s[3] if len(s) > 3 else 0.1 for s in shapes]
        self.lat = m.Lattice.batch(Lx, Lt, beta, m0, seed=seed)
        if persistent is not None:
            self.lat.set_persistent_limit(persistent)
        self.shapes = list(zip(Lx, Lt, beta, m0))

    def links_to_native(self, arrays, out=None):
        flat = np.concatenate([np.ascontiguousarray(a, dtype=np.float64).ravel() for a in arrays])
        return self.lat.pack_links(torch.from_numpy(flat), out=out)

    def spinor_to_native(self, arrays, out=None):
        flat = np.concatenate([np.ascontiguousarray(a, dtype=np.complex128).ravel() for a in arrays])
        return self.lat.pack_spinor(torch.from_numpy(flat), out=out)

    def links_from_native(self, t):
        flat = self.lat.unpack_links(t).cpu().numpy()
        return [flat[2 * o:2 * o + 2 * Lx * Lt].reshape(Lt, Lx, 2)
                for o, (Lx, Lt, _, _) in zip(self.lat.offsets, self.shapes)]

    def spinor_from_native(self, t):
        flat = self.lat.unpack_spinor(t).cpu().numpy()
        return [flat[2 * o:2 * o + 2 * Lx * Lt].reshape(Lt, Lx, 2)
                for o, (Lx, Lt, _, _) in zip(self.lat.offsets, self.shapes)]

    def set_q(self, arrays):
        self.links_to_native(arrays, out=self.lat.q)


def run_oracle_chain(Lx, Lt, beta, m0, seed, chain, n_traj, scheme, tau, n_outer, n_inner, tol,
                     fg_exact=False, quenched=False):
    q = oracle.random_links(Lx, Lt, seed, chain)
    out = []
    for t in range(n_traj):
        q, info = oracle.hmc_trajectory(q, beta, m0, seed, chain, t, scheme, tau, n_outer, n_inner,
                                        tol=tol, fg_exact=fg_exact, quenched=quenched)
        out.append((q.copy(), info))
    return out
