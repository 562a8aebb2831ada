"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds none of the method's arithmetic: only numpy random draws of the shapes the
Schwinger-model HMC works on (lexicographic layout, shape (Lt, Lx, 2)).  Random
numbers that the method itself draws (momenta, pseudofermions, hot start,
Metropolis) are not made here: each side generates them with its own Philox4x32-10.
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def random_angles(Lx, Lt, seed, scale=np.pi):
    """Link angles q uniform in [-scale, scale)."""
    return rng(seed).uniform(-scale, scale, size=(Lt, Lx, 2))


def smooth_angles(Lx, Lt, seed, scale=0.3):
    """Link angles near the identity (a weakly disordered, 'thermalised-like' field)."""
    return rng(seed).normal(0.0, scale, size=(Lt, Lx, 2))


def random_spinor(Lx, Lt, seed):
    g = rng(seed)
    return (g.normal(size=(Lt, Lx, 2)) + 1j * g.normal(size=(Lt, Lx, 2))) / np.sqrt(2.0)


def random_momenta(Lx, Lt, seed):
    return rng(seed).normal(size=(Lt, Lx, 2))


def random_gauge_transform(Lx, Lt, seed):
    """alpha(n), one angle per site, shape (Lt, Lx)."""
    return rng(seed).uniform(-np.pi, np.pi, size=(Lt, Lx))
