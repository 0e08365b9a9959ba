"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module only draws numbers: it holds none of the method's arithmetic
(no pair functions, no potentials, no Metropolis logic).  Configurations are
jittered cubic grids in the box [0, L)^3, which gives liquid-like nearest
neighbour distances without the perfect symmetry of a lattice.
"""
import numpy as np


def grid_config(n: int, L: float, seed: int, jitter: float = 0.3, dtype=np.float64) -> np.ndarray:
    """(3, n) coordinates: the first n sites of a k^3 cubic grid (k^3 >= n)
    filling the box, each moved by U(-jitter, jitter) grid spacings, wrapped
    into [0, L)."""
    rng = np.random.default_rng(seed)
    k = 1
    while k ** 3 < n:
        k += 1
    a = L / k
    idx = np.arange(n)
    ijk = np.stack([idx // (k * k), (idx // k) % k, idx % k]).astype(np.float64)
    x = a * (ijk + 0.5) + a * rng.uniform(-jitter, jitter, size=(3, n))
    x = np.mod(x, L)
    x = np.where(x >= L, x - L, x)
    x = x.astype(dtype)
    # a float32 cast can round a value just below L up to L
    x[x.astype(np.float64) >= L] = 0
    return np.ascontiguousarray(x)


def uniform_config(n: int, L: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, size=(3, n))
    return np.ascontiguousarray(np.where(x >= L, 0.0, x))


def moves(n: int, count: int, sigma: float, seed: int):
    """count random (s, delta) pairs: s uniform in [0, n), delta Gaussian with
    standard deviation sigma per component."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, size=count).astype(np.int32)
    d = rng.normal(0.0, sigma, size=(count, 3))
    return s, d
