"""splitmix64 start vectors (oracle side).

Test infrastructure: see the package docstring.

The power iteration that estimates the largest eigenvalue of D^-1 A for the
Chebyshev smoother needs a start vector. It is a function of the global node
ID only, so that it is consistent across copies of a node and independent of
element order: v(gid) = 2 u - 1 with u = (splitmix64(gid) >> 11) * 2^-53.

splitmix64 (Steele, Lea & Flood, OOPSLA 2014) is one step of the generator
seeded with the counter:
    z = gid + 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)
all modulo 2^64. The HIP library implements the same published definition in
its own code.
"""
from __future__ import annotations

import numpy as np


def splitmix64(counter: np.ndarray) -> np.ndarray:
    z = np.asarray(counter, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def start_vector(gid: np.ndarray) -> np.ndarray:
    """Values in [-1, 1) keyed by global ID."""
    u = (splitmix64(gid) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0
