"""splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014; the 64-bit finaliser popularised by Vigna), used to draw Lanczos start
vectors.  Reading: the paper does not say how the eigen-estimate is started; the
start vector entry i is the first splitmix64 output from state (seed XOR i), mapped to
[-1, 1) through its top 53 bits.

Pinned by the generator's published first outputs from state 0.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(state: int) -> int:
    """First output of splitmix64 started from `state` (pure Python integers)."""
    z = (state + GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64_array(states: np.ndarray) -> np.ndarray:
    """Vectorised splitmix64 over uint64 states (numpy wraps modulo 2^64)."""
    z = states.astype(np.uint64) + np.uint64(GAMMA)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def start_vector(n: int, seed: int) -> np.ndarray:
    """v_i = 2 * ((splitmix64(seed ^ i) >> 11) * 2^-53) - 1, i = 0..n-1."""
    i = np.arange(n, dtype=np.uint64)
    z = splitmix64_array(np.uint64(seed) ^ i)
    return 2.0 * ((z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)) - 1.0
