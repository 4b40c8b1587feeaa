"""SplitMix64 counter-based generator (Steele, Lea & Flood, OOPSLA 2014).

Every random number a workload or the method draws comes from here and is
handed to the solver (or to the oracle) as an ordinary input array, so both
sides see the same bits without sharing any arithmetic of the method.

The k-th output (k = 1, 2, ...) of a stream seeded with ``s`` is
``mix(s + k * 0x9E3779B97F4A7C15)`` where ``mix`` is the published
SplitMix64 finaliser.  Because the state advances by a constant, the k-th
draw is a pure function of (seed, k) and a whole stream is produced in one
vectorised numpy pass.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs ``offset+1 .. offset+count`` of the stream seeded with ``seed``."""
    if count < 0:
        raise ValueError("count must be >= 0")
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        state = np.uint64(seed & MASK64) + k * _GOLDEN
        return _mix(state)


def splitmix64_scalar(seed: int, k: int) -> int:
    """Pure-integer reference of the k-th output (k >= 1), for self-checks."""
    z = (seed + k * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each output times 2**-53."""
    z = splitmix64(seed, count, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [-1, 1): ``2u - 1`` with ``u`` from :func:`uniform01`."""
    return 2.0 * uniform01(seed, count, offset) - 1.0


def uniform_int(seed: int, lo: int, hi: int, count: int, offset: int = 0) -> np.ndarray:
    """Integers uniform on ``{lo, ..., hi}`` (inclusive) by scaling a U[0,1) draw."""
    u = uniform01(seed, count, offset)
    return lo + np.minimum((u * (hi - lo + 1)).astype(np.int64), hi - lo)


def he_uniform_params(seed: int, shapes) -> np.ndarray:
    """Initial parameters of a dense network, flattened in the order of
    ``shapes``: every 2-D weight (out x in) is U(-l, l) with l = sqrt(6 / in)
    drawn from stream ``seed`` at the running offset; every 1-D bias is zero."""
    parts = []
    off = 0
    for s in shapes:
        k = int(np.prod(s))
        if len(s) == 2:
            parts.append(np.sqrt(6.0 / s[1]) * uniform_pm1(seed, k, off))
        else:
            parts.append(np.zeros(k))
        off += k
    return np.concatenate(parts)
