"""Counter-based random numbers for the synthetic workloads.

SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) is used as a keyed hash: every random number is a
pure function of (seed, level, I, J, K), so the values do not depend on the
order in which boxes or cells are visited.  This module holds input
generation only; it contains none of the solver's arithmetic.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    """SplitMix64 output function applied to a uint64 array."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64(x):
    """One SplitMix64 step from state ``x``: returns mix(x + golden gamma)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(x + _GOLDEN)


def hash_keys(*keys):
    """Fold integer keys (broadcastable arrays) into one uint64 hash each."""
    h = np.uint64(0)
    for k in keys:
        k = np.asarray(k).astype(np.int64).astype(np.uint64)
        with np.errstate(over="ignore"):
            h = splitmix64(h ^ k)
    return h


def uniform01(seed, level, I, J, K):
    """U in [0, 1) keyed by (seed, level, global cell index I, J, K)."""
    h = hash_keys(seed, level, I, J, K)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
