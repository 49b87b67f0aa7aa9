"""Seeded random substreams for the synthetic scene generators.

Every generator draws from a numpy Generator whose seed is derived from one
master seed and a stream label with SplitMix64 (Steele, Lea, Flood 2014), so
that adding a new stream never shifts the draws of an existing one.
"""
import numpy as np

MASTER_SEED = 260203002

_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One SplitMix64 output step for state ``x`` (returns the mixed word)."""
    x = (x + 0x9E3779B97F4A7C15) & _M64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _label_hash(label: str) -> int:
    h = 0xCBF29CE484222325  # FNV-1a 64
    for ch in label.encode():
        h ^= ch
        h = (h * 0x100000001B3) & _M64
    return h


def substream(label: str, seed: int = MASTER_SEED) -> np.random.Generator:
    """A numpy Generator for the named substream of ``seed``."""
    s = splitmix64((seed & _M64) ^ _label_hash(label))
    return np.random.Generator(np.random.PCG64(s))
