"""Counter-based random numbers for the randomised initialisers (test
infrastructure only; see ``oracle/__init__``).

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): output n of the stream with key k is
mix64(k + (n + 1) * GOLDEN), where mix64 is the published finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)
and GOLDEN = 0x9E3779B97F4A7C15 (all arithmetic mod 2^64).  A double in
[0, 1) is (z >> 11) * 2^-53.  The key of target b under a base seed s is
mix64(s + (b + 1) * GOLDEN), i.e. output b of the base stream.

The HIP library implements the same published definition independently, so a
(seed, target) pair names the same draws on both sides.
"""
from __future__ import annotations

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def output(key: int, n: int) -> int:
    return mix64(key + ((n + 1) * GOLDEN & MASK))


def target_key(seed: int, b: int) -> int:
    return output(seed & MASK, b)


class Stream:
    """Sequential reader over one counter-based stream."""

    def __init__(self, key: int):
        self.key = key & MASK
        self.n = 0

    def next_u64(self) -> int:
        z = output(self.key, self.n)
        self.n += 1
        return z

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))
