"""Uniform sampling of distinct row/column indices for IRCUR.

Algorithm 1 draws the row set I and the column set J uniformly at random (and,
in the IRCUR-R variant of section 3.4, draws them again every iteration).  The
paper fixes neither the generator nor with/without replacement (Theorem 2 is
stated for sampling with replacement); the reading used here is: distinct
indices, sorted ascending, drawn from a documented counter-based stream so that
an independent implementation can reproduce them bit for bit.

Generator (written from its published definition, Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014; the constants are
those of the public-domain reference ``splitmix64``):

    state <- state + 0x9E3779B97F4A7C15        (mod 2^64)
    z <- state
    z <- (z xor (z >> 30)) * 0xBF58476D1CE4E5B9
    z <- (z xor (z >> 27)) * 0x94D049BB133111EB
    output z xor (z >> 31)

Stream (seed, t): the generator starts from state mix(seed xor ((t+1) * 0xD1B54A32D192ED03)),
where mix is the three-line output function above applied to a value.

Bounded draw in [0, m): the high 64 bits of the 128-bit product x * m
(multiply-shift, Lemire 2019), bias at most m / 2^64.

Distinct k-subset of [0, n): Floyd's algorithm (Bentley & Floyd, "Programming
pearls: a sample of brilliance", CACM 30(9), 1987): for j = n-k .. n-1 draw
t uniform in [0, j]; insert t unless already present, else insert j.  The set is
then sorted ascending.  I is drawn first (from [0, n1)), then J (from [0, n2)),
from the same stream.

IRCUR-F uses stream t = 0 for every iteration; IRCUR-R uses stream t = k at
iteration k+1, so both variants see the same sets in their first iteration.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_STREAM_MUL = 0xD1B54A32D192ED03


def mix64(z: int) -> int:
    """SplitMix64 output function applied to a 64-bit value."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


class SplitMix64:
    """The SplitMix64 generator on Python integers (exact 64-bit arithmetic)."""

    def __init__(self, state: int):
        self.state = state & _MASK

    def next(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK
        return mix64(self.state)

    def below(self, m: int) -> int:
        """Uniform integer in [0, m) by 64x64 -> 128 multiply-shift."""
        return (self.next() * m) >> 64


def stream(seed: int, t: int) -> SplitMix64:
    """Generator for index stream t of a run seeded with ``seed``."""
    key = (seed & _MASK) ^ (((t + 1) * _STREAM_MUL) & _MASK)
    return SplitMix64(mix64(key))


def floyd_sample(gen: SplitMix64, n: int, k: int) -> np.ndarray:
    """k distinct integers of [0, n), sorted ascending (Floyd's algorithm)."""
    if not (0 <= k <= n):
        raise ValueError("need 0 <= k <= n")
    chosen: set[int] = set()
    for j in range(n - k, n):
        t = gen.below(j + 1)
        chosen.add(j if t in chosen else t)
    return np.array(sorted(chosen), dtype=np.int64)


def draw_IJ(seed: int, t: int, n1: int, n2: int, sI: int, sJ: int):
    """Row set I then column set J from stream (seed, t)."""
    g = stream(seed, t)
    I = floyd_sample(g, n1, sI)
    J = floyd_sample(g, n2, sJ)
    return I, J


def stream_id(k: int, resample: bool) -> int:
    """Stream used by iteration k+1 (k = 0, 1, ...): 0 for IRCUR-F, k for IRCUR-R."""
    return k if resample else 0
