"""Seeded synthetic operands for the multiplication workloads.

This module only draws random limbs; it holds none of the multiplication's
arithmetic.  It feeds both the GPU library and its checker, so both see
identical inputs.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used as a counter-based stream: output i of
stream (seed, tag) is mix64(base + (i + 1) * GAMMA) where
base = mix64(seed * GAMMA + tag).  Each 64-bit output gives two 32-bit limbs,
low half first.  Operands are little-endian uint32 limb vectors.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64's output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _base(seed: int, tag: int) -> np.uint64:
    s = np.uint64(((seed * 0x9E3779B97F4A7C15) + tag) & MASK64)
    return mix64(np.array([s], dtype=np.uint64))[0]


def words(seed: int, tag: int, count: int, start: int = 0) -> np.ndarray:
    """64-bit outputs start .. start+count-1 of stream (seed, tag)."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(_base(seed, tag) + i * GAMMA)


def uniform01(seed: int, tag: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of each output."""
    return (words(seed, tag, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def random_limbs(seed: int, tag: int, n: int, top_nonzero: bool = True) -> np.ndarray:
    """n uniform limbs; the top limb is redrawn from later outputs while zero."""
    w = words(seed, tag, (n + 1) // 2)
    limbs = w.view(np.uint32)[:n].copy()  # little-endian host: low half first
    if top_nonzero and n > 0:
        k = (n + 1) // 2
        while limbs[n - 1] == 0:
            limbs[n - 1] = np.uint32(int(words(seed, tag, 1, start=k)[0]) & 0xFFFFFFFF)
            k += 1
    return limbs


def all_ones(n: int) -> np.ndarray:
    return np.full(n, 0xFFFFFFFF, dtype=np.uint32)


def single_bit(n: int, bit: int) -> np.ndarray:
    a = np.zeros(n, dtype=np.uint32)
    a[bit // 32] = np.uint32(1 << (bit % 32))
    return a


def sparse_limbs(seed: int, tag: int, n: int, density: float = 0.01) -> np.ndarray:
    """Each limb non-zero with probability `density`, value uniform in
    [1, 2^32-1]; the top limb is always non-zero."""
    keep = uniform01(seed, tag * 2 + 1, n) < density
    vals = random_limbs(seed, tag * 2 + 2, n, top_nonzero=False).astype(np.uint64)
    vals = (vals % np.uint64(0xFFFFFFFF)) + np.uint64(1)
    out = np.where(keep, vals, np.uint64(0)).astype(np.uint32)
    out[n - 1] = np.uint32(vals[n - 1])
    return out


# --------------------------------------------------------------------------
# The five workloads (seeds 1..5)
# --------------------------------------------------------------------------

def config1_uniform(n: int = 1024):
    """Two uniform 1024-limb operands, top limb non-zero (seed 1)."""
    return random_limbs(1, 1, n), random_limbs(1, 2, n)


def config1_all_ones(n: int = 1024):
    return all_ones(n), all_ones(n)


def config1_single_bit(n: int = 1024):
    """u = 2^(32(n-1)+a), v = 2^(32(n-1)+c), a and c drawn from [0, 32)."""
    a, c = (int(x) % 32 for x in words(1, 3, 2))
    return single_bit(n, 32 * (n - 1) + a), single_bit(n, 32 * (n - 1) + c)


def config2(n: int = 1 << 19):
    """Two uniform 2^19-limb (2^24-bit) operands (seed 2)."""
    return random_limbs(2, 1, n), random_limbs(2, 2, n)


def config3_sizes(count: int = 4096, lo: int = 64, hi: int = 16384, seed: int = 3):
    """Balanced sizes n = floor(exp(U[ln lo, ln(hi+1))))."""
    r = uniform01(seed, 100, count)
    n = np.floor(np.exp(math.log(lo) + r * (math.log(hi + 1) - math.log(lo)))).astype(np.int64)
    return np.clip(n, lo, hi)


def config3_operand(seed: int, tag: int, n: int) -> np.ndarray:
    """p = 0.90 uniform, 0.05 all-ones, 0.05 sparse (1% non-zero limbs)."""
    r = float(uniform01(seed, 1_000_000 + tag, 1)[0])
    if r < 0.90:
        return random_limbs(seed, tag, n)
    if r < 0.95:
        return all_ones(n)
    return sparse_limbs(seed, tag, n)


def config3(count: int = 4096, lo: int = 64, hi: int = 16384, seed: int = 3):
    """List of (u, v) pairs for the batched workload."""
    sizes = config3_sizes(count, lo, hi, seed)
    return [(config3_operand(seed, 2 * i + 10, int(n)), config3_operand(seed, 2 * i + 11, int(n)))
            for i, n in enumerate(sizes)]


def zipf_sizes(count: int, seed: int = 4, s: float = 1.2, ranks: int = 16, first_log2: int = 5):
    """Sizes 2^(first_log2 + r - 1) for rank r = 1..ranks with P(r) ~ r^-s."""
    p = np.array([r ** -s for r in range(1, ranks + 1)])
    cdf = np.cumsum(p / p.sum())
    r = uniform01(seed, 200, count)
    rank = np.minimum(np.searchsorted(cdf, r, side="right"), ranks - 1)
    return (1 << (first_log2 + rank)).astype(np.int64)


def poisson_arrivals(count: int, rate: float, seed: int = 4) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with `rate` per second."""
    r = uniform01(seed, 300, count)
    gaps = -np.log1p(-r) / rate
    return np.cumsum(gaps)


def config5(n: int = 1 << 25):
    """Two uniform 2^25-limb (2^30-bit, 128 MiB) operands (seed 5)."""
    return random_limbs(5, 1, n), random_limbs(5, 2, n)


def unbalanced(nu: int = 1 << 20, nv: int = 1 << 12):
    """Uniform operands of unequal lengths, 2^20 and 2^12 limbs by default
    (seed 6)."""
    return random_limbs(6, 1, nu), random_limbs(6, 2, nv)


def to_int(limbs) -> int:
    """Python int of a limb vector (for checks on small sizes)."""
    a = np.ascontiguousarray(limbs, dtype=np.uint32)
    return int.from_bytes(a.astype("<u4").tobytes(), "little")


def from_int(x: int, n: int) -> np.ndarray:
    """n limbs of a non-negative Python int (must fit)."""
    if x < 0 or x.bit_length() > 32 * n:
        raise ValueError("value does not fit")
    return np.frombuffer(x.to_bytes(4 * n, "little"), dtype="<u4").astype(np.uint32)
