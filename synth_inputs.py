"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers: it holds none of the multiplication's
arithmetic, so both the oracle side and the GPU side may take their inputs
from it without sharing any computation.  Every generator is
``numpy.random.Generator(PCG64(seed))``; the default base seed is 1911, with A
drawn from ``seed`` and B from ``seed + 1``.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 1911
INF = 1 << 30  # sentinel infinity of the integer semirings


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_f32(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """i.i.d. uniform[lo, hi) float32."""
    return rng(seed).uniform(lo, hi, size=shape).astype(np.float32)


def normal_f32(seed: int, shape) -> np.ndarray:
    """i.i.d. N(0, 1) float32."""
    return rng(seed).standard_normal(size=shape, dtype=np.float32)


def small_int_f32(seed: int, shape, bound: int = 8) -> np.ndarray:
    """Integers in [-bound, bound] stored as float32 (exact in bf16/fp16/fp32)."""
    return rng(seed).integers(-bound, bound + 1, size=shape).astype(np.float32)


def row_scale_exponents(seed: int, rows: int, span: float = 3.0) -> np.ndarray:
    """u_i ~ U(-span, span): row i is multiplied by 10**u_i."""
    return rng(seed).uniform(-span, span, size=rows)


def row_scaled_normal_f32(seed: int, shape, span: float = 3.0) -> np.ndarray:
    """N(0,1) matrix whose row i is scaled by 10**U(-span, span)."""
    x = normal_f32(seed, shape).astype(np.float64)
    u = row_scale_exponents(seed + 1000003, shape[0], span)
    return (x * (10.0 ** u)[:, None]).astype(np.float32)


def minplus_i32(seed: int, shape, bits: int = 20, frac_inf: float = 0.1) -> np.ndarray:
    """(min,+) operand: uniform integers in [0, 2**bits), then each entry
    independently (probability frac_inf) replaced by the sentinel INF = 2**30."""
    g = rng(seed)
    x = g.integers(0, 1 << bits, size=shape, dtype=np.int64)
    mask = g.random(size=shape) < frac_inf
    x[mask] = INF
    return x.astype(np.int32)


def maxplus_i32(seed: int, shape, bits: int = 20, frac_inf: float = 0.1) -> np.ndarray:
    """(max,+) operand: the (min,+) recipe negated, so -INF = -2**30."""
    return (-minplus_i32(seed, shape, bits, frac_inf).astype(np.int64)).astype(np.int32)


I32_MIN, I32_MAX = -(1 << 31), (1 << 31) - 1


def maxmin_i32(seed: int, shape, frac_zero: float = 0.1) -> np.ndarray:
    """(max, min) operand: uniform over all int32 values, then each entry
    independently (probability frac_zero) set to the smallest int32 (the
    semiring's zero: no edge)."""
    g = rng(seed)
    x = g.integers(I32_MIN, I32_MAX, size=shape, dtype=np.int64, endpoint=True)
    x[g.random(size=shape) < frac_zero] = I32_MIN
    return x.astype(np.int32)


def bool_i32(seed: int, shape, density: float = 0.1) -> np.ndarray:
    """Boolean operand: each entry 1 with probability density, else 0."""
    return (rng(seed).random(size=shape) < density).astype(np.int32)


def semiring_operand(sr: int, seed: int, shape, bits: int = 20, frac_inf: float = 0.1):
    """Operand for semiring kind sr (1 = (min,+), 2 = (max,+), 3 = (max, min),
    4 = Boolean (or, and))."""
    if sr == 1:
        return minplus_i32(seed, shape, bits, frac_inf)
    if sr == 2:
        return maxplus_i32(seed, shape, bits, frac_inf)
    if sr == 3:
        return maxmin_i32(seed, shape, frac_inf)
    if sr == 4:
        return bool_i32(seed, shape)
    raise ValueError("integer semiring kinds are 1 to 4")


def wide_i32(sr: int, seed: int, shape, bits: int = 20, frac_inf: float = 0.1, frac_extreme: float = 0.05):
    """Operand over the checked (wider) domain of (min,+) (sr 1) or (max,+)
    (sr 2): integers of either sign in [-2^bits, 2^bits), a fraction frac_inf
    set to the sentinel (INF, resp. -INF) and a fraction frac_extreme drawn
    from the whole domain ([-2^30, 2^30) for (min,+), [-2^30 + 1, 2^30 - 1]
    for (max,+)) so that sums reach both ends."""
    g = rng(seed)
    x = g.integers(-(1 << bits), 1 << bits, size=shape, dtype=np.int64)
    lo = -INF if sr == 1 else -INF + 1
    ext = g.integers(lo, INF, size=shape, dtype=np.int64)
    u = g.random(size=shape)
    x = np.where(u < frac_extreme, ext, x)
    x = np.where(u > 1.0 - frac_inf, INF if sr == 1 else -INF, x)
    return x.astype(np.int32)


def semiring_init(sr: int, shape) -> np.ndarray:
    """C0 filled with the additive identity (+INF for (min,+), -INF for
    (max,+), the smallest int32 for (max, min), 0 for Boolean)."""
    zero = {1: INF, 2: -INF, 3: I32_MIN, 4: 0}[sr]
    return np.full(shape, zero, dtype=np.int32)


def log_uniform_ints(seed: int, count: int, lo: int, hi: int, dims: int = 3) -> np.ndarray:
    """count x dims integers round(exp(U(ln lo, ln hi))), independently per dim."""
    g = rng(seed)
    x = np.exp(g.uniform(math.log(lo), math.log(hi), size=(count, dims)))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def batched_shapes(seed: int = BASE_SEED, count: int = 512, lo: int = 64, hi: int = 4096):
    """Uneven batch: (m, n, k) each log-uniform in [lo, hi]."""
    return log_uniform_ints(seed, count, lo, hi, 3)


def tuner_shapes(seed: int, count: int, lo: int = 128, hi: int = 16384):
    """Shapes for the schedule tuner / cost model: (m, n, k) log-uniform in [lo, hi]."""
    return log_uniform_ints(seed, count, lo, hi, 3)


def log_uniform_floats(seed: int, count: int, lo: float, hi: float) -> np.ndarray:
    g = rng(seed)
    return np.exp(g.uniform(math.log(lo), math.log(hi), size=count))
