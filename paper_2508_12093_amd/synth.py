"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws data only; it holds none of the encryption or statistics
arithmetic.  Tests, the benchmark and the CPU reference all take their inputs
from here, so every side sees the same numbers for the same seed.

Workloads (sizes as the paper's experiments, data synthetic because the
paper's datasets are not available here):
  * ``exp1_grid``          the evenly spaced [0.001, 100] grid of Sec. 6.2 (Exp. 1)
  * ``uniform_column``     values ~ U[lo, hi) (Sec. 6.3 draws on [0,100] / [0,20])
  * ``binary_cost_pair``   a binary attribute x ~ Bernoulli(p) and a heavy-tailed
                           cost y = (exp(N(9, 0.8)) + s x) / 1000 with s chosen
                           for a target correlation; shaped like the
                           smoker / charges pair of Sec. 6.4 (charges scaled by 1/1000)
  * ``lognormal_bernoulli_pair`` lognormal(0,1) + s Bernoulli(0.3), for the
                           serving mix of columns with 2^10 .. 2^20 rows
"""
from __future__ import annotations

import math

import numpy as np


def exp1_grid(n: int = 32768) -> np.ndarray:
    """The inverse-square-root test grid of Sec. 6.2 (Exp. 1): n/2 evenly
    spaced points on [0.001, 1] and n/2 on [1, 100] (32768 in the paper)."""
    h = n // 2
    return np.concatenate([np.linspace(0.001, 1.0, h), np.linspace(1.0, 100.0, n - h)])


def uniform_column(seed: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


def binary_cost_pair(seed: int, n: int = 32768, p: float = 0.2, rho: float = 0.79,
                     mu: float = 9.0, sigma: float = 0.8, divisor: float = 1000.0):
    """x ~ Bernoulli(p); y0 = exp(N(mu, sigma)); y = (y0 + s x) / divisor with
    s = rho sqrt(Var y0) / sqrt(p (1-p) (1-rho^2)), so corr(x, y) ~ rho."""
    rng = np.random.default_rng(seed)
    x = (rng.uniform(0.0, 1.0, n) < p).astype(np.float64)
    y0 = np.exp(rng.normal(mu, sigma, n))
    var_y0 = (math.exp(sigma ** 2) - 1.0) * math.exp(2 * mu + sigma ** 2)
    s = rho * math.sqrt(var_y0) / math.sqrt(p * (1 - p) * (1 - rho ** 2))
    y = (y0 + s * x) / divisor
    return x, y


def lognormal_bernoulli_pair(seed: int, n: int, p: float = 0.3, rho: float = 0.5):
    """x ~ Bernoulli(p); y = lognormal(0, 1) + s x with corr(x, y) ~ rho."""
    rng = np.random.default_rng(seed)
    x = (rng.uniform(0.0, 1.0, n) < p).astype(np.float64)
    y0 = rng.lognormal(0.0, 1.0, n)
    var_y0 = (math.e - 1.0) * math.e
    s = rho * math.sqrt(var_y0) / math.sqrt(p * (1 - p) * (1 - rho ** 2))
    return x, y0 + s * x


def slot_batch(seed: int, count: int, slots: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """`count` independent slot vectors ~ U[lo, hi)."""
    return np.random.default_rng(seed).uniform(lo, hi, (count, slots))


def split_column(values: np.ndarray, slots: int):
    """Rows into ceil(n / slots) chunks of `slots` (last one zero-padded)."""
    n = len(values)
    chunks = []
    for c in range(0, max(n, 1), slots):
        part = np.zeros(slots)
        seg = values[c:c + slots]
        part[: len(seg)] = seg
        chunks.append(part)
    return chunks
