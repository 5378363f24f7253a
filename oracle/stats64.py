"""FP64 plaintext statistics (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/ref.py``).

Population moments (ddof = 0), two passes, as defined in Sec. 5:
  ZNorm (Sec. 5.2)  z = (x - mu) / sigma
  Kurt  (Sec. 5.3)  E[(x - mu)^4] / (E[(x - mu)^2])^2   (Tab. 4/5 report it minus 3)
  Skew  (Sec. 5, "mirrors kurtosis")  E[(x - mu)^3] / sigma^3
  CV    (Sec. 5.4)  sigma / mu
  PCC   (Sec. 5.5)  Cov(x, y) / (sigma_x sigma_y)
"""
from __future__ import annotations

import numpy as np


def mean(x):
    return float(np.mean(np.asarray(x, dtype=np.float64)))


def var(x):
    x = np.asarray(x, dtype=np.float64)
    return float(np.mean((x - x.mean()) ** 2))


def zscore(x):
    x = np.asarray(x, dtype=np.float64)
    return (x - x.mean()) / np.sqrt(var(x))


def skewness(x):
    x = np.asarray(x, dtype=np.float64)
    d = x - x.mean()
    return float(np.mean(d ** 3) / np.mean(d ** 2) ** 1.5)


def kurtosis(x, excess=False):
    x = np.asarray(x, dtype=np.float64)
    d = x - x.mean()
    k = float(np.mean(d ** 4) / np.mean(d ** 2) ** 2)
    return k - 3.0 if excess else k


def cv(x):
    x = np.asarray(x, dtype=np.float64)
    return float(np.sqrt(var(x)) / x.mean())


def pearson(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    dx = x - x.mean()
    dy = y - y.mean()
    return float(np.mean(dx * dy) / np.sqrt(np.mean(dx * dx) * np.mean(dy * dy)))


def mre(approx, exact, floor_frac=1e-3):
    """Mean relative error; for vectors only entries with |y| >= floor_frac *
    max|y| count (relative error is ill-conditioned near 0)."""
    a = np.atleast_1d(np.asarray(approx, dtype=np.float64))
    e = np.atleast_1d(np.asarray(exact, dtype=np.float64))
    keep = np.abs(e) >= floor_frac * np.max(np.abs(e))
    return float(np.mean(np.abs(a[keep] - e[keep]) / np.abs(e[keep])))
