"""Chebyshev initial values for the inverse square root (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/ref.py``).

CryptoInvSqrt (Sec. 4.1, Alg. 3; Sec. 4.2, Eq. 1; Sec. 5.1, Eq. 3) starts
Newton's iteration from a Chebyshev approximation of the inverse square root.
The paper does not say which Chebyshev construction it uses; the reading taken
here is interpolation at the first-kind nodes cos(pi (k + 1/2) / (d + 1)),
which is what ``numpy.polynomial.chebyshev.chebinterpolate`` computes.  With
that reading the Experiment-1 set-up (Tab. 2: degree 31, six Newton steps,
B = 100, the 32768-point grid on [0.001, 100]) reproduces the printed MRE.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as C


def invsqrt_coeffs(a: float, b: float, degree: int, Bp: float) -> np.ndarray:
    """Coefficients c_0..c_d (first kind) of f(v) = 1/sqrt(Bp v) on [a, b],
    in the variable t = (2 v - a - b) / (b - a) on [-1, 1]."""
    if not (0.0 < a < b):
        raise ValueError("need 0 < a < b")

    def f(t):
        v = a + (b - a) * (t + 1.0) / 2.0
        return 1.0 / np.sqrt(Bp * v)

    return C.chebinterpolate(f, degree)


def paper_invsqrt_coeffs(degree: int, B: float) -> np.ndarray:
    """Eq. 3: F(x, B) = 1 / (sqrt(B) sqrt(x + 1)) on [-1, 1] (the domain map of
    Eq. 1 shifts [0, 2] onto [-1, 1]); the input is x = v/B - 1."""
    def f(x):
        return 1.0 / (np.sqrt(B) * np.sqrt(x + 1.0))

    return C.chebinterpolate(f, degree)


def paper_sqrt_coeffs(degree: int, B: float) -> np.ndarray:
    """Eq. 4: F(x, B) = sqrt(B) sqrt(x + 1) on [-1, 1]."""
    def f(x):
        return np.sqrt(B) * np.sqrt(x + 1.0)

    return C.chebinterpolate(f, degree)


def newton_invsqrt(x: np.ndarray, y: np.ndarray, iters: int) -> np.ndarray:
    """Alg. 1 (Sec. 3.3): y_i = 0.5 y_{i-1} (3 - x y_{i-1}^2)."""
    for _ in range(iters):
        y = 0.5 * y * (3.0 - x * y * y)
    return y


def g3(x):
    """g_3(x) = (35 x - 35 x^3 + 21 x^5 - 5 x^7) / 16 (Sec. 6.2)."""
    return (35.0 * x - 35.0 * x ** 3 + 21.0 * x ** 5 - 5.0 * x ** 7) / 16.0


G3_COEFFS = {1: 35.0 / 16.0, 3: -35.0 / 16.0, 5: 21.0 / 16.0, 7: -5.0 / 16.0}


def exp1_grid(n: int = 32768) -> np.ndarray:
    """Experiment 1 (Sec. 6.2): n/2 evenly spaced points on [0.001, 1] and
    n/2 on [1, 100] (16384 each in the paper)."""
    h = n // 2
    return np.concatenate([np.linspace(0.001, 1.0, h), np.linspace(1.0, 100.0, n - h)])


def exp1_model(v: np.ndarray, degree: int = 31, iters: int = 6, B: float = 100.0) -> np.ndarray:
    """FP64 model of Tab. 2's CryptoInvSqrt row: Chebyshev initial value of
    Eq. 3 on x = v/B - 1, then `iters` Newton steps on v."""
    c = paper_invsqrt_coeffs(degree, B)
    return newton_invsqrt(v, C.chebval(v / B - 1.0, c), iters)


def exp1_mre(degree: int = 31, iters: int = 6, B: float = 100.0) -> float:
    """MRE of ``exp1_model`` against 1/sqrt(v) over the Exp. 1 grid."""
    v = exp1_grid()
    y = exp1_model(v, degree, iters, B)
    ref = 1.0 / np.sqrt(v)
    return float(np.mean(np.abs(y - ref) / np.abs(ref)))


def evalmod_cos_coeffs(K: int, r: int, degree: int) -> np.ndarray:
    """Coefficients c_0..c_d (first kind) of cos(2 pi (K u - 1/4) / 2^r) on
    u in [-1, 1], interpolated at the first-kind nodes: EvalMod's polynomial
    (bootstrapping, Sec. 3.2; Sec. 3.4 names Chebyshev approximation
    of the sine in the modular reduction).  r double angles y <- 2 y^2 - 1
    turn it into cos(2 pi K u - pi/2) = sin(2 pi x) at x = K u, which is
    2 pi (x - I) + O((x - I)^3) near every integer I."""
    def f(u):
        return np.cos(2.0 * np.pi * (K * u - 0.25) / float(2 ** r))

    return C.chebinterpolate(f, degree)
