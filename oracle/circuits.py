"""Encrypted-statistics circuits of PP-STAT, oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/ref.py``).

Each function below is one fixed sequence of CKKS operations.  The GPU library
implements the same sequences independently; the two agree bit for bit because
every operation is exact integer arithmetic on the same inputs and the sequence
(including every level alignment and every constant) is fixed here:

* binary operations on operands at different levels first bring the higher
  one down to the lower level (``level_align``);
* sums over lists fold left to right;
* FP64 constants are formed exactly as written (e.g. ``1.0 / (B * n)``).

Circuits (paper references):
  mean_B      Mean(x, B) = sum x_i / (B n) (ciphertexts added, then scaled) Sec. 5.1
  variance_B  Variance(x, B) = sum (x_i / (B sqrt n))^2 - Mean(x,B)^2  Sec. 5.1, Eq. 2
  inv_sqrt    Chebyshev initial value (Alg. 3, Eq. 3) + Newton (Alg. 2, n = 2)
  invsqrt     CryptoInvSqrt of x / B slot by slot (Sec. 6.2, Exp. 1)
  zscore      Alg. 4;  kurtosis Alg. 5;  skewness (mirror of Alg. 5, Sec. 5)
  cv          Alg. 6 with a g_3-composition sign (Sec. 6.2)
  pearson     Sec. 5.5: Cov_B * InvSqrt(Var_B x) * InvSqrt(Var_B y), Eq. 2's
              pre-scaled moments, the five slot sums summed together

Readings where the paper is silent or inconsistent:
  * Newton (Alg. 2) is evaluated in a balanced order that costs two levels per
    step: y2 = y*y, p1 = w2*y, p2 = p1*y2, y = 1.5 y - p2, with w2 = (B'/2) v
    formed once.  Mathematically identical to Alg. 2 for n = 2.
  * Alg. 3 squares the initial value for n == 1 (the text: Inv = InvSqrt^2);
    for the inverse square root (n == 2) the Chebyshev value is used directly.
  * Alg. 6 calls CryptoSqrt(var, B); since Variance(x, B) = Var/B^2 the factor
    must be B^2, as in Alg. 4 and 5.  sqrt is evaluated as 2 * w2 * InvSqrt(v).
  * The PCC circuit (deferred by the paper to another work) is
    Cov * InvSqrt(Var x) * InvSqrt(Var y) with the moments in Eq. 2's
    pre-scaled form, Cov_B = E[xy]/(Bx By) - Mean(x, Bx) Mean(y, By).
  * Slots beyond the row count are zero; centred moments use a 1/n-valued row
    mask (a constant when a ciphertext is full, a plaintext vector otherwise).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import cheb
from .ref import Ciphertext, Oracle


@dataclass
class InvSqrtCfg:
    a: float = 1e-3
    b: float = 1.0
    degree: int = 7
    iters: int = 3
    coeffs: np.ndarray | None = None   # optional explicit c_0..c_d for B' = 1
    # refresh levels by bootstrapping inside InvSqrt (the evaluator's
    # ``refresh``): see ``Circuits.inv_sqrt``
    boot: bool = False

    def coeffs_for(self, Bp: float) -> np.ndarray:
        if self.coeffs is not None:
            base = np.asarray(self.coeffs, dtype=np.float64)
            return base / math.sqrt(Bp)
        return cheb.invsqrt_coeffs(self.a, self.b, self.degree, Bp)


# ----------------------------------------------------------------------------
# evaluators: encrypted (over the C oracle) and plain FP64 slots with levels
# ----------------------------------------------------------------------------
class EncEval:
    """Evaluator over encrypted oracle ciphertexts.  ``booter``: an
    ``oracle.boot.Bootstrapper`` for InvSqrt's refreshes."""

    def __init__(self, O: Oracle, rlk, gkeys, booter=None):
        self.O, self.rlk, self.gkeys = O, rlk, gkeys
        self.slots = O.P.slots
        self.booter = booter

    def refresh(self, x):
        """Level 0, then bootstrapped to the top computation level."""
        if self.booter is None:
            raise ValueError("no bootstrapper")
        return self.booter.bootstrap(self.O.level_align(x, 0))

    def level(self, x):
        return x.level

    def align(self, x, level):
        return self.O.level_align(x, level)

    def add(self, a, b):
        return self.O.add(a, b)

    def sub(self, a, b):
        return self.O.sub(a, b)

    def mul(self, a, b):
        return self.O.mul(a, b, self.rlk)

    def mul_const(self, a, c):
        return self.O.mul_const(a, c)

    def mul_int(self, a, k):
        return self.O.mul_int(a, k)

    def lincomb(self, xs, cs, level):
        return self.O.lincomb(xs, cs, level)

    def add_const(self, a, c):
        return self.O.add_const(a, c)

    def mul_vec(self, a, vec):
        pt = self.O.encode(vec, a.level)
        return self.O.mul_plain(a, pt)

    def rotsum(self, a):
        # The circuits' slot sums use the hoisted radix-8 rotate-and-sum (five
        # steps at N = 2^16), the form the library runs; tests pin it to the
        # plain definition ``Oracle.rotsum`` (serial ct + Rot(ct, 2^k)) by
        # decryption within the key-switching noise.
        return self.O.rotsum_hoisted8(a, self.gkeys)


class PlainEval:
    """FP64 model: slot vectors carrying the same level bookkeeping."""

    @dataclass
    class V:
        v: np.ndarray
        level: int

    def __init__(self, L, slots, Lc=None):
        self.L, self.slots = L, slots
        self.Lc = L if Lc is None else Lc

    def refresh(self, x):
        return PlainEval.V(x.v, self.Lc)

    def fresh(self, values):
        v = np.zeros(self.slots)
        v[: len(values)] = values
        return PlainEval.V(v, self.L)

    def level(self, x):
        return x.level

    def align(self, x, level):
        assert level <= x.level
        return PlainEval.V(x.v, level)

    def _chk(self, a, b):
        assert a.level == b.level

    def add(self, a, b):
        self._chk(a, b)
        return PlainEval.V(a.v + b.v, a.level)

    def sub(self, a, b):
        self._chk(a, b)
        return PlainEval.V(a.v - b.v, a.level)

    def mul(self, a, b):
        self._chk(a, b)
        assert a.level >= 1
        return PlainEval.V(a.v * b.v, a.level - 1)

    def mul_const(self, a, c):
        assert a.level >= 1
        return PlainEval.V(a.v * c, a.level - 1)

    def mul_int(self, a, k):
        return PlainEval.V(a.v * k, a.level)

    def lincomb(self, xs, cs, level):
        assert all(x.level > level for x in xs)
        return PlainEval.V(sum(c * x.v for x, c in zip(xs, cs)), level)

    def add_const(self, a, c):
        return PlainEval.V(a.v + c, a.level)

    def mul_vec(self, a, vec):
        return PlainEval.V(a.v * np.asarray(vec), a.level - 1)

    def rotsum(self, a):
        return PlainEval.V(np.full(self.slots, a.v.sum()), a.level)


# ----------------------------------------------------------------------------
# circuits
# ----------------------------------------------------------------------------
class Circuits:
    def __init__(self, ev):
        self.ev = ev

    # helpers ------------------------------------------------------------
    def _lower(self, a, b):
        ev = self.ev
        m = min(ev.level(a), ev.level(b))
        return ev.align(a, m), ev.align(b, m)

    def addx(self, a, b):
        return self.ev.add(*self._lower(a, b))

    def subx(self, a, b):
        return self.ev.sub(*self._lower(a, b))

    def mulx(self, a, b):
        return self.ev.mul(*self._lower(a, b))

    def sumx(self, xs):
        acc = xs[0]
        for x in xs[1:]:
            acc = self.addx(acc, x)
        return acc

    def mask_mean(self, zs, n):
        """RotSum(sum_c Z_c * mask_c) with mask_c = 1/n on rows < n, else 0:
        the full ciphertexts are added first and scaled by 1/n once; a ragged
        last one is multiplied by its 1/n row mask."""
        S = self.ev.slots
        full, terms = [], []
        for c, z in enumerate(zs):
            rows = min(S, n - c * S)
            if rows == S:
                full.append(z)
            else:
                vec = np.zeros(S)
                vec[:rows] = 1.0 / float(n)
                terms.append(self.ev.mul_vec(z, vec))
        if full:
            terms.insert(0, self.ev.mul_const(self.sumx(full), 1.0 / float(n)))
        return self.ev.rotsum(self.sumx(terms))

    # Sec. 5.1 -------------------------------------------------------------
    def mean_B(self, X, n, B):
        """Mean(x, B) = sum_i x_i / (B n)."""
        c = 1.0 / (B * float(n))
        return self.ev.rotsum(self.ev.mul_const(self.sumx(X), c))

    def variance_B(self, X, n, B, mean_term):
        """Variance(x, B) = sum (x_i / (B sqrt n))^2 - mean_term^2  (Eq. 2)."""
        c = 1.0 / (B * math.sqrt(float(n)))
        xs = [self.ev.mul_const(x, c) for x in X]
        e2 = self.ev.rotsum(self.sumx([self.ev.mul(x, x) for x in xs]))
        m2 = self.ev.mul(mean_term, mean_term)
        return self.subx(e2, m2)

    # Alg. 3 + Alg. 2 -------------------------------------------------------
    def cheb_series(self, t, coeffs, d):
        """sum_{k<=d} c_k T_k(t): T_1 = t, T_2m = 2 T_m^2 - 1,
        T_2m+1 = 2 T_m T_m+1 - T_1 (each the product of two lower terms, so
        T_k sits ceil(log2 k) levels below t), then c_1..c_d combined at one
        level below the lowest T_k with one rescale, and c_0 added."""
        ev = self.ev
        if d == 0:      # a constant initial value: 0 t + c_0 (t's level)
            return ev.add_const(ev.mul_int(t, 0), float(coeffs[0]))
        T = {1: t}
        for k in range(2, d + 1):
            if k % 2 == 0:
                m = k // 2
                T[k] = ev.add_const(ev.mul_int(ev.mul(T[m], T[m]), 2), -1.0)
            else:
                m = (k - 1) // 2
                T[k] = self.subx(ev.mul_int(self.mulx(T[m], T[m + 1]), 2), T[1])
        y = ev.lincomb([T[k] for k in range(1, d + 1)], [float(coeffs[k]) for k in range(1, d + 1)],
                       min(ev.level(T[k]) for k in range(1, d + 1)) - 1)
        return ev.add_const(y, float(coeffs[0]))

    def inv_sqrt(self, v, Bp, cfg: InvSqrtCfg, reserve: int = 0):
        """y ~ 1/sqrt(Bp v); returns (y, w2) with w2 = (Bp/2) v.

        With cfg.boot, levels are refreshed (level 0, then bootstrap; Alg. 3
        bootstraps the initial value, the rest is the reading of where the
        chain runs out): v when it has fewer levels than the affine map, the
        ladder (T_d lies ceil(log2 d) levels down) and the weighted sum take;
        the initial value always; w2 and y before a Newton step when either
        has fewer than the step's two levels; y at the end when fewer than
        `reserve` levels (what the statistic uses after InvSqrt) remain."""
        ev = self.ev
        a, b, d = cfg.a, cfg.b, cfg.degree
        coeffs = cfg.coeffs_for(Bp)
        # the affine map onto [-1, 1]; a pure shift (b - a = 2, Eq. 1's
        # x - 1 on [0, 2]) needs no product and no level
        g = 2.0 / (b - a)
        if cfg.boot:
            ladder = (d - 1).bit_length() if d >= 1 else 0      # ceil(log2 d)
            if ev.level(v) < (0 if g == 1.0 else 1) + (ladder + 1 if d >= 1 else 0):
                v = ev.refresh(v)
        t = ev.add_const(v if g == 1.0 else ev.mul_const(v, g), -(a + b) / (b - a))
        y = self.cheb_series(t, coeffs, d)
        if cfg.boot and d >= 1:
            y = ev.refresh(y)
        w2 = ev.mul_const(v, Bp / 2.0)
        for _ in range(cfg.iters):
            if cfg.boot:
                if ev.level(w2) < 2:
                    w2 = ev.refresh(w2)
                if ev.level(y) < 2:
                    y = ev.refresh(y)
            y2 = ev.mul(y, y)
            p1 = self.mulx(w2, y)
            p2 = self.mulx(p1, y2)
            y = self.subx(ev.lincomb([y], [1.5], ev.level(p2)), p2)
        if cfg.boot and ev.level(y) < reserve:
            y = ev.refresh(y)
        return y, w2

    def invsqrt(self, X, B, cfg: InvSqrtCfg):
        """CryptoInvSqrt of every slot (Sec. 4, Alg. 2-3; Sec. 6.2, Exp. 1):
        v = x / B (the scaling of the input domain), y = InvSqrt(v; B), so
        y ~ 1/sqrt(x).  One output per input ciphertext."""
        return [self.inv_sqrt(self.ev.mul_const(x, 1.0 / B), B, cfg)[0] for x in X]

    def sqrt(self, v, Bp, cfg: InvSqrtCfg, reserve: int = 0):
        """sqrt(Bp v) = 2 * w2 * InvSqrt(v; Bp)."""
        y, w2 = self.inv_sqrt(v, Bp, cfg, reserve)
        return self.ev.mul_int(self.mulx(w2, y), 2)

    def g3(self, x):
        """g_3 at depth 3: u = x^2, w = u^2; each term puts its constant on x."""
        ev = self.ev
        u = ev.mul(x, x)
        w = ev.mul(u, u)
        a1 = ev.mul_const(x, 35.0 / 16.0)
        a3 = self.mulx(ev.mul_const(x, -35.0 / 16.0), u)
        a5 = self.mulx(ev.mul_const(x, 21.0 / 16.0), w)
        a7 = self.mulx(self.mulx(ev.mul_const(x, -5.0 / 16.0), u), w)
        return self.sumx([a1, a3, a5, a7])

    def sign(self, x, k):
        for _ in range(k):
            x = self.g3(x)
        return x

    def moments_B(self, X, n, B_mean, B_var):
        """Mean(x, B_mean) and Variance(x, B_var) (Eq. 2) with one RotSum for
        both: the variance's slot sum sum (x_i / (B_var sqrt n))^2 does not
        need the mean, so the mean's sum is brought to its level and the two
        are summed together; Var = E2 - m^2 with m = Mean(x, B_var)."""
        ev = self.ev
        s1 = ev.mul_const(self.sumx(X), 1.0 / (B_mean * float(n)))
        c = 1.0 / (B_var * math.sqrt(float(n)))
        xs = [ev.mul_const(x, c) for x in X]
        s2 = self.sumx([ev.mul(x, x) for x in xs])
        muB = ev.rotsum(ev.align(s1, ev.level(s2)))
        e2 = ev.rotsum(s2)
        m = muB if B_var == B_mean else ev.mul_const(muB, B_mean / B_var)
        return muB, self.subx(e2, ev.mul(m, m))

    # statistics ------------------------------------------------------------
    def _moments_prefix(self, X, n, B):
        muB, var = self.moments_B(X, n, B, B)
        mu = self.ev.mul_const(muB, B)
        return muB, var, mu

    def zscore(self, X, n, B, cfg: InvSqrtCfg):
        """Alg. 4: (X - mu) * InvSqrt(Variance(X, B); B^2), one output per ciphertext."""
        _, var, mu = self._moments_prefix(X, n, B)
        b, _ = self.inv_sqrt(var, B * B, cfg, 1)
        return [self.mulx(self.subx(x, mu), b) for x in X]

    def kurtosis(self, X, n, B, cfg: InvSqrtCfg, excess=False):
        """Alg. 5: Mean((X - mu)^4) * InvSqrt(Variance(X,B); B^2)^4."""
        ev = self.ev
        _, var, mu = self._moments_prefix(X, n, B)
        x1 = [self.subx(x, mu) for x in X]
        x2 = [ev.mul(x, x) for x in x1]
        x4 = [ev.mul(x, x) for x in x2]
        num = self.mask_mean(x4, n)
        i, _ = self.inv_sqrt(var, B * B, cfg, 3)
        i2 = ev.mul(i, i)
        # (num i^2) i^2: every partial product stays near the result's size
        # (i^4 alone is ~1/Var^2, small enough to lose digits to the noise)
        k = self.mulx(self.mulx(num, i2), i2)
        return ev.add_const(k, -3.0) if excess else k

    def skewness(self, X, n, B, cfg: InvSqrtCfg):
        """Mirror of Alg. 5: Mean((X - mu)^3) * InvSqrt(Variance(X,B); B^2)^3."""
        ev = self.ev
        _, var, mu = self._moments_prefix(X, n, B)
        x1 = [self.subx(x, mu) for x in X]
        x2 = [ev.mul(x, x) for x in x1]
        x3 = [self.mulx(a, b) for a, b in zip(x2, x1)]
        num = self.mask_mean(x3, n)
        i, _ = self.inv_sqrt(var, B * B, cfg, 2)
        i2 = ev.mul(i, i)
        return self.mulx(self.mulx(num, i), i2)

    def cv(self, X, n, B_mean, B_var, cfg: InvSqrtCfg, sign_k=2):
        """Alg. 6: Std * InvSqrt(mu * sign(mu); B_mean)^2 * sign(mu).  With
        cfg.boot the sign is refreshed before a g_3 step (depth 3) it lacks
        the levels for and after the last step when below 3 levels; the
        inverse mean and the standard deviation keep 3 levels."""
        ev = self.ev
        muB, var = self.moments_B(X, n, B_mean, B_var)
        sg = muB
        for _ in range(sign_k):
            if cfg.boot and ev.level(sg) < 3:
                sg = ev.refresh(sg)
            sg = self.g3(sg)
        if cfg.boot and ev.level(sg) < 3:
            sg = ev.refresh(sg)
        ia, _ = self.inv_sqrt(self.mulx(muB, sg), B_mean, cfg, 3)
        mu_inv = ev.mul(ia, ia)
        sigma = self.sqrt(var, B_var * B_var, cfg, 3)
        return self.mulx(self.mulx(sigma, mu_inv), sg)

    def pearson(self, X, Y, n, Bx, By, cfg: InvSqrtCfg):
        """Sec. 5.5, Cov(X, Y) / (sd X sd Y), with every moment in Eq. 2's
        pre-scaled form: Mean(x, Bx) = sum x_i / (Bx n), Var_B = sum (x_i /
        (Bx sqrt n))^2 - Mean^2 and Cov_B = sum (x_i / (Bx sqrt n)) (y_i /
        (By sqrt n)) - Mean(x) Mean(y) = Cov / (Bx By); then
        PCC = Cov_B * InvSqrt(Var_B x; 1) * InvSqrt(Var_B y; 1).  None of the
        five slot sums depends on another, so they are formed first, brought
        to one level and summed together."""
        ev = self.ev
        sx = ev.mul_const(self.sumx(X), 1.0 / (Bx * float(n)))
        sy = ev.mul_const(self.sumx(Y), 1.0 / (By * float(n)))
        xs = [ev.mul_const(x, 1.0 / (Bx * math.sqrt(float(n)))) for x in X]
        ys = [ev.mul_const(y, 1.0 / (By * math.sqrt(float(n)))) for y in Y]
        sxx = self.sumx([ev.mul(a, a) for a in xs])
        syy = self.sumx([ev.mul(b, b) for b in ys])
        sxy = self.sumx([ev.mul(a, b) for a, b in zip(xs, ys)])
        lv = ev.level(sxx)
        mx, my, exx, eyy, exy = [ev.rotsum(ev.align(v, lv)) for v in (sx, sy, sxx, syy, sxy)]
        varx = self.subx(exx, ev.mul(mx, mx))
        vary = self.subx(eyy, ev.mul(my, my))
        cov = self.subx(exy, ev.mul(mx, my))
        ix, _ = self.inv_sqrt(varx, 1.0, cfg, 2)
        iy, _ = self.inv_sqrt(vary, 1.0, cfg, 2)
        return self.mulx(cov, ev.mul(ix, iy))
