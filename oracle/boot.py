"""CKKS bootstrapping, oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/ref.py``).

The paper relies on bootstrapping to refresh a ciphertext whose levels are
spent (Sec. 3.2; Alg. 3 bootstraps the Chebyshev initial value; Tab. 1 gives
its cost) and takes the construction from the cited work (Cheon et al. 2018,
Chen-Chillotti-Song 2019, Han-Ki 2020).  This module writes that construction
out over the oracle's operations, in this order:

  ModRaise     the level-0 ciphertext's residues mod q_0, lifted to (-q_0/2, q_0/2]
               and read mod q_0..q_L: it now decrypts to t = c + q_0 I, where
               c is the old plaintext polynomial and I a small integer one
  CoeffToSlot  the inverse decoding map BR U0^H / n (``boot_ref.c``) in
               ``len(groups)`` levels, each a baby-step giant-step sum of
               rotated diagonals and one rescale; its constant also divides by
               2 K q_0 so that the slots hold (t_k + i t_{k+n}) / (2 K q_0)
               (bit-reversed slot order)
  real/imag    re = w + conj(w), im = -X^n (w - conj(w)) (conjugation is the
               automorphism X -> X^(2N-1); X^n acts on every slot as i), so
               re, im hold u = x / K with x = t_k / q_0 in [-K, K]
  EvalMod      y = cos(2 pi (K u - 1/4) / 2^r) by Chebyshev interpolation,
               then r double angles y <- 2 y^2 - 1: y = sin(2 pi x), which is
               2 pi (x - I) = 2 pi c_k / q_0 up to a cubic term
  recombine    w' = y_re + X^n y_im
  SlotToCoeff  the decoding map U0 BR (``boot_ref.c``) in ``len(groups)``
               levels, with the constant q_0 / (2 pi Delta_0) spread evenly
               over them: the slots return to the old message at Delta_Lc.

Readings (the paper gives none of this; the design doc lists them):
  * sparse ternary secret of weight h (64), so that |I| stays below K = 16;
  * the layer groups: log2(n) layers split into three, the larger groups on
    the side of len = n; a group reaching len = n indexes its diagonals by
    offset mod n (2^g of them), any other by m in [-(2^g - 1), 2^g - 1];
  * baby steps b = 2^ceil(ceil(log2 R) / 2) for R offsets, G = ceil(R / b)
    giant steps; baby rotations hoisted (one ModUp), giant rotations plain,
    applied to the unrescaled inner sums, one rescale per group;
  * EvalMod: K = 16, r = 4 double angles, degree 27 (T-ladder depth 5, the
    combination one more, the double angles four: 10 levels);
  * every constant a group carries is folded into its plaintexts at the
    scale that takes Delta_l to Delta_{l-1} through one rescale.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cheb
from .circuits import Circuits, EncEval
from .ref import Ciphertext, Oracle, Plaintext, _p, galois_element


@dataclass
class Group:
    inverse: int          # 1: CoeffToSlot (conjugate layers), 0: SlotToCoeff
    lo: int               # layers len = 2^lo .. 2^hi
    hi: int
    level: int            # the level the group runs at (it ends one lower)
    ckind: int            # constant: 0 none, 1 CoeffToSlot's, 2 SlotToCoeff's share
    u: int                # offset unit: 2^(lo-1) slots
    m0: int               # first offset index
    b: int                # baby steps
    G: int                # giant steps

    def baby_steps(self, n):
        return [(self.u * i) % n for i in range(self.b)]

    def giant_step(self, j, n):
        return (self.u * (self.m0 + self.b * j)) % n


@dataclass
class Plan:
    K: int = 16
    r: int = 4
    degree: int = 27
    cts: list = field(default_factory=list)
    stc: list = field(default_factory=list)

    def rotations(self, n):
        """Every rotation step (mod n, nonzero) the transforms use."""
        out = set()
        for g in self.cts + self.stc:
            out.update(s for s in g.baby_steps(n) if s)
            out.update(g.giant_step(j, n) for j in range(g.G) if g.giant_step(j, n))
        return sorted(out)


def split_layers(logn: int, parts: int = 3):
    """Layer ranges (lo, hi) from the top (len = n) down; the larger parts on top."""
    q, r = divmod(logn, parts)
    sizes = [q + 1] * r + [q] * (parts - r)
    out, hi = [], logn
    for s in sizes:
        out.append((hi - s + 1, hi))
        hi -= s
    return out


def make_group(inverse, lo, hi, logn, level, ckind) -> Group:
    g = hi - lo + 1
    u = 1 << (lo - 1)
    if hi == logn:
        m0, R = 0, 1 << g
    else:
        m0, R = -((1 << g) - 1), (1 << (g + 1)) - 1
    bits = (R - 1).bit_length()
    b = 1 << ((bits + 1) // 2)
    G = -(-R // b)
    return Group(inverse, lo, hi, level, ckind, u, m0, b, G)


def make_plan(P) -> Plan:
    C, E, S = P.boot
    logn = P.slots.bit_length() - 1
    ranges = split_layers(logn, C)
    assert len(ranges) == C and S == C
    plan = Plan()
    # CoeffToSlot acts with the top layers first, at levels L, L-1, ...
    for t, (lo, hi) in enumerate(ranges):
        plan.cts.append(make_group(1, lo, hi, logn, P.L - t, 1 if t == 0 else 0))
    # SlotToCoeff acts with the bottom layers first, at levels Lc+S, ..., Lc+1
    for t, (lo, hi) in enumerate(reversed(ranges)):
        plan.stc.append(make_group(0, lo, hi, logn, P.Lc + S - t, 2))
    assert E == plan.degree.bit_length() + 1 + plan.r
    return plan


class Bootstrapper:
    def __init__(self, O: Oracle, sk, seed: int, plan: Plan | None = None, coeffs=None):
        P = O.P
        if not P.boot:
            raise ValueError("parameter set without bootstrapping levels")
        self.O, self.P = O, P
        self.plan = plan or make_plan(P)
        self.n = P.slots
        self.rlk = O.relin_key(sk, seed)
        self.gkeys = O.rotation_keys(sk, seed, self.plan.rotations(self.n))
        self.g_conj = 2 * P.N - 1
        self.gkeys[self.g_conj] = O.galois_key(sk, seed, self.g_conj)
        pl = self.plan
        self.coeffs = (np.asarray(coeffs, dtype=np.float64) if coeffs is not None
                       else cheb.evalmod_cos_coeffs(pl.K, pl.r, pl.degree))
        self.grids = {id(g): self.grid(g) for g in pl.cts + pl.stc}
        self.circ = Circuits(EncEval(O, self.rlk, self.gkeys))

    # ------------------------------------------------------------ plaintexts
    def grid_coeffs(self, g: Group):
        """Integer coefficients [G*b][N] and used flags of a group's cells."""
        P = self.P
        out = np.zeros((g.G * g.b, P.N), dtype=np.int64)
        used = np.zeros(g.G * g.b, dtype=np.int8)
        C = P.boot[0]
        rc = self.O.L.orc_boot_grid(P.ref, g.inverse, g.lo, g.hi, g.level, g.ckind, self.plan.K, C,
                                    g.u, g.m0, g.b, g.G, _p(out), _p(used))
        if rc < 0:
            raise ValueError("orc_boot_grid failed: %d" % rc)
        return out, used

    def grid(self, g: Group):
        out, used = self.grid_coeffs(g)
        return [self.O.plaintext_from_coeffs(out[c], g.level, 1.0) if used[c] else None
                for c in range(g.G * g.b)]

    # ------------------------------------------------------------ pieces
    def mod_raise(self, ct: Ciphertext) -> Ciphertext:
        """Level 0 -> level L: every residue mod q_0, centred, read mod q_0..q_L."""
        if ct.level != 0:
            raise ValueError("ModRaise takes a level-0 ciphertext")
        P, O = self.P, self.O
        q0 = P.q[0]
        out = np.zeros((2, P.L + 1, P.N), dtype=np.uint64)
        idx = np.arange(P.L + 1, dtype=np.int32)
        for c in range(2):
            x = O.intt(ct.data[c][0:1], [0])[0]
            centred = np.where(x > q0 // 2, x.astype(np.int64) - np.int64(q0), x.astype(np.int64))
            res = np.zeros((P.L + 1, P.N), dtype=np.uint64)
            O.L.orc_from_signed(P.ref, _p(np.ascontiguousarray(centred)), P.L + 1, _p(idx), _p(res))
            O.L.orc_ntt(P.ref, _p(res), P.L + 1, _p(idx))
            out[c] = res
        return Ciphertext(out, P.L, P.scale[P.L])

    def apply_galois(self, ct: Ciphertext, g: int) -> Ciphertext:
        """X -> X^g, then the key switch back to s (as ``Oracle.rotate``)."""
        O = self.O
        pa = O.automorph(ct, g)
        u0, u1 = O.keyswitch(pa.data[1], ct.level, self.gkeys[g])
        out = np.zeros_like(ct.data)
        O.L.orc_add(O.P.ref, _p(np.ascontiguousarray(pa.data[0:1])), _p(np.ascontiguousarray(u0[None])),
                    ct.level, 1, _p(out[0:1]))
        out[1] = u1
        return Ciphertext(out, ct.level, ct.scale)

    def mul_monomial(self, ct: Ciphertext, k: int, sign: int) -> Ciphertext:
        """ct * (sign X^k), exact (no level)."""
        P, O = self.P, self.O
        e = np.zeros(P.N, dtype=np.int64)
        e[k] = sign
        pt = O.plaintext_from_coeffs(e, ct.level, 1.0)
        return self.mul_pt_raw(ct, pt)

    def mul_pt_raw(self, ct: Ciphertext, pt: Plaintext) -> Ciphertext:
        out = np.zeros_like(ct.data)
        self.O.L.orc_mul_poly(self.P.ref, _p(np.ascontiguousarray(ct.data)), _p(pt.ntt), ct.level, 2, _p(out))
        return Ciphertext(out, ct.level, ct.scale)

    def lintrans(self, ct: Ciphertext, g: Group) -> Ciphertext:
        """One group: sum_j Rot_{giant j}( sum_i pt_{j,i} . Rot_{u i}(ct) ),
        then one rescale (label Delta_{l-1})."""
        O, n = self.O, self.n
        if ct.level != g.level:
            raise ValueError("group runs at level %d, ciphertext at %d" % (g.level, ct.level))
        pts = self.grids[id(g)]
        baby = O.rotate_hoisted(ct, g.baby_steps(n), self.gkeys)
        acc = None
        for j in range(g.G):
            inner = None
            for i in range(g.b):
                pt = pts[j * g.b + i]
                if pt is None:
                    continue
                t = self.mul_pt_raw(baby[i], pt)
                inner = t if inner is None else O.add(inner, t)
            if inner is None:
                continue
            r = g.giant_step(j, n)
            if r:
                inner = O.rotate(inner, r, self.gkeys)
            acc = inner if acc is None else O.add(acc, inner)
        out = np.zeros((2, ct.level, self.P.N), dtype=np.uint64)
        O.L.orc_rescale(self.P.ref, _p(np.ascontiguousarray(acc.data)), ct.level, 2, _p(out))
        return Ciphertext(out, ct.level - 1, self.P.scale[ct.level - 1])

    def coeff_to_slot(self, ct: Ciphertext) -> Ciphertext:
        for g in self.plan.cts:
            ct = self.lintrans(ct, g)
        return ct

    def slot_to_coeff(self, ct: Ciphertext) -> Ciphertext:
        for g in self.plan.stc:
            ct = self.lintrans(ct, g)
        return ct

    def eval_mod(self, ct: Ciphertext) -> Ciphertext:
        """sin(2 pi K u) of the slots u in [-1, 1]: the Chebyshev series of
        cos(2 pi (K u - 1/4) / 2^r), then r double angles."""
        c = self.circ
        y = c.cheb_series(ct, self.coeffs, self.plan.degree)
        for _ in range(self.plan.r):
            y = self.O.add_const(self.O.mul_int(self.O.mul(y, y, self.rlk), 2), -1.0)
        return y

    def split(self, w: Ciphertext):
        """(re, im) = (w + conj w, -X^n (w - conj w))."""
        cj = self.apply_galois(w, self.g_conj)
        re = self.O.add(w, cj)
        im = self.mul_monomial(self.O.sub(w, cj), self.n, -1)
        return re, im

    def bootstrap(self, ct: Ciphertext) -> Ciphertext:
        w = self.coeff_to_slot(self.mod_raise(ct))
        re, im = self.split(w)
        yr, yi = self.eval_mod(re), self.eval_mod(im)
        w2 = self.O.add(yr, self.mul_monomial(yi, self.n, 1))
        return self.slot_to_coeff(w2)


def rotation_steps(P) -> list:
    """The rotation steps whose Galois keys ``Bootstrapper`` makes (besides
    conjugation, Galois element 2N - 1)."""
    return make_plan(P).rotations(P.slots)


__all__ = ["Bootstrapper", "Group", "Plan", "make_plan", "split_layers", "rotation_steps",
           "galois_element"]
