"""CPU checks of the arithmetic identities the kernels rely on, in plain
Python integers (no library call): the row-twiddle factorisation of the
two-pass NTT, the Montgomery reduction of the base conversions' 30-bit
partial-product sums, and the exact FP64 modular product's error bound."""
import math
import random

import numpy as np
import pytest


def brv(x, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def test_row_twiddle_exponent_factorisation():
    """Table entry (R + r) 2^s + j (j < 2^s) of the row pass, N = 2^16,
    R = 2^8: brv_16 of it is brv_16((R + r) 2^s) + brv_s(j) N / 2^s, so the
    twiddle psi^brv(...) is a per-(row, stage) factor times a shared one."""
    logn, logr = 16, 8
    n, rr = 1 << logn, 1 << logr
    table = np.array([brv(m, logn) for m in range(n)], dtype=np.int64)
    for s in range(logn - logr):
        j = np.arange(1 << s, dtype=np.int64)
        shared = np.array([brv(int(x), s) for x in j], dtype=np.int64) * (n >> s)
        for r in range(rr):
            base = (rr + r) << s
            assert np.array_equal(table[base + j], table[base] + shared)


def test_row_twiddle_product_matches_the_table():
    """The same factorisation on actual twiddles: psi a primitive 2N-th root
    of unity mod a 40-bit NTT prime."""
    logn = 16
    n = 1 << logn
    # the largest prime q = 1 mod 2N below 2^40 (Miller-Rabin, bases that
    # decide every q < 3.3e24)
    def is_prime(x):
        d, e = x - 1, 0
        while d % 2 == 0:
            d, e = d // 2, e + 1
        for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41):
            y = pow(a, d, x)
            if y in (1, x - 1):
                continue
            for _ in range(e - 1):
                y = y * y % x
                if y == x - 1:
                    break
            else:
                return False
        return True
    k = ((1 << 40) - 1) // (2 * n)
    while not is_prime(k * 2 * n + 1):
        k -= 1
    q = k * 2 * n + 1
    g = 3
    while pow(g, (q - 1) // 2, q) == 1:
        g += 1
    psi = pow(g, (q - 1) // (2 * n), q)
    assert pow(psi, n, q) == q - 1
    rng = random.Random(5)
    for _ in range(200):
        r, s = rng.randrange(256), rng.randrange(8)
        j = rng.randrange(1 << s)
        m = ((256 + r) << s) + j
        want = pow(psi, brv(m, logn), q)
        rowf = pow(psi, brv((256 + r) << s, logn), q)
        comm = pow(pow(psi, n >> s, q), brv(j, s), q)
        assert rowf * comm % q == want


def acc30_redc(zs, cs, q):
    """The device's Acc30 sum of z_i c_i in 30-bit halves (a fold after
    every 8 terms), its 128-bit words after a last fold and Montgomery's
    REDC with mneg = -q^-1 mod 2^64."""
    m64 = (1 << 64) - 1
    mask = (1 << 30) - 1
    a0 = a1 = a2 = 0
    for i, (z, c) in enumerate(zip(zs, cs)):
        zl, zh, cl, ch = z & mask, z >> 30, c & mask, c >> 30
        a0 += zl * cl
        a1 += zl * ch + zh * cl
        a2 += zh * ch
        assert max(a0, a1, a2) < 1 << 64
        if i % 8 == 7:
            a1 += a0 >> 30
            a0 &= mask
            a2 += a1 >> 30
            a1 &= mask
    # REDC's final fold: the three fields then occupy disjoint bits
    a1 += a0 >> 30
    a0 &= mask
    a2 += a1 >> 30
    a1 &= mask
    assert a2 < 1 << 64
    lo2 = (a0 | (a1 << 30) | (a2 << 60)) & m64
    hi = a2 >> 4
    assert (hi << 64) + lo2 == sum(z * c for z, c in zip(zs, cs))
    mneg = (-pow(q, -1, 1 << 64)) % (1 << 64)
    mm = (lo2 * mneg) & m64
    t = hi + ((mm * q) >> 64) + int(lo2 != 0)
    return t - q if t >= q else t


@pytest.mark.parametrize("nterms", [7, 8, 9, 16])
def test_montgomery_reduction_of_conversion_sums(nterms):
    """REDC(sum z_i (c_i 2^64 mod q)) = sum z_i c_i mod q for worst-case and
    random operands: z_i below 2^60 (source residues), constants below q."""
    rng = random.Random(nterms)
    for q in (0xFFFFFFFFFFC0001, (1 << 40) - 87, (1 << 59) + 21):
        q |= 1
        for trial in range(60):
            if trial == 0:
                zs = [(1 << 60) - 1] * nterms
                cs0 = [q - 1] * nterms
            else:
                zs = [rng.randrange(1 << 60) for _ in range(nterms)]
                cs0 = [rng.randrange(q) for _ in range(nterms)]
            cs = [c * (1 << 64) % q for c in cs0]
            assert sum(z * c for z, c in zip(zs, cs)) < q << 64
            assert acc30_redc(zs, cs, q) == sum(z * c for z, c in zip(zs, cs0)) % q


def fp_mulmod(y, w, ws, q):
    """FpArith::mulmod in FP64: h = fl(y w), l = fma(y, w, -h) (exact),
    k = rint(y ws), r = fma(-k, q, h) + l."""
    h = y * w
    l = math.fma(y, w, -h) if hasattr(math, "fma") else float(int(y) * int(w) - int(h))
    k = float(round(y * ws))
    r = float(int(-k) * int(q) + int(h))   # the fma's exact result, an integer below 2^53
    return r + l, k


def test_fp64_product_with_formed_twiddles():
    """A twiddle formed as the exact product of two table entries is signed,
    |w| <= 0.51 q; with ws = fl(w fl(1/q)) the butterfly's quotient estimate
    stays within 0.032 of y w / q for |y| < 2^47.4, so y w - k q is exact and
    below 0.532 q in magnitude."""
    rng = random.Random(9)
    q = float((1 << 40) - 87)
    qinv = 1.0 / q
    worst = 0.0
    for _ in range(20000):
        a = float(rng.randrange(int(q)))
        b = float(rng.randrange(int(q)))
        w, _ = fp_mulmod(a, b, b / q, q)
        assert abs(w) <= 0.51 * q
        assert (int(w) - int(a) * int(b)) % int(q) == 0
        ws = w * qinv
        y = float(rng.randrange(-(1 << 47), 1 << 47))
        r, k = fp_mulmod(y, w, ws, q)
        assert (int(r) - int(y) * int(w)) % int(q) == 0
        worst = max(worst, abs(r) / q)
        exact = int(y) * int(w) / int(q)
        assert abs(exact - y * ws) < 0.032
    assert worst <= 0.532


def test_fp64_moddown_store_bounds():
    """The fused ModDown row pass on an FP64 prime sums u P^-1, the operand
    products (each an exact FP64 product of canonical residues) and the
    transform's unreduced output (below 10 q) into s, |s| < 12 q, and takes
    s q_l^-1 with one more exact product: the quotient estimate stays within
    0.07 of s w / q, so the result is exact and below 0.57 q in magnitude
    and one conditional addition of q makes it canonical."""
    rng = random.Random(21)
    for q in (float((1 << 40) - 87), float((1 << 44) - 17)):
        qinv = 1.0 / q
        worst = 0.0
        for _ in range(20000):
            w = float(rng.randrange(int(q)))
            ws = w * qinv
            s = float(rng.randrange(-12 * int(q) + 1, 12 * int(q)))
            r, _ = fp_mulmod(s, w, ws, q)
            assert (int(r) - int(s) * int(w)) % int(q) == 0
            assert abs(int(s) * int(w) / int(q) - s * ws) < 0.07
            worst = max(worst, abs(r) / q)
            c = r + q if r < 0 else r
            assert 0 <= c < q and int(c) == int(s) * int(w) % int(q)
        assert worst < 0.57
