"""Pins of the oracle's arithmetic: primes, parameters, NTT (CPU only).

Each check compares the oracle with something other than itself: Python big
integers, brute-force definitions, the schoolbook negacyclic product, and the
parameter budget the paper prints (Sec. 6.1).
"""
import json
import math
import os
import decimal

import numpy as np
import pytest

from oracle import ref

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def test_mulmod_matches_python_ints():
    L = ref.lib()
    rng = np.random.default_rng(1)
    for q in [(1 << 61) - 1, 1152921504606830593, 1099511480321, 1073692673, 97]:
        for _ in range(2000):
            a, b = (int(v) for v in rng.integers(0, 1 << 63, 2, dtype=np.uint64))
            assert L.orc_mulmod(a, b, q) == (a * b) % q
        for a in (0, 1, q - 1, (1 << 64) - 1):
            for b in (0, 1, q - 1, (1 << 64) - 1):
                assert L.orc_mulmod(a, b, q) == (a * b) % q


def test_miller_rabin_against_trial_division_and_known_values():
    L = ref.lib()

    def trial(n):
        if n < 2:
            return False
        i = 2
        while i * i <= n:
            if n % i == 0:
                return False
            i += 1
        return True

    for n in range(0, 3000):
        assert bool(L.orc_is_prime(n)) == trial(n), n
    # Mersenne prime 2^61-1, the largest prime below 2^64, Carmichael numbers
    assert L.orc_is_prime((1 << 61) - 1)
    assert L.orc_is_prime((1 << 64) - 59)
    for c in (561, 1105, 1729, 2465, 41041, 3215031751, 3825123056546413051):
        assert not L.orc_is_prime(c)
    assert not L.orc_is_prime(((1 << 31) - 1) * 2147483629)


@pytest.mark.parametrize("name", ["c1", "c2", "t1", "t2"])
def test_parameter_rule(name):
    P = ref.Params.preset(name)
    twoN = 2 * P.N
    assert len(set(P.q)) == len(P.q)
    for q, psi in zip(P.q, P.psi):
        assert ref.lib().orc_is_prime(q)
        assert q % twoN == 1
        assert pow(psi, P.N, q) == q - 1          # primitive 2N-th root
        assert pow(psi, twoN, q) == 1
    # q_0 is the largest prime below 2^bits that is 1 mod 2N
    bits = ref.PRESETS[name]["q0_bits"]
    assert P.q[0] < (1 << bits)
    x = P.q[0] + twoN
    while x < (1 << bits):
        assert not ref.lib().orc_is_prime(x)
        x += twoN


def test_c2_matches_paper_budget():
    """N = 2^16, Delta = 2^40, 32768 slots and log2(PQ) <= 1443 (Sec. 6.1)."""
    P = ref.Params.preset("c2")
    assert P.logN == GOLD["ring_degree_log2"]["value"]
    assert P.scale[P.L] == 2.0 ** GOLD["scale_log2"]["value"]
    assert P.slots == GOLD["slots"]["value"]
    logPQ = sum(math.log2(q) for q in P.q)
    assert logPQ <= GOLD["log2_PQ_budget"]["value"]
    assert logPQ > 1400
    for q in P.q[1:P.L + 1]:           # scale primes track Delta = 2^40
        assert abs(q / 2.0 ** 40 - 1.0) < 1e-4
    assert P.q[0].bit_length() == 60 and all(p.bit_length() == 60 for p in P.q[P.L + 1:])


@pytest.mark.parametrize("name", ["c1", "c2", "t2"])
def test_scale_schedule_high_precision(name):
    """Delta_{l-1} = Delta_l^2 / q_l: the FP64 chain stays within 1e-9 of the
    same chain in 60-digit decimal arithmetic, and every level stays within
    2^-15 of Delta."""
    P = ref.Params.preset(name)
    ctx = decimal.Context(prec=60)
    exact = decimal.Decimal(P.scale[P.L])
    for l in range(P.L, 0, -1):
        exact = ctx.divide(ctx.multiply(exact, exact), decimal.Decimal(P.q[l]))
        assert abs(float(exact) / P.scale[l - 1] - 1.0) < 1e-9
    for s in P.scale:
        assert abs(s / P.scale[P.L] - 1.0) < 2.0 ** -15


@pytest.mark.parametrize("logN", [2, 3, 4, 5])
def test_ntt_equals_definition_bruteforce(logN):
    """NTT_j = sum_k a_k psi^((2 brv(j) + 1) k) mod q, by Python big ints."""
    P = ref.Params(logN, 1, 1, 1, 50, 2.0 ** 30, 50)
    O = ref.Oracle(P)
    rng = np.random.default_rng(logN)
    N = P.N
    for pi in range(P.nprimes):
        q, psi = P.q[pi], P.psi[pi]
        a = [int(v) for v in rng.integers(0, q, N, dtype=np.uint64)]
        got = O.ntt(np.array([a], dtype=np.uint64), [pi])[0]
        for j in range(N):
            e = 2 * brv(j, logN) + 1
            want = sum(a[k] * pow(psi, e * k, q) for k in range(N)) % q
            assert int(got[j]) == want
        back = O.intt(got[None, :], [pi])[0]
        assert [int(v) for v in back] == a


@pytest.mark.parametrize("name,limbs", [("c1", [0, 1, 2, 3]), ("t1", [0, 3, 9])])
def test_ntt_convolution_vs_schoolbook(name, limbs):
    """iNTT(NTT(a) * NTT(b)) equals the schoolbook negacyclic product (N = 2^12)."""
    P = ref.Params.preset(name)
    O = ref.Oracle(P)
    L = ref.lib()
    rng = np.random.default_rng(7)
    for pi in limbs:
        q = P.q[pi]
        a = rng.integers(0, q, P.N, dtype=np.uint64)
        b = rng.integers(0, q, P.N, dtype=np.uint64)
        c = np.zeros(P.N, dtype=np.uint64)
        L.orc_negacyclic_mul(ref._p(a), ref._p(b), ref._p(c), P.N, q)
        fa = O.ntt(a[None], [pi])[0]
        fb = O.ntt(b[None], [pi])[0]
        prod = ref._mulmod_vec(fa, fb, q)
        assert np.array_equal(O.intt(prod[None], [pi])[0], c)


def test_ntt_full_size_horner_samples():
    """At N = 2^16: NTT_j equals a(psi^(2 brv(j)+1)) by Horner, for 24 sampled j."""
    P = ref.Params.preset("c2")
    O = ref.Oracle(P)
    rng = np.random.default_rng(3)
    for pi in (0, 12, P.L + 3):
        q, psi = P.q[pi], P.psi[pi]
        a = rng.integers(0, q, P.N, dtype=np.uint64)
        got = O.ntt(a[None], [pi])[0]
        coeffs = [int(v) for v in a[::-1]]
        for j in rng.integers(0, P.N, 8):
            x = pow(psi, 2 * brv(int(j), P.logN) + 1, q)
            acc = 0
            for c in coeffs:
                acc = (acc * x + c) % q
            assert int(got[j]) == acc


def test_automorphism_ntt_is_slot_permutation():
    """In NTT form X -> X^g moves slot j' to slot j with
    2 brv(j') + 1 = (2 brv(j) + 1) g (mod 2N)."""
    P = ref.Params(5, 1, 1, 1, 50, 2.0 ** 30, 50)
    O = ref.Oracle(P)
    N, logN = P.N, P.logN
    rng = np.random.default_rng(5)
    a = rng.integers(0, P.q[0], (1, N), dtype=np.uint64)
    for g in (5, 25, 2 * N - 1, 3):
        out = np.zeros_like(a)
        ref.lib().orc_automorph_ntt(P.ref, ref._p(a), ref._p(out), 1, ref._p(np.array([0], np.int32)), g)
        inv = {(2 * brv(j, logN) + 1) % (2 * N): j for j in range(N)}
        for j in range(N):
            src = inv[((2 * brv(j, logN) + 1) * g) % (2 * N)]
            assert out[0, j] == a[0, src]
