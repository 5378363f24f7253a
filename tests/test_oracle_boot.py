"""Pins of the oracle's CKKS bootstrapping (CPU only).

The transforms are pinned to the plain decoding matrix U0[j, k] =
zeta^((5^j mod 2N) k) written out here with numpy; ModRaise, conjugation and
the monomial X^n to exact identities of the decryption; EvalMod's polynomial
to the sine it approximates; the whole bootstrap to the identity on the
message (a refreshed ciphertext decrypts to what the level-0 one held).
"""
import math

import numpy as np
import pytest

from oracle import boot, cheb, ref
from oracle.ref import _p


def u0_matrix(N):
    n = N // 2
    e = np.array([pow(5, j, 2 * N) for j in range(n)], dtype=np.int64)
    k = np.arange(n, dtype=np.int64)
    return np.exp(1j * np.pi * ((e[:, None] * k[None, :]) % (2 * N)) / N)


def bitrev_perm(n):
    logn = n.bit_length() - 1
    return np.array([int(format(s, "0%db" % logn)[::-1], 2) for s in range(n)])


def group_matrix(N, inverse, lo, hi):
    n = N // 2
    cap = 256
    offs = np.zeros(cap, dtype=np.int32)
    re = np.zeros((cap, n))
    im = np.zeros((cap, n))
    cnt = ref.lib().orc_boot_group_diags(N, inverse, lo, hi, cap, _p(offs), _p(re), _p(im))
    assert cnt > 0
    M = np.zeros((n, n), dtype=complex)
    rows = np.arange(n)
    for c in range(cnt):
        M[rows, (rows + offs[c]) % n] += re[c] + 1j * im[c]
    return M, offs[:cnt]


@pytest.mark.parametrize("logN", [4, 6, 8])
def test_special_fft_layers_equal_decoding_matrix(logN):
    """U0 BR = (StC groups, applied bottom first) and BR U0^H / n = (CtS
    groups, applied top first), for the group split the bootstrap uses."""
    N = 1 << logN
    n = N // 2
    logn = n.bit_length() - 1
    U = u0_matrix(N)
    BR = np.eye(n)[bitrev_perm(n)]           # (BR x)_s = x_brv(s)
    ranges = boot.split_layers(logn, 3 if logn >= 3 else logn)
    stc = np.eye(n, dtype=complex)
    for lo, hi in reversed(ranges):
        stc = group_matrix(N, 0, lo, hi)[0] @ stc
    cts = np.eye(n, dtype=complex)
    for lo, hi in ranges:
        cts = group_matrix(N, 1, lo, hi)[0] @ cts
    assert np.max(np.abs(stc - U @ BR)) < 1e-12 * n
    assert np.max(np.abs(cts - BR @ U.conj().T / n)) < 1e-12
    # and U0 U0^H = n I, the fact CoeffToSlot rests on
    assert np.max(np.abs(U @ U.conj().T - n * np.eye(n))) < 1e-9 * n


def test_single_layer_is_a_butterfly():
    """One layer by hand: len = 2 pairs (x_2t, x_2t+1) -> (x + w y, x - w y)
    with w = zeta^(n/2 * (5^0 mod 8)) = zeta^(n/2)."""
    N = 16
    n = N // 2
    M, offs = group_matrix(N, 0, 1, 1)
    w = np.exp(1j * np.pi * (n // 2) / N)
    want = np.zeros((n, n), dtype=complex)
    for t in range(0, n, 2):
        want[t, t], want[t, t + 1] = 1, w
        want[t + 1, t], want[t + 1, t + 1] = 1, -w
    assert np.max(np.abs(M - want)) < 1e-15
    assert sorted(int(o) for o in offs) == [0, 1, n - 1]


@pytest.fixture(scope="module")
def b1():
    P = ref.Params.preset("b1")
    O = ref.Oracle(P)
    sk, pk = O.keygen(11)
    B = boot.Bootstrapper(O, sk, 12)
    return P, O, sk, pk, B


def test_boot_chain(b1):
    """The bootstrappable chain: every prime distinct, prime, = 1 mod 2N and
    below 2^60; the scale rule holds wherever two ciphertexts are multiplied
    (EvalMod's and the computation levels), the transform levels carry their
    labels; the depth splits 11 + 3 + 10 + 3 = 27."""
    P = b1[0]
    assert (P.L, P.Lc, P.boot) == (27, 11, (3, 10, 3))
    assert len(set(P.q)) == P.nprimes
    for q in P.q:
        assert q < 2 ** 60 and q % (2 * P.N) == 1 and ref.lib().orc_is_prime(q)
    C, E, S = P.boot
    canon = list(range(1, P.Lc + 1)) + list(range(P.Lc + S + 1, P.L - C + 1))
    for l in canon:
        assert P.scale[l - 1] == P.scale[l] * P.scale[l] / P.q[l]
    assert P.scale[P.Lc] == 2.0 ** 40
    assert [P.scale[P.Lc + i] for i in (1, 2)] == [2.0 ** 46, 2.0 ** 52]
    assert all(P.scale[l] == 2.0 ** 58 for l in range(P.L - C, P.L + 1))
    for l in range(P.Lc + S, P.L - C + 1):
        assert abs(math.log2(P.scale[l]) - 58) < 1e-3


def test_sparse_secret(b1):
    P, O, sk, *_ = b1
    s = sk.s_coef.astype(int)
    assert np.count_nonzero(s) == P.h and set(np.unique(s)) <= {-1, 0, 1}
    s2, _ = O.keygen(11)
    assert np.array_equal(s2.s_coef, sk.s_coef)
    s3, _ = O.keygen(12)
    assert not np.array_equal(s3.s_coef, sk.s_coef)
    # positions come from a shuffle of all N indices: both halves are hit
    nz = np.flatnonzero(s)
    assert nz.min() < P.N // 4 and nz.max() > 3 * P.N // 4


def decrypt_exact(O, ct, sk):
    """Centred integer coefficients of <ct, s> over the ciphertext's modulus
    (Python integers)."""
    return O.crt_centred(O.intt(O.decrypt_ntt(ct, sk), list(range(ct.level + 1))))


def test_mod_raise(b1):
    """<raised, s> = <ct, s> mod q_0 exactly, and |<raised, s>| < K q_0."""
    P, O, sk, pk, B = b1
    m = np.random.default_rng(3).uniform(-1, 1, P.slots)
    ct = O.encrypt(O.encode(m, 0), pk, 13)
    t = decrypt_exact(O, B.mod_raise(ct), sk)
    t0 = decrypt_exact(O, ct, sk)
    q0 = P.q[0]
    assert all((int(a) - int(b)) % q0 == 0 for a, b in zip(t, t0))
    assert max(abs(int(a)) for a in t) < B.plan.K * q0


def slots_complex(O, ct, sk):
    P = O.P
    c = np.ascontiguousarray(O.decrypt_coeffs(ct, sk))
    re, im = np.zeros(P.slots), np.zeros(P.slots)
    O.L.orc_decode_coeffs_complex(P.ref, _p(c), ct.scale, _p(re), _p(im))
    return re + 1j * im


def test_conjugation_and_monomial(b1):
    """X -> X^(2N-1) conjugates every slot; X^n multiplies every slot by i."""
    P, O, sk, pk, B = b1
    rng = np.random.default_rng(4)
    zr, zi = rng.uniform(-1, 1, P.slots), rng.uniform(-1, 1, P.slots)
    lv = P.Lc
    coeffs = np.zeros(P.N, dtype=np.int64)
    O.L.orc_encode_coeffs_complex(P.ref, _p(zr), _p(zi), P.slots, P.scale[lv], _p(coeffs))
    ct = O.encrypt(O.plaintext_from_coeffs(coeffs, lv, P.scale[lv]), pk, 14)
    z = zr + 1j * zi
    tol = 1e-6
    assert np.max(np.abs(slots_complex(O, ct, sk) - z)) < tol
    assert np.max(np.abs(slots_complex(O, B.apply_galois(ct, 2 * P.N - 1), sk) - z.conj())) < tol
    assert np.max(np.abs(slots_complex(O, B.mul_monomial(ct, P.slots, 1), sk) - 1j * z)) < tol
    assert np.max(np.abs(slots_complex(O, B.mul_monomial(ct, P.slots, -1), sk) + 1j * z)) < tol


def test_evalmod_polynomial():
    """The Chebyshev series of cos(2 pi (K u - 1/4) / 2^r) followed by r
    double angles is sin(2 pi K u) on [-1, 1] (closed form), and near each
    integer x = K u it is 2 pi (x - I) to within the cubic term."""
    K, r, d = 16, 4, 27
    c = cheb.evalmod_cos_coeffs(K, r, d)
    u = np.linspace(-1, 1, 100001)
    y = np.polynomial.chebyshev.chebval(u, c)
    for _ in range(r):
        y = 2 * y * y - 1
    assert np.max(np.abs(y - np.sin(2 * np.pi * K * u))) < 1e-11
    I = np.arange(-K + 1, K)
    eps = 1e-6
    x = I + eps
    y = np.polynomial.chebyshev.chebval(x / K, c)
    for _ in range(r):
        y = 2 * y * y - 1
    assert np.max(np.abs(y - 2 * np.pi * eps)) < 1e-11


def test_grid_plaintexts_decode_to_rotated_diagonals(b1):
    """Each baby-step giant-step plaintext decodes, at the scale dp that takes
    Delta_l to Delta_{l-1} through one rescale (dp = Delta_{l-1} q_l /
    Delta_l), to its diagonal rotated back by the giant step, times the
    group constant c; its integers were rounded at S = dp c."""
    P, O, sk, pk, B = b1
    n = P.slots
    for g in (B.plan.cts[0], B.plan.cts[2], B.plan.stc[1]):
        coeffs, used = B.grid_coeffs(g)
        M, _ = group_matrix(P.N, g.inverse, g.lo, g.hi)
        S = ref.lib().orc_boot_group_factor(P.ref, g.level, g.ckind, B.plan.K, P.boot[0])
        dp = P.scale[g.level - 1] * P.q[g.level] / P.scale[g.level]
        c = S / dp
        if g.ckind == 1:
            assert abs(c - P.scale[P.L] / (2 * B.plan.K * P.q[0])) < 1e-15 * c
        if g.ckind == 2:
            assert abs(c ** 3 - P.q[0] / (2 * math.pi * P.scale[0])) < 1e-12 * c ** 3
        rows = np.arange(n)
        for j in range(g.G):
            for i in range(g.b):
                cell = j * g.b + i
                k = (g.u * (g.m0 + g.b * j + i)) % n
                d = M[rows, (rows + k) % n]
                assert bool(used[cell]) == bool(np.any(np.abs(d) > 0))
                if not used[cell]:
                    continue
                gj = g.giant_step(j, n)
                want = c * d[(rows - gj) % n]
                re, im = np.zeros(n), np.zeros(n)
                O.L.orc_decode_coeffs_complex(P.ref, _p(np.ascontiguousarray(coeffs[cell])), dp, _p(re), _p(im))
                # rounding N integer coefficients: at most N / 2 / dp, about sqrt(N) / dp
                assert np.max(np.abs(re + 1j * im - want)) < 16 * math.sqrt(P.N) / dp + 1e-13 * abs(c)


def test_bootstrap_refreshes(b1):
    """A level-0 ciphertext refreshed to level Lc decrypts to its message
    (max error 2^-19 of a [-1, 1] message; about 2^-21.2 measured), and
    the result computes on: its square decrypts to m^2."""
    P, O, sk, pk, B = b1
    m = np.random.default_rng(5).uniform(-1, 1, P.slots)
    ct = O.encrypt(O.encode(m, 0), pk, 15)
    out = B.bootstrap(ct)
    assert out.level == P.Lc and out.scale == P.scale[P.Lc]
    got = O.decrypt(out, sk)
    assert np.max(np.abs(got - m)) < 2.0 ** -19
    sq = O.mul(out, out, B.rlk)
    assert np.max(np.abs(O.decrypt(sq, sk) - m * m)) < 2.0 ** -18


def test_kurtosis_with_refreshes(b1):
    """Kurtosis at the paper's InvSqrt (degree 31 on [0, 2], six Newton
    steps, B = 20) on 11 computation levels: InvSqrt refreshes by
    bootstrapping and the result agrees with the FP64 closed form to 1e-4;
    without the refreshes the circuit runs out of levels."""
    from oracle import circuits as C, stats64
    P, O, sk, pk, B = b1
    gk = dict(B.gkeys)
    gk.update(O.rotation_keys(sk, 12, [s for s in O.rotsum_hoisted8_steps()
                                       if ref.galois_element(s, P.N) not in gk]))
    circ = C.Circuits(C.EncEval(O, B.rlk, gk, booter=B))
    n = 3000
    x = np.random.default_rng(3).uniform(0, 20, n)
    X = [O.encrypt(O.encode(x[k:k + P.slots], P.Lc), pk, 100 + k) for k in range(0, n, P.slots)]
    coeffs = cheb.paper_invsqrt_coeffs(31, 1.0)
    cfg = C.InvSqrtCfg(a=0.0, b=2.0, degree=31, iters=6, coeffs=coeffs, boot=True)
    k = circ.kurtosis(X, n, 20.0, cfg)
    assert abs(O.decrypt(k, sk)[0] / stats64.kurtosis(x) - 1) < 1e-4
    with pytest.raises(ref.LevelError):
        circ.kurtosis(X, n, 20.0, C.InvSqrtCfg(a=0.0, b=2.0, degree=31, iters=6, coeffs=coeffs))
