"""Pins of the oracle's CKKS operations: decryption identities, exact CRT
checks of key switching and rescale, rotations (CPU only)."""
import math

import numpy as np
import pytest

from oracle import ref


@pytest.fixture(scope="module", params=["c1", "t1"])
def env(request):
    P = ref.Params.preset(request.param)
    O = ref.Oracle(P)
    sk, pk = O.keygen(1)
    rlk = O.relin_key(sk, 2)
    gk = O.rotation_keys(sk, 3, O.rotsum_hoisted8_steps() + [3, 5])
    return P, O, sk, pk, rlk, gk


def fresh_std(P):
    """std of one slot's fresh public-key noise: N sigma sqrt(2/3) / Delta."""
    return P.N * 3.2 * math.sqrt(2.0 / 3.0) / P.scale[P.L]


def enc(O, pk, m, seed, level=None):
    return O.encrypt(O.encode(m, level), pk, seed)


def test_decrypt_encrypt(env):
    P, O, sk, pk, *_ = env
    m = np.random.default_rng(1).uniform(0, 1, P.slots)
    ct = enc(O, pk, m, 10)
    assert np.max(np.abs(O.decrypt(ct, sk) - m)) < 8 * fresh_std(P)
    ct2 = O.encrypt_sk(O.encode(m), sk, 11)
    assert np.max(np.abs(O.decrypt(ct2, sk) - m)) < 8 * fresh_std(P)


def test_keyswitch_exact_crt(env):
    """u0 + u1 s - d s' is a small integer polynomial (exact CRT over Q_l)."""
    P, O, sk, pk, rlk, gk = env
    l = P.L
    rng = np.random.default_rng(2)
    d = np.stack([rng.integers(0, P.q[i], P.N, dtype=np.uint64) for i in range(l + 1)])
    u0, u1 = O.keyswitch(d, l, rlk)
    res = np.zeros_like(u0)
    for i in range(l + 1):
        q = P.q[i]
        s = sk.s_ntt[i]
        s2 = ref._mulmod_vec(s, s, q)
        lhs = (u0[i].astype(object) + ref._mulmod_vec(u1[i], s, q).astype(object)) % q
        rhs = ref._mulmod_vec(d[i], s2, q).astype(object)
        res[i] = ((lhs - rhs) % q).astype(np.uint64)
    e = O.crt_centred(O.intt(res, list(range(l + 1))))
    Q = 1
    for q in P.q[: l + 1]:
        Q *= q
    ev = np.array([int(v) for v in e], dtype=np.float64)
    assert np.max(np.abs(ev)) < 2 ** 12      # Q is at least 2^99 for both presets
    assert Q > 2 ** 99
    # ModDown rounds to nearest: no systematic offset (a floor would leave a
    # mean near -(1 + sum s)/2 on every coefficient)
    assert abs(ev.mean()) < 3.0


def test_rescale_is_rounded_division(env):
    """Rescale equals round(X / q_l) mod Q_{l-1}, X the CRT integer."""
    P, O, sk, *_ = env
    l = P.L
    rng = np.random.default_rng(3)
    X = np.stack([rng.integers(0, P.q[i], P.N, dtype=np.uint64) for i in range(l + 1)])
    out = np.zeros((1, l, P.N), dtype=np.uint64)
    ref.lib().orc_rescale(P.ref, ref._p(np.ascontiguousarray(X[None])), l, 1, ref._p(out))
    xs = O.crt_centred(O.intt(X, list(range(l + 1))))
    got = O.crt_centred(O.intt(out[0], list(range(l))))
    ql = P.q[l]
    Qm = 1
    for q in P.q[:l]:
        Qm *= q
    for k in range(0, P.N, 97):
        want = (2 * int(xs[k]) + ql) // (2 * ql)
        assert (int(got[k]) - want) % Qm == 0


def test_mul_add_const_ops(env):
    P, O, sk, pk, rlk, gk = env
    rng = np.random.default_rng(4)
    a = rng.uniform(-1, 1, P.slots)
    b = rng.uniform(-1, 1, P.slots)
    ca, cb = enc(O, pk, a, 20), enc(O, pk, b, 21)
    tol = 64 * fresh_std(P)
    m = O.mul(ca, cb, rlk)
    assert m.level == P.L - 1 and m.scale == P.scale[P.L - 1]
    assert np.max(np.abs(O.decrypt(m, sk) - a * b)) < tol
    assert np.max(np.abs(O.decrypt(O.mul_const(ca, -0.75), sk) + 0.75 * a)) < tol
    assert np.max(np.abs(O.decrypt(O.add_const(ca, 0.25), sk) - (a + 0.25))) < tol
    assert np.max(np.abs(O.decrypt(O.mul_int(ca, 3), sk) - 3 * a)) < tol
    assert np.max(np.abs(O.decrypt(O.sub(ca, cb), sk) - (a - b))) < tol
    pt = O.encode(b, P.L)
    assert np.max(np.abs(O.decrypt(O.mul_plain(ca, pt), sk) - a * b)) < tol
    al = O.level_align(ca, 0)
    assert al.level == 0 and al.scale == P.scale[0]
    assert np.max(np.abs(O.decrypt(al, sk) - a)) < tol
    with pytest.raises(ref.LevelError):
        O.add(ca, m)


def test_lincomb(env):
    """sum_k c_k ct_k with one rescale: a single term one level up is exactly
    Mul(P) by the constant; terms at different levels decrypt to the
    weighted sum of their messages."""
    P, O, sk, pk, rlk, gk = env
    rng = np.random.default_rng(9)
    a, b = rng.uniform(-1, 1, P.slots), rng.uniform(-1, 1, P.slots)
    ca, cb = enc(O, pk, a, 40), enc(O, pk, b, 41)
    one = O.lincomb([ca], [-0.75], P.L - 1)
    ref_ = O.mul_const(ca, -0.75)
    assert one.level == ref_.level and one.scale == ref_.scale
    assert np.array_equal(one.data, ref_.data)
    tol = 64 * fresh_std(P)
    cb_low = O.level_align(cb, P.L - 1)            # a term one level lower
    out = O.lincomb([ca, cb_low, ca], [0.5, -1.25, 0.125], P.L - 2)
    assert out.level == P.L - 2 and out.scale == P.scale[P.L - 2]
    assert np.max(np.abs(O.decrypt(out, sk) - (0.625 * a - 1.25 * b))) < 4 * tol
    with pytest.raises(ref.LevelError):
        O.lincomb([cb_low], [1.0], P.L - 1)


def test_rotations(env):
    P, O, sk, pk, rlk, gk = env
    m = np.random.default_rng(5).uniform(0, 1, P.slots)
    ct = enc(O, pk, m, 30)
    tol = 64 * fresh_std(P)
    r3 = O.rotate(ct, 3, gk)
    assert np.max(np.abs(O.decrypt(r3, sk) - np.roll(m, -3))) < tol
    r35 = O.rotate(r3, 5, gk)
    assert np.max(np.abs(O.decrypt(r35, sk) - np.roll(m, -8))) < tol
    h = O.rotate_hoisted(ct, [3, 5], gk)
    assert np.max(np.abs(O.decrypt(h[0], sk) - np.roll(m, -3))) < tol
    assert np.max(np.abs(O.decrypt(h[1], sk) - np.roll(m, -5))) < tol
    s = O.rotsum(ct, gk)
    assert np.max(np.abs(O.decrypt(s, sk) - m.sum())) < m.sum() * 1e-4
    assert 9 not in O.rotsum_hoisted8_steps() + [3, 5]
    with pytest.raises(KeyError):
        O.rotate(ct, 9, gk)


def test_rotsum_plan_covers_every_slot_once(env):
    """RotSum's steps multiply out to every shift 0..slots-1 exactly once:
    the product over steps of (1 + X^s + ... + X^{(radix-1) s}) is
    1 + X + ... + X^{slots-1}."""
    P, O = env[0], env[1]
    poly = np.zeros(P.slots, dtype=np.int64)
    poly[0] = 1
    for s, rad in O.rotsum_hoisted8_plan():
        nxt = np.zeros_like(poly)
        for k in range(rad):
            nxt += np.roll(poly, k * s)
        poly = nxt
    assert np.array_equal(poly, np.ones(P.slots, dtype=np.int64))
    assert sorted(set(O.rotsum_hoisted8_steps())) == sorted(O.rotsum_hoisted8_steps())


def test_rotsum_step_sums_rotations(env):
    """The hoisted step ct + rot(ct, s) + rot(ct, 2s) + rot(ct, 3s) (one
    ModUp, one ModDown) decrypts to the slot-wise sum of the rotated
    messages, and agrees with separate rotations up to the noise."""
    P, O, sk, pk, rlk, gk = env
    m = np.random.default_rng(6).uniform(-1, 1, P.slots)
    ct = enc(O, pk, m, 31)
    s = 1
    want = sum(np.roll(m, -k * s) for k in range(4))
    got = O.rotsum_step(ct, s, 4, gk)
    tol = 64 * fresh_std(P)
    assert np.max(np.abs(O.decrypt(got, sk) - want)) < 4 * tol
    sep = ct
    for k in range(1, 4):
        sep = O.add(sep, O.rotate(ct, k * s, gk))
    assert np.max(np.abs(O.decrypt(got, sk) - O.decrypt(sep, sk))) < 4 * tol
    two = O.rotsum_step(ct, 2, 2, gk)
    assert np.max(np.abs(O.decrypt(two, sk) - (m + np.roll(m, -2)))) < 2 * tol
    eight = O.rotsum_step(ct, 1, 8, gk)       # seven keys in one extended sum
    want8 = sum(np.roll(m, -k) for k in range(8))
    assert np.max(np.abs(O.decrypt(eight, sk) - want8)) < 8 * tol


def test_rotsum_serial_definition_and_hoisted8_pin(env):
    """The plain rotate-and-sum (log2(N/2) steps ct <- ct + Rot(ct, 2^k);
    the slot sums of Eq. 2) leaves the sum of all slots in every slot, and
    the hoisted radix-8 form the circuits use decrypts to the same integer
    polynomial up to the key-switching rounding.

    Bound: a rounding ModDown of u returns round(u/P) - v with 0 <= v < K
    (fast conversion without correction), so one key switch adds at most
    B = (K + 1/2)(1 + ||s||_1) + 1 to a decrypted coefficient (the key's
    own error times ModUp(d)/P is below 1 at these parameters).  Each
    serial step doubles what came before, so its total is below slots * B;
    the radix-8 form adds one ModDown per step and stays below that too.
    The two decryptions therefore differ by at most 2 slots B, while one
    dropped rotation term would move a coefficient by about Delta/2."""
    P, O, sk, pk, rlk, gk = env
    m = np.random.default_rng(7).uniform(0, 1, P.slots)
    ct = enc(O, pk, m, 40)
    serial = O.rotsum(ct, gk)
    fused = O.rotsum_hoisted8(ct, gk)
    assert len(O.rotsum_serial_steps()) == P.slots.bit_length() - 1
    assert set(O.rotsum_serial_steps()) <= set(O.rotsum_hoisted8_steps())
    cs = O.decrypt_coeffs(serial, sk)
    cf = O.decrypt_coeffs(fused, sk)
    s1 = int(np.abs(sk.s_coef.astype(np.int64)).sum())
    B = (P.K + 0.5) * (1 + s1) + 1
    diff = np.abs(cs - cf)
    assert diff.max() <= 2 * P.slots * B
    assert diff.max() < P.scale[P.L] / 64
    total = m.sum()
    for c in (serial, fused):
        got = O.decrypt(c, sk)
        assert np.max(np.abs(got - total)) < 2 * P.slots * B / P.scale[P.L] + 1e-9 * total
    # the first serial step alone: ct + Rot(ct, 1) holds m_j + m_{j+1}
    one = O.add(ct, O.rotate(ct, 1, gk))
    assert np.max(np.abs(O.decrypt(one, sk) - (m + np.roll(m, -1)))) < 64 * fresh_std(P)
