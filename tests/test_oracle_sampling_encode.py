"""Pins of the oracle's seeded sampling and its canonical-embedding encoder."""
import decimal

import numpy as np
import pytest

from oracle import ref


def test_splitmix64_published_first_outputs():
    """SplitMix64 (Steele, Lea, Flood 2014) started from state 0 outputs
    0xE220A8397B1DCDAF, then 0x6E789E6AA1B965F4, then 0x06C45D188009454F."""
    L = ref.lib()
    g = 0x9E3779B97F4A7C15
    assert L.orc_splitmix64_next(0) == 0xE220A8397B1DCDAF
    assert L.orc_splitmix64_next(g) == 0x6E789E6AA1B965F4
    assert L.orc_splitmix64_next((2 * g) % (1 << 64)) == 0x06C45D188009454F


def test_ternary_frequencies():
    s = np.zeros(1 << 16, dtype=np.int8)
    ref.lib().orc_sample_ternary(11, 1, len(s), ref._p(s))
    assert set(np.unique(s)) == {-1, 0, 1}
    for v in (-1, 0, 1):
        assert abs(np.mean(s == v) - 1 / 3) < 0.01


def test_uniform_range_and_mean():
    q = 1152921504606830593
    a = np.zeros(1 << 16, dtype=np.uint64)
    ref.lib().orc_sample_uniform(5, 2, 3, q, len(a), ref._p(a))
    assert int(a.max()) < q
    assert abs(float(np.mean(a.astype(np.float64))) / q - 0.5) < 0.01
    b = np.zeros_like(a)
    ref.lib().orc_sample_uniform(5, 2, 4, q, len(b), ref._p(b))   # another limb: another stream
    assert not np.array_equal(a, b)


def test_dg_table_against_decimal_probabilities():
    """Thresholds T_x / 2^64 equal the cumulative probabilities of the
    discrete Gaussian (sigma 3.2, |e| <= 19), computed here with 40-digit
    decimal exp instead of the C library's."""
    thr = np.zeros(19, dtype=np.uint64)
    ref.lib().orc_dg_table(ref._p(thr))
    D = decimal.Decimal
    ctx = decimal.Context(prec=40)
    s2 = D(2) * D("3.2") * D("3.2")
    w = [D(1)] + [D(2) * ctx.exp(-D(x * x) / s2) for x in range(1, 20)]
    total = sum(w)
    cum = D(0)
    for x in range(19):
        cum += w[x]
        assert abs(float(cum / total) - int(thr[x]) / 2.0 ** 64) < 1e-14
    assert all(np.diff(thr.astype(object)) > 0)


def test_dg_moments():
    e = np.zeros(1 << 17, dtype=np.int64)
    ref.lib().orc_sample_dg(9, 3, len(e), ref._p(e))
    assert np.abs(e).max() <= 19
    assert abs(e.std() - 3.2) < 0.05
    assert abs(e.mean()) < 0.05


@pytest.mark.parametrize("logN", [4, 5, 6])
def test_encode_matches_direct_sum(logN):
    """p_k = (2/N) Re sum_j m_j xi_j^(-k) with xi_j = exp(i pi 5^j / N); the
    direct complex sum in numpy agrees with the FFT encoder to within 1."""
    P = ref.Params(logN, 1, 1, 1, 50, 2.0 ** 30, 50)
    O = ref.Oracle(P)
    N, n = P.N, P.N // 2
    m = np.random.default_rng(logN).uniform(-1, 1, n)
    got = O.encode_coeffs(m, 2.0 ** 30)
    e = np.array([pow(5, j, 2 * N) for j in range(n)])
    k = np.arange(N)
    xi = np.exp(-1j * np.pi * np.outer(e, k) / N)
    p = (2.0 / N) * np.real(m @ xi)
    want = np.round(p * 2.0 ** 30)
    assert np.max(np.abs(got - want)) <= 1


def test_constant_vector_encodes_to_constant_polynomial():
    P = ref.Params.preset("c1")
    O = ref.Oracle(P)
    for c in (0.5, -0.37, 3.0):
        got = O.encode_coeffs(np.full(P.slots, c), P.scale[P.L])
        assert got[0] == ref.round_half_away(c * P.scale[P.L])
        assert np.all(got[1:] == 0)


def test_decode_encode_roundtrip_and_unit_vectors():
    P = ref.Params.preset("c1")
    O = ref.Oracle(P)
    s = P.scale[P.L]
    m = np.random.default_rng(0).uniform(-1, 1, P.slots)
    back = O.decode_coeffs(O.encode_coeffs(m, s), s)
    assert np.max(np.abs(back - m)) < P.N / s
    for j in (0, 1, 777, P.slots - 1):
        u = np.zeros(P.slots)
        u[j] = 1.0
        back = O.decode_coeffs(O.encode_coeffs(u, s), s)
        assert abs(back[j] - 1) < 1e-6 and np.max(np.abs(np.delete(back, j))) < 1e-6
