"""Pins of the oracle's statistics layer: FP64 closed forms, the paper's
Tab. 2 number, g_3, and the circuits (FP64 model and encrypted)."""
import json
import os

import numpy as np
import pytest

from oracle import cheb, circuits as C, ref, stats64 as S
from paper_2508_12093_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# --------------------------------------------------------------- closed forms
def test_fp64_stat_closed_forms():
    rng = np.random.default_rng(0)
    x = rng.lognormal(0, 1, 5000)
    z = S.zscore(x)
    assert abs(z.mean()) < 1e-12 and abs(z.var() - 1) < 1e-12
    assert abs(S.pearson(x, 3 * x + 2) - 1) < 1e-12
    assert abs(S.pearson(x, -0.5 * x + 7) + 1) < 1e-12
    sym = np.concatenate([x, -x])
    assert abs(S.skewness(sym)) < 1e-12
    two = np.array([-1.0, 1.0] * 100)
    assert abs(S.kurtosis(two) - 1) < 1e-12 and abs(S.kurtosis(two, excess=True) + 2) < 1e-12
    p = 0.2
    b = np.array([1.0] * 200 + [0.0] * 800)
    assert abs(S.kurtosis(b) - (1 - 3 * p * (1 - p)) / (p * (1 - p))) < 1e-12
    assert abs(S.cv(4.0 * x) - S.cv(x)) < 1e-12
    for f in (S.skewness, S.kurtosis, S.cv):
        assert abs(f(2.5 * x) - f(x)) < 1e-10


# --------------------------------------------------------- paper's numbers
def test_tab2_cryptoinvsqrt_mre():
    """Tab. 2: CryptoInvSqrt on the Exp-1 grid (B = 100, 6 Newton steps) has
    MRE 5.08e-5.  The FP64 model with a degree-31 first-kind Chebyshev
    initial value of Eq. 3 lands within 1% of it; degrees 30 and 32 do not."""
    paper = GOLD["exp1_cryptoinvsqrt_mre"]["value"]
    iters = GOLD["exp1_newton_iters"]["value"]
    B = GOLD["exp1_B"]["value"]
    g = GOLD["exp1_grid"]["value"]
    grid = cheb.exp1_grid()
    assert len(grid) == g["low"][2] + g["high"][2]
    assert grid[0] == g["low"][0] and grid[-1] == g["high"][1]
    assert abs(cheb.exp1_mre(31, iters, B) / paper - 1) < 0.01
    for d in (30, 32):
        assert abs(cheb.exp1_mre(d, iters, B) / paper - 1) > 0.1


def test_g3_coefficients_and_shape():
    gold = GOLD["g3_coeffs_times_16"]["value"]
    for k, v in gold.items():
        assert cheb.G3_COEFFS[int(k)] * 16 == v
    x = np.linspace(-1, 1, 201)
    assert np.allclose(cheb.g3(-x), -cheb.g3(x))
    assert cheb.g3(1.0) == 1.0 and cheb.g3(-1.0) == -1.0
    h = 1e-6       # g3'(x) = 35/16 (1 - x^2)^3
    for t in (0.0, 0.3, 0.9):
        d = (cheb.g3(t + h) - cheb.g3(t - h)) / (2 * h)
        assert abs(d - 35 / 16 * (1 - t * t) ** 3) < 1e-6
    assert 5e-5 < 1 - cheb.g3(cheb.g3(0.6)) < 1e-4


def test_invsqrt_chebyshev_interpolates_and_newton_converges():
    a, b, d = 1e-3, 1.0, 7
    c = cheb.invsqrt_coeffs(a, b, d, 1.0)
    nodes = np.cos(np.pi * (np.arange(d + 1) + 0.5) / (d + 1))
    v = a + (b - a) * (nodes + 1) / 2
    assert np.allclose(np.polynomial.chebyshev.chebval(nodes, c), 1 / np.sqrt(v), rtol=1e-12)
    vs = np.linspace(0.0053, 1.0, 20000)
    t = (2 * vs - a - b) / (b - a)
    y0 = np.polynomial.chebyshev.chebval(t, c)
    e2 = np.abs(cheb.newton_invsqrt(vs, y0, 2) * np.sqrt(vs) - 1)
    e3 = np.abs(cheb.newton_invsqrt(vs, y0, 3) * np.sqrt(vs) - 1)
    assert np.max(e3) < 5e-4                       # worst near v = 0.033
    assert np.max(e3[vs >= 0.05]) < 1e-4
    assert np.all(e3 <= 1.5 * e2 ** 2 * 1.01 + 1e-15)   # Newton's quadratic step
    c20 = cheb.invsqrt_coeffs(a, b, d, 20.0)
    assert np.allclose(c20, c / np.sqrt(20.0))


# ------------------------------------------------------------- FP64 circuits
def _levels_and_values(n=32768):
    x, y = synth.binary_cost_pair(0, n)
    ev = C.PlainEval(24, 32768)
    cc = C.Circuits(ev)
    cfg = C.InvSqrtCfg()
    X, Y = [ev.fresh(x)], [ev.fresh(y)]
    return x, y, {
        "zscore": cc.zscore(Y, n, 20.0, cfg)[0],
        "kurt": cc.kurtosis(Y, n, 20.0, cfg),
        "skew": cc.skewness(Y, n, 20.0, cfg),
        "cv": cc.cv(Y, n, 20.0, 20.0, cfg),
        "pcc": cc.pearson(X, Y, n, 1.0, 20.0, cfg),
    }


def _sqrt1px_aliased(degree):
    """Coefficients of the degree-d interpolant of sqrt(1 + x) at the d + 1
    first-kind Chebyshev nodes, from the closed-form series
    sqrt(1 + x) = (2 sqrt 2 / pi) (1 + 2 sum_k (-1)^(k+1) T_k(x) / (4k^2 - 1))
    (the cosine series of sqrt 2 cos(theta / 2), x = cos theta) and the
    aliasing of T_(2m n +- k) onto (-1)^m T_k at those n = d + 1 nodes."""
    n = degree + 1
    amp = 2.0 * np.sqrt(2.0) / np.pi

    def a(k):
        k = np.asarray(k, dtype=np.float64)
        return np.where(k == 0, amp, amp * 2.0 * (-1.0) ** (k + 1) / (4.0 * k * k - 1.0))

    m = np.arange(1, 400001, dtype=np.float64)
    sign = (-1.0) ** m
    c = np.empty(n)
    c[0] = a(0) + np.sum(sign * a(2 * m * n))
    for k in range(1, n):
        c[k] = a(k) + np.sum(sign * (a(2 * m * n - k) + a(2 * m * n + k)))
    return c


@pytest.mark.parametrize("degree,B", [(7, 1.0), (7, 20.0), (31, 100.0)])
def test_paper_sqrt_coefficients_closed_form(degree, B):
    """Eq. 4 (CryptoSqrt's initial polynomial sqrt(B) sqrt(x + 1) on
    [-1, 1]): the oracle's interpolated coefficients equal the closed-form
    Chebyshev series with its aliasing summed, and the polynomial matches
    the function at the nodes."""
    got = cheb.paper_sqrt_coeffs(degree, B)
    want = np.sqrt(B) * _sqrt1px_aliased(degree)
    assert np.max(np.abs(got - want)) < 1e-12 * np.sqrt(B)
    nodes = np.cos(np.pi * (np.arange(degree + 1) + 0.5) / (degree + 1))
    assert np.allclose(np.polynomial.chebyshev.chebval(nodes, got), np.sqrt(B * (nodes + 1.0)),
                       rtol=0, atol=1e-13 * np.sqrt(B))


def test_plain_circuits_match_fp64_and_depths():
    x, y, r = _levels_and_values()
    assert S.mre(r["zscore"].v, S.zscore(y)) < 1e-6
    assert abs(r["kurt"].v[0] / S.kurtosis(y) - 1) < 1e-6
    assert abs(r["skew"].v[0] / S.skewness(y) - 1) < 1e-6
    assert abs(r["cv"].v[0] / S.cv(y) - 1) < 1e-6
    assert abs(r["pcc"].v[0] / S.pearson(x, y) - 1) < 1e-5      # v_x = 0.16: Newton residual 1.2e-6
    depth = {k: 24 - v.level for k, v in r.items()}
    assert depth == {"zscore": 15, "kurt": 17, "skew": 16, "cv": 23, "pcc": 16}


def _exp1_cfg():
    """Exp. 1 (Sec. 6.2): Eq. 3's Chebyshev initial value, degree 31 on the
    domain map [0, 2] -> [-1, 1], six Newton steps."""
    return C.InvSqrtCfg(a=0.0, b=2.0, degree=31, iters=6,
                        coeffs=cheb.paper_invsqrt_coeffs(31, 1.0))


def test_plain_invsqrt_circuit_is_exp1_model():
    """The CryptoInvSqrt circuit (v = x/B, then InvSqrt(v; B)) in FP64 with
    levels equals the closed-form Tab. 2 model slot by slot, reaches the
    printed MRE, and consumes 19 of the 24 levels (no bootstrapping; the
    domain map of Eq. 1 is a pure shift and costs no level)."""
    v = cheb.exp1_grid()
    assert np.array_equal(v, synth.exp1_grid())     # the benchmark's input
    ev = C.PlainEval(24, len(v))
    y = C.Circuits(ev).invsqrt([ev.fresh(v)], 100.0, _exp1_cfg())[0]
    assert np.max(np.abs(y.v / cheb.exp1_model(v) - 1)) < 1e-9
    assert abs(S.mre(y.v, 1.0 / np.sqrt(v)) / GOLD["exp1_cryptoinvsqrt_mre"]["value"] - 1) < 0.01
    assert 24 - y.level == 19


# ------------------------------------------------------ encrypted circuits
@pytest.fixture(scope="module")
def t2():
    P = ref.Params.preset("t2")
    O = ref.Oracle(P)
    sk, pk = O.keygen(101)
    rlk = O.relin_key(sk, 102)
    gk = O.rotation_keys(sk, 103, O.rotsum_hoisted8_steps())
    return P, O, sk, pk, C.Circuits(C.EncEval(O, rlk, gk))


@pytest.mark.slow
def test_encrypted_statistics_match_fp64(t2):
    P, O, sk, pk, cc = t2
    n = 1500                                   # ragged: 1500 of 2048 slots
    x, y = synth.binary_cost_pair(0, n)
    ex, ey = O.encrypt(O.encode(x), pk, 201), O.encrypt(O.encode(y), pk, 202)
    cfg = C.InvSqrtCfg()
    dec = lambda c: O.decrypt(c, sk)
    assert abs(dec(cc.pearson([ex], [ey], n, 1.0, 20.0, cfg))[0] / S.pearson(x, y) - 1) < 1e-3
    assert abs(dec(cc.kurtosis([ey], n, 20.0, cfg))[0] / S.kurtosis(y) - 1) < 1e-3
    assert abs(dec(cc.skewness([ey], n, 20.0, cfg))[0] / S.skewness(y) - 1) < 1e-3
    assert abs(dec(cc.cv([ey], n, 20.0, 20.0, cfg))[0] / S.cv(y) - 1) < 1e-3
    z = dec(cc.zscore([ey], n, 20.0, cfg)[0])[:n]
    assert S.mre(z, S.zscore(y)) < 1e-3


@pytest.mark.slow
def test_encrypted_closed_forms(t2):
    P, O, sk, pk, cc = t2
    n = P.slots
    x = np.random.default_rng(8).uniform(0, 1, n)
    ex = O.encrypt(O.encode(x), pk, 301)
    ey = O.encrypt(O.encode(-2.0 * x + 1.5), pk, 302)
    cfg = C.InvSqrtCfg()
    pcc = O.decrypt(cc.pearson([ex], [ey], n, 1.0, 1.0, cfg), sk)[0]
    assert abs(pcc + 1) < 1e-3
    z = O.decrypt(cc.zscore([ex], n, 1.0, cfg)[0], sk)
    assert abs(z.mean()) < 1e-3 and abs(z.var() - 1) < 1e-3
    half = x[: n // 2]
    sym = np.concatenate([half, 1.0 - half])   # symmetric about 0.5
    es = O.encrypt(O.encode(sym), pk, 303)
    assert abs(O.decrypt(cc.skewness([es], n, 1.0, cfg), sk)[0]) < 1e-3


@pytest.mark.slow
def test_encrypted_invsqrt_exp1(t2):
    """Encrypted CryptoInvSqrt on a 2048-point version of the Exp. 1 grid:
    each slot within 1e-4 of the FP64 model (the ladder and the unconverged
    Newton steps near x = 0.001 amplify the encryption noise to about 3e-5;
    elsewhere 1e-8), MRE against 1/sqrt(x) that of the model to 1e-6, 19
    levels consumed."""
    P, O, sk, pk, cc = t2
    v = cheb.exp1_grid(P.slots)
    y = cc.invsqrt([O.encrypt(O.encode(v), pk, 401)], 100.0, _exp1_cfg())[0]
    assert y.level == P.L - 19
    got = O.decrypt(y, sk)
    model = cheb.exp1_model(v)
    assert np.max(np.abs(got / model - 1)) < 1e-4
    ref = 1.0 / np.sqrt(v)
    assert abs(S.mre(got, ref) - S.mre(model, ref)) < 1e-6


def test_config1_mean_variance():
    """Config 1: N = 2^12, 2048 slots ~ U[0,1): Mean (B=1) and Variance (Eq. 2)."""
    P = ref.Params.preset("c1")
    O = ref.Oracle(P)
    sk, pk = O.keygen(1)
    rlk = O.relin_key(sk, 101)
    gk = O.rotation_keys(sk, 102, O.rotsum_hoisted8_steps())
    x = synth.uniform_column(1, P.slots)
    ct = O.encrypt(O.encode(x), pk, 201)
    cc = C.Circuits(C.EncEval(O, rlk, gk))
    mu = cc.mean_B([ct], P.slots, 1.0)
    var = cc.variance_B([ct], P.slots, 1.0, mu)
    assert var.level == 0
    assert abs(O.decrypt(mu, sk)[0] / S.mean(x) - 1) < 1e-3
    assert abs(O.decrypt(var, sk)[0] / S.var(x) - 1) < 1e-3
