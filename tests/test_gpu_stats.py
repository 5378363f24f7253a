"""GPU statistics: the library's encrypted circuits equal the oracle's bit for
bit (same coefficient table), and decrypt to the FP64 statistics within 1e-3
relative error at the paper's parameters (MI355X only)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import Pair  # noqa: E402

from oracle import cheb, circuits as C, stats64 as S  # noqa: E402
from paper_2508_12093_amd import ffi, synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-3       # relative error bound on decrypted statistics


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return abs(a - b) / abs(b)


# ----------------------------------------------------- t2: bit-exact circuits
@pytest.fixture(scope="module")
def t2():
    _gpu()
    print("\n[stats] preset t2 (N=2^12, L=24)", flush=True)
    p = Pair("t2", steps=())
    p.add_rotsum_keys()
    p.cc = C.Circuits(C.EncEval(p.O, p.orlk, p.ogk))
    base = cheb.invsqrt_coeffs(1e-3, 1.0, 7, 1.0)
    p.cfg = ffi.ppst_invsqrt_cfg_default(coeffs=base)
    p.ocfg = C.InvSqrtCfg(coeffs=base)
    return p


def test_t2_statistics_bit_exact(t2):
    p = t2
    n = 1500                                  # ragged: 1500 rows in 2048 slots
    x, y = synth.binary_cost_pair(0, n)
    cx, ox = p.encrypt(x, 201)
    cy, oy = p.encrypt(y, 202)
    print("[stats] mean/variance", flush=True)
    p.same(ffi.ppst_stat_mean(p.ctx, p.evk, [cy], n, 20.0), p.cc.mean_B([oy], n, 20.0))
    mu = p.cc.mean_B([oy], n, 20.0)
    p.same(ffi.ppst_stat_variance(p.ctx, p.evk, [cy], n, 20.0), p.cc.variance_B([oy], n, 20.0, mu))
    print("[stats] pearson", flush=True)
    pcc = ffi.ppst_stat_pearson(p.ctx, p.evk, [cx], [cy], n, 1.0, 20.0, p.cfg)
    p.same(pcc, p.cc.pearson([ox], [oy], n, 1.0, 20.0, p.ocfg))
    assert rel(p.decrypt(pcc)[0], S.pearson(x, y)) < TOL
    print("[stats] kurtosis/skewness", flush=True)
    k = ffi.ppst_stat_kurtosis(p.ctx, p.evk, [cy], n, 20.0, p.cfg, excess=True)
    p.same(k, p.cc.kurtosis([oy], n, 20.0, p.ocfg, excess=True))
    assert rel(p.decrypt(k)[0], S.kurtosis(y, excess=True)) < TOL
    s = ffi.ppst_stat_skewness(p.ctx, p.evk, [cy], n, 20.0, p.cfg)
    p.same(s, p.cc.skewness([oy], n, 20.0, p.ocfg))
    assert rel(p.decrypt(s)[0], S.skewness(y)) < TOL
    print("[stats] cv/zscore", flush=True)
    cv = ffi.ppst_stat_cv(p.ctx, p.evk, [cy], n, 20.0, 20.0, p.cfg)
    p.same(cv, p.cc.cv([oy], n, 20.0, 20.0, p.ocfg))
    assert rel(p.decrypt(cv)[0], S.cv(y)) < TOL
    z = ffi.ppst_stat_zscore(p.ctx, p.evk, [cy], n, 20.0, p.cfg)
    p.same(z[0], p.cc.zscore([oy], n, 20.0, p.ocfg)[0])
    assert S.mre(p.decrypt(z[0])[:n], S.zscore(y)) < TOL


def test_t2_multi_ciphertext_column(t2):
    """A column longer than one ciphertext (5000 rows = 3 ciphertexts, the
    last one ragged): per-ciphertext terms are added before one RotSum."""
    p = t2
    n = 5000
    x, y = synth.binary_cost_pair(3, n)
    S_ = p.P.slots
    xs, ys = synth.split_column(x, S_), synth.split_column(y, S_)
    cxs, oxs, cys, oys = [], [], [], []
    for i, (a, b) in enumerate(zip(xs, ys)):
        c, o = p.encrypt(a, 300 + i)
        cxs.append(c)
        oxs.append(o)
        c, o = p.encrypt(b, 400 + i)
        cys.append(c)
        oys.append(o)
    pcc = ffi.ppst_stat_pearson(p.ctx, p.evk, cxs, cys, n, 1.0, 20.0, p.cfg)
    p.same(pcc, p.cc.pearson(oxs, oys, n, 1.0, 20.0, p.ocfg))
    assert rel(p.decrypt(pcc)[0], S.pearson(x, y)) < TOL
    z = ffi.ppst_stat_zscore(p.ctx, p.evk, cys, n, 20.0, p.cfg)
    zz = np.concatenate([p.decrypt(c) for c in z])[:n]
    assert S.mre(zz, S.zscore(y)) < TOL
    # the per-ciphertext constant products and level alignments run batched
    # on the device; every output equals the oracle's one-by-one sequence
    for a, b in zip(z, p.cc.zscore(oys, n, 20.0, p.ocfg)):
        p.same(a, b)
    mu = p.cc.mean_B(oys, n, 20.0)
    p.same(ffi.ppst_stat_variance(p.ctx, p.evk, cys, n, 20.0),
           p.cc.variance_B(oys, n, 20.0, mu))
    p.same(ffi.ppst_stat_skewness(p.ctx, p.evk, cys, n, 20.0, p.cfg),
           p.cc.skewness(oys, n, 20.0, p.ocfg))
    p.same(ffi.ppst_stat_kurtosis(p.ctx, p.evk, cys, n, 20.0, p.cfg, excess=True),
           p.cc.kurtosis(oys, n, 20.0, p.ocfg, excess=True))
    for a, b in zip(ffi.ppst_stat_invsqrt(p.ctx, p.evk, cys, 20.0, p.cfg),
                    p.cc.invsqrt(oys, 20.0, p.ocfg)):
        p.same(a, b)


def test_t2_column_longer_than_one_launch_group(t2):
    """A column of 66 ciphertexts (the last one ragged): the n-ary sum runs
    two launches (64 terms, then the rest accumulated), the constant products
    five rescale groups and the squares five product groups; mean and
    variance equal the oracle's left-to-right sequence bit for bit."""
    p = t2
    S_ = p.P.slots
    n = 65 * S_ + 100
    y = synth.lognormal_bernoulli_pair(17, n)[1] / 4.0
    cys, oys = [], []
    for i, v in enumerate(synth.split_column(y, S_)):
        c, o = p.encrypt(v, 5000 + i)
        cys.append(c)
        oys.append(o)
    assert len(cys) == 66
    print("[stats] 66-ciphertext mean/variance", flush=True)
    mean = ffi.ppst_stat_mean(p.ctx, p.evk, cys, n, 2.0)
    omu = p.cc.mean_B(oys, n, 2.0)
    p.same(mean, omu)
    p.same(ffi.ppst_stat_variance(p.ctx, p.evk, cys, n, 2.0), p.cc.variance_B(oys, n, 2.0, omu))
    assert rel(p.decrypt(mean)[0], y.mean() / 2.0) < TOL


def test_t2_closed_forms(t2):
    """PCC(x, a x + b) = sign(a); z-score has mean 0, variance 1; a symmetric
    sample has skewness 0 (absolute error 1e-3)."""
    p = t2
    n = p.P.slots
    x = synth.uniform_column(8, n)
    cx, _ = p.encrypt(x, 501)
    cy, _ = p.encrypt(-2.0 * x + 1.5, 502)
    assert abs(p.decrypt(ffi.ppst_stat_pearson(p.ctx, p.evk, [cx], [cy], n, 1.0, 1.0, p.cfg))[0] + 1) < TOL
    z = p.decrypt(ffi.ppst_stat_zscore(p.ctx, p.evk, [cx], n, 1.0, p.cfg)[0])
    assert abs(z.mean()) < TOL and abs(z.var() - 1) < TOL
    half = x[: n // 2]
    cs, _ = p.encrypt(np.concatenate([half, 1.0 - half]), 503)
    assert abs(p.decrypt(ffi.ppst_stat_skewness(p.ctx, p.evk, [cs], n, 1.0, p.cfg))[0]) < TOL


def _exp1_cfgs():
    """Exp. 1 (Sec. 6.2): Eq. 3's degree-31 Chebyshev initial value on the
    domain map [0, 2] -> [-1, 1], six Newton steps; the same table both sides."""
    base = cheb.paper_invsqrt_coeffs(31, 1.0)
    return (ffi.ppst_invsqrt_cfg_default(coeffs=base, a=0.0, b=2.0, degree=31, iters=6),
            C.InvSqrtCfg(a=0.0, b=2.0, degree=31, iters=6, coeffs=base))


def test_t2_invsqrt_bit_exact(t2):
    """CryptoInvSqrt on two ciphertexts (evaluated side by side by the
    library, one after the other by the oracle): bit-exact, 19 levels."""
    p = t2
    cfg, ocfg = _exp1_cfgs()
    v = cheb.exp1_grid(p.P.slots)
    c1, o1 = p.encrypt(v, 701)
    c2_, o2 = p.encrypt(v[::-1].copy(), 702)
    print("[stats] invsqrt degree 31, 6 Newton steps", flush=True)
    got = ffi.ppst_stat_invsqrt(p.ctx, p.evk, [c1, c2_], 100.0, cfg)
    want = p.cc.invsqrt([o1, o2], 100.0, ocfg)
    assert want[0].level == p.P.L - 19
    p.same(got[0], want[0])
    p.same(got[1], want[1])
    assert np.max(np.abs(p.decrypt(got[0]) / cheb.exp1_model(v) - 1)) < 1e-4


def test_t2_invsqrt_degree_63_and_limits(t2):
    """A degree-63 Chebyshev ladder (62 products, its 63-term weighted sum
    over eleven launches of six terms) stays bit-exact; degree 512 and a
    negative interval start are refused."""
    p = t2
    base = cheb.invsqrt_coeffs(0.05, 1.0, 63, 1.0)
    cfg = ffi.ppst_invsqrt_cfg_default(coeffs=base, a=0.05, b=1.0, degree=63, iters=2)
    ocfg = C.InvSqrtCfg(a=0.05, b=1.0, degree=63, iters=2, coeffs=base)
    v = synth.uniform_column(21, p.P.slots, 0.05, 1.0)
    c, o = p.encrypt(v, 711)
    got = ffi.ppst_stat_invsqrt(p.ctx, p.evk, [c], 1.0, cfg)[0]
    p.same(got, p.cc.invsqrt([o], 1.0, ocfg)[0])
    assert np.max(np.abs(p.decrypt(got) * np.sqrt(v) - 1)) < 1e-3
    for bad in (ffi.ppst_invsqrt_cfg_default(degree=512), ffi.ppst_invsqrt_cfg_default(a=-0.5)):
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_stat_invsqrt(p.ctx, p.evk, [c], 1.0, bad)
        assert e.value.name == "EDOMAIN"


def test_t2_depth_errors(t2):
    p = t2
    x = synth.uniform_column(9, 100)
    low, _ = p.encrypt(x, 601, level=10)
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_stat_cv(p.ctx, p.evk, [low], 100, 1.0, 1.0, p.cfg)
    assert e.value.name == "ELEVEL"
    bad = ffi.ppst_invsqrt_cfg_default(a=-1.0)
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_stat_kurtosis(p.ctx, p.evk, [low], 100, 1.0, bad)
    assert e.value.name == "EDOMAIN"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_stat_mean(p.ctx, p.evk, [low], 5000, 1.0)
    assert e.value.name == "EINVAL"


# ------------------------------------------------ c2: the paper's parameters
@pytest.fixture(scope="module")
def c2():
    _gpu()
    print("\n[stats] preset c2 (N=2^16, L=24)", flush=True)
    ctx = ffi.ppst_context_create("c2")
    sk, pk = ffi.ppst_keygen(ctx, 101)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 102, evk)
    ffi.ppst_evk_add_rotsum(ctx, sk, 103, evk)
    return ctx, sk, pk, evk


def test_c2_config2_statistics_within_tolerance(c2):
    """Two 32768-row columns: x ~ Bernoulli(0.2), y lognormal cost with
    corr ~ 0.79; Chebyshev degree 7 on [1e-3, 1] + 3 Newton steps, B_y = 20,
    B_x = 1.  Decrypted statistics within 1e-3 of FP64."""
    ctx, sk, pk, evk = c2
    x, y = synth.binary_cost_pair(0)
    n = len(x)
    cx = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, x, 24), 201)
    cy = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, y, 24), 202)
    dec = lambda c: ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, c))
    cfg = ffi.ppst_invsqrt_cfg_default()
    got = {
        "pearson": dec(ffi.ppst_stat_pearson(ctx, evk, [cx], [cy], n, 1.0, 20.0, cfg))[0],
        "kurtosis": dec(ffi.ppst_stat_kurtosis(ctx, evk, [cy], n, 20.0, cfg))[0],
        "skewness": dec(ffi.ppst_stat_skewness(ctx, evk, [cy], n, 20.0, cfg))[0],
        "cv": dec(ffi.ppst_stat_cv(ctx, evk, [cy], n, 20.0, 20.0, cfg))[0],
    }
    want = {"pearson": S.pearson(x, y), "kurtosis": S.kurtosis(y), "skewness": S.skewness(y),
            "cv": S.cv(y)}
    for k in got:
        print("[stats] %-9s %.8f vs %.8f  rel %.2e" % (k, got[k], want[k], rel(got[k], want[k])), flush=True)
        assert rel(got[k], want[k]) < TOL, k
    z = dec(ffi.ppst_stat_zscore(ctx, evk, [cy], n, 20.0, cfg)[0])
    assert S.mre(z, S.zscore(y)) < TOL


def test_c2_exp1_invsqrt_replay(c2):
    """Tab. 2's CryptoInvSqrt row at the paper's parameters without
    bootstrapping: the 32768-point grid on [0.001, 100], B = 100, degree 31,
    six Newton steps fit 19 of the 24 levels; the decrypted MRE against
    1/sqrt(x) equals the FP64 model's (5.11e-5; printed 5.08e-5) to 3e-6
    (the encryption noise, amplified near x = 0.001 where the Newton steps
    have not converged, adds about 1e-6)."""
    ctx, sk, pk, evk = c2
    cfg, _ = _exp1_cfgs()
    v = cheb.exp1_grid()
    ct = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, v, 24), 801)
    y = ffi.ppst_stat_invsqrt(ctx, evk, [ct], 100.0, cfg)[0]
    got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, y))
    ref = 1.0 / np.sqrt(v)
    mre, model = S.mre(got, ref), S.mre(cheb.exp1_model(v), ref)
    print("[stats] Exp. 1 replay: MRE %.4e (FP64 model %.4e)" % (mre, model), flush=True)
    assert abs(mre - model) < 3e-6


def test_c2_exp2_replay_one_million_rows(c2):
    """Tab. 3's workloads without bootstrapping: 10^6 rows (31 ciphertexts,
    the last ragged); ZNorm on U[0, 100] (B = 100), skewness, kurtosis and
    PCC on U[0, 20] (B = 20) with Exp. 1's InvSqrt; CV with B_mean = 16,
    B_var = 20 and the default InvSqrt.  Each within 1e-3 of FP64 (relative;
    absolute for the skewness, which is about 2e-4 for a uniform sample, so
    its relative error is ill-conditioned, as Tab. 3's spread shows)."""
    ctx, sk, pk, evk = c2
    n, slots = 1_000_000, 32768
    x100 = synth.uniform_column(11, n, 0.0, 100.0)
    x20 = synth.uniform_column(12, n, 0.0, 20.0)
    y20 = 0.5 * (x20 + synth.uniform_column(13, n, 0.0, 20.0))

    def enc(v, seed):
        return [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, c, 24), seed + k)
                for k, c in enumerate(synth.split_column(v, slots))]

    dec = lambda c: ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, c))
    c100, c20, cy = enc(x100, 40000), enc(x20, 41000), enc(y20, 42000)
    assert len(c100) == 31
    e1, _ = _exp1_cfgs()
    z = np.concatenate([dec(c) for c in ffi.ppst_stat_zscore(ctx, evk, c100, n, 100.0, e1)])[:n]
    got = {
        "zscore": S.mre(z, S.zscore(x100)),
        "skewness": abs(dec(ffi.ppst_stat_skewness(ctx, evk, c20, n, 20.0, e1))[0] - S.skewness(x20)),
        "kurtosis": rel(dec(ffi.ppst_stat_kurtosis(ctx, evk, c20, n, 20.0, e1))[0], S.kurtosis(x20)),
        "cv": rel(dec(ffi.ppst_stat_cv(ctx, evk, c20, n, 16.0, 20.0, ffi.ppst_invsqrt_cfg_default()))[0],
                  S.cv(x20)),
        "pearson": rel(dec(ffi.ppst_stat_pearson(ctx, evk, c20, cy, n, 20.0, 20.0, e1))[0],
                       S.pearson(x20, y20)),
    }
    for k, v in got.items():
        print("[stats] Exp. 2 %-8s error %.3e" % (k, v), flush=True)
        assert v < TOL, k
