"""Bootstrapping on the GPU through the C-ABI against the oracle.

At N = 2^12 ("b1", the bootstrappable chain of "b2") every stage is compared
bit for bit with ``oracle/boot.py`` on the same keys and inputs: the sparse
secret, ModRaise, conjugation and X^n, CoeffToSlot, the split into real and
imaginary parts, EvalMod, SlotToCoeff and the whole refresh.  EvalMod takes
the oracle's Chebyshev coefficients (an input; the library's own
interpolation agrees to 1e-14, tests/test_abi_host.py).  At N = 2^16 ("b2")
the refresh is checked by what holds at any size: it decrypts to the
message, lands on level Lc, and computes on.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import Pair  # noqa: E402

from oracle import boot, cheb, ref, stats64  # noqa: E402
from oracle import circuits as C  # noqa: E402
from paper_2508_12093_amd import ffi, synth  # noqa: E402

pytestmark = pytest.mark.gpu

BOOT_SEED = 21


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def bp():
    _torch()
    p = Pair("b1", steps=())
    print("b1: keys, plaintexts", flush=True)
    coeffs = cheb.evalmod_cos_coeffs(16, 4, 27)
    ffi.ppst_evk_add_boot(p.ctx, p.sk, BOOT_SEED, p.evk)
    p.bt = ffi.ppst_boot_create(p.ctx, coeffs)
    p.OB = boot.Bootstrapper(p.O, p.osk, BOOT_SEED, coeffs=coeffs)
    # the oracle's Bootstrapper makes its own relinearisation key from the
    # same seed; the library's comes from Pair (seed 12): use that one
    p.OB.rlk = p.orlk
    p.OB.circ.ev.rlk = p.orlk
    return p


def level0(p, seed):
    m = synth.uniform_column(seed, p.P.slots, -1, 1)
    ct, oct_ = p.encrypt(m, 100 + seed, level=0)
    return m, ct, oct_


def test_sparse_secret_and_keys(bp):
    p = bp
    s = p.osk.s_coef
    assert np.count_nonzero(s) == 64
    assert np.array_equal(ffi.ppst_sk_export(p.ctx, p.sk), p.osk.s_ntt)
    g = 2 * p.P.N - 1
    assert np.array_equal(ffi.ppst_evk_export(p.ctx, p.evk, g), p.OB.gkeys[g])
    r = boot.rotation_steps(p.P)[3]
    ge = ref.galois_element(r, p.P.N)
    assert np.array_equal(ffi.ppst_evk_export(p.ctx, p.evk, ge), p.OB.gkeys[ge])


def test_mod_raise_conj_monomial(bp):
    p = bp
    _, ct, oct_ = level0(p, 1)
    p.same(ct, oct_)
    raised = ffi.ppst_mod_raise(p.ctx, ct)
    oraised = p.OB.mod_raise(oct_)
    p.same(raised, oraised)
    cj = ffi.ppst_apply_galois(p.ctx, p.evk, raised, 2 * p.P.N - 1)
    p.same(cj, p.OB.apply_galois(oraised, 2 * p.P.N - 1))
    for k, sign in ((p.P.slots, 1), (p.P.slots, -1), (5, 1)):
        p.same(ffi.ppst_mul_monomial(p.ctx, raised, k, sign), p.OB.mul_monomial(oraised, k, sign))


def test_stages_bit_exact(bp):
    p = bp
    _, ct, oct_ = level0(p, 2)
    raised = ffi.ppst_mod_raise(p.ctx, ct)
    oraised = p.OB.mod_raise(oct_)
    w = ffi.ppst_boot_coeff_to_slot(p.ctx, p.evk, p.bt, raised)
    ow = p.OB.coeff_to_slot(oraised)
    p.same(w, ow)
    re, im = ffi.ppst_boot_split(p.ctx, p.evk, p.bt, w)
    ore, oim = p.OB.split(ow)
    p.same(re, ore)
    p.same(im, oim)
    yr, yi = ffi.ppst_boot_eval_mod(p.ctx, p.evk, p.bt, [re, im])
    oyr, oyi = p.OB.eval_mod(ore), p.OB.eval_mod(oim)
    p.same(yr, oyr)
    p.same(yi, oyi)
    out = ffi.ppst_boot_slot_to_coeff(p.ctx, p.evk, p.bt, yr, yi)
    p.same(out, p.OB.slot_to_coeff(p.O.add(oyr, p.OB.mul_monomial(oyi, p.P.slots, 1))))


def test_bootstrap_bit_exact_and_refreshes(bp):
    p = bp
    m, ct, oct_ = level0(p, 3)
    out = ffi.ppst_bootstrap(p.ctx, p.evk, p.bt, ct)
    oout = p.OB.bootstrap(oct_)
    p.same(out, oout)
    assert out.level == p.P.Lc
    got = p.decrypt(out)
    assert np.max(np.abs(got - m)) < 2.0 ** -19
    # the refreshed ciphertext computes on
    sq = ffi.ppst_mul(p.ctx, p.evk, out, out)
    assert np.max(np.abs(p.decrypt(sq) - m * m)) < 2.0 ** -18


def test_bootstrap_errors(bp):
    p = bp
    _, ct, _ = level0(p, 4)
    raised = ffi.ppst_mod_raise(p.ctx, ct)
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_bootstrap(p.ctx, p.evk, p.bt, raised)          # not level 0
    assert e.value.name == "ELEVEL"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_mul(p.ctx, p.evk, raised, raised)              # a transform level
    assert e.value.name == "ESCALE"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_apply_galois(p.ctx, p.evk, raised, 4)          # even element
    assert e.value.name == "EINVAL"
    with pytest.raises(ffi.PpstError):
        ffi.ppst_boot_create(p.ctx, np.zeros(5))                # wrong coefficient count
    other = ffi.ppst_context_create("c1")
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_boot_create(other)
    assert e.value.name == "EINVAL"
    # the raised exceptions' tracebacks hold this frame: drop the handles now
    # rather than whenever the cycle collector runs
    del e, other, raised, ct


EXP1_COEFFS = cheb.paper_invsqrt_coeffs(31, 1.0)


def exp2_columns(seed, n):
    """Sec. 6.3's kurtosis / PCC data: x ~ U[0, 20], y = (x + u) / 2, u ~ U[0, 20]."""
    x = synth.uniform_column(seed, n, 0.0, 20.0)
    y = 0.5 * (x + synth.uniform_column(seed + 1, n, 0.0, 20.0))
    return x, y


@pytest.fixture(scope="module")
def bstat(bp):
    """bp with the RotSum keys the statistics need: the library adds them
    after the bootstrapping keys (existing Galois elements keep their key),
    the oracle's dictionary is built the same way."""
    p = bp
    p.ogk = dict(p.OB.gkeys)
    p.add_rotsum_keys()
    p.ev = C.EncEval(p.O, p.orlk, p.ogk, booter=p.OB)
    p.circ = C.Circuits(p.ev)
    return p


def test_b1_statistics_with_refreshes_bit_exact(bstat):
    """Kurtosis and PCC over a two-ciphertext column at the paper's InvSqrt
    (Eq. 3's degree 31 on [0, 2], six Newton steps, B = 20): 11 levels do
    not hold it, so InvSqrt refreshes by bootstrapping.  The library and
    the oracle agree bit for bit; the values agree with FP64 to 1e-4."""
    p = bstat
    n = 3000
    x, y = exp2_columns(50, n)

    def enc(v, seed):
        cts, octs = [], []
        for k in range(0, n, p.P.slots):
            c, o = p.encrypt(v[k:k + p.P.slots], seed + k, level=p.P.Lc)
            cts.append(c)
            octs.append(o)
        return cts, octs

    X, OX = enc(x, 600)
    Y, OY = enc(y, 700)
    cfg = ffi.ppst_invsqrt_cfg_default(coeffs=EXP1_COEFFS, a=0.0, b=2.0, degree=31, iters=6, boot=p.bt)
    ocfg = C.InvSqrtCfg(a=0.0, b=2.0, degree=31, iters=6, coeffs=EXP1_COEFFS, boot=True)
    print("b1 kurtosis with refreshes", flush=True)
    k = ffi.ppst_stat_kurtosis(p.ctx, p.evk, X, n, 20.0, cfg)
    ok = p.circ.kurtosis(OX, n, 20.0, ocfg)
    p.same(k, ok)
    assert abs(p.decrypt(k)[0] / stats64.kurtosis(x) - 1) < 1e-4
    print("b1 PCC with refreshes", flush=True)
    r = ffi.ppst_stat_pearson(p.ctx, p.evk, X, Y, n, 20.0, 20.0, cfg)
    orr = p.circ.pearson(OX, OY, n, 20.0, 20.0, ocfg)
    p.same(r, orr)
    assert abs(p.decrypt(r)[0] / stats64.pearson(x, y) - 1) < 1e-4


def test_b1_cv_and_comparator_with_refreshes_bit_exact(bstat):
    """CV at Exp. 2's B = 20 with a three-fold g_3 sign (mu / B = 0.5) and
    the paper's InvSqrt, its sign refreshed between compositions; and the
    HEaaN-STAT comparator of Exp. 1 (y_0 = 1, a degree-0 initial value, 21
    Newton steps on x / 100).  Bit-exact with the oracle; CV within 1e-4 of
    FP64, the comparator's MRE below 1e-6 on a 2048-point Exp. 1 grid."""
    p = bstat
    n = 3000
    x, _ = exp2_columns(70, n)
    X, OX = [], []
    for k in range(0, n, p.P.slots):
        c, o = p.encrypt(x[k:k + p.P.slots], 1000 + k, level=p.P.Lc)
        X.append(c)
        OX.append(o)
    cfg = ffi.ppst_invsqrt_cfg_default(coeffs=EXP1_COEFFS, a=0.0, b=2.0, degree=31, iters=6,
                                       sign_k=3, boot=p.bt)
    ocfg = C.InvSqrtCfg(a=0.0, b=2.0, degree=31, iters=6, coeffs=EXP1_COEFFS, boot=True)
    print("b1 CV with refreshes", flush=True)
    r = ffi.ppst_stat_cv(p.ctx, p.evk, X, n, 20.0, 20.0, cfg)
    p.same(r, p.circ.cv(OX, n, 20.0, 20.0, ocfg, sign_k=3))
    assert abs(p.decrypt(r)[0] / stats64.cv(x) - 1) < 1e-4
    print("b1 HEaaN-STAT comparator", flush=True)
    g = np.concatenate([np.linspace(0.001, 1.0, 1024), np.linspace(1.0, 100.0, 1024)])
    cg, og = p.encrypt(g, 1100, level=p.P.Lc)
    hcfg = ffi.ppst_invsqrt_cfg_default(coeffs=np.array([1.0]), a=0.0, b=2.0, degree=0, iters=21,
                                        boot=p.bt)
    y = ffi.ppst_stat_invsqrt(p.ctx, p.evk, [cg], 100.0, hcfg)[0]
    oy = p.circ.invsqrt([og], 100.0, C.InvSqrtCfg(a=0.0, b=2.0, degree=0, iters=21,
                                                   coeffs=np.array([1.0]), boot=True))[0]
    p.same(y, oy)
    assert np.mean(np.abs(p.decrypt(y) * np.sqrt(g) - 1.0)) < 1e-6


def test_b1_cv_full_range_sign_bit_exact(bstat):
    """CV with a negative mean and with a mean near zero: the sign of mu / B
    by Exp. 1's seven-fold g_3 composition (G_3^(7), 21 levels, so it
    refreshes twice), mu / B = -0.5 and -0.1.  Bit-exact with the oracle;
    within 1e-3 of FP64 (the sign's error at 0.1 is below 1e-9)."""
    p = bstat
    n = 2048
    cfg = ffi.ppst_invsqrt_cfg_default(coeffs=EXP1_COEFFS, a=0.0, b=2.0, degree=31, iters=6,
                                       sign_k=7, boot=p.bt)
    ocfg = C.InvSqrtCfg(a=0.0, b=2.0, degree=31, iters=6, coeffs=EXP1_COEFFS, boot=True)
    for lo, hi, seed in ((-18.0, -2.0, 1200), (-12.0, 8.0, 1300)):
        x = synth.uniform_column(seed, n, lo, hi)
        c, o = p.encrypt(x, seed + 1, level=p.P.Lc)
        print("b1 CV with G_3^(7), mean %.3f" % float(np.mean(x)), flush=True)
        r = ffi.ppst_stat_cv(p.ctx, p.evk, [c], n, 20.0, 20.0, cfg)
        p.same(r, p.circ.cv([o], n, 20.0, 20.0, ocfg, sign_k=7))
        want = stats64.cv(x)                     # sigma / mu, negative here
        assert want < 0
        assert abs(p.decrypt(r)[0] / want - 1) < 1e-3


def test_b2_bootstrap_refreshes():
    """N = 2^16: the refresh of a full [-1, 1] column decrypts to it (max
    error 2^-15, about 2^-17 measured), lands on level 11 and computes on;
    the library's own EvalMod coefficients."""
    _torch()
    print("b2: keys, plaintexts", flush=True)
    ctx = ffi.ppst_context_create("b2")
    sk, pk = ffi.ppst_keygen(ctx, 31)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 32, evk)
    ffi.ppst_evk_add_boot(ctx, sk, 33, evk)
    bt = ffi.ppst_boot_create(ctx)
    n = 1 << 15
    m = synth.uniform_column(7, n, -1, 1)
    ct = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, m, 0), 34)
    print("b2: bootstrap", flush=True)
    out = ffi.ppst_bootstrap(ctx, evk, bt, ct)
    assert out.level == 11
    got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, out), n)
    err = np.max(np.abs(got - m))
    print("b2 refresh max error 2^%.2f" % np.log2(err), flush=True)
    assert err < 2.0 ** -15
    sq = ffi.ppst_mul(ctx, evk, out, out)
    got2 = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, sq), n)
    assert np.max(np.abs(got2 - m * m)) < 2.0 ** -14


def test_b2_statistics_with_bootstrapping_one_million_rows():
    """The full pipeline at N = 2^16: kurtosis and PCC of 2^20-row columns
    (32 ciphertexts at level 11) with the paper's InvSqrt (degree 31, six
    Newton steps), which 11 levels cannot hold, so InvSqrt bootstraps.
    Decrypted values within 1e-3 relative of FP64."""
    _torch()
    print("b2 pipeline: keys, plaintexts", flush=True)
    ctx = ffi.ppst_context_create("b2")
    sk, pk = ffi.ppst_keygen(ctx, 41)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 42, evk)
    ffi.ppst_evk_add_boot(ctx, sk, 43, evk)
    ffi.ppst_evk_add_rotsum(ctx, sk, 44, evk)
    bt = ffi.ppst_boot_create(ctx)
    n = 1 << 20
    slots = ctx.info.slots
    x, y = exp2_columns(60, n)

    def enc(v, seed):
        return [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, c, 11), seed + k)
                for k, c in enumerate(synth.split_column(v, slots))]

    X, Y = enc(x, 800), enc(y, 900)
    cfg = ffi.ppst_invsqrt_cfg_default(coeffs=EXP1_COEFFS, a=0.0, b=2.0, degree=31, iters=6, boot=bt)
    print("b2 pipeline: kurtosis", flush=True)
    k = ffi.ppst_stat_kurtosis(ctx, evk, X, n, 20.0, cfg)
    kv = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, k), 1)[0]
    print("b2 kurtosis %.6f fp64 %.6f" % (kv, stats64.kurtosis(x)), flush=True)
    assert abs(kv / stats64.kurtosis(x) - 1) < 1e-3
    print("b2 pipeline: PCC", flush=True)
    r = ffi.ppst_stat_pearson(ctx, evk, X, Y, n, 20.0, 20.0, cfg)
    rv = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, r), 1)[0]
    print("b2 PCC %.6f fp64 %.6f" % (rv, stats64.pearson(x, y)), flush=True)
    assert abs(rv / stats64.pearson(x, y) - 1) < 1e-3
