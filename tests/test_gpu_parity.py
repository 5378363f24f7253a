"""GPU parity: every RNS-CKKS primitive of the library, called through the
C-ABI, equals the oracle bit for bit from the same seeds (MI355X only)."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import Pair  # noqa: E402

from oracle import ref  # noqa: E402
from paper_2508_12093_amd import ffi, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module", params=["c1", "t1"])
def pair(request):
    _torch()
    print("\n[parity] preset", request.param, flush=True)
    return Pair(request.param)


# ------------------------------------------------------------------ NTT
@pytest.mark.parametrize("name", ["c1", "t1", "c2"])
def test_raw_ntt_matches_oracle(name):
    torch = _torch()
    print("\n[ntt] preset", name, flush=True)
    ctx = ffi.ppst_context_create(name)
    P = ref.Params.preset(name)
    O = ref.Oracle(P)
    info = ctx.info
    rng = np.random.default_rng(1)
    first = 0 if name != "c2" else 20          # c2: a prime window that spans q_20..p_2
    nl = min(info.nprimes - first, 9)
    a = np.stack([rng.integers(0, P.q[first + i], P.N, dtype=np.uint64) for i in range(nl)])
    t = torch.from_numpy(a.view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    ffi.ppst_ntt_forward(ctx, t.data_ptr(), nl, first)
    ffi.ppst_sync(ctx)
    got = t.cpu().numpy().view(np.uint64)
    want = O.ntt(a, list(range(first, first + nl)))
    assert np.array_equal(got, want)
    ffi.ppst_ntt_inverse(ctx, t.data_ptr(), nl, first)
    ffi.ppst_sync(ctx)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), a)


@pytest.mark.parametrize("name,ncol,nrow", [("c1", 1, 5), ("c2", 11, 12)])
def test_every_ntt_variant_matches_oracle(name, ncol, nrow):
    """Each register-radix / workgroup-shape variant the autotuner can pick
    gives the canonical NTT (bit-exact) and inverts; an index past the
    tables is rejected."""
    torch = _torch()
    ctx = ffi.ppst_context_create(name)
    P = ref.Params.preset(name)
    O = ref.Oracle(P)
    rng = np.random.default_rng(2)
    nl = 3
    a = np.stack([rng.integers(0, P.q[i], P.N, dtype=np.uint64) for i in range(nl)])
    want = O.ntt(a, list(range(nl)))
    print("\n[ntt-variants]", name, ffi.ppst_ntt_plan(ctx)[:120], flush=True)
    for c in range(ncol):
        for r in range(nrow):
            ffi.ppst_ntt_set_plan(ctx, c, r)
            t = torch.from_numpy(a.view(np.int64).copy()).cuda()
            torch.cuda.synchronize()
            ffi.ppst_ntt_forward(ctx, t.data_ptr(), nl, 0)
            ffi.ppst_sync(ctx)
            assert np.array_equal(t.cpu().numpy().view(np.uint64), want), (c, r)
            ffi.ppst_ntt_inverse(ctx, t.data_ptr(), nl, 0)
            ffi.ppst_sync(ctx)
            assert np.array_equal(t.cpu().numpy().view(np.uint64), a), (c, r)
    with pytest.raises(ffi.PpstError):
        ffi.ppst_ntt_set_plan(ctx, 0, nrow)


# ------------------------------------------------------------ keys / enc
def test_keys_bit_exact(pair):
    p = pair
    assert np.array_equal(ffi.ppst_sk_export(p.ctx, p.sk), p.osk.s_ntt)
    assert np.array_equal(ffi.ppst_pk_export(p.ctx, p.pk), p.opk)
    assert np.array_equal(ffi.ppst_evk_export(p.ctx, p.evk, 0), p.orlk)
    g = ref.galois_element(3, p.P.N)
    assert np.array_equal(ffi.ppst_evk_export(p.ctx, p.evk, g), p.ogk[g])
    assert np.array_equal(ffi.ppst_context_dg_table(p.ctx), ffi.ppst_dg_thresholds())


def test_encrypt_decrypt(pair):
    p = pair
    m = synth.uniform_column(5, p.P.slots, -1, 1)
    ct, oct_ = p.encrypt(m, 21)
    p.same(ct, oct_)
    for level in (0, 1):
        c2, o2 = p.encrypt(m, 22, level)
        p.same(c2, o2)
    std = p.P.N * 3.2 * math.sqrt(2 / 3) / p.P.scale[p.P.L]
    assert np.max(np.abs(p.decrypt(ct) - m)) < 8 * std
    pt = ffi.ppst_encode(p.ctx, m, p.P.L)
    cs = ffi.ppst_encrypt_sk(p.ctx, p.sk, pt, 23)
    p.same(cs, p.O.encrypt_sk(p.O.encode(m), p.osk, 23))
    # library decryption equals the oracle's c0 + c1 s
    dec = ffi.ppst_plaintext_export(p.ctx, ffi.ppst_decrypt(p.ctx, p.sk, ct), p.P.L)
    assert np.array_equal(dec, p.O.decrypt_ntt(oct_, p.osk))


# --------------------------------------------------------------- ops
def test_linear_ops(pair):
    p = pair
    a = synth.uniform_column(6, p.P.slots, -1, 1)
    b = synth.uniform_column(7, p.P.slots, -1, 1)
    ca, oa = p.encrypt(a, 31)
    cb, ob = p.encrypt(b, 32)
    p.same(ffi.ppst_add(p.ctx, ca, cb), p.O.add(oa, ob))
    p.same(ffi.ppst_sub(p.ctx, ca, cb), p.O.sub(oa, ob))
    p.same(ffi.ppst_add_const(p.ctx, ca, -0.3125), p.O.add_const(oa, -0.3125))
    p.same(ffi.ppst_mul_int(p.ctx, ca, -3), p.O.mul_int(oa, -3))
    p.same(ffi.ppst_mul_const(p.ctx, ca, 0.7071), p.O.mul_const(oa, 0.7071))
    p.same(ffi.ppst_rescale(p.ctx, ca), p.O.rescale(oa))
    for lvl in range(p.P.L):
        p.same(ffi.ppst_level_align(p.ctx, ca, lvl), p.O.level_align(oa, lvl))
    pt = ffi.ppst_encode(p.ctx, b, p.P.L)
    p.same(ffi.ppst_mul_plain(p.ctx, ca, pt), p.O.mul_plain(oa, p.O.encode(b, p.P.L)))


def test_lincomb(pair):
    """Weighted sums with one rescale: one term equals Mul(P) by the
    constant; eight terms over three levels (two launches of the term loop)
    equal the oracle's bit for bit; a term below level + 1 is refused."""
    p = pair
    L = p.P.L
    cts, octs = [], []
    for i in range(3):
        c, o = p.encrypt(synth.uniform_column(40 + i, p.P.slots, -1, 1), 60 + i)
        cts.append(c)
        octs.append(o)
    p.same(ffi.ppst_lincomb(p.ctx, [cts[0]], [0.7071], L - 1), p.O.mul_const(octs[0], 0.7071))
    if L >= 2:
        low = [ffi.ppst_level_align(p.ctx, c, L - 1) for c in cts]
        olow = [p.O.level_align(o, L - 1) for o in octs]
        terms = [cts[0], low[1], cts[2], low[0], cts[1], low[2], cts[0], low[1]]
        oterms = [octs[0], olow[1], octs[2], olow[0], octs[1], olow[2], octs[0], olow[1]]
        cs = [0.5, -1.25, 0.125, 3.0, -0.0625, 0.75, 2.5e-3, -7.0]
        p.same(ffi.ppst_lincomb(p.ctx, terms, cs, L - 2), p.O.lincomb(oterms, cs, L - 2))
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_lincomb(p.ctx, [low[0]], [1.0], L - 1)
        assert e.value.name == "ELEVEL"


def test_mul_relin_rescale(pair):
    p = pair
    a = synth.uniform_column(8, p.P.slots, -1, 1)
    b = synth.uniform_column(9, p.P.slots, -1, 1)
    ca, oa = p.encrypt(a, 41)
    cb, ob = p.encrypt(b, 42)
    d = ffi.ppst_tensor(p.ctx, ca, cb)
    od = p.O.tensor(oa, ob)
    assert np.array_equal(ffi.ppst_ct_export(p.ctx, d), od)
    r = ffi.ppst_relin(p.ctx, p.evk, d)
    p.same(r, p.O.relin(od, p.P.L, p.orlk, oa.scale * ob.scale))
    m = ffi.ppst_mul(p.ctx, p.evk, ca, cb)
    om = p.O.mul(oa, ob, p.orlk)
    p.same(m, om)
    # every level down to 1
    cur, ocur = m, om
    while cur.level >= 1:
        cur = ffi.ppst_mul(p.ctx, p.evk, cur, cur)
        ocur = p.O.mul(ocur, ocur, p.orlk)
        p.same(cur, ocur)
    assert np.max(np.abs(p.decrypt(m) - a * b)) < 1e-3


def test_rotations(pair):
    p = pair
    m = synth.uniform_column(10, p.P.slots, 0, 1)
    ct, oct_ = p.encrypt(m, 51)
    for r in p.steps:
        p.same(ffi.ppst_rotate(p.ctx, p.evk, ct, r), p.O.rotate(oct_, r, p.ogk))
    low, olow = ffi.ppst_level_align(p.ctx, ct, 1), p.O.level_align(oct_, 1)
    p.same(ffi.ppst_rotate(p.ctx, p.evk, low, 3), p.O.rotate(olow, 3, p.ogk))
    hs = ffi.ppst_rotate_hoisted(p.ctx, p.evk, ct, p.steps)
    ohs = p.O.rotate_hoisted(oct_, p.steps, p.ogk)
    for h, oh in zip(hs, ohs):
        p.same(h, oh)
    assert np.max(np.abs(p.decrypt(hs[1]) - np.roll(m, -3))) < 1e-3


def test_rotsum(pair):
    p = pair
    p.add_rotsum_keys()
    m = synth.uniform_column(11, p.P.slots, 0, 1) / p.P.slots
    ct, oct_ = p.encrypt(m, 61)
    s = ffi.ppst_rotsum(p.ctx, p.evk, ct)
    p.same(s, p.O.rotsum_hoisted8(oct_, p.ogk))
    assert abs(p.decrypt(s)[0] - m.sum()) < 1e-3
    # the plain definition: serial ct + Rot(ct, 2^k)
    s2 = ffi.ppst_rotsum_serial(p.ctx, p.evk, ct)
    p.same(s2, p.O.rotsum(oct_, p.ogk))
    assert abs(p.decrypt(s2)[0] - m.sum()) < 1e-3
    low, olow = ffi.ppst_level_align(p.ctx, ct, 0), p.O.level_align(oct_, 0)
    p.same(ffi.ppst_rotsum_serial(p.ctx, p.evk, low), p.O.rotsum(olow, p.ogk))


def test_rotsum_batch_matches_oracle(pair):
    """Rotate-and-sum of 1 to 6 ciphertexts at once (every lane count the
    multi-key inner product groups differently) equals the oracle's RotSum
    of each, bit for bit."""
    p = pair
    p.add_rotsum_keys()
    cts, octs = [], []
    for i in range(6):
        m = synth.uniform_column(140 + i, p.P.slots, 0, 1) / p.P.slots
        c, o = p.encrypt(m, 140 + i)
        cts.append(c)
        octs.append(p.O.rotsum_hoisted8(o, p.ogk))
    for n in range(1, 7):
        for o, oc in zip(ffi.ppst_rotsum_batch(p.ctx, p.evk, cts[:n]), octs[:n]):
            p.same(o, oc)
    assert ffi.ppst_rotsum_batch(p.ctx, p.evk, []) == []


def test_mul_batch_equals_single(pair):
    p = pair
    cts = [p.encrypt(synth.uniform_column(70 + i, p.P.slots, -1, 1), 70 + i)[0] for i in range(5)]
    a, b = cts, cts[1:] + cts[:1]
    outs = ffi.ppst_mul_batch(p.ctx, p.evk, a, b)
    for x, y, o in zip(a, b, outs):
        single = ffi.ppst_mul(p.ctx, p.evk, x, y)
        assert np.array_equal(ffi.ppst_ct_export(p.ctx, o), ffi.ppst_ct_export(p.ctx, single))


def test_mul_const_batch_matches_oracle(pair):
    """Constant products of 18 ciphertexts (two launch groups, the second
    ragged) equal the oracle's mul_const bit for bit, at the top level and one
    below; mixed levels are refused and an empty list gives no outputs."""
    p = pair
    cts, octs = [], []
    for i in range(18):
        c, o = p.encrypt(synth.uniform_column(120 + i, p.P.slots, -1, 1), 120 + i)
        cts.append(c)
        octs.append(o)
    for k in (0.7071, -3.25):
        for o, oc in zip(ffi.ppst_mul_const_batch(p.ctx, cts, k), octs):
            p.same(o, p.O.mul_const(oc, k))
    if p.P.L >= 2:
        low = [ffi.ppst_rescale(p.ctx, c) for c in cts[:3]]
        olow = [p.O.rescale(o) for o in octs[:3]]
        for o, oc in zip(ffi.ppst_mul_const_batch(p.ctx, low, 0.5), olow):
            p.same(o, p.O.mul_const(oc, 0.5))
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_mul_const_batch(p.ctx, [cts[0], low[0]], 0.5)
        assert e.value.name == "ESCALE"
    assert ffi.ppst_mul_const_batch(p.ctx, [], 0.5) == []


def test_rotate_batch_equals_single(pair):
    """Several ciphertexts rotated by one step in one key switch equal the
    oracle's rotations bit for bit (and the identity step copies)."""
    p = pair
    cts, octs = [], []
    for i in range(3):
        c, o = p.encrypt(synth.uniform_column(97 + i, p.P.slots, -1, 1), 97 + i)
        cts.append(c)
        octs.append(o)
    for r in (3, p.P.slots):
        outs = ffi.ppst_rotate_batch(p.ctx, p.evk, cts, r)
        for o, oc in zip(outs, octs):
            p.same(o, p.O.rotate(oc, r, p.ogk) if r != p.P.slots else oc)
    assert ffi.ppst_rotate_batch(p.ctx, p.evk, [], 3) == []


def test_rotation_under_every_ntt_variant(pair):
    """Rotations read their input through the Galois permutation inside the
    first pass of the inverse NTT; every variant of that pass (LDS-staged and
    direct-load) gives the oracle's ciphertext."""
    p = pair
    m = synth.uniform_column(95, p.P.slots, -1, 1)
    ct, oct_ = p.encrypt(m, 95)
    want = p.O.rotate(oct_, 3, p.ogk)
    nrow = 5                                   # N = 2^12: one pass, five variants
    for r in range(nrow):
        ffi.ppst_ntt_set_plan(p.ctx, 0, r)
        p.same(ffi.ppst_rotate(p.ctx, p.evk, ct, 3), want)
        p.same(ffi.ppst_mul(p.ctx, p.evk, ct, ct), p.O.mul(oct_, oct_, p.orlk))
    ffi.ppst_ntt_autotune(p.ctx)


def test_rotate_hoisted_batch_equals_single(pair):
    """Batched hoisted rotations equal the one-ciphertext hoisted form bit for
    bit (which the oracle pins in test_rotations), for every ciphertext and
    step, including a step that is the identity."""
    p = pair
    cts = [p.encrypt(synth.uniform_column(90 + i, p.P.slots, -1, 1), 90 + i)[0] for i in range(5)]
    steps = list(p.steps) + [p.P.slots]
    outs = ffi.ppst_rotate_hoisted_batch(p.ctx, p.evk, cts, steps)
    assert len(outs) == len(cts) and all(len(o) == len(steps) for o in outs)
    for ct, row in zip(cts, outs):
        single = ffi.ppst_rotate_hoisted(p.ctx, p.evk, ct, steps)
        for o, s1 in zip(row, single):
            assert np.array_equal(ffi.ppst_ct_export(p.ctx, o), ffi.ppst_ct_export(p.ctx, s1))
    assert ffi.ppst_rotate_hoisted_batch(p.ctx, p.evk, [], steps) == []


def test_error_statuses(pair):
    p = pair
    m = synth.uniform_column(12, 16, 0, 1)
    ct, _ = p.encrypt(m, 81)
    low = ffi.ppst_level_align(p.ctx, ct, 0)
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_add(p.ctx, ct, low)
    assert e.value.name == "ESCALE"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_mul(p.ctx, p.evk, low, low)
    assert e.value.name == "ELEVEL"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_rotate(p.ctx, p.evk, ct, 9)      # neither a fixture step nor a RotSum step
    assert e.value.name == "ENOKEY"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_level_align(p.ctx, low, 1)
    assert e.value.name == "ELEVEL"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_encode(p.ctx, np.zeros(p.P.slots + 1), p.P.L)
    assert e.value.name == "EINVAL"


# ---------------------------------------------------- full-size spot checks
@pytest.fixture(scope="module")
def c2pair():
    _torch()
    print("\n[parity] preset c2 (N=2^16, L=24)", flush=True)
    return Pair("c2", steps=(1,))


def test_c2_hmult_and_rotation_bit_exact(c2pair):
    """N = 2^16, level 24 (the configuration the benchmark times): one
    HMult+relin+rescale and one rotation against the oracle, all residues."""
    p = c2pair
    x, y = synth.binary_cost_pair(0)
    cx, ox = p.encrypt(x, 91)
    cy, oy = p.encrypt(y / 100.0, 92)
    p.same(cx, ox)
    m = ffi.ppst_mul(p.ctx, p.evk, cx, cy)
    om = p.O.mul(ox, oy, p.orlk)
    p.same(m, om)
    r = ffi.ppst_rotate(p.ctx, p.evk, cy, 1)
    orot = p.O.rotate(oy, 1, p.ogk)
    p.same(r, orot)
    assert np.max(np.abs(p.decrypt(m) - x * y / 100.0)) < 1e-4
    assert np.max(np.abs(p.decrypt(r) - np.roll(y / 100.0, -1))) < 1e-4
    # the same under fixed plans: LDS-staged passes, then direct-load passes
    # (the Galois read sits in the first inverse row pass)
    for col, row in [(2, 4), (6, 6), (5, 9), (0, 1), (7, 2), (8, 3)]:
        ffi.ppst_ntt_set_plan(p.ctx, col, row)
        p.same(ffi.ppst_mul(p.ctx, p.evk, cx, cy), om)
        p.same(ffi.ppst_rotate(p.ctx, p.evk, cy, 1), orot)
        if (col, row) == (2, 4):
            # batched constant products: the rescale's last pass under a fixed plan
            for o, oc in zip(ffi.ppst_mul_const_batch(p.ctx, [cx, cy], 0.375), [ox, oy]):
                p.same(o, p.O.mul_const(oc, 0.375))
    ffi.ppst_ntt_autotune(p.ctx)


def test_c2_rotsum_bit_exact(c2pair):
    """Rotate-and-sum at N = 2^16, level 24 (five hoisted radix-8 steps, seven
    Galois keys each) equals the oracle's in every residue, alone and as five
    lanes of one batch (the five-lane multi-key inner product)."""
    p = c2pair
    print("\n[parity] c2 RotSum: 35 Galois keys on both sides, oracle RotSum", flush=True)
    p.add_rotsum_keys()
    m = synth.uniform_column(11, p.P.slots, 0, 1) / p.P.slots
    ct, oct_ = p.encrypt(m, 61)
    ors = p.O.rotsum_hoisted8(oct_, p.ogk)
    s = ffi.ppst_rotsum(p.ctx, p.evk, ct)
    p.same(s, ors)
    for o in ffi.ppst_rotsum_batch(p.ctx, p.evk, [ct] * 5):
        p.same(o, ors)
    assert abs(p.decrypt(s)[0] - m.sum()) < 1e-3


def test_c2_rotsum_serial_bit_exact(c2pair):
    """The plain rotate-and-sum at N = 2^16, level 24: fifteen serial steps
    ct + Rot(ct, 2^k) equal the oracle's definition in every residue, and the
    five-step hoisted form decrypts to the same sum."""
    p = c2pair
    print("\n[parity] c2 serial RotSum (15 rotations on both sides)", flush=True)
    p.add_rotsum_keys()
    m = synth.uniform_column(12, p.P.slots, 0, 1) / p.P.slots
    ct, oct_ = p.encrypt(m, 62)
    s = ffi.ppst_rotsum_serial(p.ctx, p.evk, ct)
    p.same(s, p.O.rotsum(oct_, p.ogk))
    fused = ffi.ppst_rotsum(p.ctx, p.evk, ct)
    a, b = p.decrypt(s), p.decrypt(fused)
    # every slot sums the encryption noise of all N/2 slots: fresh noise has
    # std N sigma sqrt(2/3) / Delta = 1.6e-7 per slot, so the sum's std is
    # sqrt(32768) x 1.6e-7 = 2.9e-5; 3e-4 is about ten of them
    ea, eb, ab = (float(np.max(np.abs(a - m.sum()))), float(np.max(np.abs(b - m.sum()))),
                  float(np.max(np.abs(a - b))))
    print("serial %.2e, hoisted %.2e, between %.2e" % (ea, eb, ab), flush=True)
    assert ea < 3e-4 and eb < 3e-4 and ab < 3e-4


def test_c2_primitives_bit_exact(c2pair):
    """N = 2^16, L = 24: standalone tensor, relinearisation and rescale, the
    plaintext product, level alignment to 23, 12 and 0, and a weighted sum
    over terms at three levels equal the oracle bit for bit."""
    p = c2pair
    print("\n[parity] c2 primitives", flush=True)
    a = synth.uniform_column(21, p.P.slots, -1, 1)
    b = synth.uniform_column(22, p.P.slots, -1, 1)
    ca, oa = p.encrypt(a, 121)
    cb, ob = p.encrypt(b, 122)
    L = p.P.L
    d = ffi.ppst_tensor(p.ctx, ca, cb)
    od = p.O.tensor(oa, ob)
    assert np.array_equal(ffi.ppst_ct_export(p.ctx, d), od)
    r = ffi.ppst_relin(p.ctx, p.evk, d)
    orl = p.O.relin(od, L, p.orlk, oa.scale * ob.scale)
    p.same(r, orl)
    p.same(ffi.ppst_rescale(p.ctx, r), p.O.rescale(orl))
    p.same(ffi.ppst_rescale(p.ctx, ca), p.O.rescale(oa))
    pt = ffi.ppst_encode(p.ctx, b, L)
    p.same(ffi.ppst_mul_plain(p.ctx, ca, pt), p.O.mul_plain(oa, p.O.encode(b, L)))
    lows, olows = {}, {}
    for lvl in (23, 12, 0):
        lows[lvl] = ffi.ppst_level_align(p.ctx, ca, lvl)
        olows[lvl] = p.O.level_align(oa, lvl)
        p.same(lows[lvl], olows[lvl])
    pt12 = ffi.ppst_encode(p.ctx, b, 12)
    p.same(ffi.ppst_mul_plain(p.ctx, lows[12], pt12),
           p.O.mul_plain(olows[12], p.O.encode(b, 12)))
    b23, ob23 = ffi.ppst_level_align(p.ctx, cb, 23), p.O.level_align(ob, 23)
    terms = [ca, lows[23], cb, b23, lows[12]]
    oterms = [oa, olows[23], ob, ob23, olows[12]]
    cs = [0.5, -1.25, 0.125, 3.0, -0.0625]
    got = ffi.ppst_lincomb(p.ctx, terms, cs, 11)
    p.same(got, p.O.lincomb(oterms, cs, 11))
    want = 0.5 * a - 1.25 * a + 0.125 * b + 3.0 * b - 0.0625 * a
    assert np.max(np.abs(p.decrypt(got) - want)) < 1e-4


def test_c2_hoisted_rotation_bit_exact(c2pair):
    """Hoisted rotations by 1, 3 and 16 at N = 2^16 (one ModUp, the
    automorphism on the extended digits) equal the oracle's hoisted form."""
    p = c2pair
    p.add_rotsum_keys()                      # 3 and 16 are RotSum steps
    m = synth.uniform_column(23, p.P.slots, -1, 1)
    ct, oct_ = p.encrypt(m, 123)
    steps = [1, 3, 16]
    for h, oh in zip(ffi.ppst_rotate_hoisted(p.ctx, p.evk, ct, steps),
                     p.O.rotate_hoisted(oct_, steps, p.ogk)):
        p.same(h, oh)


def test_c2_batch_items_match_oracle(c2pair):
    """One item of a batched product and one of a batched hoisted rotation at
    N = 2^16 against the oracle itself (not against the library's own
    one-ciphertext forms)."""
    p = c2pair
    p.add_rotsum_keys()
    cts, octs = [], []
    for i in range(3):
        c, o = p.encrypt(synth.uniform_column(130 + i, p.P.slots, -1, 1), 130 + i)
        cts.append(c)
        octs.append(o)
    outs = ffi.ppst_mul_batch(p.ctx, p.evk, cts, cts[1:] + cts[:1])
    p.same(outs[1], p.O.mul(octs[1], octs[2], p.orlk))
    rows = ffi.ppst_rotate_hoisted_batch(p.ctx, p.evk, cts, [2, 5])
    p.same(rows[2][1], p.O.rotate_hoisted(octs[2], [5], p.ogk)[0])


def test_c2_pearson_matches_oracle_digest(c2pair):
    """The headline latency workload: Pearson on the config-2 columns
    (x ~ Bernoulli(0.2), y lognormal with corr 0.79; Bx = 1, By = 20,
    degree-7 Chebyshev on [1e-3, 1] + 3 Newton steps) at N = 2^16, L = 24.
    The result ciphertext equals the oracle's residue for residue: the
    oracle's output (about 90 s of host time) is stored as a SHA-256 digest
    by tests/golden/make_c2_pearson.py, which calls only the oracle."""
    import hashlib
    import json
    from oracle import cheb, stats64 as S
    p = c2pair
    with open(os.path.join(os.path.dirname(__file__), "golden", "c2_pearson.json")) as f:
        g = json.load(f)
    spec = g["spec"]
    assert (p.name, 11, 12, 13) == (spec["preset"], spec["key_seed"], spec["relin_seed"],
                                    spec["galois_seed"])
    p.add_rotsum_keys()
    x, y = synth.binary_cost_pair(spec["data_seed"])
    cx = ffi.ppst_encrypt(p.ctx, p.pk, ffi.ppst_encode(p.ctx, x, p.P.L), spec["enc_seed_x"])
    cy = ffi.ppst_encrypt(p.ctx, p.pk, ffi.ppst_encode(p.ctx, y, p.P.L), spec["enc_seed_y"])
    base = cheb.invsqrt_coeffs(spec["a"], spec["b"], spec["degree"], 1.0)
    cfg = ffi.ppst_invsqrt_cfg_default(coeffs=base)
    print("\n[parity] c2 Pearson vs the oracle's digest", flush=True)
    out = ffi.ppst_stat_pearson(p.ctx, p.evk, [cx], [cy], len(x), spec["Bx"], spec["By"], cfg)
    words = ffi.ppst_ct_export(p.ctx, out)
    assert out.level == g["level"] and float(out.scale).hex() == g["scale_hex"]
    assert list(words.shape) == g["shape"]
    assert hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest() == g["sha256"]
    got = p.decrypt(out)[0]
    assert abs(got - g["decrypted"]) < 1e-9
    assert abs(got - S.pearson(x, y)) / abs(S.pearson(x, y)) < 1e-3


@pytest.mark.parametrize("name", ["t1", "c2"])
def test_ntt_plan_round_trip(name):
    """A plan written by ppst_ntt_plan loads back unchanged (so an autotuning
    can be saved and reused); malformed text is refused and leaves the
    plan as it was."""
    _torch()
    ctx = ffi.ppst_context_create(name)
    tuned = ffi.ppst_ntt_plan(ctx)
    ffi.ppst_ntt_set_plan(ctx, 0, 1)
    ffi.ppst_ntt_load_plan(ctx, tuned)
    assert ffi.ppst_ntt_plan(ctx) == tuned
    for bad in ["fwd[b0] nonsense", tuned.split(";", 1)[1], "fwd[b9] x y;"]:
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_ntt_load_plan(ctx, bad)
        assert e.value.name == "EINVAL"
        assert ffi.ppst_ntt_plan(ctx) == tuned
