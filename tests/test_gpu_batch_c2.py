"""The batched forms at the paper's parameters (N = 2^16, L = 24, dnum = 3):
64 independent products through ppst_mul_batch equal the one-ciphertext
path bit for bit, and 16 hoisted rotations of each of several ciphertexts
through ppst_rotate_hoisted_batch (sampled) equal ppst_rotate_hoisted
(MI355X only).
The one-ciphertext forms are pinned to the oracle in test_gpu_parity."""
import numpy as np
import pytest

from paper_2508_12093_amd import ffi, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[batch] preset c2", flush=True)
    ctx = ffi.ppst_context_create("c2")
    sk, pk = ffi.ppst_keygen(ctx, 1001)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 1002, evk)
    steps = list(range(1, 17))
    ffi.ppst_evk_add_galois(ctx, sk, steps, 1003, evk)
    slots = ctx.info.N // 2
    vals = synth.slot_batch(7, 64, slots)
    cts = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, vals[i], 24), 2000 + i) for i in range(64)]
    return ctx, sk, evk, steps, vals, cts


def _same(ctx, a, b):
    return np.array_equal(ffi.ppst_ct_export(ctx, a), ffi.ppst_ct_export(ctx, b))


def test_mul_batch_64_equals_plain(c2):
    ctx, sk, evk, steps, vals, cts = c2
    a, b = cts, cts[1:] + cts[:1]
    print("[batch] 64 products, batched and one at a time", flush=True)
    outs = ffi.ppst_mul_batch(ctx, evk, a, b)
    for i in range(64):
        assert _same(ctx, outs[i], ffi.ppst_mul(ctx, evk, a[i], b[i])), i
    got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, outs[5]))
    assert np.max(np.abs(got - vals[5] * vals[6])) < 1e-4


def test_rotate_hoisted_batch_16_steps(c2):
    ctx, sk, evk, steps, vals, cts = c2
    sub = cts[:18]        # two ModUp groups of 16 and 2 ciphertexts
    print("[batch] 18 ciphertexts x 16 hoisted rotations", flush=True)
    outs = ffi.ppst_rotate_hoisted_batch(ctx, evk, sub, steps)
    for i in (0, 2, 15, 16, 17):
        single = ffi.ppst_rotate_hoisted(ctx, evk, sub[i], steps)
        for k in range(len(steps)):
            assert _same(ctx, outs[i][k], single[k]), (i, k)
    got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, outs[2][6]))
    assert np.max(np.abs(got - np.roll(vals[2], -7))) < 1e-4
