"""ppst_mul_noalloc (HMult+relin+rescale into caller memory, no device
allocation) against ppst_mul through the C ABI: bit for bit on two calls in a
row, the second at a lower level (a smaller input), at N = 2^12 and 2^16."""
import numpy as np
import pytest

from paper_2508_12093_amd import ffi, synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def _check(torch, ctx, evk, pk, levels, seed):
    info = ctx.info
    N = info.N
    outs = []
    for k, lvl in enumerate(levels):
        a = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, synth.uniform_column(seed + k, info.slots, -1, 1), lvl),
                             seed + 10 + k)
        b = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, synth.uniform_column(seed + 20 + k, info.slots, -1, 1), lvl),
                             seed + 30 + k)
        want = ffi.ppst_ct_export(ctx, ffi.ppst_mul(ctx, evk, a, b))
        out = torch.full((2, lvl, N), -1, dtype=torch.int64, device="cuda")
        ffi.ppst_sync(ctx)
        torch.cuda.synchronize()
        print("[no-alloc] N=%d level %d" % (N, lvl), flush=True)
        ffi.ppst_mul_noalloc(ctx, evk, ffi.ppst_ct_device_ptr(a), ffi.ppst_ct_device_ptr(b), lvl,
                             out.data_ptr())
        ffi.ppst_sync(ctx)
        got = out.cpu().numpy().view(np.uint64)
        assert got.shape == want.shape
        diff = int(np.sum(got != want))
        assert diff == 0, "%d of %d residues differ at level %d" % (diff, got.size, lvl)
        outs.append(got)
    return outs


@pytest.mark.parametrize("name,levels", [("t1", (6, 3)), ("c2", (24, 9))])
def test_mul_noalloc_equals_mul(name, levels):
    torch = _torch()
    ctx = ffi.ppst_context_create(name)
    sk, pk = ffi.ppst_keygen(ctx, 5)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 6, evk)
    _check(torch, ctx, evk, pk, levels, 100)


def test_mul_noalloc_refusals():
    torch = _torch()
    ctx = ffi.ppst_context_create("t1")
    sk, pk = ffi.ppst_keygen(ctx, 5)
    evk = ffi.ppst_evk_create(ctx)
    N, L = ctx.info.N, ctx.info.L
    a = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, np.zeros(4), L), 1)
    pa = ffi.ppst_ct_device_ptr(a)
    out = torch.zeros((2, L, N), dtype=torch.int64, device="cuda")
    with pytest.raises(ffi.PpstError) as e:            # no relinearisation key yet
        ffi.ppst_mul_noalloc(ctx, evk, pa, pa, L, out.data_ptr())
    assert e.value.name == "ENOKEY"
    ffi.ppst_evk_add_relin(ctx, sk, 6, evk)
    for lvl in (0, L + 1):
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_mul_noalloc(ctx, evk, pa, pa, lvl, out.data_ptr())
        assert e.value.name == "ELEVEL"
    with pytest.raises(ffi.PpstError) as e:            # output on top of an operand
        ffi.ppst_mul_noalloc(ctx, evk, pa, pa, L, pa + 8 * N)
    assert e.value.name == "EINVAL"
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_mul_noalloc(ctx, evk, 0, pa, L, out.data_ptr())
    assert e.value.name == "EINVAL"
    ffi.ppst_sync(ctx)


def test_mul_noalloc_refuses_shapes_beyond_its_scratch():
    """A parameter set whose level-L product needs more than the 144 MiB
    array (N = 2^16, 40 levels, 8 special primes: 448 limbs of 512 KiB) is
    refused before any key is looked up or any kernel runs."""
    torch = _torch()
    import os
    os.environ["PPST_NTT_AUTOTUNE"] = "0"
    try:
        params = ffi.Params(16, 40, 8, 3, 60, 60, float(2 ** 40))
        ctx = ffi.ppst_context_create(params)
    finally:
        del os.environ["PPST_NTT_AUTOTUNE"]
    evk = ffi.ppst_evk_create(ctx)
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_mul_noalloc(ctx, evk, out.data_ptr(), out.data_ptr(), 40, out.data_ptr() + 64)
    assert e.value.name == "EINVAL" and "scratch" in str(e.value)
    ffi.ppst_sync(ctx)
