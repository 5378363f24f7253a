"""The boundary's memory hooks and imports through the C ABI: a context whose
every device block comes from torch's caching allocator computes the same
bits as the oracle; keys and plaintexts exported by one context and imported
by another (the paper's client and server roles) give the same results."""
import numpy as np
import pytest

from gpu_common import Pair
from paper_2508_12093_amd import ffi, synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def test_torch_allocator_hooks_bit_exact():
    """c1 on torch-allocated memory: product, rotation and RotSum equal the
    oracle's; the blocks really come from torch's allocator (its allocated
    byte count rises while the context lives and falls once it and its
    objects are gone)."""
    torch = _torch()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ref_pair = Pair("c1", steps=(1,))            # the oracle side and its keys
    O = ref_pair.O
    ctx = ffi.ppst_context_create("c1", alloc="torch")
    grown = torch.cuda.memory_allocated() - base
    assert grown > 0, "the context's tables did not come from torch's allocator"
    sk, pk = ffi.ppst_keygen(ctx, 11)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 12, evk)
    ffi.ppst_evk_add_rotsum(ctx, sk, 13, evk)
    ref_pair.add_rotsum_keys()
    x = synth.uniform_column(3, ref_pair.P.slots, -1, 1)
    y = synth.uniform_column(4, ref_pair.P.slots, -1, 1)
    cx = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, x, ref_pair.P.L), 21)
    cy = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, y, ref_pair.P.L), 22)
    ox = O.encrypt(O.encode(x), ref_pair.opk, 21)
    oy = O.encrypt(O.encode(y), ref_pair.opk, 22)
    m = ffi.ppst_mul(ctx, evk, cx, cy)
    om = O.mul(ox, oy, ref_pair.orlk)
    assert np.array_equal(ffi.ppst_ct_export(ctx, m), om.data)
    r = ffi.ppst_rotate(ctx, evk, m, 1)
    assert np.array_equal(ffi.ppst_ct_export(ctx, r), O.rotate(om, 1, ref_pair.ogk).data)
    s = ffi.ppst_rotsum(ctx, evk, cx)
    assert np.array_equal(ffi.ppst_ct_export(ctx, s), O.rotsum_hoisted8(ox, ref_pair.ogk).data)
    peak = torch.cuda.memory_allocated() - base
    assert peak >= grown
    ffi.ppst_sync(ctx)
    del m, r, s, cx, cy, evk, sk, pk, ctx
    import gc
    gc.collect()
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated() - base
    print("[hooks] torch bytes: tables %d, peak %d, after release %d" % (grown, peak, after), flush=True)
    assert after < peak


def test_key_and_plaintext_import_round_trip():
    """Keys and a plaintext exported from the client's context and imported
    into a second (server) context give bit-identical products, rotations and
    plaintext products; malformed imports are refused."""
    _torch()
    client = ffi.ppst_context_create("t1")
    server = ffi.ppst_context_create("t1")
    info = client.info
    sk, pk = ffi.ppst_keygen(client, 31)
    evk = ffi.ppst_evk_create(client)
    ffi.ppst_evk_add_relin(client, sk, 32, evk)
    ffi.ppst_evk_add_galois(client, sk, [1, 5], 33, evk)
    g1 = 5                                      # Galois element of a rotation by one slot
    sevk = ffi.ppst_evk_create(server)
    ffi.ppst_evk_import(server, sevk, 0, ffi.ppst_evk_export(client, evk, 0))
    ffi.ppst_evk_import(server, sevk, g1, ffi.ppst_evk_export(client, evk, g1))
    spk = ffi.ppst_pk_import(server, ffi.ppst_pk_export(client, pk))
    assert np.array_equal(ffi.ppst_pk_export(server, spk), ffi.ppst_pk_export(client, pk))
    x = synth.uniform_column(5, info.slots, -1, 1)
    pt = ffi.ppst_encode(client, x, info.L)
    c = ffi.ppst_encrypt(client, pk, pt, 41)
    s = ffi.ppst_encrypt(server, spk, ffi.ppst_encode(server, x, info.L), 41)
    assert np.array_equal(ffi.ppst_ct_export(client, c), ffi.ppst_ct_export(server, s))
    same = lambda a, b: np.array_equal(ffi.ppst_ct_export(client, a), ffi.ppst_ct_export(server, b))
    assert same(ffi.ppst_mul(client, evk, c, c), ffi.ppst_mul(server, sevk, s, s))
    assert same(ffi.ppst_rotate(client, evk, c, 1), ffi.ppst_rotate(server, sevk, s, 1))
    words = ffi.ppst_plaintext_export(client, pt, info.L)
    spt = ffi.ppst_plaintext_import(server, words, info.L, client.scales[info.L])
    assert same(ffi.ppst_mul_plain(client, c, pt), ffi.ppst_mul_plain(server, s, spt))
    assert np.allclose(ffi.ppst_decode(server, spt), x, atol=1e-6)
    with pytest.raises(ffi.PpstError) as e:          # rotation by 5 was never imported
        ffi.ppst_rotate(server, sevk, s, 5)
    assert e.value.name == "ENOKEY"
    bad = ffi.ppst_evk_export(client, evk, 0)
    bad[0, 0, 0, 0] = client.primes[0]       # not reduced
    for args, name in [((sevk, 0, bad), "EINVAL"), ((sevk, 4, ffi.ppst_evk_export(client, evk, 0)), "EINVAL"),
                       ((sevk, 0, bad[:1]), "EINVAL")]:
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_evk_import(server, *args)
        assert e.value.name == name
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_plaintext_import(server, words, info.L + 1, 1.0)
    assert e.value.name in ("EINVAL", "ELEVEL")
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_pk_import(server, ffi.ppst_pk_export(client, pk)[:, :1])
    assert e.value.name == "EINVAL"
