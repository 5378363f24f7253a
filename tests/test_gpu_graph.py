"""Recorded HIP graphs of evaluation calls: every replay equals the eager
result bit for bit, with eager work and synchronisation between replays,
outputs released early stay valid, and host-bound calls are refused while
recording (MI355X only)."""
import contextlib
import gc
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import Pair  # noqa: E402

from paper_2508_12093_amd import ffi, synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def t1():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[graph] preset t1", flush=True)
    return Pair("t1")


def _exp(p, c):
    return ffi.ppst_ct_export(p.ctx, c)


@contextlib.contextmanager
def no_collection():
    """Python's cycle collector may destroy handles of other contexts (kept
    alive by earlier tests' tracebacks) at any moment; a context's
    destruction synchronises and frees device memory, which HIP does not
    allow while a stream capture is open.  Collect first, hold it off while
    recording."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def test_graph_replays_equal_eager(t1):
    p = t1
    cts = [p.encrypt(synth.uniform_column(300 + i, p.P.slots, -1, 1), 300 + i)[0] for i in range(3)]
    a, b = cts, cts[1:] + cts[:1]

    def work():
        m = ffi.ppst_mul_batch(p.ctx, p.evk, a, b)
        r = ffi.ppst_rotate(p.ctx, p.evk, m[0], 3)
        s = ffi.ppst_add(p.ctx, r, m[1])
        h = ffi.ppst_rotate_hoisted_batch(p.ctx, p.evk, cts, [1, 5])
        return m, r, s, h

    em, er, es, eh = work()
    want = [_exp(p, c) for c in em] + [_exp(p, er), _exp(p, es)] + [_exp(p, c) for row in eh for c in row]

    with no_collection():
        ffi.ppst_graph_begin(p.ctx)
        try:
            gm, gr, gs, gh = work()
        finally:
            g = ffi.ppst_graph_end(p.ctx)
    del gr                      # released early: the graph keeps its memory
    for rep in range(4):
        print("[graph] replay", rep, flush=True)
        g.launch()
        ffi.ppst_sync(p.ctx)
        got = [_exp(p, c) for c in gm] + [_exp(p, gs)] + [_exp(p, c) for row in gh for c in row]
        ref = want[:3] + want[4:]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), rep
        # eager work between replays reuses the pool but not the graph's blocks
        junk = [ffi.ppst_mul(p.ctx, p.evk, cts[0], cts[1]) for _ in range(3)]
        ffi.ppst_sync(p.ctx)
        del junk
    g = None


def test_recording_refuses_host_calls(t1):
    p = t1
    ct, _ = p.encrypt(synth.uniform_column(310, 16, 0, 1), 310)
    gc.collect()
    gc.disable()
    ffi.ppst_graph_begin(p.ctx)
    try:
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_decrypt(p.ctx, p.sk, ct)
        assert e.value.name == "EINVAL"
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_sync(p.ctx)
        assert e.value.name == "EINVAL"
        with pytest.raises(ffi.PpstError) as e:
            ffi.ppst_graph_begin(p.ctx)
        assert e.value.name == "EINVAL"
        out = ffi.ppst_add(p.ctx, ct, ct)
    finally:
        g = ffi.ppst_graph_end(p.ctx)
        gc.enable()
    g.launch()
    ffi.ppst_sync(p.ctx)
    assert np.array_equal(_exp(p, out), _exp(p, ffi.ppst_add(p.ctx, ct, ct)))
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_graph_end(p.ctx)
    assert e.value.name == "EINVAL"


def test_forked_contexts_overlap_and_agree(t1):
    """Products issued round-robin on contexts forked onto their own streams
    (as the 4-stream benchmark does) equal the one-stream results."""
    p = t1
    cts = [p.encrypt(synth.uniform_column(320 + i, p.P.slots, -1, 1), 320 + i)[0] for i in range(6)]
    forks = [ffi.ppst_context_fork(p.ctx) for _ in range(3)]
    got = [ffi.ppst_mul(forks[i % 3], p.evk, cts[i], cts[(i + 1) % 6]) for i in range(6)]
    for f in forks:
        ffi.ppst_sync(f)
    for i in range(6):
        want = ffi.ppst_mul(p.ctx, p.evk, cts[i], cts[(i + 1) % 6])
        assert np.array_equal(_exp(p, got[i]), _exp(p, want)), i
