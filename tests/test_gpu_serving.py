"""Serving: queries over resident columns are admitted as slots and memory
free up, run concurrently on worker streams, and give the same result
ciphertext alone and in the mix (MI355X only)."""
import os
import sys
import threading

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

from oracle import stats64 as S  # noqa: E402
from paper_2508_12093_amd import ffi, synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[serving] preset t2 (N=2^12, L=24)", flush=True)
    ctx = ffi.ppst_context_create("t2")
    sk, pk = ffi.ppst_keygen(ctx, 5)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 6, evk)
    ffi.ppst_evk_add_rotsum(ctx, sk, 7, evk)
    slots = ctx.info.slots
    cols = {}
    for name, n, seed in [("a", 1000, 1), ("b", 2048, 2), ("c", 5000, 3)]:
        x, y = synth.lognormal_bernoulli_pair(seed, n)
        cx = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, v, 24), 100 * seed + i)
              for i, v in enumerate(synth.split_column(x / 4.0, slots))]
        cy = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, v, 24), 100 * seed + 50 + i)
              for i, v in enumerate(synth.split_column(y / 4.0, slots))]
        cols[name] = (n, x / 4.0, y / 4.0, cx, cy)
    return ctx, sk, evk, cols


def direct(ctx, evk, kind, cx, cy, n, B, B2, cfg):
    if kind == ffi.Q_MEAN:
        return ffi.ppst_stat_mean(ctx, evk, cx, n, B)
    if kind == ffi.Q_VARIANCE:
        return ffi.ppst_stat_variance(ctx, evk, cx, n, B)
    if kind == ffi.Q_ZSCORE:
        return ffi.ppst_stat_zscore(ctx, evk, cx, n, B, cfg)[0]
    if kind == ffi.Q_CV:
        return ffi.ppst_stat_cv(ctx, evk, cx, n, B, B2, cfg)
    if kind == ffi.Q_PEARSON:
        return ffi.ppst_stat_pearson(ctx, evk, cx, cy, n, B, B2, cfg)
    if kind == ffi.Q_SKEWNESS:
        return ffi.ppst_stat_skewness(ctx, evk, cx, n, B, cfg)
    return ffi.ppst_stat_kurtosis(ctx, evk, cx, n, B, cfg)


def test_mixed_stream_equals_alone(env):
    ctx, sk, evk, cols = env
    cfg = ffi.ppst_invsqrt_cfg_default()
    srv = ffi.ppst_server_create(ctx, evk, 8 << 30, 4)
    ids = {}
    for name, (n, x, y, cx, cy) in cols.items():
        ids[name] = (ffi.ppst_server_register_column(srv, cx, n), ffi.ppst_server_register_column(srv, cy, n))
    # bounds: x ~ Bernoulli(0.3)/4, y lognormal/4 + shift: Var/B^2 and mean/B inside [1e-3, 1]
    plan = []
    for rep in range(2):
        for name in cols:
            plan += [(ffi.Q_MEAN, name, 1.0, 1.0), (ffi.Q_VARIANCE, name, 2.0, 2.0),
                     (ffi.Q_ZSCORE, name, 2.0, 2.0), (ffi.Q_CV, name, 1.0, 2.0),
                     (ffi.Q_PEARSON, name, 1.0, 2.0), (ffi.Q_SKEWNESS, name, 2.0, 2.0),
                     (ffi.Q_KURTOSIS, name, 2.0, 2.0)]
    # CV reads column y (lognormal, positive mean); the others read x except Pearson (x, y)
    tickets = []
    for kind, name, B, B2 in plan:
        cx_id, cy_id = ids[name]
        col = cy_id if kind in (ffi.Q_CV, ffi.Q_SKEWNESS, ffi.Q_KURTOSIS, ffi.Q_ZSCORE) else cx_id
        tickets.append(ffi.ppst_server_submit(srv, kind, col, cy_id, B, B2, cfg))
    results = [ffi.ppst_server_wait(srv, t) for t in tickets]
    overlap = 0
    for i, ((kind, name, B, B2), (rc, ct, st)) in enumerate(zip(plan, results)):
        assert rc == 0, (kind, name, ffi.lib().ppst_last_error())
        assert st.t_submit <= st.t_admit <= st.t_done
        n, x, y, cx, cy = cols[name]
        colx = cy if kind in (ffi.Q_CV, ffi.Q_SKEWNESS, ffi.Q_KURTOSIS, ffi.Q_ZSCORE) else cx
        alone = direct(ctx, evk, kind, colx, cy, n, B, B2, cfg)
        assert np.array_equal(ffi.ppst_ct_export(ctx, ct), ffi.ppst_ct_export(ctx, alone)), (kind, name)
        # overlap: another query admitted before this one finished
        for j, (_, _, st2) in enumerate(results):
            if j != i and st2.t_admit < st.t_done and st2.t_admit > st.t_admit:
                overlap += 1
                break
    assert overlap > 0, "no two queries were in flight together"
    info = ffi.ppst_server_info(srv)
    print("[serving] merged rotate-and-sums:", info, flush=True)
    assert info["merged_lanes"] >= info["merged_launches"] > 0
    # decrypted values are the statistics
    n, x, y, cx, cy = cols["c"]
    rc, ct, _ = results[[k for k, p in enumerate(plan) if p[0] == ffi.Q_PEARSON and p[1] == "c"][0]]
    got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, ct))[0]
    assert abs(got - S.pearson(x, y)) / abs(S.pearson(x, y)) < 1e-3


def test_admission_by_memory(env):
    ctx, sk, evk, cols = env
    cfg = ffi.ppst_invsqrt_cfg_default()
    n, x, y, cx, cy = cols["b"]
    tiny = ffi.ppst_server_create(ctx, evk, 1 << 20, 2)          # 1 MiB: nothing fits
    cid = ffi.ppst_server_register_column(tiny, cx, n)
    with pytest.raises(ffi.PpstError) as e:
        ffi.ppst_server_submit(tiny, ffi.Q_MEAN, cid, 0, 1.0, 1.0, cfg)
    assert e.value.name == "ENOMEM"
    del tiny
    # a budget for exactly one query at a time: everything still completes, in order
    probe = ffi.ppst_server_create(ctx, evk, 8 << 30, 1)
    pid = ffi.ppst_server_register_column(probe, cx, n)
    rc, ct, st = ffi.ppst_server_wait(probe, ffi.ppst_server_submit(probe, ffi.Q_VARIANCE, pid, 0, 1.0, 1.0, cfg))
    one = st.bytes_reserved
    del probe
    srv = ffi.ppst_server_create(ctx, evk, one + one // 2, 4)
    cid = ffi.ppst_server_register_column(srv, cx, n)
    ts = [ffi.ppst_server_submit(srv, ffi.Q_VARIANCE, cid, 0, 1.0, 1.0, cfg) for _ in range(4)]
    res = [ffi.ppst_server_wait(srv, t) for t in ts]
    assert all(r[0] == 0 for r in res)
    for a, b in zip(res, res[1:]):            # serialized by the budget
        assert b[2].t_admit >= a[2].t_done
    ref = ffi.ppst_ct_export(ctx, res[0][1])
    assert all(np.array_equal(ffi.ppst_ct_export(ctx, r[1]), ref) for r in res)


def test_estimates_cover_peaks(env):
    """Each query's admission estimate covers the device memory its worker
    actually held (queries run one at a time, no merging)."""
    ctx, sk, evk, cols = env
    cfg = ffi.ppst_invsqrt_cfg_default()
    srv = ffi.ppst_server_create(ctx, evk, 8 << 30, 1, merge=False)
    n, x, y, cx, cy = cols["c"]
    cid, yid = ffi.ppst_server_register_column(srv, cx, n), ffi.ppst_server_register_column(srv, cy, n)
    for kind, col, B, B2 in [(ffi.Q_MEAN, cid, 1.0, 1.0), (ffi.Q_VARIANCE, cid, 2.0, 2.0),
                             (ffi.Q_ZSCORE, yid, 2.0, 2.0), (ffi.Q_CV, yid, 1.0, 2.0),
                             (ffi.Q_PEARSON, cid, 1.0, 2.0), (ffi.Q_KURTOSIS, yid, 2.0, 2.0)]:
        rc, ct, st = ffi.ppst_server_wait(srv, ffi.ppst_server_submit(srv, kind, col, yid, B, B2, cfg))
        assert rc == 0
        print("[serving] kind %d: estimate %d, peak %d bytes" % (kind, st.bytes_reserved, st.bytes_peak),
              flush=True)
        assert 0 < st.bytes_peak <= st.bytes_reserved, (kind, st.bytes_peak, st.bytes_reserved)
    assert ffi.ppst_server_info(srv)["merged_launches"] == 0
    free = ffi.ppst_server_create(ctx, evk, 0, 1)         # admission by the device's free memory
    assert ffi.ppst_server_info(free)["budget"] > (1 << 30)


def test_bad_queries(env):
    ctx, sk, evk, cols = env
    cfg = ffi.ppst_invsqrt_cfg_default()
    srv = ffi.ppst_server_create(ctx, evk, 8 << 30, 2)
    with pytest.raises(ffi.PpstError):
        ffi.ppst_server_submit(srv, ffi.Q_MEAN, 12345, 0, 1.0, 1.0, cfg)
    n, x, y, cx, cy = cols["a"]
    cid = ffi.ppst_server_register_column(srv, cx, n)
    bad = ffi.ppst_invsqrt_cfg_default(a=-1.0)
    t = ffi.ppst_server_submit(srv, ffi.Q_ZSCORE, cid, 0, 1.0, 1.0, bad)
    rc, ct, st = ffi.ppst_server_wait(srv, t)
    assert rc == -7 and ct is None            # EDOMAIN from the worker, server keeps going
    t = ffi.ppst_server_submit(srv, ffi.Q_MEAN, cid, 0, 1.0, 1.0, cfg)
    assert ffi.ppst_server_wait(srv, t)[0] == 0
    with pytest.raises(ffi.PpstError) as e:      # collected already
        ffi.ppst_server_poll(srv, t)
    assert e.value.name == "EINVAL"


def test_poll_does_not_block(env):
    """ppst_server_poll reports pending work without blocking and turns true
    once the query is done; the result is then collected by wait."""
    ctx, sk, evk, cols = env
    cfg = ffi.ppst_invsqrt_cfg_default()
    n, x, y, cx, cy = cols["b"]
    srv = ffi.ppst_server_create(ctx, evk, 8 << 30, 1)
    cid = ffi.ppst_server_register_column(srv, cx, n)
    ts = [ffi.ppst_server_submit(srv, ffi.Q_ZSCORE, cid, 0, 1.0, 1.0, cfg) for _ in range(3)]
    assert not ffi.ppst_server_poll(srv, ts[-1])   # one slot: the last one is still queued
    rc, ct, st = ffi.ppst_server_wait(srv, ts[-1])
    assert rc == 0
    assert all(ffi.ppst_server_poll(srv, t) for t in ts[:-1])   # served before it, in order
    assert all(ffi.ppst_server_wait(srv, t)[0] == 0 for t in ts[:-1])


def test_register_right_after_encryption(env):
    """Columns registered while their encryptions may still be running on the
    caller's stream are copied complete: every mean matches FP64."""
    ctx, sk, evk, cols = env
    slots = ctx.info.slots
    pk = ffi.ppst_keygen(ctx, 5)[1]
    srv = ffi.ppst_server_create(ctx, evk, 8 << 30, 4)
    cfg = ffi.ppst_invsqrt_cfg_default()
    fresh = []
    for seed in range(4):
        n = 3 * slots - 100
        y = synth.lognormal_bernoulli_pair(40 + seed, n)[1] / 4.0
        cy = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, v, 24), 900 + 10 * seed + i)
              for i, v in enumerate(synth.split_column(y, slots))]
        fresh.append((ffi.ppst_server_register_column(srv, cy, n), n, y))   # no sync before
    ts = [ffi.ppst_server_submit(srv, ffi.Q_MEAN, cid, 0, 1.0, 1.0, cfg) for cid, _, _ in fresh]
    for t, (cid, n, y) in zip(ts, fresh):
        rc, ct, st = ffi.ppst_server_wait(srv, t)
        got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, ct))[0]
        assert rc == 0 and abs(got - y.mean()) < 1e-3 * max(1.0, abs(y.mean()))


def test_zscore_query_returns_every_ciphertext(env):
    """A served ZNorm over a 3-ciphertext column hands back all three z-score
    ciphertexts (wait_all), each equal to the direct call's; a too-small
    output array is refused without collecting the query."""
    ctx, sk, evk, cols = env
    cfg = ffi.ppst_invsqrt_cfg_default()
    n, x, y, cx, cy = cols["c"]
    srv = ffi.ppst_server_create(ctx, evk, 8 << 30, 2)
    cid = ffi.ppst_server_register_column(srv, cy, n)
    t = ffi.ppst_server_submit(srv, ffi.Q_ZSCORE, cid, 0, 2.0, 2.0, cfg)
    assert ffi.ppst_server_output_count(srv, t) == len(cy) == 3
    rc, outs, st = ffi.ppst_server_wait_all(srv, t, cap=2)
    assert rc == -1 and outs == []
    rc, outs, st = ffi.ppst_server_wait_all(srv, t)
    assert rc == 0 and len(outs) == 3
    alone = ffi.ppst_stat_zscore(ctx, evk, cy, n, 2.0, cfg)
    for a, b in zip(outs, alone):
        assert np.array_equal(ffi.ppst_ct_export(ctx, a), ffi.ppst_ct_export(ctx, b))
    z = np.concatenate([ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, c)) for c in outs])[:n]
    assert S.mre(z, S.zscore(y)) < 1e-3
    t = ffi.ppst_server_submit(srv, ffi.Q_MEAN, cid, 0, 1.0, 1.0, cfg)
    assert ffi.ppst_server_output_count(srv, t) == 1
    rc, outs, st = ffi.ppst_server_wait_all(srv, t)
    assert rc == 0 and len(outs) == 1


def test_results_outlive_the_server(env):
    """Result ciphertexts stay usable after the server that produced them is
    destroyed, and releasing them afterwards (the last use of the worker's
    memory pool, whose stream is gone) leaves the device working."""
    ctx, sk, evk, cols = env
    cfg = ffi.ppst_invsqrt_cfg_default()
    n, x, y, cx, cy = cols["c"]
    srv = ffi.ppst_server_create(ctx, evk, 8 << 30, 2)
    cid = ffi.ppst_server_register_column(srv, cy, n)
    ts = [ffi.ppst_server_submit(srv, ffi.Q_MEAN, cid, 0, 1.0, 1.0, cfg) for _ in range(3)]
    outs = [ffi.ppst_server_wait(srv, t)[1] for t in ts]
    del srv
    for ct in outs:
        assert abs(ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, ct))[0] - y.mean()) < 1e-3
    del outs, ct
    again = ffi.ppst_stat_mean(ctx, evk, cy, n, 1.0)
    assert abs(ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, again))[0] - y.mean()) < 1e-3


def test_c2_mixed_stream_equals_alone():
    """N = 2^16, L = 24, config-2 columns (x ~ Bernoulli(0.2), lognormal y):
    mean, variance, z-score, CV and Pearson twice each on 8 workers, their
    rotate-and-sums merged across queries, give the same result ciphertexts
    as the same calls made one at a time."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[serving] preset c2", flush=True)
    ctx = ffi.ppst_context_create("c2")
    sk, pk = ffi.ppst_keygen(ctx, 15)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 16, evk)
    ffi.ppst_evk_add_rotsum(ctx, sk, 17, evk)
    x, y = synth.binary_cost_pair(3)
    n, L = len(x), ctx.info.L
    cx = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, x, L), 301)]
    cy = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, y, L), 302)]
    cfg = ffi.ppst_invsqrt_cfg_default()
    srv = ffi.ppst_server_create(ctx, evk, 0, 8)
    xid, yid = ffi.ppst_server_register_column(srv, cx, n), ffi.ppst_server_register_column(srv, cy, n)
    # y: mean ~18, variance ~300 -> Var/B^2 in [1e-3, 1] with B = 20, mean/B_mean in [0.6, 1.1] with 25
    plan = [(ffi.Q_MEAN, 20.0, 20.0), (ffi.Q_VARIANCE, 20.0, 20.0), (ffi.Q_ZSCORE, 20.0, 20.0),
            (ffi.Q_CV, 25.0, 20.0), (ffi.Q_PEARSON, 1.0, 20.0)] * 2
    tickets = [ffi.ppst_server_submit(srv, k, xid if k == ffi.Q_PEARSON else yid, yid, B, B2, cfg)
               for k, B, B2 in plan]
    res = [ffi.ppst_server_wait(srv, t) for t in tickets]
    info = ffi.ppst_server_info(srv)
    print("[serving] c2 merged rotate-and-sums:", info, flush=True)
    for (k, B, B2), (rc, ct, st) in zip(plan, res):
        assert rc == 0, (k, ffi.lib().ppst_last_error())
        alone = direct(ctx, evk, k, cx if k == ffi.Q_PEARSON else cy, cy, n, B, B2, cfg)
        assert np.array_equal(ffi.ppst_ct_export(ctx, ct), ffi.ppst_ct_export(ctx, alone)), k
    assert info["multi_query_launches"] > 0, info
    got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, res[4][1]))[0]
    assert abs(got - S.pearson(x, y)) / abs(S.pearson(x, y)) < 1e-3
