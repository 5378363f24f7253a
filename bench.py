#!/usr/bin/env python3
"""Benchmark of the encrypted-statistics hot path on one MI355X.

Headline metric: HMult+relin (+ rescale) per second at N = 2^16, level 24
(the paper's N, Delta and modulus budget; 24 levels of 40-bit primes, 7
special primes, dnum = 3).  One timed step is one batch of 64 independent
ciphertext products (slot values ~ U[-1, 1)) through the per-ciphertext path;
inputs are resident in HBM before the timed region.

Reported beside it on the same JSON line: rotations/s at level 24, the
batched and hoisted forms, p50/p99 latency of an encrypted Pearson
correlation on two 32768-row columns (binary x, lognormal y, corr ~ 0.79) with
its relative error, the roofline of the dominant kernel (forward NTT, timed
with HIP events on the library's stream), and the CPU reference timed on the
host cores.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU ceiling: 256 CUs x 64 lanes x 2.4 GHz = 39.32 T lane-operations/s
# (FP64 fused multiply-add issues at that full rate: 78.6 TFLOP/s).
VALU_PEAK = 256 * 64 * 2.4e9
# One forward butterfly on the FP64 path (every 40-bit prime of the chain):
# 6 operations for the exact product r = y w - k q (mul, fma, mul, rint, fma,
# add) and 2 for the outputs x + r, x - r (the path keeps residues unreduced
# between stages, so there is no reduction step).
OPS_PER_BFLY = 8
BFLY_PEAK_G = VALU_PEAK / OPS_PER_BFLY / 1e9
# HBM bytes per 25-limb forward NTT from FETCH_SIZE + WRITE_SIZE counters
# (rocprofv3 --pmc, one counter per run), scaled by the same counters on a
# plain copy of known size.  The figure belongs to the NTT source it was taken
# with (its SHA-256 below); for any other source the traffic is reported as
# null.
NTT_TRAFFIC = {"bytes": 55823626,
               "source_sha256": "b44b006d8ebd757dc0c360ac372d09d4a5aa0a0f663dff2da86641f7f81acfb4"}
# Algorithmic HBM bytes of the other key-switching kernels of one plain
# product at level 24 (N = 2^16, K = 7, dnum = 3; a limb is 512 KiB): the key
# inner product reads 3 digit limbs and 6 key limbs per extended limb (32)
# and writes 2 (352 limbs), alone or fused with the row pass of the digits'
# forward NTT (the pass's own input is the same 3 digit limbs); ModUp reads d2's 25 limbs and writes the 71
# extension limbs; the ModDown correction reads 2 x 8 limbs and writes
# 2 x 24; the tensor reads 4 x 25 and writes 3 x 25; ModUp inside the
# digits' column pass reads the 25 scaled limbs and writes the 69 extension
# limbs column-transformed.
LIMB = 1 << 19
# (a product from its operands: the ModDown + rescale's last pass reads
# corr, u, a0, a1, b0, b1 and writes the output, 2 x 24 limbs each but the
# operands' 4 x 24, per item: 240 limbs)
KS_KERNELS = {"k_ntt_row_mdr<8, 2, 4>": ("hbm", 240 * LIMB), "k_ks_inner_kernel<1>": ("hbm", 352 * LIMB), "k_ntt_row_ks<8, 2, 4>": ("hbm", 352 * LIMB),
              "k_ntt_col_modup<3, 16, 9>": ("alu", 94 * LIMB), "k_modup_kernel<9>": ("alu", 96 * LIMB),
              "k_mdr_corr_kernel<8>": ("alu", 64 * LIMB), "k_tensor_kernel": ("hbm", 175 * LIMB)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--pearson-runs", type=int, default=30)
    ap.add_argument("--cpu-runs", type=int, default=5,
                    help="repetitions per operation of the oracle timed on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-pearson", action="store_true",
                    help="skip timing the oracle's encrypted Pearson on the config-2 columns "
                         "(about 20 s at 16 host threads, plus its key generation)")
    ap.add_argument("--quick", action="store_true", help="short run for profiling")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the roofline kernel and a copy of known size")
    ap.add_argument("--ntt-variants", default=None,
                    help="column,row variant indices of the roofline kernel (default %d,%d)"
                    % (NTT_COL_VARIANT, NTT_ROW_VARIANT))
    ap.add_argument("--boot-runs", type=int, default=5,
                    help="timed bootstraps at N=2^16 (0: skip the bootstrapping leg)")
    ap.add_argument("--only", choices=["plain", "batched", "pearson", "boot"], default=None,
                    help="time one form of the 64-product step alone (for kernel profiles)")
    ap.add_argument("--no-exp2", action="store_true",
                    help="skip the 1M-row statistics replay of Sec. 6.3")
    ap.add_argument("--serving-queries", type=int, default=200,
                    help="queries per load point of the serving loop (0: skip)")
    ap.add_argument("--serving-slots", type=int, default=8,
                    help="queries in flight at once (worker streams)")
    ap.add_argument("--serving-loads", type=str, default="0.5,0.9",
                    help="offered loads as fractions of the measured saturation rate")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2508_12093_amd import ffi, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.kernels_only:
        kernels_only(args)
        return
    if args.quick:
        args.steps, args.warmup, args.pearson_runs = min(args.steps, 3), 1, 3
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    sptr = ctypes.c_void_p(stream.cuda_stream)
    ctx = ffi.ppst_context_create("c2", stream=sptr)
    info = ctx.info
    L, N = info.L, info.N
    log("context N=%d L=%d K=%d dnum=%d" % (N, L, info.K, info.dnum))
    log("NTT plan:", ffi.ppst_ntt_plan(ctx))

    sk, pk = ffi.ppst_keygen(ctx, 1001)
    evk = ffi.ppst_evk_create(ctx)
    ffi.ppst_evk_add_relin(ctx, sk, 1002, evk)
    ffi.ppst_evk_add_rotsum(ctx, sk, 1003, evk)
    hoist_steps = list(range(1, 17))
    ffi.ppst_evk_add_galois(ctx, sk, hoist_steps, 1003, evk)
    log("keys ready")

    B = args.batch
    vals = synth.slot_batch(7, B, info.slots)
    cts = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, vals[i], L), 2000 + i) for i in range(B)]
    ffi.ppst_sync(ctx)
    log("%d ciphertexts resident at level %d" % (B, L))

    def sync():
        ffi.ppst_sync(ctx)
        torch.cuda.synchronize()

    # ------------------------------------------------ headline: HMult+relin
    def step_mul():
        outs = [ffi.ppst_mul(ctx, evk, cts[i], cts[(i + 1) % B]) for i in range(B)]
        return outs

    if args.only == "boot":
        print(json.dumps({"only": "boot", "bootstrap": boot_bench(stream, max(1, args.boot_runs))}))
        return
    if args.only == "pearson":
        x, y = synth.binary_cost_pair(0)
        cx = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, x, L), 3001)
        cy = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, y, L), 3002)
        cfg = ffi.ppst_invsqrt_cfg_default()
        ffi.ppst_stat_pearson(ctx, evk, [cx], [cy], len(x), 1.0, 20.0, cfg)
        sync()
        t = time.perf_counter()
        for _ in range(args.steps):
            res = ffi.ppst_stat_pearson(ctx, evk, [cx], [cy], len(x), 1.0, 20.0, cfg)
        sync()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        log("Pearson: %.2f ms" % ms)
        print(json.dumps({"only": "pearson", "ms": round(ms, 3), "steps": args.steps}))
        return
    if args.only:
        fn = step_mul if args.only == "plain" else (
            lambda: ffi.ppst_mul_batch(ctx, evk, cts, cts[1:] + cts[:1]))
        fn()
        sync()
        t = time.perf_counter()
        for _ in range(args.steps):
            keep = fn()
        sync()
        rate = B * args.steps / (time.perf_counter() - t)
        del keep
        log("%s HMult+relin+rescale: %.0f /s" % (args.only, rate))
        print(json.dumps({"only": args.only, "hmult_per_s": round(rate, 2), "steps": args.steps}))
        return

    for _ in range(args.warmup):
        step_mul()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        keep = step_mul()
    sync()
    t1 = time.perf_counter()
    del keep
    ms_step = (t1 - t0) * 1e3 / args.steps
    hmult_s = B * args.steps / (t1 - t0)
    log("HMult+relin+rescale: %.3f ms / step of %d -> %.0f /s" % (ms_step, B, hmult_s))

    # the same 64 products spread over 4 contexts with their own streams
    # (one ciphertext per launch; independent products overlap on the GPU)
    forks = [ffi.ppst_context_fork(ctx) for _ in range(4)]

    def step_mul_streams():
        return [ffi.ppst_mul(forks[i % 4], evk, cts[i], cts[(i + 1) % B]) for i in range(B)]

    def sync_all():
        for f in forks:
            ffi.ppst_sync(f)
        sync()

    step_mul_streams()
    sync_all()
    t = time.perf_counter()
    for _ in range(args.steps):
        keep = step_mul_streams()
    sync_all()
    ms4_s = B * args.steps / (time.perf_counter() - t)
    del keep
    log("HMult+relin+rescale on 4 streams: %.0f /s" % ms4_s)

    # check one product against the plaintext
    got = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, ffi.ppst_mul(ctx, evk, cts[0], cts[1])))
    hmult_err = float(np.max(np.abs(got - vals[0] * vals[1])))

    def timed(fn, reps):
        fn()
        sync()
        t = time.perf_counter()
        for _ in range(reps):
            keep = fn()
        sync()
        return (time.perf_counter() - t) / reps

    # ------------------------------------------------------ rotations
    rot_t = timed(lambda: [ffi.ppst_rotate(ctx, evk, cts[i], 1 + (i % 15)) for i in range(B)],
                  max(1, args.steps // 2))
    rot_s = B / rot_t
    log("rotation: %.0f /s" % rot_s)

    # ----------------------------------------------- batched / hoisted forms
    bm_t = timed(lambda: ffi.ppst_mul_batch(ctx, evk, cts, cts[1:] + cts[:1]), max(1, args.steps // 2))
    bm_s = B / bm_t
    log("batched HMult: %.0f /s" % bm_s)

    # the same two steps recorded once into HIP graphs and replayed
    def record(fn):
        ffi.ppst_graph_begin(ctx)
        try:
            outs = fn()
        finally:
            g = ffi.ppst_graph_end(ctx)
        return g, outs

    g_plain, keep_p = record(step_mul)
    gp_t = timed(g_plain.launch, max(1, args.steps // 2))
    g_batch, keep_b = record(lambda: ffi.ppst_mul_batch(ctx, evk, cts, cts[1:] + cts[:1]))
    gb_t = timed(g_batch.launch, max(1, args.steps // 2))
    gp_s, gb_s = B / gp_t, B / gb_t
    log("graph-replayed HMult: plain %.0f /s, batched %.0f /s" % (gp_s, gb_s))
    del g_plain, g_batch, keep_p, keep_b
    nh = min(B, 8)
    ho_t = timed(lambda: [ffi.ppst_rotate_hoisted(ctx, evk, cts[i], hoist_steps) for i in range(nh)], 1)
    ho_s = nh * len(hoist_steps) / ho_t
    log("hoisted rotations: %.0f /s" % ho_s)
    hb_t = timed(lambda: ffi.ppst_rotate_hoisted_batch(ctx, evk, cts, hoist_steps), 1)
    hb_s = B * len(hoist_steps) / hb_t
    log("batched hoisted rotations (%d x %d): %.0f /s" % (B, len(hoist_steps), hb_s))

    # --------------------------------------------- Pearson latency (config 2)
    x, y = synth.binary_cost_pair(0)
    n = len(x)
    cx = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, x, L), 3001)
    cy = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, y, L), 3002)
    cfg = ffi.ppst_invsqrt_cfg_default()
    lat = []
    res = None
    for r in range(args.pearson_runs + 1):
        sync()
        t = time.perf_counter()
        res = ffi.ppst_stat_pearson(ctx, evk, [cx], [cy], n, 1.0, 20.0, cfg)
        sync()
        if r > 0:
            lat.append((time.perf_counter() - t) * 1e3)
    pcc = float(ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, res))[0])
    ref_pcc = float(np.corrcoef(x, y)[0, 1])
    lat = np.array(lat)
    log("Pearson p50 %.2f ms p99 %.2f ms, value %.6f (fp64 %.6f)" % (
        np.percentile(lat, 50), np.percentile(lat, 99), pcc, ref_pcc))

    # ------------------- CryptoInvSqrt replay of Sec. 6.2, Exp. 1 (Tab. 2 row)
    # 32768-point grid on [0.001, 100], B = 100, Eq. 3's degree-31 Chebyshev
    # initial value on [0, 2] and six Newton steps: 19 levels, no bootstrap.
    grid = synth.exp1_grid(info.slots)
    cg = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, grid, L), 3003)
    e1cfg = ffi.ppst_invsqrt_cfg_default(a=0.0, b=2.0, degree=31, iters=6)
    e1lat, e1 = [], None
    for r in range(args.pearson_runs + 1):
        sync()
        t = time.perf_counter()
        e1 = ffi.ppst_stat_invsqrt(ctx, evk, [cg], 100.0, e1cfg)[0]
        sync()
        if r > 0:
            e1lat.append((time.perf_counter() - t) * 1e3)
    e1v = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, e1))
    e1_mre = float(np.mean(np.abs(e1v * np.sqrt(grid) - 1.0)))
    e1_p50 = float(np.percentile(e1lat, 50))
    log("Exp. 1 CryptoInvSqrt (32768 points, degree 31, 6 Newton): p50 %.2f ms, MRE %.3e" % (
        e1_p50, e1_mre))
    del cg, e1

    exp2 = None if args.no_exp2 else exp2_replay(ctx, pk, sk, evk, sync)

    serving = None
    if args.serving_queries > 0:
        loads = [float(v) for v in args.serving_loads.split(",") if v]
        serving = serving_bench(ctx, pk, sk, evk, args.serving_queries, loads,
                                nslots=args.serving_slots)
    boot = boot_bench(stream, args.boot_runs) if args.boot_runs > 0 else None
    rf = measure_ntt(ctx, stream, reps=10 if args.quick else 50)
    peaks = measure_peaks(stream)

    out = {
        "metric": "HMult+relin/sec and rotations/sec at N=2^16; p50/p99 encrypted-Pearson latency",
        "value": round(hmult_s, 2),
        "unit": "HMult+relin/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "RNS-CKKS N=2^16, L=24 (q0 60-bit, 24x~40-bit, 7x60-bit special primes, "
                        "dnum=3, Delta=2^40): %d independent HMult+relin+rescale at level 24 per "
                        "step, slots ~U[-1,1); Pearson on two 32768-row columns" % B,
            "ring_degree": N, "levels": L, "batch": B,
        },
        "rotations_per_s": round(rot_s, 2),
        "hmult_4streams_per_s": round(ms4_s, 2),
        "hmult_batched_per_s": round(bm_s, 2),
        "hmult_graph_per_s": round(gp_s, 2),
        "hmult_batched_graph_per_s": round(gb_s, 2),
        "rotations_hoisted_per_s": round(ho_s, 2),
        "rotations_hoisted_batched_per_s": round(hb_s, 2),
        "pearson_p50_ms": round(float(np.percentile(lat, 50)), 3),
        "pearson_p99_ms": round(float(np.percentile(lat, 99)), 3),
        "pearson_runs": len(lat),
        "pearson_value": pcc,
        "pearson_rel_err": abs(pcc - ref_pcc) / abs(ref_pcc),
        "hmult_max_slot_err": hmult_err,
        "exp1_invsqrt_p50_ms": round(e1_p50, 3),
        "exp1_invsqrt_mre": e1_mre,
        "roofline": rf,
        "roofline_kernels": profiled_kernels(),
        "peaks": peaks,
    }
    if exp2 is not None:
        out["exp2"] = exp2
    if serving is not None:
        out["serving"] = serving
    if boot is not None:
        out["bootstrap"] = boot
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_runs, not args.no_cpu_pearson)
    print(json.dumps(out), flush=True)


def _mre(approx, exact, floor_frac=1e-3):
    """Mean relative error over the entries with |exact| >= floor_frac max|exact|."""
    import numpy as np
    a, e = np.atleast_1d(approx), np.atleast_1d(exact)
    keep = np.abs(e) >= floor_frac * np.max(np.abs(e))
    return float(np.mean(np.abs(a[keep] - e[keep]) / np.abs(e[keep])))


def exp2_replay(ctx, pk, sk, evk, sync, n: int = 1_000_000):
    """Sec. 6.3 (Tab. 3) without bootstrapping: one million rows (31
    ciphertexts), ZNorm on U[0, 100] with B = 100, skewness, kurtosis and PCC
    on U[0, 20] with B = 20, using Exp. 1's InvSqrt (Eq. 3's degree-31
    Chebyshev on [0, 2], six Newton steps); CV on U[0, 20] with B_var = 20,
    B_mean = 16 (the g_3 sign needs mean/B_mean >= 0.6) and the degree-7 /
    three-step InvSqrt so that it fits 24 levels.  The PCC pair is
    y = (x + u) / 2 with u ~ U[0, 20] (correlation 1/sqrt 2)."""
    import numpy as np

    from paper_2508_12093_amd import ffi, synth
    info = ctx.info
    L, slots = info.L, info.slots
    x100 = synth.uniform_column(11, n, 0.0, 100.0)
    x20 = synth.uniform_column(12, n, 0.0, 20.0)
    y20 = 0.5 * (x20 + synth.uniform_column(13, n, 0.0, 20.0))

    def enc(v, seed):
        return [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, c, L), seed + k)
                for k, c in enumerate(synth.split_column(v, slots))]

    c100, c20, cy = enc(x100, 40000), enc(x20, 41000), enc(y20, 42000)
    dec = lambda c: ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, c))
    e1 = ffi.ppst_invsqrt_cfg_default(a=0.0, b=2.0, degree=31, iters=6)
    dflt = ffi.ppst_invsqrt_cfg_default()

    def moments(v):
        d = v - v.mean()
        m2, m3, m4 = np.mean(d ** 2), np.mean(d ** 3), np.mean(d ** 4)
        return d / np.sqrt(m2), m3 / m2 ** 1.5, m4 / m2 ** 2, np.sqrt(m2) / v.mean()

    z_ref = moments(x100)[0]
    _, sk_ref, ku_ref, cv_ref = moments(x20)
    runs = {
        "zscore": (lambda: ffi.ppst_stat_zscore(ctx, evk, c100, n, 100.0, e1), z_ref),
        "skewness": (lambda: ffi.ppst_stat_skewness(ctx, evk, c20, n, 20.0, e1), sk_ref),
        "kurtosis": (lambda: ffi.ppst_stat_kurtosis(ctx, evk, c20, n, 20.0, e1), ku_ref),
        "cv": (lambda: ffi.ppst_stat_cv(ctx, evk, c20, n, 16.0, 20.0, dflt), cv_ref),
        "pearson": (lambda: ffi.ppst_stat_pearson(ctx, evk, c20, cy, n, 20.0, 20.0, e1),
                    float(np.corrcoef(x20, y20)[0, 1])),
    }
    res = {"rows": n, "ciphertexts": len(c100)}
    for name, (fn, ref) in runs.items():
        sync()
        t = time.perf_counter()
        r = fn()
        sync()
        ms = (time.perf_counter() - t) * 1e3
        if isinstance(r, list):
            got = np.concatenate([dec(c) for c in r])[:n]
        else:
            got = dec(r)[0]
        err = _mre(got, ref)
        res[name] = {"ms": round(ms, 2), "mre": err, "abs_err": float(np.max(np.abs(got - ref)))}
        log("Exp. 2 %-8s %8.2f ms  MRE %.3e  abs %.3e" % (name, ms, err, res[name]["abs_err"]))
        del r
    return res


SERVING_ROWS = [1 << 10, 1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20]


def serving_bench(ctx, pk, sk, evk, nq: int, loads, seed: int = 4, nslots: int = 8):
    """Continuous-batching server over resident columns of 2^10..2^20 rows
    (1..32 ciphertexts): x ~ Bernoulli(0.3), y = (lognormal(0, 1) + s x) / 4
    with corr ~ 0.5.  Query kinds uniform over mean, variance, z-score, CV and
    Pearson, column sizes uniform over the six; first every query at once
    (saturation throughput), then Poisson arrivals at the given fractions of
    that rate.  Latency = arrival to result ready (server timestamps)."""
    import threading

    import numpy as np

    from paper_2508_12093_amd import ffi, synth

    def fp64(kind, B, x, y):
        """The statistic each query kind returns (mean / B, Var / B^2, z_0, CV, PCC)."""
        m, v = y.mean(), y.var()
        return {ffi.Q_MEAN: m / B, ffi.Q_VARIANCE: v / (B * B), ffi.Q_ZSCORE: (y[0] - m) / np.sqrt(v),
                ffi.Q_CV: np.sqrt(v) / m, ffi.Q_PEARSON: float(np.corrcoef(x, y)[0, 1])}[kind]

    info = ctx.info
    slots, L = info.slots, info.L
    data = {}
    for i, n in enumerate(SERVING_ROWS):
        x, y = synth.lognormal_bernoulli_pair(seed + i, n)
        y = y / 4.0
        cx = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, v, L), 10000 * (i + 1) + k)
              for k, v in enumerate(synth.split_column(x, slots))]
        cy = [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, v, L), 10000 * (i + 1) + 5000 + k)
              for k, v in enumerate(synth.split_column(y, slots))]
        data[n] = (cx, cy, x, y)
    ffi.ppst_sync(ctx)

    def open_server(merge):
        # admission by the device's free memory (budget 0)
        s = ffi.ppst_server_create(ctx, evk, 0, nslots, merge=merge)
        c = {n: (ffi.ppst_server_register_column(s, cx, n), ffi.ppst_server_register_column(s, cy, n), x, y)
             for n, (cx, cy, x, y) in data.items()}
        return s, c

    srv, cols = open_server(True)
    cfg = ffi.ppst_invsqrt_cfg_default()
    # (kind, column, bounds): Var/B^2 inside [1e-3, 1] and mean/B_mean inside [0.6, 1.1]
    kinds = [(ffi.Q_MEAN, "y", 1.0, 1.0), (ffi.Q_VARIANCE, "y", 2.0, 2.0), (ffi.Q_ZSCORE, "y", 2.0, 2.0),
             (ffi.Q_CV, "y", 0.8, 2.0), (ffi.Q_PEARSON, "x", 1.0, 2.0)]
    rng = np.random.default_rng(seed)

    def plan(count):
        return [(kinds[rng.integers(len(kinds))], SERVING_ROWS[rng.integers(len(SERVING_ROWS))])
                for _ in range(count)]

    def submit(q):
        (kind, which, B, B2), n = q
        xid, yid = cols[n][0], cols[n][1]
        return ffi.ppst_server_submit(srv, kind, xid if which == "x" else yid, yid, B, B2, cfg)

    def run(queries, rate):
        tickets = [None] * len(queries)
        gaps = rng.exponential(1.0 / rate, len(queries)) if rate else np.zeros(len(queries))

        failure = []

        def feeder():
            t0 = time.perf_counter()
            at = 0.0
            try:
                for i, q in enumerate(queries):
                    at += gaps[i]
                    d = t0 + at - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    tickets[i] = submit(q)
            except BaseException as e:        # a refused submission ends the run
                failure.append(e)

        th = threading.Thread(target=feeder)
        t_start = time.perf_counter()
        th.start()
        res = []
        for i in range(len(queries)):
            while tickets[i] is None and not failure:
                time.sleep(1e-4)
            if tickets[i] is None:
                break
            res.append(ffi.ppst_server_wait(srv, tickets[i]))
        th.join()
        if failure:
            raise failure[0]
        wall = time.perf_counter() - t_start
        failed = [r[0] for r in res if r[0] != 0]
        if failed:
            log("serving: %d of %d queries failed (first status %d)" % (len(failed), len(res), failed[0]))
        lat = np.array([(r[2].t_done - r[2].t_submit) * 1e3 for r in res if r[0] == 0])
        return res, lat, wall, len(failed)

    # warm-up: every (kind, size) once
    run([(k, n) for k in kinds for n in SERVING_ROWS], None)
    sat_q = plan(nq)
    res, lat, wall, nfail = run(sat_q, None)
    sat_rate = len(sat_q) / wall
    log("serving: saturation %.1f queries/s over %d queries" % (sat_rate, len(sat_q)))
    # spot-check decrypted values of the saturation run against FP64
    errs = []
    for (q, r) in [qr for qr in zip(sat_q, res) if qr[1][0] == 0][:12]:
        (kind, which, B, B2), n = q
        x, y = cols[n][2], cols[n][3]
        got = float(ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, r[1]))[0])
        want = fp64(kind, B, x, y)
        errs.append(abs(got - want) / max(abs(want), 1.0))   # relative, absolute below 1
    del res                                   # the results' blocks go back to the pools
    points = []
    for f in loads:
        rate = f * sat_rate
        _, lat, wall, nf = run(plan(nq), rate)
        nfail += nf
        points.append({"offered_qps": round(rate, 2), "achieved_qps": round(nq / wall, 2),
                       "p50_ms": round(float(np.percentile(lat, 50)), 2),
                       "p99_ms": round(float(np.percentile(lat, 99)), 2), "queries": nq,
                       "failed": nf})
        log("serving: offered %.1f q/s -> p50 %.1f ms, p99 %.1f ms" % (
            rate, points[-1]["p50_ms"], points[-1]["p99_ms"]))
    info = ffi.ppst_server_info(srv)
    t = time.perf_counter()
    del srv
    log("serving: server closed in %.1f s; merged rotate-and-sums %s" % (time.perf_counter() - t, info))
    # the same saturation run without merging the queries' rotate-and-sums
    srv, cols = open_server(False)
    run([(k, n) for k in kinds for n in SERVING_ROWS], None)
    _, _, wall0, nf0 = run(sat_q, None)
    nfail += nf0
    sat0 = len(sat_q) / wall0
    log("serving: saturation without merging %.1f queries/s" % sat0)
    del srv
    return {"saturation_qps": round(sat_rate, 2), "saturation_qps_no_merge": round(sat0, 2),
            "queries_per_point": nq, "budget_bytes": info["budget"],
            "merged_rotsum_launches": info["merged_launches"], "merged_rotsum_lanes": info["merged_lanes"],
            "multi_query_rotsum_launches": info["multi_query_launches"],
            "rows": SERVING_ROWS, "kinds": "mean,variance,zscore,cv,pearson", "slots": nslots,
            "loads": points, "failed": nfail, "spot_max_err": float(max(errs)) if errs else None}


# The roofline kernel is timed under a fixed variant pair (the one the
# autotuner picks for 25-limb forward transforms on MI355X in most runs), so
# that the same kernels appear in the rocprofv3 profiles of --kernels-only.
NTT_COL_VARIANT, NTT_ROW_VARIANT = 5, 7      # col:E3,SB16,D / row:E2,SB4,D


def boot_bench(stream, runs: int):
    """Bootstrapping at N=2^16 ("b2": 11 computation levels under 16
    bootstrapping levels, sparse secret): a level-0 ciphertext of 32768
    slots ~U[-1,1) refreshed to level 11, `runs` times after one warm-up;
    inputs resident in HBM.  Reports ms per bootstrap, bootstraps/s, the
    setup time (keys and the transforms' plaintexts) and the refresh error."""
    import numpy as np
    import torch

    from paper_2508_12093_amd import ffi, synth

    sptr = ctypes.c_void_p(stream.cuda_stream)
    t = time.perf_counter()
    bctx = ffi.ppst_context_create("b2", stream=sptr)
    sk, pk = ffi.ppst_keygen(bctx, 5001)
    evk = ffi.ppst_evk_create(bctx)
    ffi.ppst_evk_add_relin(bctx, sk, 5002, evk)
    ffi.ppst_evk_add_boot(bctx, sk, 5003, evk)
    keys_s = time.perf_counter() - t
    t = time.perf_counter()
    bt = ffi.ppst_boot_create(bctx)
    plain_s = time.perf_counter() - t
    n = bctx.info.slots
    m = synth.uniform_column(5004, n, -1, 1)
    ct = ffi.ppst_encrypt(bctx, pk, ffi.ppst_encode(bctx, m, 0), 5005)
    out = ffi.ppst_bootstrap(bctx, evk, bt, ct)

    def sync():
        ffi.ppst_sync(bctx)
        torch.cuda.synchronize()

    sync()
    t = time.perf_counter()
    for _ in range(runs):
        out = ffi.ppst_bootstrap(bctx, evk, bt, ct)
    sync()
    ms = (time.perf_counter() - t) * 1e3 / runs
    got = ffi.ppst_decode(bctx, ffi.ppst_decrypt(bctx, sk, out), n)
    err = float(np.max(np.abs(got - m)))
    log("bootstrap (N=2^16, L=27 -> 11): %.2f ms, %.1f /s, max error 2^%.2f; setup keys %.1f s, "
        "plaintexts %.1f s" % (ms, 1e3 / ms, np.log2(err), keys_s, plain_s))
    res = {"workload": "bootstrap of one ciphertext, N=2^16, level 0 -> 11 of L=27 (3 CoeffToSlot, "
                       "10 EvalMod, 3 SlotToCoeff levels), h=64, 32768 slots ~U[-1,1)",
           "ms_per_bootstrap": round(ms, 3), "bootstraps_per_s": round(1e3 / ms, 3), "runs": runs,
           "max_abs_err": err, "err_log2": round(float(np.log2(err)), 2),
           "setup_keys_s": round(keys_s, 2), "setup_plaintexts_s": round(plain_s, 2),
           "paper_lattigo_ms": 43478.77}
    # config 5: kurtosis and PCC of 2^20-row columns (32 ciphertexts at
    # level 11) with the paper's InvSqrt (Eq. 3's degree 31 on [0, 2], six
    # Newton steps, B = 20; Sec. 6.3's U[0, 20] data), whose depth exceeds
    # the 11 levels, so InvSqrt refreshes by bootstrapping
    del out, ct
    ffi.ppst_evk_add_rotsum(bctx, sk, 5006, evk)
    rows = 1 << 20
    x = synth.uniform_column(5010, rows, 0.0, 20.0)
    y = 0.5 * (x + synth.uniform_column(5011, rows, 0.0, 20.0))

    def enc(v, seed):
        return [ffi.ppst_encrypt(bctx, pk, ffi.ppst_encode(bctx, c, 11), seed + k)
                for k, c in enumerate(synth.split_column(v, n))]

    X, Y = enc(x, 6000), enc(y, 7000)
    # the library's own Eq. 3 coefficients (a = 0, b = 2)
    cfg = ffi.ppst_invsqrt_cfg_default(a=0.0, b=2.0, degree=31, iters=6, boot=bt)
    dx, dy = x - x.mean(), y - y.mean()
    kurt_ref = float(np.mean(dx ** 4) / np.mean(dx ** 2) ** 2)
    pcc_ref = float(np.mean(dx * dy) / np.sqrt(np.mean(dx * dx) * np.mean(dy * dy)))
    pipe = {"workload": "kurtosis and PCC of 2^20-row columns (32 ciphertexts at level 11), "
                        "U[0,20] data, B=20, InvSqrt degree 31 + 6 Newton steps with "
                        "bootstrapping refreshes, N=2^16"}
    for name, fn, ref in (
            ("kurtosis", lambda: ffi.ppst_stat_kurtosis(bctx, evk, X, rows, 20.0, cfg), kurt_ref),
            ("pearson", lambda: ffi.ppst_stat_pearson(bctx, evk, X, Y, rows, 20.0, 20.0, cfg),
             pcc_ref)):
        fn()
        sync()
        b0 = ffi.ppst_boot_count(bt)
        t = time.perf_counter()
        r = fn()
        sync()
        ms_s = (time.perf_counter() - t) * 1e3
        v = float(ffi.ppst_decode(bctx, ffi.ppst_decrypt(bctx, sk, r), 1)[0])
        pipe[name] = {"ms": round(ms_s, 2), "bootstraps": ffi.ppst_boot_count(bt) - b0,
                      "value": v, "rel_err": abs(v / ref - 1)}
        log("config 5 %-8s %8.2f ms, %d bootstraps, rel err %.2e" % (
            name, ms_s, pipe[name]["bootstraps"], pipe[name]["rel_err"]))
    res["pipeline"] = pipe
    del X, Y
    res["exp1"] = exp1_boot(bctx, pk, sk, evk, bt, sync)
    res["exp2"] = exp2_boot(bctx, pk, sk, evk, bt, sync)
    del bt, evk, sk, pk, bctx
    return res


def _timed_stat(bt, sync, fn):
    from paper_2508_12093_amd import ffi
    fn()
    sync()
    b0 = ffi.ppst_boot_count(bt)
    t = time.perf_counter()
    r = fn()
    sync()
    return r, (time.perf_counter() - t) * 1e3, ffi.ppst_boot_count(bt) - b0


def exp1_boot(ctx, pk, sk, evk, bt, sync):
    """Sec. 6.2 (Tab. 2) at the paper's settings on the bootstrappable chain:
    the 32768-point grid on [0.001, 100], B = 100; CryptoInvSqrt = Eq. 3's
    degree 31 on [0, 2] and six Newton steps, and the HEaaN-STAT comparator
    (y_0 = 1, 21 Newton steps on x / 100), both with refreshes; MRE against
    1/sqrt(x), bootstraps counted."""
    import numpy as np

    from paper_2508_12093_amd import ffi, synth
    grid = synth.exp1_grid(ctx.info.slots)
    cg = ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, grid, 11), 5100)
    out = {"workload": "32768-point grid on [0.001, 100] at level 11 of b2, B = 100"}
    for name, cfg in (
            ("cryptoinvsqrt", ffi.ppst_invsqrt_cfg_default(a=0.0, b=2.0, degree=31, iters=6, boot=bt)),
            ("heaan_stat", ffi.ppst_invsqrt_cfg_default(coeffs=np.array([1.0]), a=0.0, b=2.0, degree=0,
                                                         iters=21, boot=bt))):
        r, ms, nb = _timed_stat(bt, sync, lambda: ffi.ppst_stat_invsqrt(ctx, evk, [cg], 100.0, cfg))
        v = ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, r[0]))
        mre = float(np.mean(np.abs(v * np.sqrt(grid) - 1.0)))
        out[name] = {"ms": round(ms, 2), "bootstraps": nb, "mre": mre}
        log("Exp. 1 with bootstrapping %-14s %8.2f ms, %d bootstraps, MRE %.3e" % (name, ms, nb, mre))
    return out


def exp2_boot(ctx, pk, sk, evk, bt, sync, n: int = 1_000_000):
    """Sec. 6.3 (Tab. 3) at the paper's settings on the bootstrappable chain:
    10^6 rows (31 ciphertexts at level 11); ZNorm on U[0, 100] with B = 100;
    skewness, kurtosis, CV (three-fold g_3 sign) and PCC on U[0, 20] with
    B = 20; CryptoInvSqrt of Exp. 1; refreshes where the 11 levels run out."""
    import numpy as np

    from paper_2508_12093_amd import ffi, synth
    slots = ctx.info.slots
    x100 = synth.uniform_column(5211, n, 0.0, 100.0)
    x20 = synth.uniform_column(5212, n, 0.0, 20.0)
    y20 = 0.5 * (x20 + synth.uniform_column(5213, n, 0.0, 20.0))

    def enc(v, seed):
        return [ffi.ppst_encrypt(ctx, pk, ffi.ppst_encode(ctx, c, 11), seed + k)
                for k, c in enumerate(synth.split_column(v, slots))]

    c100, c20, cy = enc(x100, 52000), enc(x20, 53000), enc(y20, 54000)
    cfg = ffi.ppst_invsqrt_cfg_default(a=0.0, b=2.0, degree=31, iters=6, sign_k=3, boot=bt)

    def moments(v):
        d = v - v.mean()
        m2, m3, m4 = np.mean(d ** 2), np.mean(d ** 3), np.mean(d ** 4)
        return d / np.sqrt(m2), m3 / m2 ** 1.5, m4 / m2 ** 2, np.sqrt(m2) / v.mean()

    z_ref = moments(x100)[0]
    _, sk_ref, ku_ref, cv_ref = moments(x20)
    dec = lambda c: ffi.ppst_decode(ctx, ffi.ppst_decrypt(ctx, sk, c))
    runs = {
        "zscore": (lambda: ffi.ppst_stat_zscore(ctx, evk, c100, n, 100.0, cfg), z_ref),
        "skewness": (lambda: ffi.ppst_stat_skewness(ctx, evk, c20, n, 20.0, cfg), sk_ref),
        "kurtosis": (lambda: ffi.ppst_stat_kurtosis(ctx, evk, c20, n, 20.0, cfg), ku_ref),
        "cv": (lambda: ffi.ppst_stat_cv(ctx, evk, c20, n, 20.0, 20.0, cfg), cv_ref),
        "pearson": (lambda: ffi.ppst_stat_pearson(ctx, evk, c20, cy, n, 20.0, 20.0, cfg),
                    float(np.corrcoef(x20, y20)[0, 1])),
    }
    res = {"workload": "10^6 rows (31 ciphertexts at level 11 of b2), Sec. 6.3 settings, "
                       "InvSqrt degree 31 + 6 Newton steps with refreshes, CV sign g_3^(3)"}
    for name, (fn, ref) in runs.items():
        r, ms, nb = _timed_stat(bt, sync, fn)
        got = np.concatenate([dec(c) for c in r])[:n] if isinstance(r, list) else dec(r)[0]
        err = _mre(got, ref)
        res[name] = {"ms": round(ms, 2), "bootstraps": nb, "mre": err,
                     "abs_err": float(np.max(np.abs(got - ref)))}
        log("Exp. 2 with bootstrapping %-8s %8.2f ms, %d bootstraps, MRE %.3e" % (name, ms, nb, err))
        del r
    return res


def _ntt_source_sha():
    import hashlib
    path = os.path.join(ROOT, "paper_2508_12093_amd", "csrc", "ntt.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measure_ntt(ctx, stream, reps: int, variants=None):
    """Forward NTT (column pass + row pass) of one 25-limb polynomial at
    N = 2^16, timed with HIP events on the library's stream.  Leaves the
    context on the fixed plan.

    Algorithmic work per launch pair: 25 (N/2) log2 N butterflies and
    25 MiB of HBM traffic (one read and one write of each 512 KiB limb).
    Floors: 8 FP64 VALU operations per butterfly at 39.3 T/s, and 25 MiB at
    8 TB/s; the larger floor names the bound."""
    import numpy as np
    import torch

    from paper_2508_12093_amd import ffi

    info = ctx.info
    L, N = info.L, info.N
    limbs = L + 1
    rng = np.random.default_rng(5)
    primes = ctx.primes
    ffi.ppst_ntt_set_plan(ctx, *(variants or (NTT_COL_VARIANT, NTT_ROW_VARIANT)))
    plan = ffi.ppst_ntt_plan(ctx).split(";")[0]
    host = np.stack([rng.integers(0, primes[i % limbs], N, dtype=np.uint64) for i in range(2 * limbs)])
    dev = torch.from_numpy(host.view(np.int64).copy()).cuda()
    ffi.ppst_sync(ctx)
    torch.cuda.synchronize()
    half = limbs * N * 8
    for _ in range(3):
        ffi.ppst_ntt_forward(ctx, dev.data_ptr(), limbs, 0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ffi.ppst_ntt_forward(ctx, dev.data_ptr(), limbs, 0)
        ffi.ppst_ntt_forward(ctx, dev.data_ptr() + half, limbs, 0)
    e1.record(stream)
    ffi.ppst_sync(ctx)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / (2 * reps)           # per 25-limb forward NTT
    butterflies = limbs * (N // 2) * info.logN               # N/2 log2 N per limb
    alg_bytes = 2 * limbs * N * 8                            # read + write each limb once
    g_bfly = butterflies / sec / 1e9
    alu_floor = butterflies / (BFLY_PEAK_G * 1e9)
    hbm_floor = alg_bytes / (HBM_PEAK_GBS * 1e9)
    stale = NTT_TRAFFIC["source_sha256"] != _ntt_source_sha()
    log("forward NTT (25 limbs, 2 passes): %.2f us, %.1f G butterflies/s (%.3f of %.0f), "
        "%.0f GB/s of algorithmic bytes (%.3f of HBM)" % (
            sec * 1e6, g_bfly, g_bfly / BFLY_PEAK_G, BFLY_PEAK_G, alg_bytes / sec / 1e9,
            alg_bytes / sec / 1e9 / HBM_PEAK_GBS))
    alu = alu_floor >= hbm_floor
    gbs = alg_bytes / sec / 1e9
    return {
        "kernel": "forward NTT of 25 limbs at N=2^16 (column pass + row pass; %s)" % plan.strip(),
        "bound": "alu" if alu else "hbm",
        "achieved": round(g_bfly, 1) if alu else round(gbs, 1),
        "peak": round(BFLY_PEAK_G, 1) if alu else HBM_PEAK_GBS,
        "unit": "G butterflies/s" if alu else "GB/s",
        "frac": round(g_bfly / BFLY_PEAK_G, 4) if alu else round(gbs / HBM_PEAK_GBS, 4),
        "alu_frac": round(g_bfly / BFLY_PEAK_G, 4),
        "traffic": None if stale else NTT_TRAFFIC["bytes"],
        "us_per_launch_pair": round(sec * 1e6, 3),
        "butterflies_per_launch_pair": butterflies,
        "alg_bytes_per_launch_pair": alg_bytes,
        "alu_floor_us": round(alu_floor * 1e6, 3),
        "hbm_floor_us": round(hbm_floor * 1e6, 3),
        "hbm_algorithmic_GBs": round(alg_bytes / sec / 1e9, 1),
        "hbm_frac": round(alg_bytes / sec / 1e9 / HBM_PEAK_GBS, 4),
    }


def profiled_kernels():
    """Roofline entries of the plain product's other large kernels, from the
    committed rocprofv3 counter summary (profiles/hmult_c2_plain_valu_traffic.md):
    average duration, VALU busy fraction and counted HBM bytes per launch,
    against the algorithmic bytes above (8 TB/s)."""
    path = os.path.join(ROOT, "profiles", "hmult_c2_plain_valu_traffic.md")
    out = []
    try:
        rows = [l for l in open(path).read().splitlines() if l.startswith("| `")]
    except OSError:
        return out
    for l in rows:
        cells = [c.strip() for c in l.strip("|").split("|")]
        name = cells[0].strip("`")
        if name not in KS_KERNELS:
            continue
        bound, alg = KS_KERNELS[name]
        us = float(cells[3])
        fetch, write = (float(v) for v in cells[9].split("+"))
        out.append({"kernel": name, "bound": bound, "us": us, "alg_bytes": alg,
                    "achieved_GBs": round(alg / (us * 1e-6) / 1e9, 1),
                    "hbm_frac": round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                    "valu_busy": float(cells[8]), "traffic": int((fetch + write) * 1e6),
                    "source": "profiles/hmult_c2_plain_valu_traffic.md"})
    return out


def measure_peaks(stream):
    """Measured ceilings beside the published ones (libppstat_probe.so):
    a 1 GiB device copy, and eight independent chains per work-item of FP64
    fused multiply-adds and of v_mad_u64_u32, over 2^19 work-items (eight
    waves per SIMD).  HIP events on `stream`."""
    import torch

    from paper_2508_12093_amd import ffi

    pl = ffi.probe_lib()
    sp = ctypes.c_void_p(stream.cuda_stream)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    threads, iters = 1 << 19, 2048
    outd = torch.empty(threads, dtype=torch.float64, device="cuda")
    outi = torch.empty(threads, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    def timed(launch, reps):
        launch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            launch()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    def chk(rc):
        if rc != 0:
            raise RuntimeError("probe launch failed (%d)" % rc)

    t_copy = timed(lambda: chk(pl.ppst_probe_copy(ctypes.c_void_p(src.data_ptr()),
                                                  ctypes.c_void_p(dst.data_ptr()), nbytes, sp)), 10)
    t_fma = timed(lambda: chk(pl.ppst_probe_fma_f64(ctypes.c_void_p(outd.data_ptr()), threads,
                                                    iters, sp)), 5)
    t_mad = timed(lambda: chk(pl.ppst_probe_mad_u64_u32(ctypes.c_void_p(outi.data_ptr()), threads,
                                                        iters, sp)), 5)
    ops = 8 * threads * iters
    out = {"copy_GBs": round(2 * nbytes / t_copy / 1e9, 1),
           "fp64_fma_T_per_s": round(ops / t_fma / 1e12, 3),
           "mad_u64_u32_T_per_s": round(ops / t_mad / 1e12, 3),
           "valu_peak_T_per_s": round(VALU_PEAK / 1e12, 3),
           "hbm_peak_GBs": HBM_PEAK_GBS}
    log("peaks: copy %.0f GB/s, FP64 FMA %.2f T/s, v_mad_u64_u32 %.2f T/s (VALU slots %.2f T/s)" % (
        out["copy_GBs"], out["fp64_fma_T_per_s"], out["mad_u64_u32_T_per_s"], VALU_PEAK / 1e12))
    del src, dst, outd, outi
    return out


def kernels_only(args):
    """Only the roofline kernel and a plain copy of known size (for
    rocprofv3 kernel statistics and FETCH_SIZE / WRITE_SIZE counters)."""
    import torch

    from paper_2508_12093_amd import ffi

    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    os.environ["PPST_NTT_AUTOTUNE"] = "0"      # the profile holds only the timed launches
    ctx = ffi.ppst_context_create("c2", stream=ctypes.c_void_p(stream.cuda_stream))
    variants = tuple(int(v) for v in args.ntt_variants.split(",")) if args.ntt_variants else None
    rf = measure_ntt(ctx, stream, reps=20, variants=variants)
    n = 64 << 20                                             # 64 Mi int64 = 512 MiB
    a = torch.ones(n, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"roofline": rf, "copy_bytes_each_way": n * 8}), flush=True)


def _cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, ValueError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(runs: int, pearson: bool = False):
    """The CPU reference (the plain C oracle, built on this host at -O2
    -march=native) timed on the host at N = 2^16, level 24: medians of `runs`
    repetitions of a 25-limb NTT, an HMult+relin+rescale and a rotation, at
    one OpenMP thread and at every core of the process's CPU share, each in a
    child process (oracle/timing.py).  With `pearson`, also one encrypted
    Pearson on the config-2 columns at every core, beside FP64 NumPy."""
    import subprocess
    import tempfile

    from oracle import ref

    tmp = tempfile.mkdtemp(prefix="ppst_oracle_")
    so = ref.build_native(os.path.join(tmp, "libckks_ref_native.so"))
    share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = int(os.environ.get("OMP_NUM_THREADS", share))
    legs = {}
    for threads in sorted({1, cores}):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads), PPST_ORACLE_SO=so)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "oracle", "timing.py"), "--runs", str(runs)],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode != 0:
            raise RuntimeError("oracle timing failed:\n" + r.stderr[-2000:])
        legs[threads] = json.loads(r.stdout.strip().splitlines()[-1])
        log("oracle at %d thread(s): NTT(25 limbs) %.1f ms, HMult %.0f ms, rotation %.0f ms" % (
            threads, legs[threads]["ntt25_ms"], legs[threads]["hmult_ms"], legs[threads]["rotation_ms"]))
    top, one = legs[cores], legs[1]
    extra = {}
    if pearson:
        import numpy as np

        from paper_2508_12093_amd import synth
        cols = os.path.join(tmp, "c2_columns.npy")
        np.save(cols, np.stack(synth.binary_cost_pair(0)))
        env = dict(os.environ, OMP_NUM_THREADS=str(cores), PPST_ORACLE_SO=so)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "oracle", "timing.py"), "--pearson", cols],
                           env=env, capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            raise RuntimeError("oracle Pearson timing failed:\n" + r.stderr[-2000:])
        extra["pearson"] = json.loads(r.stdout.strip().splitlines()[-1])
        log("oracle Pearson at %d threads: %.1f s (FP64 NumPy %.0f us)" % (
            cores, extra["pearson"]["pearson_s"], extra["pearson"]["fp64_numpy_pearson_us"]))
    return {"value": top["hmult_per_s"], "unit": "HMult+relin/s", "cores": cores, "kind": "oracle",
            "sample": "median of %d runs each of a 25-limb NTT, an HMult+relin+rescale and a rotation "
                      "at N=2^16, level 24 (%.1f s timed at %d threads, %.1f s at 1)" % (
                          runs, top["timed_s"], cores, one["timed_s"]),
            "cpu_model": _cpu_model(), "build": "gcc -O2 -march=native -fopenmp",
            "per_op_ms": {"ntt25": top["ntt25_ms"], "hmult": top["hmult_ms"], "rotation": top["rotation_ms"]},
            "rotations_per_s": top["rotations_per_s"],
            "single_thread": {"hmult_per_s": one["hmult_per_s"], "rotations_per_s": one["rotations_per_s"],
                              "per_op_ms": {"ntt25": one["ntt25_ms"], "hmult": one["hmult_ms"],
                                            "rotation": one["rotation_ms"]}}, **extra}


if __name__ == "__main__":
    main()
