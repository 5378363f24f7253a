"""Host timing of the oracle (the CPU baseline beside the GPU figures).

TEST INFRASTRUCTURE ONLY (see ``oracle/ref.py``): run as a child process by
the ``cpu_baseline`` leg of ``bench.py`` and by nothing else.

At N = 2^16, level 24 (the preset the GPU headline runs on) it times the
median of ``--runs`` repetitions of: one forward NTT of a 25-limb
polynomial, one HMult (tensor + relinearisation + rescale) and one rotation,
with the OpenMP thread count the process was started with, and prints one
JSON line.  Keys and ciphertexts are made before any timing.

With ``--pearson FILE`` it times instead one encrypted Pearson correlation
on the two columns stored in FILE (an .npy array of shape [2][n], written by
the caller: the config-2 columns, x ~ Bernoulli(0.2) against a lognormal
cost column), with Bx = 1, By = 20, a degree-7 Chebyshev start on [1e-3, 1]
and 3 Newton steps (the circuit of Sec. 5.5), and the FP64 NumPy Pearson of
the same columns.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=5)
    ap.add_argument("--preset", default="c2")
    ap.add_argument("--pearson", default=None, metavar="FILE")
    args = ap.parse_args()
    if args.pearson:
        pearson(args.preset, args.pearson)
        return

    import numpy as np

    from oracle import ref

    P = ref.Params.preset(args.preset)
    O = ref.Oracle(P)
    sk, pk = O.keygen(1)
    rlk = O.relin_key(sk, 2)
    gk = O.rotation_keys(sk, 3, [1])
    rng = np.random.default_rng(1)              # slot values U[-1, 1): timing only
    a = O.encrypt(O.encode(rng.uniform(-1.0, 1.0, P.slots)), pk, 3)
    b = O.encrypt(O.encode(rng.uniform(-1.0, 1.0, P.slots)), pk, 4)
    poly = np.ascontiguousarray(a.data[0])
    limbs = list(range(P.L + 1))

    def median(fn):
        ts = []
        for _ in range(args.runs):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), float(np.sum(ts))

    ntt_s, ntt_tot = median(lambda: O.ntt(poly, limbs))
    mul_s, mul_tot = median(lambda: O.mul(a, b, rlk))
    rot_s, rot_tot = median(lambda: O.rotate(a, 1, gk))
    print(json.dumps({
        "threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0),
        "runs": args.runs,
        "ntt25_ms": round(ntt_s * 1e3, 3),
        "hmult_ms": round(mul_s * 1e3, 2),
        "rotation_ms": round(rot_s * 1e3, 2),
        "hmult_per_s": round(1.0 / mul_s, 4),
        "rotations_per_s": round(1.0 / rot_s, 4),
        "timed_s": round(ntt_tot + mul_tot + rot_tot, 2),
        "library": os.path.basename(ref.lib()._name),
    }), flush=True)


def pearson(preset: str, path: str):
    import numpy as np

    from oracle import cheb, circuits as C, ref, stats64 as S

    P = ref.Params.preset(preset)
    O = ref.Oracle(P)
    sk, pk = O.keygen(11)
    rlk = O.relin_key(sk, 12)
    gk = O.rotation_keys(sk, 13, O.rotsum_hoisted8_steps())
    x, y = np.load(path)
    ox = O.encrypt(O.encode(x), pk, 91)
    oy = O.encrypt(O.encode(y), pk, 92)
    cfg = C.InvSqrtCfg(coeffs=cheb.invsqrt_coeffs(1e-3, 1.0, 7, 1.0))
    cc = C.Circuits(C.EncEval(O, rlk, gk))
    t = time.perf_counter()
    out = cc.pearson([ox], [oy], len(x), 1.0, 20.0, cfg)
    enc_s = time.perf_counter() - t
    ts = []
    for _ in range(20):
        t = time.perf_counter()
        want = S.pearson(x, y)
        ts.append(time.perf_counter() - t)
    got = float(O.decrypt(out, sk)[0])
    print(json.dumps({
        "threads": int(os.environ.get("OMP_NUM_THREADS", "0") or 0),
        "pearson_s": round(enc_s, 2),
        "pearson_rel_err": abs(got - want) / abs(want),
        "fp64_numpy_pearson_us": round(float(np.median(ts)) * 1e6, 1),
        "rows": len(x),
    }), flush=True)


if __name__ == "__main__":
    main()
