"""Writes c2_pearson.json: the oracle's encrypted Pearson correlation on the
config-2 columns at N = 2^16, L = 24 (Sec. 5.5 circuit, Eq. 2's pre-scaled
moments), as the SHA-256 of its residues plus level, scale and decrypted
value.  The oracle takes about a minute and a half for it on 8 host cores,
too long for a GPU test to run beside the library, so the GPU test compares
the library's ciphertext with this digest instead.

Calls only the oracle and the seeded input generators:
    python tests/golden/make_c2_pearson.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cheb, circuits as C, ref, stats64 as S  # noqa: E402
from paper_2508_12093_amd import synth  # noqa: E402

# the seeds and bounds the GPU test uses (its Pair defaults and encryption seeds)
SPEC = dict(preset="c2", key_seed=11, relin_seed=12, galois_seed=13, data_seed=0,
            enc_seed_x=91, enc_seed_y=92, Bx=1.0, By=20.0, a=1e-3, b=1.0, degree=7)


def digest(words: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


def main():
    s = SPEC
    P = ref.Params.preset(s["preset"])
    O = ref.Oracle(P)
    sk, pk = O.keygen(s["key_seed"])
    rlk = O.relin_key(sk, s["relin_seed"])
    gk = O.rotation_keys(sk, s["galois_seed"], O.rotsum_hoisted8_steps())
    x, y = synth.binary_cost_pair(s["data_seed"])
    ox = O.encrypt(O.encode(x), pk, s["enc_seed_x"])
    oy = O.encrypt(O.encode(y), pk, s["enc_seed_y"])
    base = cheb.invsqrt_coeffs(s["a"], s["b"], s["degree"], 1.0)
    cc = C.Circuits(C.EncEval(O, rlk, gk))
    out = cc.pearson([ox], [oy], len(x), s["Bx"], s["By"], C.InvSqrtCfg(coeffs=base))
    val = float(O.decrypt(out, sk)[0])
    rec = dict(spec=s, level=out.level, scale_hex=float(out.scale).hex(),
               shape=list(out.data.shape), sha256=digest(out.data), decrypted=val,
               fp64=float(S.pearson(x, y)))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_pearson.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
