"""CPU oracle for textbook RNS-CKKS: Python front end of ``ckks_ref.c``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library (``paper_2508_12093_amd``) and never imports it.

The paper (PP-STAT, Sec. 3.1) treats CKKS as a black box with Add(C), Add(P),
Mul(C), Mul(P) and Rot; it names the level, the depth and the scale Delta but
no arithmetic below that.  What follows is textbook RNS-CKKS with hybrid key
switching, in the plainest form:

* ``Oracle.add/sub``           Add(C)/Sub(C)                (Sec. 3.1)
* ``Oracle.add_const``         Add(P) with a constant      (Sec. 3.1)
* ``Oracle.mul_const/mul_plain`` Mul(P), then rescale       (Sec. 3.1)
* ``Oracle.mul``               Mul(C) = tensor + relinearise + rescale (Sec. 3.1)
* ``Oracle.rotate``            Rot, cyclic slot rotation   (Sec. 3.1)
* ``Oracle.rotsum``            the slot sums inside Mean/Variance (Eq. 2, Sec. 5.1):
                               log2(N/2) serial steps ct <- ct + Rot(ct, 2^k)
* ``Oracle.rotsum_hoisted8``   the same sum in hoisted radix-8 steps (the
                               form the statistics circuits use)
* ``Oracle.level_align``       bringing two operands to a common level

Every ciphertext at level l carries the canonical scale Delta_l, with
Delta_L = Delta and Delta_{l-1} = Delta_l^2 / q_l (FP64, that order).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_ref.c")
_SRCS = [_SRC, os.path.join(_HERE, "boot_ref.c")]
_HDR = os.path.join(_HERE, "ckks_ref.h")
_SO = os.path.join(_HERE, "libckks_ref.so")

MAXP = 64

# stream purposes (shared by nothing: the library defines its own copy of the
# sampling specification)
PUR_SK, PUR_PK_A, PUR_PK_E, PUR_KSK_A, PUR_KSK_E = 1, 2, 3, 4, 5
PUR_ENC_V, PUR_ENC_E0, PUR_ENC_E1, PUR_SKE_A, PUR_SKE_E = 6, 7, 8, 9, 10


def build(force: bool = False) -> str:
    """Compile ckks_ref.c and boot_ref.c with gcc into oracle/libckks_ref.so
    (portable flags: the file travels to other hosts)."""
    newest = max(os.path.getmtime(f) for f in _SRCS + [_HDR])
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-I" + _HERE,
               "-o", tmp] + _SRCS + ["-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def build_sanitized(out: str) -> str:
    """The same sources with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc; UB aborts).  Load it by starting a process with PPST_ORACLE_SO set
    to `out` and gcc's libasan preloaded (``gcc -print-file-name=libasan.so``)."""
    cmd = ["gcc", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I" + _HERE, "-o", out] + _SRCS + ["-lquadmath", "-lm"]
    subprocess.check_call(cmd)
    return out


def build_native(out: str) -> str:
    """The same source for the host that builds it (never shipped
    elsewhere): -O2 -march=native, the fastest of -O2 / -O3 with and without
    -march=native on this code (-O3 runs the 128-bit remainder loops about
    1.5x slower).  Load it by starting a process with PPST_ORACLE_SO set to
    `out`."""
    cmd = ["gcc", "-O2", "-march=native", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-I" + _HERE, "-o", out] + _SRCS + ["-lquadmath", "-lm"]
    subprocess.check_call(cmd)
    return out


class OrcParams(ctypes.Structure):
    _fields_ = [("logN", ctypes.c_int32), ("N", ctypes.c_int32), ("L", ctypes.c_int32),
                ("K", ctypes.c_int32), ("dnum", ctypes.c_int32), ("alpha", ctypes.c_int32),
                ("q", ctypes.c_uint64 * MAXP), ("psi", ctypes.c_uint64 * MAXP),
                ("scale", ctypes.c_double * MAXP)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        override = os.environ.get("PPST_ORACLE_SO")
        if not override:
            build()
        L = ctypes.CDLL(override or _SO)
        u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        vp = ctypes.c_void_p
        PP = ctypes.POINTER(OrcParams)
        sig = {
            "orc_is_prime": (ctypes.c_int, [u64]),
            "orc_mulmod": (u64, [u64, u64, u64]),
            "orc_powmod": (u64, [u64, u64, u64]),
            "orc_params_make": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, dbl, ctypes.c_int, PP]),
            "orc_ntt_limb": (None, [PP, ctypes.c_int, vp]),
            "orc_intt_limb": (None, [PP, ctypes.c_int, vp]),
            "orc_ntt": (None, [PP, vp, ctypes.c_int, vp]),
            "orc_intt": (None, [PP, vp, ctypes.c_int, vp]),
            "orc_negacyclic_mul": (None, [vp, vp, vp, ctypes.c_int, u64]),
            "orc_stream_word": (u64, [u64, u64, u64, u64]),
            "orc_sample_ternary": (None, [u64, u64, ctypes.c_int, vp]),
            "orc_sample_uniform": (None, [u64, u64, u64, u64, ctypes.c_int, vp]),
            "orc_dg_table": (None, [vp]),
            "orc_sample_dg": (None, [u64, u64, ctypes.c_int, vp]),
            "orc_encode_coeffs": (ctypes.c_int, [PP, vp, ctypes.c_int, dbl, vp]),
            "orc_decode_coeffs": (ctypes.c_int, [PP, vp, dbl, vp]),
            "orc_encode_coeffs_complex": (ctypes.c_int, [PP, vp, vp, ctypes.c_int, dbl, vp]),
            "orc_decode_coeffs_complex": (ctypes.c_int, [PP, vp, dbl, vp, vp]),
            "orc_from_signed": (None, [PP, vp, ctypes.c_int, vp, vp]),
            "orc_keygen_secret": (None, [PP, u64, vp, vp]),
            "orc_keygen_public": (None, [PP, u64, vp, vp]),
            "orc_keygen_ksk": (None, [PP, u64, u64, vp, vp, vp]),
            "orc_automorph_coeff": (None, [vp, vp, ctypes.c_int, u64, u64]),
            "orc_automorph_ntt": (None, [PP, vp, vp, ctypes.c_int, vp, u64]),
            "orc_galois_secret": (None, [PP, vp, u64, vp]),
            "orc_encrypt_pk": (None, [PP, u64, vp, vp, ctypes.c_int, vp]),
            "orc_encrypt_sk": (None, [PP, u64, vp, vp, ctypes.c_int, vp]),
            "orc_decrypt": (None, [PP, vp, vp, ctypes.c_int, vp]),
            "orc_keyswitch": (None, [PP, ctypes.c_int, vp, vp, vp, vp]),
            "orc_add": (None, [PP, vp, vp, ctypes.c_int, ctypes.c_int, vp]),
            "orc_sub": (None, [PP, vp, vp, ctypes.c_int, ctypes.c_int, vp]),
            "orc_mul_int": (None, [PP, vp, i64, ctypes.c_int, ctypes.c_int, vp]),
            "orc_add_int": (None, [PP, vp, i64, ctypes.c_int, vp]),
            "orc_mul_poly": (None, [PP, vp, vp, ctypes.c_int, ctypes.c_int, vp]),
            "orc_tensor": (None, [PP, vp, vp, ctypes.c_int, vp]),
            "orc_rescale": (None, [PP, vp, ctypes.c_int, ctypes.c_int, vp]),
            "orc_rotate_hoisted": (None, [PP, ctypes.c_int, vp, vp, u64, vp]),
            "orc_rotsum_step": (None, [PP, ctypes.c_int, vp, vp, vp, ctypes.c_int, vp]),
            "orc_round_half_away": (i64, [dbl]),
            "orc_mulmod_vec": (None, [vp, vp, vp, ctypes.c_int, u64]),
            "orc_splitmix64_next": (u64, [u64]),
            "orc_params_make_boot": (ctypes.c_int, [ctypes.c_int] * 8 + [dbl, dbl, ctypes.c_int, PP]),
            "orc_keygen_secret_sparse": (ctypes.c_int, [PP, u64, ctypes.c_int, vp, vp]),
            "orc_boot_group_diags": (ctypes.c_int, [ctypes.c_int] * 5 + [vp, vp, vp]),
            "orc_boot_group_factor": (dbl, [PP] + [ctypes.c_int] * 4),
            "orc_boot_grid": (ctypes.c_int, [PP] + [ctypes.c_int] * 11 + [vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# parameter presets (the paper fixes N = 2^16, Delta = 2^40, log2 PQ = 1443 and
# 32768 slots, Sec. 6.1; the prime chain, dnum and the special primes are the
# documented reading: q_0 near 2^60, q_1..q_24 near 2^40, 7 special primes)
# ----------------------------------------------------------------------------
PRESETS = {
    # N=2^12, q0 40-bit, two 30-bit primes, Delta=2^30, one 60-bit special prime
    "c1": dict(logN=12, L=2, K=1, dnum=3, q0_bits=40, delta=2.0 ** 30, p_bits=60),
    # N=2^16, q0 60-bit, 24 primes near 2^40, 7 special 60-bit primes, dnum=3
    "c2": dict(logN=16, L=24, K=7, dnum=3, q0_bits=60, delta=2.0 ** 40, p_bits=60),
    # small test preset with the c2 prime shapes: multi-limb digits, ragged last digit
    "t1": dict(logN=12, L=6, K=3, dnum=3, q0_bits=60, delta=2.0 ** 40, p_bits=60),
    # the c2 prime chain (L=24, dnum=3, 7 special primes) at N=2^12, for circuits
    "t2": dict(logN=12, L=24, K=7, dnum=3, q0_bits=60, delta=2.0 ** 40, p_bits=60),
    # bootstrappable chain (orc_params_make_boot): 11 computation levels at
    # Delta = 2^40 under 3 SlotToCoeff, 10 EvalMod (Delta_b = 2^58) and 3
    # CoeffToSlot levels (L = 27), sparse secret of weight 64, dnum = 4; q_0
    # of 55 bits, so that q_0 / Delta_0 = 2^15 (a refreshed message carries
    # EvalMod's error times q_0 / Delta_0; the sine's cubic term grows as
    # that ratio falls)
    "b2": dict(logN=16, Lc=11, boot=(3, 10, 3), K=8, dnum=4, q0_bits=55, delta=2.0 ** 40,
               delta_b=2.0 ** 58, p_bits=60, h=64),
    # the b2 chain at N=2^12
    "b1": dict(logN=12, Lc=11, boot=(3, 10, 3), K=8, dnum=4, q0_bits=55, delta=2.0 ** 40,
               delta_b=2.0 ** 58, p_bits=60, h=64),
}


class Params:
    def __init__(self, logN, L=None, K=1, dnum=1, q0_bits=60, delta=2.0 ** 40, p_bits=60,
                 Lc=None, boot=None, delta_b=None, h=0):
        self.c = OrcParams()
        if boot is None:
            rc = lib().orc_params_make(logN, L, K, dnum, q0_bits, float(delta), p_bits, ctypes.byref(self.c))
        else:
            C, E, S = boot
            L = Lc + C + E + S
            rc = lib().orc_params_make_boot(logN, Lc, C, E, S, K, dnum, q0_bits, float(delta),
                                            float(delta_b), p_bits, ctypes.byref(self.c))
        if rc != 0:
            raise ValueError("parameter derivation failed: %d" % rc)
        self.logN, self.N, self.L, self.K = logN, 1 << logN, L, K
        self.dnum, self.alpha = dnum, self.c.alpha
        self.nprimes = L + 1 + K
        self.q = [int(self.c.q[i]) for i in range(self.nprimes)]
        self.psi = [int(self.c.psi[i]) for i in range(self.nprimes)]
        self.scale = [float(self.c.scale[i]) for i in range(L + 1)]
        self.slots = self.N // 2
        self.h = h                      # secret weight; 0: uniform ternary
        self.boot = boot                # (CoeffToSlot, EvalMod, SlotToCoeff) levels
        self.Lc = Lc if boot is not None else L

    @classmethod
    def preset(cls, name):
        return cls(**PRESETS[name])

    @property
    def ref(self):
        return ctypes.byref(self.c)


@dataclass
class Plaintext:
    coeffs: np.ndarray      # int64 [N], the integer polynomial
    ntt: np.ndarray         # uint64 [l+1][N], NTT form
    level: int
    scale: float


@dataclass
class Ciphertext:
    data: np.ndarray        # uint64 [2][l+1][N], NTT form
    level: int
    scale: float

    def copy(self):
        return Ciphertext(self.data.copy(), self.level, self.scale)


@dataclass
class SecretKey:
    s_coef: np.ndarray      # int8 [N]
    s_ntt: np.ndarray       # uint64 [L+1+K][N]


class LevelError(ValueError):
    pass


def galois_element(r: int, N: int) -> int:
    """g = 5^(r mod N/2) mod 2N: the automorphism X -> X^g rotates slots by r."""
    n = N // 2
    return pow(5, r % n, 2 * N)


class Oracle:
    """Evaluator over the C oracle.  Keys are generated from explicit seeds."""

    def __init__(self, params: Params):
        self.P = params
        self.L = lib()

    # ------------------------------------------------------------------ NTT
    def ntt(self, a: np.ndarray, pidx) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64).copy()
        idx = np.ascontiguousarray(pidx, dtype=np.int32)
        self.L.orc_ntt(self.P.ref, _p(a), len(idx), _p(idx))
        return a

    def intt(self, a: np.ndarray, pidx) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64).copy()
        idx = np.ascontiguousarray(pidx, dtype=np.int32)
        self.L.orc_intt(self.P.ref, _p(a), len(idx), _p(idx))
        return a

    # ---------------------------------------------------------------- keys
    def keygen(self, seed: int):
        P = self.P
        s_coef = np.zeros(P.N, dtype=np.int8)
        s_ntt = np.zeros((P.nprimes, P.N), dtype=np.uint64)
        if P.h:
            if self.L.orc_keygen_secret_sparse(P.ref, seed, P.h, _p(s_coef), _p(s_ntt)) != 0:
                raise ValueError("bad secret weight")
        else:
            self.L.orc_keygen_secret(P.ref, seed, _p(s_coef), _p(s_ntt))
        pk = np.zeros((2, P.L + 1, P.N), dtype=np.uint64)
        self.L.orc_keygen_public(P.ref, seed, _p(s_ntt), _p(pk))
        return SecretKey(s_coef, s_ntt), pk

    def _ksk(self, sk: SecretKey, seed: int, keyid: int, sp_ntt: np.ndarray):
        P = self.P
        key = np.zeros((P.dnum, 2, P.nprimes, P.N), dtype=np.uint64)
        self.L.orc_keygen_ksk(P.ref, seed, keyid, _p(sk.s_ntt), _p(sp_ntt), _p(key))
        return key

    def relin_key(self, sk: SecretKey, seed: int):
        """KS key from s^2 to s (key id 0)."""
        P = self.P
        s2 = np.zeros_like(sk.s_ntt)
        for t in range(P.nprimes):
            s2[t] = _mulmod_vec(sk.s_ntt[t], sk.s_ntt[t], P.q[t])
        return self._ksk(sk, seed, 0, s2)

    def galois_key(self, sk: SecretKey, seed: int, g: int):
        """KS key from s(X^g) to s (key id g)."""
        sp = np.zeros_like(sk.s_ntt)
        self.L.orc_galois_secret(self.P.ref, _p(sk.s_coef), g, _p(sp))
        return self._ksk(sk, seed, g, sp)

    def rotation_keys(self, sk: SecretKey, seed: int, steps):
        return {galois_element(r, self.P.N): self.galois_key(sk, seed, galois_element(r, self.P.N))
                for r in steps}

    def rotsum_hoisted8_plan(self):
        """Steps (s, radix) of the hoisted radix-8 rotate-and-sum over the N/2
        slots: radix 8 while three or more bits of the slot index remain,
        then one step of radix 4 or 2 for the bits left."""
        bits = self.P.slots.bit_length() - 1
        plan, b = [], 0
        while b < bits:
            take = min(3, bits - b)
            plan.append((1 << b, 1 << take))
            b += take
        return plan

    def rotsum_hoisted8_steps(self):
        """Rotation steps whose Galois keys the hoisted radix-8 rotate-and-sum
        needs: k s, 0 < k < radix.  They include every power of two below
        N/2, so the same keys serve the plain ``rotsum``."""
        return [k * s for s, rad in self.rotsum_hoisted8_plan() for k in range(1, rad)]

    def rotsum_serial_steps(self):
        """Rotation steps of the plain ``rotsum``: 2^k for 2^k < N/2."""
        return [1 << k for k in range(self.P.slots.bit_length() - 1)]

    # ------------------------------------------------------------- encoding
    def encode_coeffs(self, m, scale: float) -> np.ndarray:
        m = np.ascontiguousarray(m, dtype=np.float64)
        out = np.zeros(self.P.N, dtype=np.int64)
        rc = self.L.orc_encode_coeffs(self.P.ref, _p(m), len(m), float(scale), _p(out))
        if rc != 0:
            raise ValueError("too many slots")
        return out

    def plaintext_from_coeffs(self, coeffs: np.ndarray, level: int, scale: float) -> Plaintext:
        P = self.P
        coeffs = np.ascontiguousarray(coeffs, dtype=np.int64)
        idx = np.arange(level + 1, dtype=np.int32)
        res = np.zeros((level + 1, P.N), dtype=np.uint64)
        self.L.orc_from_signed(P.ref, _p(coeffs), level + 1, _p(idx), _p(res))
        self.L.orc_ntt(P.ref, _p(res), level + 1, _p(idx))
        return Plaintext(coeffs, res, level, scale)

    def encode(self, m, level: int | None = None) -> Plaintext:
        level = self.P.L if level is None else level
        scale = self.P.scale[level]
        return self.plaintext_from_coeffs(self.encode_coeffs(m, scale), level, scale)

    def decode_coeffs(self, coeffs: np.ndarray, scale: float) -> np.ndarray:
        coeffs = np.ascontiguousarray(coeffs, dtype=np.int64)
        out = np.zeros(self.P.slots, dtype=np.float64)
        self.L.orc_decode_coeffs(self.P.ref, _p(coeffs), float(scale), _p(out))
        return out

    # ------------------------------------------------------ encrypt/decrypt
    def encrypt(self, pt: Plaintext, pk: np.ndarray, seed: int) -> Ciphertext:
        P = self.P
        ct = np.zeros((2, pt.level + 1, P.N), dtype=np.uint64)
        self.L.orc_encrypt_pk(P.ref, seed, _p(np.ascontiguousarray(pk)), _p(pt.ntt), pt.level, _p(ct))
        return Ciphertext(ct, pt.level, pt.scale)

    def encrypt_sk(self, pt: Plaintext, sk: SecretKey, seed: int) -> Ciphertext:
        P = self.P
        ct = np.zeros((2, pt.level + 1, P.N), dtype=np.uint64)
        self.L.orc_encrypt_sk(P.ref, seed, _p(sk.s_ntt), _p(pt.ntt), pt.level, _p(ct))
        return Ciphertext(ct, pt.level, pt.scale)

    def decrypt_ntt(self, ct: Ciphertext, sk: SecretKey) -> np.ndarray:
        P = self.P
        out = np.zeros((ct.level + 1, P.N), dtype=np.uint64)
        self.L.orc_decrypt(P.ref, _p(sk.s_ntt), _p(ct.data), ct.level, _p(out))
        return out

    def crt_centred(self, limbs: np.ndarray) -> np.ndarray:
        """Exact CRT of coefficient-form limbs over q_0..q_l, centred in
        (-Q/2, Q/2], as Python integers (object array)."""
        nl = limbs.shape[0]
        qs = self.P.q[:nl]
        Q = 1
        for q in qs:
            Q *= q
        X = np.zeros(limbs.shape[1], dtype=object)
        for i, q in enumerate(qs):
            Qi = Q // q
            inv = pow(Qi % q, -1, q)
            X = X + ((limbs[i].astype(object) * inv) % q) * Qi
        X = X % Q
        return np.where(X > Q // 2, X - Q, X)

    def decrypt_coeffs(self, ct: Ciphertext, sk: SecretKey) -> np.ndarray:
        """Centred integer coefficients of c0 + c1 s (exact CRT over all limbs)."""
        pt = self.decrypt_ntt(ct, sk)
        c = self.crt_centred(self.intt(pt, list(range(ct.level + 1))))
        if any(abs(int(v)) >= 2 ** 63 for v in (c.max(), c.min())):
            raise OverflowError("decrypted coefficient exceeds 63 bits")
        return c.astype(np.int64)

    def decrypt(self, ct: Ciphertext, sk: SecretKey) -> np.ndarray:
        return self.decode_coeffs(self.decrypt_coeffs(ct, sk), ct.scale)

    # ------------------------------------------------------------ linear ops
    def _check_same(self, a: Ciphertext, b: Ciphertext):
        if a.level != b.level:
            raise LevelError("level mismatch %d vs %d" % (a.level, b.level))
        if a.scale != b.scale:
            raise LevelError("scale mismatch")

    def add(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        self._check_same(a, b)
        out = np.zeros_like(a.data)
        self.L.orc_add(self.P.ref, _p(a.data), _p(b.data), a.level, 2, _p(out))
        return Ciphertext(out, a.level, a.scale)

    def sub(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        self._check_same(a, b)
        out = np.zeros_like(a.data)
        self.L.orc_sub(self.P.ref, _p(a.data), _p(b.data), a.level, 2, _p(out))
        return Ciphertext(out, a.level, a.scale)

    def const_int(self, c: float, level: int) -> int:
        """round_half_away(c * Delta_l): one FP64 product, then round."""
        return round_half_away(float(c) * self.P.scale[level])

    def add_const(self, a: Ciphertext, c: float) -> Ciphertext:
        k = self.const_int(c, a.level)
        out = a.data.copy()
        self.L.orc_add_int(self.P.ref, _p(a.data[0].copy()), k, a.level, _p(out[0]))
        return Ciphertext(np.ascontiguousarray(out), a.level, a.scale)

    def mul_int(self, a: Ciphertext, k: int) -> Ciphertext:
        out = np.zeros_like(a.data)
        self.L.orc_mul_int(self.P.ref, _p(a.data), int(k), a.level, 2, _p(out))
        return Ciphertext(out, a.level, a.scale)

    def rescale(self, a: Ciphertext) -> Ciphertext:
        if a.level < 1:
            raise LevelError("cannot rescale at level 0")
        P = self.P
        out = np.zeros((2, a.level, P.N), dtype=np.uint64)
        self.L.orc_rescale(P.ref, _p(a.data), a.level, 2, _p(out))
        return Ciphertext(out, a.level - 1, P.scale[a.level - 1])

    def mul_const(self, a: Ciphertext, c: float) -> Ciphertext:
        """Mul(P) by a constant: multiply by round(c Delta_l), then rescale."""
        if a.level < 1:
            raise LevelError("no level left")
        k = self.const_int(c, a.level)
        out = np.zeros_like(a.data)
        self.L.orc_mul_int(self.P.ref, _p(a.data), k, a.level, 2, _p(out))
        return self.rescale(Ciphertext(out, a.level, a.scale))

    def lincomb_int(self, a: Ciphertext, c: float, level: int) -> int:
        """The integer that carries c * a to scale Delta_{level+1}^2 at level
        level + 1: round_half_away(c Delta_{level+1} (Delta_{level+1} / Delta_l))."""
        D = self.P.scale
        return round_half_away(float(c) * D[level + 1] * (D[level + 1] / D[a.level]))

    def lincomb(self, cts, cs, level: int) -> Ciphertext:
        """sum_k c_k ct_k at `level` with one rescale: every ct_k (level >
        `level`) is cut to q_0..q_{level+1}, multiplied by the integer of
        ``lincomb_int``, the products added, and the sum rescaled by
        q_{level+1} (scale Delta_{level+1}^2 / q_{level+1} = Delta_level)."""
        if not cts or len(cts) != len(cs):
            raise ValueError("need matching ciphertexts and constants")
        lv1 = level + 1
        acc = None
        for a, c in zip(cts, cs):
            if a.level < lv1:
                raise LevelError("a term is below the combination's level + 1")
            cut = Ciphertext(np.ascontiguousarray(a.data[:, : lv1 + 1, :]), lv1, self.P.scale[lv1])
            t = self.mul_int(cut, self.lincomb_int(a, c, level))
            acc = t if acc is None else self.add(acc, t)
        return self.rescale(acc)

    def mul_plain(self, a: Ciphertext, pt: Plaintext) -> Ciphertext:
        """Mul(P) by a plaintext vector encoded at (l, Delta_l), then rescale."""
        if pt.level != a.level:
            raise LevelError("plaintext level mismatch")
        if a.level < 1:
            raise LevelError("no level left")
        out = np.zeros_like(a.data)
        self.L.orc_mul_poly(self.P.ref, _p(a.data), _p(pt.ntt), a.level, 2, _p(out))
        return self.rescale(Ciphertext(out, a.level, a.scale))

    def level_align(self, a: Ciphertext, level: int) -> Ciphertext:
        """Bring a to a lower level: keep q_0..q_{l'+1}, multiply by
        K = round(Delta_{l'} q_{l'+1} / Delta_l), rescale by q_{l'+1}."""
        if level == a.level:
            return a
        if level > a.level or level < 0:
            raise LevelError("cannot raise a level")
        P = self.P
        keep = np.ascontiguousarray(a.data[:, : level + 2, :])
        kint = round_half_away((P.scale[level] * float(P.q[level + 1])) / P.scale[a.level])
        out = np.zeros_like(keep)
        self.L.orc_mul_int(P.ref, _p(keep), kint, level + 1, 2, _p(out))
        r = self.rescale(Ciphertext(out, level + 1, P.scale[level + 1]))
        return Ciphertext(r.data, level, P.scale[level])

    # --------------------------------------------------------- key switching
    def keyswitch(self, d: np.ndarray, level: int, key: np.ndarray):
        P = self.P
        d = np.ascontiguousarray(d, dtype=np.uint64)
        u0 = np.zeros((level + 1, P.N), dtype=np.uint64)
        u1 = np.zeros((level + 1, P.N), dtype=np.uint64)
        self.L.orc_keyswitch(P.ref, level, _p(d), _p(np.ascontiguousarray(key)), _p(u0), _p(u1))
        return u0, u1

    def tensor(self, a: Ciphertext, b: Ciphertext) -> np.ndarray:
        self._check_same(a, b)
        d = np.zeros((3, a.level + 1, self.P.N), dtype=np.uint64)
        self.L.orc_tensor(self.P.ref, _p(a.data), _p(b.data), a.level, _p(d))
        return d

    def relin(self, d: np.ndarray, level: int, rlk: np.ndarray, scale: float) -> Ciphertext:
        u0, u1 = self.keyswitch(d[2], level, rlk)
        out = np.zeros((2, level + 1, self.P.N), dtype=np.uint64)
        sum_ = np.stack([d[0], d[1]])
        ks = np.stack([u0, u1])
        self.L.orc_add(self.P.ref, _p(np.ascontiguousarray(sum_)), _p(np.ascontiguousarray(ks)), level, 2, _p(out))
        return Ciphertext(out, level, scale)

    def mul_norelin(self, a: Ciphertext, b: Ciphertext) -> np.ndarray:
        return self.tensor(a, b)

    def mul(self, a: Ciphertext, b: Ciphertext, rlk: np.ndarray) -> Ciphertext:
        """Mul(C): tensor, relinearise, rescale (level l -> l-1)."""
        self._check_same(a, b)
        if a.level < 1:
            raise LevelError("no level left")
        d = self.tensor(a, b)
        c = self.relin(d, a.level, rlk, a.scale * b.scale)
        return self.rescale(c)

    def automorph(self, a: Ciphertext, g: int) -> Ciphertext:
        P = self.P
        nl = a.level + 1
        idx = np.arange(nl, dtype=np.int32)
        out = np.zeros_like(a.data)
        for c in range(2):
            src = np.ascontiguousarray(a.data[c])
            dst = np.zeros_like(src)
            self.L.orc_automorph_ntt(P.ref, _p(src), _p(dst), nl, _p(idx), g)
            out[c] = dst
        return Ciphertext(out, a.level, a.scale)

    def rotate(self, a: Ciphertext, r: int, gkeys: dict) -> Ciphertext:
        """Rot by r: phi_g then key switch of phi_g(c1) with the key for s(X^g)."""
        g = galois_element(r, self.P.N)
        if g == 1:
            return a.copy()
        if g not in gkeys:
            raise KeyError("no Galois key for step %d" % r)
        pa = self.automorph(a, g)
        u0, u1 = self.keyswitch(pa.data[1], a.level, gkeys[g])
        out = np.zeros_like(a.data)
        self.L.orc_add(self.P.ref, _p(np.ascontiguousarray(pa.data[0:1])), _p(np.ascontiguousarray(u0[None])),
                       a.level, 1, _p(out[0:1]))
        out[1] = u1
        return Ciphertext(out, a.level, a.scale)

    def rotate_hoisted(self, a: Ciphertext, rs, gkeys: dict):
        """Rotations sharing one ModUp of c1; the automorphism is applied to the
        extended digits after ModUp (a distinct, equally valid key switch)."""
        P = self.P
        outs = []
        for r in rs:
            g = galois_element(r, P.N)
            if g == 1:
                outs.append(a.copy())
                continue
            out = np.zeros_like(a.data)
            self.L.orc_rotate_hoisted(P.ref, a.level, _p(a.data), _p(np.ascontiguousarray(gkeys[g])), g, _p(out))
            outs.append(Ciphertext(out, a.level, a.scale))
        return outs

    def rotsum(self, a: Ciphertext, gkeys: dict) -> Ciphertext:
        """Rotate-and-sum by its definition: for k = 0 .. log2(N/2) - 1,
        ct <- ct + Rot(ct, 2^k), with Rot the plain rotation above.  After
        the k-th step slot j holds the sum of slots j .. j + 2^(k+1) - 1, so
        at the end every slot holds the sum of all N/2 slots (the slot sums
        of Mean and Variance, Eq. 2 and Sec. 5.1; Rot is Sec. 3.1's)."""
        ct = a
        for r in self.rotsum_serial_steps():
            ct = self.add(ct, self.rotate(ct, r, gkeys))
        return ct

    def rotsum_step(self, a: Ciphertext, s: int, radix: int, gkeys: dict) -> Ciphertext:
        """ct + sum_{0<k<radix} rot(ct, k s), the key switches hoisted: one
        ModUp of c1, the permuted inner products added in the extended basis,
        one ModDown (``orc_rotsum_step``).  It differs from the sum of plain
        rotations only in how the ModDown rounds (a distinct, equally valid
        key switch); the tests pin it to ``rotsum`` by decryption."""
        P = self.P
        gs = np.array([galois_element(k * s, P.N) for k in range(1, radix)], dtype=np.uint64)
        keys = [np.ascontiguousarray(gkeys[int(g)]) for g in gs]
        ptrs = (ctypes.c_void_p * len(keys))(*[k.ctypes.data for k in keys])
        out = np.zeros_like(a.data)
        self.L.orc_rotsum_step(P.ref, a.level, _p(np.ascontiguousarray(a.data)), ptrs, _p(gs),
                               len(keys), _p(out))
        return Ciphertext(out, a.level, a.scale)

    def rotsum_hoisted8(self, a: Ciphertext, gkeys: dict) -> Ciphertext:
        """Rotate-and-sum in the steps of ``rotsum_hoisted8_plan``:
        ct <- ct + sum_{0<k<radix} rot(ct, k s), each step hoisted
        (``rotsum_step``).  Five steps instead of fifteen at N = 2^16; the
        same sum as ``rotsum`` up to the key-switching noise."""
        ct = a
        for s, rad in self.rotsum_hoisted8_plan():
            ct = self.rotsum_step(ct, s, rad, gkeys)
        return ct


def round_half_away(v: float) -> int:
    """Round half away from zero (C llround) of an FP64 value."""
    return int(lib().orc_round_half_away(float(v)))


def _mulmod_vec(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.zeros_like(a)
    lib().orc_mulmod_vec(_p(a), _p(b), _p(out), len(a), q)
    return out
