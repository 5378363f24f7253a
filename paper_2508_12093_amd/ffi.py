"""ctypes binding of libppstat.so (include/ppstat.h).

Argument marshalling only: every function below forwards to the C entry point
of the same name; the arithmetic runs in the library's HIP kernels.  PyTorch,
when present, provides the stream the context runs on.  Loading fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PPST_LIBRARY: another build of the same library (the sanitizer builds of
# build.py); the in-tree one otherwise
LIB_PATH = os.environ.get("PPST_LIBRARY") or os.path.join(_HERE, "libppstat.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ppstat.h")

PPST_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ELEVEL", -3: "ESCALE", -4: "ENOKEY", -5: "ENOMEM",
          -6: "EDEVICE", -7: "EDOMAIN"}

Q_MEAN, Q_VARIANCE, Q_ZSCORE, Q_CV, Q_PEARSON, Q_SKEWNESS, Q_KURTOSIS = range(7)


class PpstError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code
        self.name = STATUS.get(code, "?")


class Params(ctypes.Structure):
    _fields_ = [("logN", ctypes.c_int32), ("L", ctypes.c_int32), ("K", ctypes.c_int32),
                ("dnum", ctypes.c_int32), ("q0_bits", ctypes.c_int32), ("p_bits", ctypes.c_int32),
                ("scale", ctypes.c_double), ("h", ctypes.c_int32), ("boot_cts", ctypes.c_int32),
                ("boot_evalmod", ctypes.c_int32), ("boot_stc", ctypes.c_int32),
                ("boot_scale", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("logN", "N", "L", "K", "dnum", "alpha", "nprimes", "slots")]


class InvSqrtCfg(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("degree", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("sign_k", ctypes.c_int32),
                ("coeffs", ctypes.POINTER(ctypes.c_double)), ("boot", ctypes.c_void_p)]


class Query(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("col_x", ctypes.c_uint64), ("col_y", ctypes.c_uint64),
                ("B", ctypes.c_double), ("B2", ctypes.c_double), ("cfg", InvSqrtCfg)]


class QueryStats(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("bytes_reserved", ctypes.c_uint64),
                ("bytes_peak", ctypes.c_uint64)]


HooksAlloc = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
HooksFree = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class DeviceHooks(ctypes.Structure):
    _fields_ = [("alloc", HooksAlloc), ("free", HooksFree), ("user", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_pp = ctypes.POINTER(ctypes.c_void_p)
_u64, _i32, _i64, _dbl, _sz = ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_cfgp = ctypes.POINTER(InvSqrtCfg)

_SIGS = {
    "ppst_last_error": (ctypes.c_char_p, []),
    "ppst_params_preset": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(Params)]),
    "ppst_params_derive": (ctypes.c_int, [ctypes.POINTER(Params), _vp, _vp, _vp, _sz]),
    "ppst_dg_thresholds": (ctypes.c_int, [_vp, _sz]),
    "ppst_rotsum_steps": (ctypes.c_int, [_vp, _vp, _sz, ctypes.POINTER(ctypes.c_size_t)]),
    "ppst_encode_coeffs": (ctypes.c_int, [ctypes.POINTER(Params), _vp, _sz, _i32, _vp, _sz]),
    "ppst_stream_key": (_u64, [_u64, _u64, _u64]),
    "ppst_chebyshev_invsqrt": (ctypes.c_int, [_dbl, _dbl, _i32, _dbl, _vp, _sz]),
    "ppst_context_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(DeviceHooks), _vp, _pp]),
    "ppst_context_fork": (ctypes.c_int, [_vp, _vp, _pp]),
    "ppst_context_destroy": (ctypes.c_int, [_vp]),
    "ppst_sync": (ctypes.c_int, [_vp]),
    "ppst_context_info": (ctypes.c_int, [_vp, ctypes.POINTER(Info)]),
    "ppst_context_primes": (ctypes.c_int, [_vp, _vp, _sz]),
    "ppst_context_scales": (ctypes.c_int, [_vp, _vp, _sz]),
    "ppst_context_dg_table": (ctypes.c_int, [_vp, _vp, _sz]),
    "ppst_context_stream": (ctypes.c_int, [_vp, _pp]),
    "ppst_keygen": (ctypes.c_int, [_vp, _u64, _pp, _pp]),
    "ppst_secret_key_destroy": (ctypes.c_int, [_vp]),
    "ppst_public_key_destroy": (ctypes.c_int, [_vp]),
    "ppst_evk_create": (ctypes.c_int, [_vp, _pp]),
    "ppst_evk_destroy": (ctypes.c_int, [_vp]),
    "ppst_evk_add_relin": (ctypes.c_int, [_vp, _vp, _u64, _vp]),
    "ppst_evk_add_galois": (ctypes.c_int, [_vp, _vp, _vp, _sz, _u64, _vp]),
    "ppst_evk_add_rotsum": (ctypes.c_int, [_vp, _vp, _u64, _vp]),
    "ppst_evk_export": (ctypes.c_int, [_vp, _vp, _u64, _vp, _sz]),
    "ppst_evk_import": (ctypes.c_int, [_vp, _vp, _u64, _vp, _sz]),
    "ppst_pk_export": (ctypes.c_int, [_vp, _vp, _vp, _sz]),
    "ppst_pk_import": (ctypes.c_int, [_vp, _vp, _sz, _pp]),
    "ppst_sk_export": (ctypes.c_int, [_vp, _vp, _vp, _sz]),
    "ppst_encode": (ctypes.c_int, [_vp, _vp, _sz, _i32, _pp]),
    "ppst_plaintext_from_coeffs": (ctypes.c_int, [_vp, _vp, _i32, _dbl, _pp]),
    "ppst_plaintext_coeffs": (ctypes.c_int, [_vp, _vp, _sz]),
    "ppst_plaintext_export": (ctypes.c_int, [_vp, _vp, _vp, _sz]),
    "ppst_plaintext_import": (ctypes.c_int, [_vp, _vp, _i32, _dbl, _pp]),
    "ppst_decode": (ctypes.c_int, [_vp, _vp, _vp, _sz]),
    "ppst_plaintext_destroy": (ctypes.c_int, [_vp]),
    "ppst_encrypt": (ctypes.c_int, [_vp, _vp, _vp, _u64, _pp]),
    "ppst_encrypt_sk": (ctypes.c_int, [_vp, _vp, _vp, _u64, _pp]),
    "ppst_decrypt": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_ciphertext_destroy": (ctypes.c_int, [_vp]),
    "ppst_ct_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_dbl), ctypes.POINTER(_i32)]),
    "ppst_ct_export": (ctypes.c_int, [_vp, _vp, _vp, _sz]),
    "ppst_ct_import": (ctypes.c_int, [_vp, _vp, _i32, _dbl, _i32, _pp]),
    "ppst_ct_device_ptr": (ctypes.c_int, [_vp, _pp]),
    "ppst_add": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_sub": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_add_const": (ctypes.c_int, [_vp, _vp, _dbl, _pp]),
    "ppst_mul_const": (ctypes.c_int, [_vp, _vp, _dbl, _pp]),
    "ppst_mul_int": (ctypes.c_int, [_vp, _vp, _i64, _pp]),
    "ppst_mul_plain": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_mul": (ctypes.c_int, [_vp, _vp, _vp, _vp, _pp]),
    "ppst_mul_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "ppst_tensor": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_relin": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_rescale": (ctypes.c_int, [_vp, _vp, _pp]),
    "ppst_rotate": (ctypes.c_int, [_vp, _vp, _vp, _i32, _pp]),
    "ppst_rotate_hoisted": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, _pp]),
    "ppst_rotsum": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_rotsum_serial": (ctypes.c_int, [_vp, _vp, _vp, _pp]),
    "ppst_level_align": (ctypes.c_int, [_vp, _vp, _i32, _pp]),
    "ppst_lincomb": (ctypes.c_int, [_vp, _pp, _vp, _sz, _i32, _pp]),
    "ppst_mul_batch": (ctypes.c_int, [_vp, _vp, _pp, _pp, _sz, _pp]),
    "ppst_mul_const_batch": (ctypes.c_int, [_vp, _pp, _sz, _dbl, _pp]),
    "ppst_rotsum_batch": (ctypes.c_int, [_vp, _vp, _pp, _sz, _pp]),
    "ppst_rotate_hoisted_batch": (ctypes.c_int, [_vp, _vp, _pp, _sz, _vp, _sz, _pp]),
    "ppst_boot_create": (ctypes.c_int, [_vp, _vp, _sz, _pp]),
    "ppst_boot_destroy": (ctypes.c_int, [_vp]),
    "ppst_evk_add_boot": (ctypes.c_int, [_vp, _vp, _u64, _vp]),
    "ppst_boot_count": (ctypes.c_int, [_vp, ctypes.POINTER(_u64)]),
    "ppst_boot_rotations": (ctypes.c_int, [_vp, _vp, _sz, ctypes.POINTER(ctypes.c_size_t)]),
    "ppst_boot_group_info": (ctypes.c_int, [_vp, _i32, _i32, _vp]),
    "ppst_boot_group_coeffs": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _sz]),
    "ppst_evalmod_coeffs": (ctypes.c_int, [_i32, _i32, _i32, _vp, _sz]),
    "ppst_bootstrap": (ctypes.c_int, [_vp, _vp, _vp, _vp, _pp]),
    "ppst_mod_raise": (ctypes.c_int, [_vp, _vp, _pp]),
    "ppst_apply_galois": (ctypes.c_int, [_vp, _vp, _vp, _u64, _pp]),
    "ppst_mul_monomial": (ctypes.c_int, [_vp, _vp, _i32, _i32, _pp]),
    "ppst_boot_coeff_to_slot": (ctypes.c_int, [_vp, _vp, _vp, _vp, _pp]),
    "ppst_boot_split": (ctypes.c_int, [_vp, _vp, _vp, _vp, _pp, _pp]),
    "ppst_boot_eval_mod": (ctypes.c_int, [_vp, _vp, _vp, _pp, _sz, _pp]),
    "ppst_boot_slot_to_coeff": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _pp]),
    "ppst_rotate_batch": (ctypes.c_int, [_vp, _vp, _pp, _sz, ctypes.c_int32, _pp]),
    "ppst_graph_begin": (ctypes.c_int, [_vp]),
    "ppst_graph_end": (ctypes.c_int, [_vp, _pp]),
    "ppst_graph_launch": (ctypes.c_int, [_vp]),
    "ppst_graph_destroy": (ctypes.c_int, [_vp]),
    "ppst_invsqrt_cfg_default": (ctypes.c_int, [_cfgp]),
    "ppst_stat_mean": (ctypes.c_int, [_vp, _vp, _pp, _sz, _sz, _dbl, _pp]),
    "ppst_stat_variance": (ctypes.c_int, [_vp, _vp, _pp, _sz, _sz, _dbl, _pp]),
    "ppst_stat_invsqrt": (ctypes.c_int, [_vp, _vp, _pp, _sz, _dbl, _cfgp, _pp]),
    "ppst_stat_zscore": (ctypes.c_int, [_vp, _vp, _pp, _sz, _sz, _dbl, _cfgp, _pp]),
    "ppst_stat_kurtosis": (ctypes.c_int, [_vp, _vp, _pp, _sz, _sz, _dbl, _cfgp, _i32, _pp]),
    "ppst_stat_skewness": (ctypes.c_int, [_vp, _vp, _pp, _sz, _sz, _dbl, _cfgp, _pp]),
    "ppst_stat_cv": (ctypes.c_int, [_vp, _vp, _pp, _sz, _sz, _dbl, _dbl, _cfgp, _pp]),
    "ppst_stat_pearson": (ctypes.c_int, [_vp, _vp, _pp, _pp, _sz, _sz, _dbl, _dbl, _cfgp, _pp]),
    "ppst_ntt_autotune": (ctypes.c_int, [_vp]),
    "ppst_ntt_plan": (ctypes.c_int, [_vp, ctypes.c_char_p, _sz]),
    "ppst_ntt_load_plan": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "ppst_ntt_set_plan": (ctypes.c_int, [_vp, _i32, _i32]),
    "ppst_ntt_forward": (ctypes.c_int, [_vp, _vp, _i32, _i32]),
    "ppst_ntt_inverse": (ctypes.c_int, [_vp, _vp, _i32, _i32]),
    "ppst_server_create": (ctypes.c_int, [_vp, _vp, _sz, _i32, ctypes.c_uint32, _pp]),
    "ppst_server_info": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "ppst_server_register_column": (ctypes.c_int, [_vp, _pp, _sz, _sz, ctypes.POINTER(_u64)]),
    "ppst_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(Query), ctypes.POINTER(_u64)]),
    "ppst_server_wait": (ctypes.c_int, [_vp, _u64, _pp, ctypes.POINTER(QueryStats)]),
    "ppst_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "ppst_server_output_count": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(ctypes.c_size_t)]),
    "ppst_server_wait_all": (ctypes.c_int, [_vp, _u64, _pp, _sz, ctypes.POINTER(ctypes.c_size_t),
                                            ctypes.POINTER(QueryStats)]),
    "ppst_server_destroy": (ctypes.c_int, [_vp]),
}

_lib = None


def _runtime_first():
    """Load torch (when installed) before the library: torch ships its own HIP
    runtime, and loading it first makes the process use that one runtime for
    both (the library's libamdhip64.so.7 dependency resolves to the copy
    already loaded); loaded the other way round, the library's device calls
    have failed to find the GPU."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """Load libppstat.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libppstat.so is not built (run __graft_entry__.build())")
        _runtime_first()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


PROBE_PATH = os.path.join(_HERE, "libppstat_probe.so")
PROBE_HEADER = os.path.join(os.path.dirname(_HERE), "include", "ppstat_probe.h")
_probe = None


def probe_lib():
    """Load libppstat_probe.so, the peak-rate microbenchmarks
    (include/ppstat_probe.h); raises if it has not been built."""
    global _probe
    if _probe is None:
        if not os.path.exists(PROBE_PATH):
            raise RuntimeError("libppstat_probe.so is not built (run __graft_entry__.build())")
        _runtime_first()
        L = ctypes.CDLL(PROBE_PATH)
        for name, args in {"ppst_probe_copy": [_vp, _vp, _sz, _vp],
                           "ppst_probe_fma_f64": [_vp, _sz, ctypes.c_int, _vp],
                           "ppst_probe_mad_u64_u32": [_vp, _sz, ctypes.c_int, _vp]}.items():
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = args
        _probe = L
    return _probe


def header_symbols(header: str = HEADER):
    """Names of the functions a header (by default include/ppstat.h) declares."""
    text = open(header).read()
    return sorted(set(re.findall(r"\b(ppst_[a-z0-9_]+)\s*\(", text)))


def _chk(rc):
    if rc != PPST_OK:
        msg = lib().ppst_last_error()
        raise PpstError(rc, msg.decode() if msg else "")


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _out():
    return ctypes.c_void_p()


# ---------------------------------------------------------------- handles
class _Handle:
    _destroy = None

    def __init__(self, ptr, owner=None):
        self.ptr = ptr
        self.owner = owner            # keeps the context alive

    def __del__(self):
        if getattr(self, "ptr", None) and self._destroy and _lib is not None:
            getattr(_lib, self._destroy)(self.ptr)
            self.ptr = None

    @property
    def _as_parameter_(self):
        return self.ptr


class Context(_Handle):
    _destroy = "ppst_context_destroy"

    @property
    def info(self):
        i = Info()
        _chk(lib().ppst_context_info(self, ctypes.byref(i)))
        return i

    @property
    def primes(self):
        i = self.info
        out = np.zeros(i.nprimes, dtype=np.uint64)
        _chk(lib().ppst_context_primes(self, _p(out), len(out)))
        return [int(v) for v in out]

    @property
    def scales(self):
        i = self.info
        out = np.zeros(i.L + 1, dtype=np.float64)
        _chk(lib().ppst_context_scales(self, _p(out), len(out)))
        return [float(v) for v in out]


class SecretKey(_Handle):
    _destroy = "ppst_secret_key_destroy"


class PublicKey(_Handle):
    _destroy = "ppst_public_key_destroy"


class EvalKeys(_Handle):
    _destroy = "ppst_evk_destroy"


class Plaintext(_Handle):
    _destroy = "ppst_plaintext_destroy"


class Ciphertext(_Handle):
    _destroy = "ppst_ciphertext_destroy"

    @property
    def level(self):
        l, s, n = _i32(), _dbl(), _i32()
        _chk(lib().ppst_ct_info(self, ctypes.byref(l), ctypes.byref(s), ctypes.byref(n)))
        return l.value

    @property
    def scale(self):
        l, s, n = _i32(), _dbl(), _i32()
        _chk(lib().ppst_ct_info(self, ctypes.byref(l), ctypes.byref(s), ctypes.byref(n)))
        return s.value

    @property
    def npoly(self):
        l, s, n = _i32(), _dbl(), _i32()
        _chk(lib().ppst_ct_info(self, ctypes.byref(l), ctypes.byref(s), ctypes.byref(n)))
        return n.value


class Server(_Handle):
    _destroy = "ppst_server_destroy"


# ------------------------------------------------------------- functions
def ppst_params_preset(name: str) -> Params:
    p = Params()
    _chk(lib().ppst_params_preset(name.encode(), ctypes.byref(p)))
    return p


def ppst_params_derive(params: Params):
    n = params.L + 1 + params.K
    primes = np.zeros(n, dtype=np.uint64)
    roots = np.zeros(n, dtype=np.uint64)
    scales = np.zeros(params.L + 1, dtype=np.float64)
    _chk(lib().ppst_params_derive(ctypes.byref(params), _p(primes), _p(roots), _p(scales), n))
    return [int(v) for v in primes], [int(v) for v in roots], [float(v) for v in scales]


def ppst_dg_thresholds():
    out = np.zeros(19, dtype=np.uint64)
    _chk(lib().ppst_dg_thresholds(_p(out), 19))
    return out


def ppst_rotsum_steps(params) -> list:
    """Rotation steps whose Galois keys ppst_rotsum needs (host only)."""
    n = ctypes.c_size_t()
    _chk(lib().ppst_rotsum_steps(ctypes.byref(params), None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), dtype=np.int32)
    _chk(lib().ppst_rotsum_steps(ctypes.byref(params), _p(out), n.value, ctypes.byref(n)))
    return [int(v) for v in out[:n.value]]


def ppst_encode_coeffs(params: Params, values, level: int):
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = np.zeros(1 << params.logN, dtype=np.int64)
    _chk(lib().ppst_encode_coeffs(ctypes.byref(params), _p(v), len(v), level, _p(out), len(out)))
    return out


def ppst_chebyshev_invsqrt(a: float, b: float, degree: int, Bp: float):
    out = np.zeros(degree + 1, dtype=np.float64)
    _chk(lib().ppst_chebyshev_invsqrt(a, b, degree, Bp, _p(out), out.size))
    return out


def ppst_stream_key(seed: int, purpose: int, limb: int) -> int:
    return int(lib().ppst_stream_key(seed, purpose, limb))


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


# ctypes callbacks handed to the library stay alive for the whole process:
# its pools may return memory through them until their last context is gone
_HOOK_REFS = []


def torch_device_hooks() -> DeviceHooks:
    """ppst_device_hooks backed by torch's caching allocator: every device
    block the library takes (ciphertexts, keys, tables, scratch) comes from
    torch.cuda.caching_allocator_alloc on the stream the library names, and
    goes back through caching_allocator_delete.  A failed allocation returns
    NULL, on which the library releases its own cached blocks and retries
    before reporting ENOMEM.  Contexts made with these hooks should be
    destroyed before the interpreter shuts down."""
    import torch
    dev = torch.cuda.current_device()

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=int(stream or 0))
        except Exception:
            return None

    def free(ptr, nbytes, stream, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    h = DeviceHooks(HooksAlloc(alloc), HooksFree(free), None)
    _HOOK_REFS.append(h)
    return h


def ppst_context_create(params, stream=None, use_torch_stream=True, alloc: str = "library") -> Context:
    """Create a context; by default it runs on torch's current stream.
    alloc="torch" takes every device block from torch's caching allocator
    (torch_device_hooks); "library" lets the library's own pool call
    hipMalloc."""
    if isinstance(params, str):
        params = ppst_params_preset(params)
    if stream is None and use_torch_stream:
        stream = _torch_stream()
    if alloc not in ("library", "torch"):
        raise ValueError("alloc must be 'library' or 'torch'")
    hooks = ctypes.byref(torch_device_hooks()) if alloc == "torch" else None
    out = _out()
    _chk(lib().ppst_context_create(ctypes.byref(params), hooks, stream, ctypes.byref(out)))
    return Context(out.value)


def ppst_context_fork(ctx: Context, stream=None) -> Context:
    out = _out()
    _chk(lib().ppst_context_fork(ctx, stream, ctypes.byref(out)))
    return Context(out.value)


def ppst_sync(ctx: Context):
    _chk(lib().ppst_sync(ctx))


def ppst_context_dg_table(ctx: Context):
    out = np.zeros(19, dtype=np.uint64)
    _chk(lib().ppst_context_dg_table(ctx, _p(out), 19))
    return out


def ppst_context_stream(ctx: Context) -> int:
    out = _out()
    _chk(lib().ppst_context_stream(ctx, ctypes.byref(out)))
    return out.value or 0


def ppst_keygen(ctx: Context, seed: int):
    sk, pk = _out(), _out()
    _chk(lib().ppst_keygen(ctx, seed, ctypes.byref(sk), ctypes.byref(pk)))
    return SecretKey(sk.value, ctx), PublicKey(pk.value, ctx)


def ppst_evk_create(ctx: Context) -> EvalKeys:
    out = _out()
    _chk(lib().ppst_evk_create(ctx, ctypes.byref(out)))
    return EvalKeys(out.value, ctx)


def ppst_evk_add_relin(ctx, sk, seed, evk):
    _chk(lib().ppst_evk_add_relin(ctx, sk, seed, evk))


def ppst_evk_add_galois(ctx, sk, steps, seed, evk):
    s = np.ascontiguousarray(steps, dtype=np.int32)
    _chk(lib().ppst_evk_add_galois(ctx, sk, _p(s), len(s), seed, evk))


def ppst_evk_add_rotsum(ctx, sk, seed, evk):
    _chk(lib().ppst_evk_add_rotsum(ctx, sk, seed, evk))


def ppst_evk_export(ctx: Context, evk: EvalKeys, galois: int):
    i = ctx.info
    out = np.zeros((i.dnum, 2, i.nprimes, i.N), dtype=np.uint64)
    _chk(lib().ppst_evk_export(ctx, evk, galois, _p(out), out.size))
    return out


def ppst_evk_import(ctx: Context, evk: EvalKeys, galois: int, words: np.ndarray):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    _chk(lib().ppst_evk_import(ctx, evk, galois, _p(w), w.size))


def ppst_pk_import(ctx: Context, words: np.ndarray) -> PublicKey:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    out = _out()
    _chk(lib().ppst_pk_import(ctx, _p(w), w.size, ctypes.byref(out)))
    return PublicKey(out.value, ctx)


def ppst_pk_export(ctx: Context, pk: PublicKey):
    i = ctx.info
    out = np.zeros((2, i.L + 1, i.N), dtype=np.uint64)
    _chk(lib().ppst_pk_export(ctx, pk, _p(out), out.size))
    return out


def ppst_sk_export(ctx: Context, sk: SecretKey):
    i = ctx.info
    out = np.zeros((i.nprimes, i.N), dtype=np.uint64)
    _chk(lib().ppst_sk_export(ctx, sk, _p(out), out.size))
    return out


def ppst_encode(ctx: Context, values, level: int) -> Plaintext:
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = _out()
    _chk(lib().ppst_encode(ctx, _p(v), len(v), level, ctypes.byref(out)))
    return Plaintext(out.value, ctx)


def ppst_plaintext_from_coeffs(ctx: Context, coeffs, level: int, scale: float) -> Plaintext:
    c = np.ascontiguousarray(coeffs, dtype=np.int64)
    out = _out()
    _chk(lib().ppst_plaintext_from_coeffs(ctx, _p(c), level, scale, ctypes.byref(out)))
    return Plaintext(out.value, ctx)


def ppst_plaintext_coeffs(ctx: Context, pt: Plaintext):
    out = np.zeros(ctx.info.N, dtype=np.int64)
    _chk(lib().ppst_plaintext_coeffs(pt, _p(out), len(out)))
    return out


def ppst_plaintext_export(ctx: Context, pt: Plaintext, level: int):
    out = np.zeros((level + 1, ctx.info.N), dtype=np.uint64)
    _chk(lib().ppst_plaintext_export(ctx, pt, _p(out), out.size))
    return out


def ppst_plaintext_import(ctx: Context, words: np.ndarray, level: int, scale: float) -> Plaintext:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    if w.size != (level + 1) * ctx.info.N:
        raise PpstError(-1, "expected [level+1][N] words")
    out = _out()
    _chk(lib().ppst_plaintext_import(ctx, _p(w), level, scale, ctypes.byref(out)))
    return Plaintext(out.value, ctx)


def ppst_decode(ctx: Context, pt: Plaintext, n: int | None = None):
    n = ctx.info.slots if n is None else n
    out = np.zeros(n, dtype=np.float64)
    _chk(lib().ppst_decode(ctx, pt, _p(out), n))
    return out


def ppst_encrypt(ctx, pk, pt, seed) -> Ciphertext:
    out = _out()
    _chk(lib().ppst_encrypt(ctx, pk, pt, seed, ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_encrypt_sk(ctx, sk, pt, seed) -> Ciphertext:
    out = _out()
    _chk(lib().ppst_encrypt_sk(ctx, sk, pt, seed, ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_decrypt(ctx, sk, ct) -> Plaintext:
    out = _out()
    _chk(lib().ppst_decrypt(ctx, sk, ct, ctypes.byref(out)))
    return Plaintext(out.value, ctx)


def ppst_ct_export(ctx: Context, ct: Ciphertext):
    out = np.zeros((ct.npoly, ct.level + 1, ctx.info.N), dtype=np.uint64)
    _chk(lib().ppst_ct_export(ctx, ct, _p(out), out.size))
    return out


def ppst_ct_import(ctx: Context, data: np.ndarray, level: int, scale: float) -> Ciphertext:
    d = np.ascontiguousarray(data, dtype=np.uint64)
    out = _out()
    _chk(lib().ppst_ct_import(ctx, _p(d), level, scale, d.shape[0], ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_mul_noalloc(ctx: Context, evk, a_ptr: int, b_ptr: int, level: int, out_ptr: int):
    """Device addresses in, device address out (see the header)."""
    _chk(lib().ppst_mul_noalloc(ctx, evk, ctypes.c_void_p(a_ptr), ctypes.c_void_p(b_ptr), level,
                                ctypes.c_void_p(out_ptr)))


def ppst_ct_device_ptr(ct: Ciphertext) -> int:
    out = _out()
    _chk(lib().ppst_ct_device_ptr(ct, ctypes.byref(out)))
    return out.value


def _unary(name):
    def f(ctx, *args):
        out = _out()
        _chk(getattr(lib(), name)(ctx, *args, ctypes.byref(out)))
        return Ciphertext(out.value, ctx)
    f.__name__ = name
    return f


ppst_add = _unary("ppst_add")
ppst_sub = _unary("ppst_sub")
ppst_add_const = _unary("ppst_add_const")
ppst_mul_const = _unary("ppst_mul_const")
ppst_mul_int = _unary("ppst_mul_int")
ppst_mul_plain = _unary("ppst_mul_plain")
ppst_mul = _unary("ppst_mul")
ppst_tensor = _unary("ppst_tensor")
ppst_relin = _unary("ppst_relin")
ppst_rescale = _unary("ppst_rescale")
ppst_rotate = _unary("ppst_rotate")
ppst_rotsum = _unary("ppst_rotsum")
ppst_rotsum_serial = _unary("ppst_rotsum_serial")
ppst_level_align = _unary("ppst_level_align")
ppst_mod_raise = _unary("ppst_mod_raise")
ppst_apply_galois = _unary("ppst_apply_galois")
ppst_mul_monomial = _unary("ppst_mul_monomial")
ppst_bootstrap = _unary("ppst_bootstrap")
ppst_boot_coeff_to_slot = _unary("ppst_boot_coeff_to_slot")
ppst_boot_slot_to_coeff = _unary("ppst_boot_slot_to_coeff")


# ---------------------------------------------------------- bootstrapping
class Boot(_Handle):
    _destroy = "ppst_boot_destroy"


def ppst_boot_create(ctx, coeffs=None):
    out = _out()
    if coeffs is None:
        _chk(lib().ppst_boot_create(ctx, None, 0, ctypes.byref(out)))
    else:
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        _chk(lib().ppst_boot_create(ctx, _p(c), c.size, ctypes.byref(out)))
    return Boot(out.value, ctx)


def ppst_boot_count(bt) -> int:
    n = _u64()
    _chk(lib().ppst_boot_count(bt, ctypes.byref(n)))
    return int(n.value)


def ppst_evk_add_boot(ctx, sk, seed, evk):
    _chk(lib().ppst_evk_add_boot(ctx, sk, seed, evk))


def ppst_boot_rotations(params) -> list:
    n = ctypes.c_size_t()
    _chk(lib().ppst_boot_rotations(ctypes.byref(params), None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), dtype=np.int32)
    _chk(lib().ppst_boot_rotations(ctypes.byref(params), _p(out), n.value, ctypes.byref(n)))
    return [int(v) for v in out[:n.value]]


def ppst_boot_group_info(params, transform: int, group: int) -> dict:
    d = np.zeros(9, dtype=np.int32)
    _chk(lib().ppst_boot_group_info(ctypes.byref(params), transform, group, _p(d)))
    keys = ("inverse", "lo", "hi", "level", "ckind", "u", "m0", "b", "G")
    return {k: int(v) for k, v in zip(keys, d)}


def ppst_boot_group_coeffs(params, transform: int, group: int):
    """(coefficients [b G][N] int64, used [b G] uint8) of a group's plaintexts."""
    g = ppst_boot_group_info(params, transform, group)
    cells = g["b"] * g["G"]
    out = np.zeros((cells, 1 << params.logN), dtype=np.int64)
    used = np.zeros(cells, dtype=np.uint8)
    _chk(lib().ppst_boot_group_coeffs(ctypes.byref(params), transform, group, _p(out), _p(used), cells))
    return out, used


def ppst_evalmod_coeffs(K: int, r: int, degree: int):
    out = np.zeros(degree + 1, dtype=np.float64)
    _chk(lib().ppst_evalmod_coeffs(K, r, degree, _p(out), out.size))
    return out


def ppst_boot_split(ctx, evk, bt, w):
    re, im = _out(), _out()
    _chk(lib().ppst_boot_split(ctx, evk, bt, w, ctypes.byref(re), ctypes.byref(im)))
    return Ciphertext(re.value, ctx), Ciphertext(im.value, ctx)


def ppst_boot_eval_mod(ctx, evk, bt, lanes):
    outs = (ctypes.c_void_p * len(lanes))()
    _chk(lib().ppst_boot_eval_mod(ctx, evk, bt, _ptrs(lanes), len(lanes), outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(lanes))]


def ppst_lincomb(ctx, cts, cs, level):
    out = _out()
    c = np.ascontiguousarray(cs, dtype=np.float64)
    _chk(lib().ppst_lincomb(ctx, _ptrs(cts), c.ctypes.data, len(cts), level, ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_rotate_hoisted(ctx, evk, ct, steps):
    s = np.ascontiguousarray(steps, dtype=np.int32)
    outs = (ctypes.c_void_p * len(s))()
    _chk(lib().ppst_rotate_hoisted(ctx, evk, ct, _p(s), len(s), outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(s))]


def _ptrs(cts):
    arr = (ctypes.c_void_p * len(cts))()
    for i, c in enumerate(cts):
        arr[i] = c.ptr
    return arr


def ppst_mul_batch(ctx, evk, a, b):
    outs = (ctypes.c_void_p * len(a))()
    _chk(lib().ppst_mul_batch(ctx, evk, _ptrs(a), _ptrs(b), len(a), outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(a))]


def ppst_mul_const_batch(ctx, cts, c):
    outs = (ctypes.c_void_p * max(1, len(cts)))()
    _chk(lib().ppst_mul_const_batch(ctx, _ptrs(cts), len(cts), c, outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(cts))]


def ppst_rotsum_batch(ctx, evk, cts):
    outs = (ctypes.c_void_p * max(1, len(cts)))()
    _chk(lib().ppst_rotsum_batch(ctx, evk, _ptrs(cts), len(cts), outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(cts))]


def ppst_rotate_batch(ctx, evk, cts, r):
    outs = (ctypes.c_void_p * max(1, len(cts)))()
    _chk(lib().ppst_rotate_batch(ctx, evk, _ptrs(cts), len(cts), r, outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(cts))]


def ppst_rotate_hoisted_batch(ctx, evk, cts, steps):
    """Rotations of every ciphertext by every step; result[i][k] = cts[i]
    rotated by steps[k]."""
    s = np.ascontiguousarray(steps, dtype=np.int32)
    n, m = len(cts), len(s)
    outs = (ctypes.c_void_p * max(1, n * m))()
    _chk(lib().ppst_rotate_hoisted_batch(ctx, evk, _ptrs(cts), n, _p(s), m, outs))
    return [[Ciphertext(outs[i * m + k], ctx) for k in range(m)] for i in range(n)]


class Graph(_Handle):
    """A recorded sequence of evaluation calls (ppst_graph_*)."""
    _destroy = "ppst_graph_destroy"

    def launch(self):
        _chk(lib().ppst_graph_launch(self))


def ppst_graph_begin(ctx):
    _chk(lib().ppst_graph_begin(ctx))


def ppst_graph_end(ctx) -> Graph:
    out = _out()
    _chk(lib().ppst_graph_end(ctx, ctypes.byref(out)))
    return Graph(out.value, ctx)


def ppst_invsqrt_cfg_default(coeffs=None, boot=None, **kw) -> InvSqrtCfg:
    """boot: a Boot handle (ppst_boot_create) for InvSqrt with refreshes."""
    cfg = InvSqrtCfg()
    _chk(lib().ppst_invsqrt_cfg_default(ctypes.byref(cfg)))
    for k, v in kw.items():
        setattr(cfg, k, v)
    if boot is not None:
        cfg._boot = boot
        cfg.boot = boot.ptr
    if coeffs is not None:
        arr = np.ascontiguousarray(coeffs, dtype=np.float64)
        cfg._keep = arr
        cfg.coeffs = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return cfg


def ppst_stat_mean(ctx, evk, col, nrows, B):
    out = _out()
    _chk(lib().ppst_stat_mean(ctx, evk, _ptrs(col), len(col), nrows, B, ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_stat_variance(ctx, evk, col, nrows, B):
    out = _out()
    _chk(lib().ppst_stat_variance(ctx, evk, _ptrs(col), len(col), nrows, B, ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_stat_invsqrt(ctx, evk, xs, B, cfg=None):
    outs = (ctypes.c_void_p * len(xs))()
    cfg = cfg or ppst_invsqrt_cfg_default()
    _chk(lib().ppst_stat_invsqrt(ctx, evk, _ptrs(xs), len(xs), B, ctypes.byref(cfg), outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(xs))]


def ppst_stat_zscore(ctx, evk, col, nrows, B, cfg=None):
    outs = (ctypes.c_void_p * len(col))()
    cfg = cfg or ppst_invsqrt_cfg_default()
    _chk(lib().ppst_stat_zscore(ctx, evk, _ptrs(col), len(col), nrows, B, ctypes.byref(cfg), outs))
    return [Ciphertext(outs[i], ctx) for i in range(len(col))]


def ppst_stat_kurtosis(ctx, evk, col, nrows, B, cfg=None, excess=False):
    out = _out()
    cfg = cfg or ppst_invsqrt_cfg_default()
    _chk(lib().ppst_stat_kurtosis(ctx, evk, _ptrs(col), len(col), nrows, B, ctypes.byref(cfg),
                                  int(excess), ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_stat_skewness(ctx, evk, col, nrows, B, cfg=None):
    out = _out()
    cfg = cfg or ppst_invsqrt_cfg_default()
    _chk(lib().ppst_stat_skewness(ctx, evk, _ptrs(col), len(col), nrows, B, ctypes.byref(cfg),
                                  ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_stat_cv(ctx, evk, col, nrows, B_mean, B_var, cfg=None):
    out = _out()
    cfg = cfg or ppst_invsqrt_cfg_default()
    _chk(lib().ppst_stat_cv(ctx, evk, _ptrs(col), len(col), nrows, B_mean, B_var, ctypes.byref(cfg),
                            ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_stat_pearson(ctx, evk, colx, coly, nrows, Bx, By, cfg=None):
    out = _out()
    cfg = cfg or ppst_invsqrt_cfg_default()
    _chk(lib().ppst_stat_pearson(ctx, evk, _ptrs(colx), _ptrs(coly), len(colx), nrows, Bx, By,
                                 ctypes.byref(cfg), ctypes.byref(out)))
    return Ciphertext(out.value, ctx)


def ppst_ntt_autotune(ctx: Context):
    _chk(lib().ppst_ntt_autotune(ctx))


def ppst_ntt_plan(ctx: Context) -> str:
    buf = ctypes.create_string_buffer(4096)
    _chk(lib().ppst_ntt_plan(ctx, buf, 4096))
    return buf.value.decode()


def ppst_ntt_set_plan(ctx: Context, col: int, row: int):
    _chk(lib().ppst_ntt_set_plan(ctx, col, row))


def ppst_ntt_load_plan(ctx: Context, plan: str):
    _chk(lib().ppst_ntt_load_plan(ctx, plan.encode()))


def ppst_ntt_forward(ctx: Context, dev_ptr: int, nlimbs: int, first_prime: int):
    _chk(lib().ppst_ntt_forward(ctx, ctypes.c_void_p(dev_ptr), nlimbs, first_prime))


def ppst_ntt_inverse(ctx: Context, dev_ptr: int, nlimbs: int, first_prime: int):
    _chk(lib().ppst_ntt_inverse(ctx, ctypes.c_void_p(dev_ptr), nlimbs, first_prime))


SERVER_NO_MERGE = 1


def ppst_server_create(ctx, evk, hbm_budget: int, slots: int, merge: bool = True) -> Server:
    """hbm_budget 0: the device's free memory at creation less 2 GiB."""
    out = _out()
    _chk(lib().ppst_server_create(ctx, evk, hbm_budget, slots, 0 if merge else SERVER_NO_MERGE,
                                  ctypes.byref(out)))
    s = Server(out.value, ctx)
    s.evk = evk
    return s


def ppst_server_info(srv: Server) -> dict:
    v = [ctypes.c_uint64() for _ in range(4)]
    _chk(lib().ppst_server_info(srv, *[ctypes.byref(x) for x in v]))
    return {"budget": v[0].value, "merged_launches": v[1].value, "merged_lanes": v[2].value,
            "multi_query_launches": v[3].value}


def ppst_server_register_column(srv: Server, cts, nrows: int) -> int:
    cid = _u64()
    _chk(lib().ppst_server_register_column(srv, _ptrs(cts), len(cts), nrows, ctypes.byref(cid)))
    return cid.value


def ppst_server_submit(srv: Server, kind: int, col_x: int, col_y: int = 0, B: float = 1.0,
                       B2: float = 1.0, cfg: InvSqrtCfg | None = None) -> int:
    q = Query()
    q.kind, q.col_x, q.col_y, q.B, q.B2 = kind, col_x, col_y, B, B2
    q.cfg = cfg or ppst_invsqrt_cfg_default()
    t = _u64()
    _chk(lib().ppst_server_submit(srv, ctypes.byref(q), ctypes.byref(t)))
    return t.value


def ppst_server_poll(srv, ticket) -> bool:
    done = ctypes.c_int32(0)
    _chk(lib().ppst_server_poll(srv, ticket, ctypes.byref(done)))
    return bool(done.value)


def ppst_server_output_count(srv: Server, ticket: int) -> int:
    n = ctypes.c_size_t()
    _chk(lib().ppst_server_output_count(srv, ticket, ctypes.byref(n)))
    return n.value


def ppst_server_wait_all(srv: Server, ticket: int, cap: int | None = None):
    """Returns (status, list of ciphertexts, stats); cap defaults to the
    query's output count."""
    cap = ppst_server_output_count(srv, ticket) if cap is None else cap
    outs = (ctypes.c_void_p * max(1, cap))()
    n = ctypes.c_size_t()
    st = QueryStats()
    rc = lib().ppst_server_wait_all(srv, ticket, outs, cap, ctypes.byref(n), ctypes.byref(st))
    return rc, [Ciphertext(outs[i], srv.owner) for i in range(n.value)], st


def ppst_server_wait(srv: Server, ticket: int):
    """Returns (status, ciphertext or None, stats)."""
    out = _out()
    st = QueryStats()
    rc = lib().ppst_server_wait(srv, ticket, ctypes.byref(out), ctypes.byref(st))
    ct = Ciphertext(out.value, srv.owner) if out.value else None
    return rc, ct, st
