"""ctypes loader for ckks_oracle.c (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile the oracle's C with gcc (no GPU code, no shared sources)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    lib = ctypes.CDLL(build())
    u64, u32, i64, sz = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.c_void_p
    sig = {
        "orc_mulmod": (u64, [u64, u64, u64]),
        "orc_powmod": (u64, [u64, u64, u64]),
        "orc_invmod": (u64, [u64, u64]),
        "orc_reduce_i64": (u64, [i64, u64]),
        "orc_is_prime": (ctypes.c_int, [u64]),
        "orc_ntt_tables": (None, [u32, u64, u64, P, P]),
        "orc_ntt": (None, [P, u32, u64, P]),
        "orc_intt": (None, [P, u32, u64, P]),
        "orc_vec_add": (None, [P, P, P, sz, u64]),
        "orc_vec_sub": (None, [P, P, P, sz, u64]),
        "orc_vec_neg": (None, [P, P, sz, u64]),
        "orc_vec_mul": (None, [P, P, P, sz, u64]),
        "orc_vec_mul_scalar": (None, [P, u64, P, sz, u64]),
        "orc_vec_reduce_i64": (None, [P, P, sz, u64]),
        "orc_poly_mul": (None, [P, P, P, u32, u64, P, P, P]),
        "orc_automorphism": (None, [P, P, u32, u64, u64]),
        "orc_base_convert": (None, [P, u32, P, P, u32, P, u32]),
        "orc_rescale_limb": (None, [P, P, P, sz, u64, u64]),
        "orc_chacha_quarter": (None, [P]),
        "orc_chacha20_block": (None, [P, u32, P, P]),
        "orc_stream_words": (None, [P, u32, u64, u64, sz, P]),
        "orc_sample_ternary": (None, [P, u32, u64, sz, P]),
        "orc_sample_gauss": (None, [P, u32, u64, sz, P, P]),
        "orc_sample_uniform": (None, [P, u32, u64, u32, u32, u64, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def ptr(a):
    """Data pointer of a C-contiguous numpy array."""
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data


def u64arr(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
