"""Thin ctypes binding of include/vr.h (argument marshalling only).

Every operation runs in libvr.so's HIP kernels; this module converts numpy
arrays and Python numbers to C arguments and wraps handles so that they are
freed with the matching vr_free_* call.  There is no CPU fallback: without the
built library (python -m paper_2512_18646_amd.build) or without a gfx950
device, loading or creating a context raises.

PyTorch, when importable, is imported before the library so the process holds
a single HIP runtime, and torch's current stream can be passed as `stream`.
"""
import ctypes
import os

import numpy as np

try:  # one HIP runtime per process: torch's, when torch is present
    import torch  # noqa: F401
    _HAVE_TORCH = True
except Exception:  # pragma: no cover
    _HAVE_TORCH = False

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvr.so")

VR_OK, VR_EINVAL, VR_ESECURITY, VR_ELEVEL, VR_ESCALE, VR_ENOKEY, VR_ENOMEM, VR_EDEVICE, VR_EBUSY, \
    VR_ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
_NAMES = {VR_EINVAL: "EINVAL", VR_ESECURITY: "ESECURITY", VR_ELEVEL: "ELEVEL", VR_ESCALE: "ESCALE",
          VR_ENOKEY: "ENOKEY", VR_ENOMEM: "ENOMEM", VR_EDEVICE: "EDEVICE", VR_EBUSY: "EBUSY",
          VR_ECANCELED: "ECANCELED"}


class VRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


class vr_cnn_desc(ctypes.Structure):
    _fields_ = [("C_in", ctypes.c_uint32), ("h", ctypes.c_uint32), ("w", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("C_out", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("stride", ctypes.c_uint32), ("K", ctypes.c_void_p), ("bias", ctypes.c_void_p),
                ("square", ctypes.c_uint32), ("fc_w", ctypes.c_void_p), ("fc_bias", ctypes.c_void_p),
                ("fc_out", ctypes.c_uint32), ("fc_block", ctypes.c_uint32)]


class vr_matmul_cost(ctypes.Structure):
    _fields_ = [("feasible", ctypes.c_uint32), ("transposed", ctypes.c_uint32), ("client_cts", ctypes.c_uint64),
                ("key_switches", ctypes.c_uint64), ("tensors", ctypes.c_uint64), ("est_us", ctypes.c_double)]


MATMUL_FORMS = ("column_split", "column_block", "outer")


class vr_params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("n_p", ctypes.c_uint32),
                ("dnum", ctypes.c_uint32), ("q_bits", ctypes.POINTER(ctypes.c_uint32)),
                ("p_bits", ctypes.POINTER(ctypes.c_uint32)), ("log2_scale", ctypes.c_double),
                ("sigma", ctypes.c_double), ("allow_insecure", ctypes.c_uint32)]


P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
U32, U64, I32, DBL, SZ = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t

# name -> argument types (all return vr_status unless listed in _VOID)
_SIGS = {
    "vr_context_create": [ctypes.POINTER(vr_params), ctypes.c_int, PP],
    "vr_context_moduli": [P, P, SZ],
    "vr_context_info": [P, P, ctypes.POINTER(DBL)],
    "vr_context_set_stream": [P, P],
    "vr_context_set_allocator": [P, P, P, P],
    "vr_context_mem_info": [P, ctypes.POINTER(SZ), ctypes.POINTER(SZ)],
    "vr_context_trim": [P],
    "vr_context_set_tuning": [P, ctypes.c_char_p, ctypes.c_char_p],
    "vr_context_tuning_report": [P, ctypes.c_char_p, SZ],
    "vr_keygen": [P, P, P, SZ, PP, PP],
    "vr_keys_add_rotations": [P, P, P, P, P, SZ],
    "vr_encode": [P, P, SZ, U32, DBL, PP],
    "vr_encrypt": [P, P, P, P, U64, PP],
    "vr_encrypt_columns": [P, P, P, U32, U32, U32, U32, U32, U32, P, U64, PP],
    "vr_encrypt_matrix_columns": [P, P, P, U32, U32, U32, U32, U32, U32, P, U64, PP],
    "vr_decrypt": [P, P, P, PP],
    "vr_decode": [P, P, P, SZ],
    "vr_add": [P, P, P, PP, P],
    "vr_sub": [P, P, P, PP, P],
    "vr_mul_const": [P, P, DBL, DBL, PP, P],
    "vr_add_const": [P, P, DBL, PP, P],
    "vr_mul_plain": [P, P, P, PP, P],
    "vr_tensor": [P, P, P, PP, P],
    "vr_relinearize": [P, P, P, PP, P],
    "vr_mul": [P, P, P, P, PP, P],
    "vr_rescale": [P, P, PP, P],
    "vr_relin_rescale": [P, P, P, PP, P],
    "vr_mul_rescale": [P, P, P, P, PP, P],
    "vr_mod_drop": [P, P, U32, PP, P],
    "vr_rotate": [P, P, P, I32, PP, P],
    "vr_rotate_many": [P, P, P, P, SZ, PP, P],
    "vr_rotate_batch": [P, P, PP, SZ, I32, PP, P],
    "vr_rotate_noalloc": [P, P, P, U32, I32, P, P],
    "vr_poly_eval": [P, P, PP, SZ, P, U32, PP, P],
    "vr_conv2d_encw": [P, P, PP, U32, U32, U32, U32, PP, PP, U32, U32, U32, PP, P],
    "vr_matmul_block": [P, P, PP, PP, U32, U32, U32, PP, P],
    "vr_matmul_plan": [P, U32, U32, U32, U32, U64, P, ctypes.POINTER(U32)],
    "vr_fc_encw": [P, P, PP, U32, PP, PP, U32, U32, PP, P],
    "vr_dense": [P, PP, U32, P, P, U32, PP, P],
    "vr_matmul": [P, P, PP, PP, U32, U32, U32, PP, P],
    "vr_matmul_outer": [P, P, PP, PP, U32, U32, U32, PP, P],
    "vr_conv2d": [P, P, PP, U32, U32, U32, U32, P, P, U32, U32, U32, PP, P],
    "vr_conv2d_sets": [P, P, PP, U32, U32, U32, U32, U32, P, P, U32, U32, U32, PP, P],
    "vr_square": [P, P, PP, SZ, PP, P],
    "vr_fc": [P, P, PP, U32, U32, PP, P, U32, U32, PP, P],
    "vr_encode_fc_weights": [P, P, U32, U32, U32, U32, U32, U32, U32, PP],
    "vr_ct_export": [P, P, P, SZ, P, P, P],
    "vr_ct_import": [P, P, U32, U32, DBL, PP],
    "vr_pt_export": [P, P, P, SZ, P, P],
    "vr_pt_import": [P, P, U32, DBL, PP],
    "vr_sk_export": [P, P, P, SZ],
    "vr_ct_meta": [P, P, P, P],
    "vr_swk_export": [P, P, U32, P, SZ],
    "vr_ntt": [P, P, U32, P, ctypes.c_int, P],
    "vr_profile_start": [P, ctypes.c_char_p, SZ],
    "vr_profile_stop": [P, ctypes.POINTER(DBL), ctypes.POINTER(U64), ctypes.POINTER(U64),
                        ctypes.POINTER(U32)],
    "vr_cnn_forward": [P, P, P, PP, U32, PP, P],
    "vr_graph_create": [P, P, P, PP, U32, PP],
    "vr_graph_set_inputs": [P, PP, SZ, P],
    "vr_graph_launch": [P, P],
    "vr_graph_outputs": [P, PP, SZ, ctypes.POINTER(SZ)],
    "vr_graph_destroy": [P],
    "vr_batch_create": [P, P, PP],
    "vr_batch_add_cnn": [P, P, PP, U32, ctypes.POINTER(U32)],
    "vr_batch_add_matmul": [P, PP, PP, U32, U32, U32, ctypes.POINTER(U32)],
    "vr_batch_add_matmul_outer": [P, PP, PP, U32, U32, U32, ctypes.POINTER(U32)],
    "vr_batch_run": [P, P],
    "vr_batch_capture": [P],
    "vr_batch_launch": [P, P],
    "vr_batch_outputs": [P, U32, PP, SZ, ctypes.POINTER(SZ)],
    "vr_batch_destroy": [P],
    "vr_srv_create": [P, SZ, U32, PP],
    "vr_srv_destroy": [P],
    "vr_srv_register_session": [P, P, ctypes.POINTER(U64)],
    "vr_srv_register_conv_model": [P, U32, U32, U32, U32, P, P, U32, U32, U32, U32,
                                   ctypes.POINTER(U32)],
    "vr_srv_register_model": [P, P, ctypes.POINTER(U32)],
    "vr_srv_submit": [P, U64, U32, PP, SZ, U32, ctypes.POINTER(U64)],
    "vr_srv_cancel": [P, U64],
    "vr_srv_reset_stats": [P],
    "vr_srv_poll": [P, U64, ctypes.c_int, PP, SZ, ctypes.POINTER(SZ), ctypes.POINTER(ctypes.c_int)],
    "vr_srv_stats": [P, ctypes.POINTER(DBL), ctypes.POINTER(DBL), ctypes.POINTER(DBL),
                     ctypes.POINTER(U64), ctypes.POINTER(U64), ctypes.POINTER(U64)],
    "vr_context_destroy": [P],
    "vr_free_ciphertext": [P],
    "vr_free_plaintext": [P],
    "vr_free_keys": [P, P],
    "vr_last_error": [],
}
_VOID = {"vr_context_destroy", "vr_srv_destroy", "vr_graph_destroy", "vr_batch_destroy", "vr_free_ciphertext", "vr_free_plaintext", "vr_free_keys"}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libvr.so is not built: run `python -m paper_2512_18646_amd.build` "
                          "(the product path has no CPU fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None if name in _VOID else (ctypes.c_char_p if name == "vr_last_error" else ctypes.c_int)
    return lib


lib = _load()


def exported_symbols():
    return sorted(_SIGS)


def _seed(seed):
    """A seed as the four host words of its 256-bit ChaCha20 key (an integer
    below 2^256; seed[0] holds bits 0..63)."""
    seed = int(seed)
    if not 0 <= seed < 1 << 256:
        raise ValueError("seed must be a 256-bit non-negative integer")
    return (ctypes.c_uint64 * 4)(*[(seed >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(4)])


def _check(rc):
    if rc != VR_OK:
        raise VRError(rc, (lib.vr_last_error() or b"").decode())


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream   # torch.cuda.Stream


def _ptr_array(handles):
    arr = (ctypes.c_void_p * max(1, len(handles)))()
    for i, h in enumerate(handles):
        arr[i] = h.h if hasattr(h, "h") else h
    return arr


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ------------------------------------------------------------------ handles

class Ciphertext:
    __slots__ = ("h", "ctx")

    def __init__(self, h, ctx):
        self.h, self.ctx = h, ctx

    def __del__(self):
        if self.h and lib is not None:   # lib is None once the interpreter is tearing down
            lib.vr_free_ciphertext(self.h)
            self.h = None

    @property
    def meta(self):
        nc, lv, sc = U32(), U32(), DBL()
        _check(lib.vr_ct_meta(self.h, ctypes.byref(nc), ctypes.byref(lv), ctypes.byref(sc)))
        return nc.value, lv.value, sc.value

    @property
    def level(self):
        return self.meta[1]

    @property
    def scale(self):
        return self.meta[2]

    def export(self):
        """Coefficient-domain limbs, uint64 [ncomp][level+1][N] (synchronises)."""
        nc, lv, _ = self.meta
        out = np.empty((nc, lv + 1, self.ctx.n), dtype=np.uint64)
        _check(lib.vr_ct_export(self.ctx.h, self.h, out.ctypes.data, out.size, None, None, None))
        return out


class Plaintext:
    __slots__ = ("h", "ctx", "level", "scale")

    def __init__(self, h, ctx, level, scale):
        self.h, self.ctx, self.level, self.scale = h, ctx, level, scale

    def __del__(self):
        if self.h and lib is not None:
            lib.vr_free_plaintext(self.h)
            self.h = None

    def export(self):
        out = np.empty((self.level + 1, self.ctx.n), dtype=np.uint64)
        _check(lib.vr_pt_export(self.ctx.h, self.h, out.ctypes.data, out.size, None, None))
        return out


class Keys:
    def __init__(self, sk, ek, ctx):
        self.sk, self.ek, self.ctx = sk, ek, ctx

    def __del__(self):
        if (self.sk or self.ek) and lib is not None:
            lib.vr_free_keys(self.sk, self.ek)
            self.sk = self.ek = None

    def secret_coeffs(self):
        out = np.empty(self.ctx.n, dtype=np.int8)
        _check(lib.vr_sk_export(self.ctx.h, self.sk, out.ctypes.data, self.ctx.n))
        return out

    def switching_key(self, galois=0):
        """Coefficient-domain key [dnum][2][n_q + n_p][N] (galois 0: relinearisation)."""
        c = self.ctx
        out = np.empty((c.dnum, 2, len(c.q) + len(c.p), c.n), dtype=np.uint64)
        _check(lib.vr_swk_export(c.h, self.ek, galois, out.ctypes.data, out.size))
        return out

    def add_rotations(self, seed, steps):
        st = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
        _check(lib.vr_keys_add_rotations(self.ctx.h, self.sk, self.ek, _seed(seed), st.ctypes.data, st.size))


class Context:
    """RNS-CKKS context on one GPU (see vr_context_create)."""

    def __init__(self, log_n, q_bits, p_bits, dnum, log2_scale, sigma=3.2, allow_insecure=False,
                 device=0):
        qb = (U32 * len(q_bits))(*q_bits)
        pb = (U32 * len(p_bits))(*p_bits)
        prm = vr_params(log_n, len(q_bits), len(p_bits), dnum, qb, pb, log2_scale, sigma,
                        1 if allow_insecure else 0)
        h = ctypes.c_void_p()
        _check(lib.vr_context_create(ctypes.byref(prm), device, ctypes.byref(h)))
        self.h = h.value
        info = (U32 * 8)()
        sc = DBL()
        _check(lib.vr_context_info(self.h, info, ctypes.byref(sc)))
        self.log_n, self.slots, n_q, n_p, self.dnum, self.alpha, secure, self.total_bits = list(info)
        self.n = 1 << self.log_n
        self.secure = bool(secure)
        self.scale = sc.value
        mods = np.zeros(n_q + n_p, dtype=np.uint64)
        _check(lib.vr_context_moduli(self.h, mods.ctypes.data, mods.size))
        self.q = [int(x) for x in mods[:n_q]]
        self.p = [int(x) for x in mods[n_q:]]
        self.L = n_q - 1

    @classmethod
    def from_params(cls, p, device=0):
        """From any object with log_n, q_bits, p_bits, dnum, log2_scale, allow_insecure."""
        return cls(p.log_n, list(p.q_bits), list(p.p_bits), p.dnum, p.log2_scale,
                   allow_insecure=getattr(p, "allow_insecure", False), device=device)

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.vr_context_destroy(self.h)
            self.h = None

    def set_stream(self, stream):
        _check(lib.vr_context_set_stream(self.h, _stream(stream)))

    def use_torch_allocator(self):
        """Device memory from PyTorch's caching allocator (vr_context_set_allocator
        with torch.cuda.caching_allocator_alloc / _delete on the stream the
        library uses the memory on), so the library and the framework share
        one pool.  Graph capture needs the built-in allocator."""
        import torch
        alloc_t = ctypes.CFUNCTYPE(ctypes.c_void_p, SZ, ctypes.c_void_p, ctypes.c_void_p)
        free_t = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
        dev = torch.cuda.current_device()

        def alloc(nbytes, stream, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
            except RuntimeError:
                return None

        def free(ptr, stream, user):
            torch.cuda.caching_allocator_delete(ptr)
        self._alloc_cbs = (alloc_t(alloc), free_t(free))   # kept alive with the context
        _check(lib.vr_context_set_allocator(self.h, ctypes.cast(self._alloc_cbs[0], ctypes.c_void_p),
                                            ctypes.cast(self._alloc_cbs[1], ctypes.c_void_p), None))

    def use_builtin_allocator(self):
        _check(lib.vr_context_set_allocator(self.h, None, None, None))

    def mem_info(self):
        """(reserved, in_use) bytes of the built-in caching allocator."""
        r, u = SZ(), SZ()
        _check(lib.vr_context_mem_info(self.h, ctypes.byref(r), ctypes.byref(u)))
        return r.value, u.value

    def trim(self):
        _check(lib.vr_context_trim(self.h))

    def set_tuning(self, knob, value):
        _check(lib.vr_context_set_tuning(self.h, knob.encode(), value.encode()))

    def tuning_report(self):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib.vr_context_tuning_report(self.h, buf, len(buf)))
        return buf.value.decode()

    def profile_start(self, kernel_class, max_launches=65536):
        _check(lib.vr_profile_start(self.h, kernel_class.encode(), max_launches))

    def profile_stop(self):
        """(total_ms, launches, units, dropped) of the profiled kernel class."""
        ms, la, un, dr = DBL(), U64(), U64(), U32()
        _check(lib.vr_profile_stop(self.h, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(un),
                                   ctypes.byref(dr)))
        return ms.value, la.value, un.value, bool(dr.value)

    # ------------------------------------------------------------ client
    def keygen(self, seed, rot_steps=()):
        st = np.ascontiguousarray(np.asarray(list(rot_steps), dtype=np.int32))
        sk, ek = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib.vr_keygen(self.h, _seed(seed), st.ctypes.data if st.size else None, st.size,
                             ctypes.byref(sk), ctypes.byref(ek)))
        return Keys(sk.value, ek.value, self)

    def encode(self, x, level, scale=None):
        x = _f64(x)
        scale = self.scale if scale is None else float(scale)
        h = ctypes.c_void_p()
        _check(lib.vr_encode(self.h, x.ctypes.data if x.size else None, x.size, level, scale, ctypes.byref(h)))
        return Plaintext(h.value, self, level, scale)

    def encrypt(self, keys, pt, seed, ct_id):
        h = ctypes.c_void_p()
        _check(lib.vr_encrypt(self.h, keys.ek, pt.h, _seed(seed), ct_id, ctypes.byref(h)))
        return Ciphertext(h.value, self)

    def encrypt_columns(self, keys, X, pad, level, seed, first_ct_id):
        X = _f64(X)
        B, C, h, w = X.shape
        arr = (ctypes.c_void_p * (C * w))()
        _check(lib.vr_encrypt_columns(self.h, keys.ek, X.ctypes.data, B, C, h, w, pad, level, _seed(seed),
                                      first_ct_id, arr))
        return [Ciphertext(arr[i], self) for i in range(C * w)]

    def encrypt_matrix_columns(self, keys, M, role, m, p, level, seed, first_ct_id):
        M = _f64(M)
        rows, cols = M.shape
        n = cols if role in (0, 2, 4) else rows
        if role == 2:
            n = self.outer_tiles(m, p)[2] * cols
        elif role in (4, 5):
            n = self.block_shape(m, n, p)[3]
        arr = (ctypes.c_void_p * n)()
        _check(lib.vr_encrypt_matrix_columns(self.h, keys.ek, M.ctypes.data, rows, cols, role, m, p,
                                             level, _seed(seed), first_ct_id, arr))
        return [Ciphertext(arr[i], self) for i in range(n)]

    def decrypt(self, keys, ct):
        h = ctypes.c_void_p()
        _check(lib.vr_decrypt(self.h, keys.sk, ct.h, ctypes.byref(h)))
        _, lv, sc = ct.meta
        return Plaintext(h.value, self, lv, sc)

    def decode(self, pt, n=None):
        n = self.slots if n is None else n
        out = np.empty(n, dtype=np.float64)
        _check(lib.vr_decode(self.h, pt.h, out.ctypes.data, n))
        return out

    # ------------------------------------------------------------ server
    def _unary(self, fn, *args, stream=None):
        h = ctypes.c_void_p()
        _check(fn(self.h, *args, ctypes.byref(h), _stream(stream)))
        return Ciphertext(h.value, self)

    def add(self, a, b, stream=None):
        return self._unary(lib.vr_add, a.h, b.h, stream=stream)

    def sub(self, a, b, stream=None):
        return self._unary(lib.vr_sub, a.h, b.h, stream=stream)

    def mul_const(self, a, c, c_scale, stream=None):
        return self._unary(lib.vr_mul_const, a.h, float(c), float(c_scale), stream=stream)

    def add_const(self, a, c, stream=None):
        return self._unary(lib.vr_add_const, a.h, float(c), stream=stream)

    def mul_plain(self, a, pt, stream=None):
        return self._unary(lib.vr_mul_plain, a.h, pt.h, stream=stream)

    def tensor(self, a, b, stream=None):
        return self._unary(lib.vr_tensor, a.h, b.h, stream=stream)

    def relinearize(self, keys, a, stream=None):
        return self._unary(lib.vr_relinearize, keys.ek, a.h, stream=stream)

    def mul(self, keys, a, b, stream=None):
        return self._unary(lib.vr_mul, keys.ek, a.h, b.h, stream=stream)

    def rescale(self, a, stream=None):
        return self._unary(lib.vr_rescale, a.h, stream=stream)

    def relin_rescale(self, keys, a, stream=None):
        """Relinearisation and rescale as one ModDown by P q_l (level - 1)."""
        return self._unary(lib.vr_relin_rescale, keys.ek, a.h, stream=stream)

    def mul_rescale(self, keys, a, b, stream=None):
        return self._unary(lib.vr_mul_rescale, keys.ek, a.h, b.h, stream=stream)

    def mod_drop(self, a, level, stream=None):
        return self._unary(lib.vr_mod_drop, a.h, level, stream=stream)

    def rotate(self, keys, a, step, stream=None):
        return self._unary(lib.vr_rotate, keys.ek, a.h, int(step), stream=stream)

    def rotate_many(self, keys, a, steps, stream=None):
        st = np.ascontiguousarray(np.asarray(list(steps), dtype=np.int32))
        arr = (ctypes.c_void_p * max(1, st.size))()
        _check(lib.vr_rotate_many(self.h, keys.ek, a.h, st.ctypes.data, st.size, arr, _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(st.size)]

    def rotate_batch(self, keys, cts, step, stream=None):
        arr = (ctypes.c_void_p * len(cts))()
        _check(lib.vr_rotate_batch(self.h, keys.ek, _ptr_array(cts), len(cts), int(step), arr,
                                   _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(len(cts))]

    def rotate_noalloc(self, keys, in_ptr, level, step, out_ptr, stream=None):
        """vr_rotate_noalloc: device limbs [2][level+1][N] at in_ptr rotated into
        out_ptr, with no device allocation (integer device addresses)."""
        _check(lib.vr_rotate_noalloc(self.h, keys.ek, ctypes.c_void_p(in_ptr), int(level), int(step),
                                     ctypes.c_void_p(out_ptr), _stream(stream)))

    # ------------------------------------------------------------ layers
    def matmul(self, keys, A, Bbar, m, n, p, stream=None):
        Pp = 1                  # P' (M' when m < p: the transposed product)
        while Pp < min(m, p):
            Pp *= 2
        arr = (ctypes.c_void_p * Pp)()
        _check(lib.vr_matmul(self.h, keys.ek, _ptr_array(A), _ptr_array(Bbar), m, n, p, arr,
                             _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(Pp)]

    def block_shape(self, m, n, p):
        """(P', Mb, c, nb) of the column-block form (the sizes vr_matmul_block
        and roles 4 / 5 use: block size, columns per ciphertext, ciphertexts
        per operand), for sizing the handle arrays."""
        Pp = 1
        while Pp < p:
            Pp *= 2
        Mb = Pp * -(-(m + Pp - 1) // Pp)
        n2 = 1
        while n2 < n:
            n2 *= 2
        c = 1
        while 2 * c * Mb <= self.slots and c < n2:
            c *= 2
        return Pp, Mb, c, -(-n // c)

    def matmul_block(self, keys, A, Bbar, m, n, p, stream=None):
        Pp = 1
        while Pp < p:
            Pp *= 2
        arr = (ctypes.c_void_p * Pp)()
        _check(lib.vr_matmul_block(self.h, keys.ek, _ptr_array(A), _ptr_array(Bbar), m, n, p, arr,
                                   _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(Pp)]

    def matmul_plan(self, m, n, p, level, max_client_cts=0):
        """(chosen form name, {form: cost dict}) of the cost-model planner."""
        costs = (vr_matmul_cost * 3)()
        chosen = U32()
        _check(lib.vr_matmul_plan(self.h, m, n, p, level, max_client_cts, costs, ctypes.byref(chosen)))
        out = {}
        for f, c in zip(MATMUL_FORMS, costs):
            out[f] = {k: getattr(c, k) for k, _ in vr_matmul_cost._fields_}
        return MATMUL_FORMS[chosen.value], out

    def outer_tiles(self, m, p):
        """(P', R, T) of the outer-product product: column padding, rows per
        ciphertext, row tiles."""
        Pp = 1
        while Pp < p:
            Pp *= 2
        R = max(1, self.slots // Pp)
        return Pp, R, -(-m // R)

    def matmul_outer(self, keys, A, B, m, n, p, stream=None):
        T = self.outer_tiles(m, p)[2]
        arr = (ctypes.c_void_p * T)()
        _check(lib.vr_matmul_outer(self.h, keys.ek, _ptr_array(A), _ptr_array(B), m, n, p, arr,
                                   _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(T)]

    def conv2d(self, keys, cols, C_in, h, w, pad, K, bias, stride, stream=None):
        K = _f64(K)
        bias = _f64(bias)
        C_out, _, k, _ = K.shape
        wo = (w + 2 * pad - k) // stride + 1
        arr = (ctypes.c_void_p * (C_out * wo))()
        _check(lib.vr_conv2d(self.h, keys.ek, _ptr_array(cols), C_in, h, w, pad, K.ctypes.data,
                             bias.ctypes.data, C_out, k, stride, arr, _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(C_out * wo)]

    def conv2d_sets(self, keys, cols, n_sets, C_in, h, w, pad, K, bias, stride, stream=None):
        """cols = every set's C_in*w columns, set after set."""
        K = _f64(K)
        bias = _f64(bias)
        C_out, _, k, _ = K.shape
        wo = (w + 2 * pad - k) // stride + 1
        arr = (ctypes.c_void_p * (n_sets * C_out * wo))()
        _check(lib.vr_conv2d_sets(self.h, keys.ek, _ptr_array(cols), n_sets, C_in, h, w, pad,
                                  K.ctypes.data, bias.ctypes.data, C_out, k, stride, arr,
                                  _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(n_sets * C_out * wo)]

    def square(self, keys, cts, stream=None):
        arr = (ctypes.c_void_p * len(cts))()
        _check(lib.vr_square(self.h, keys.ek, _ptr_array(cts), len(cts), arr, _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(len(cts))]

    def conv2d_encw(self, keys, cols, C_in, h, w, pad, K_ct, bias_ct, C_out, k, stride, stream=None):
        wo = (w + 2 * pad - k) // stride + 1
        arr = (ctypes.c_void_p * (C_out * wo))()
        _check(lib.vr_conv2d_encw(self.h, keys.ek, _ptr_array(cols), C_in, h, w, pad, _ptr_array(K_ct),
                                  _ptr_array(bias_ct), C_out, k, stride, arr, _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(C_out * wo)]

    def fc_encw(self, keys, Y, W_ct, bias_ct, block, stream=None):
        n_out = len(bias_ct)
        arr = (ctypes.c_void_p * n_out)()
        _check(lib.vr_fc_encw(self.h, keys.ek, _ptr_array(Y), len(Y), _ptr_array(W_ct), _ptr_array(bias_ct),
                              n_out, block, arr, _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(n_out)]

    def poly_eval(self, keys, cts, coeffs, stream=None):
        c = _f64(coeffs)
        arr = (ctypes.c_void_p * len(cts))()
        _check(lib.vr_poly_eval(self.h, keys.ek, _ptr_array(cts), len(cts), c.ctypes.data, c.size - 1, arr,
                                _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(len(cts))]

    def dense(self, cts, W, bias, stream=None):
        W, b = _f64(W), _f64(bias)
        n_out = b.size
        if W.size != n_out * len(cts):
            raise ValueError("dense: W must be n_out x n_in")
        arr = (ctypes.c_void_p * n_out)()
        _check(lib.vr_dense(self.h, _ptr_array(cts), len(cts), W.ctypes.data, b.ctypes.data, n_out, arr,
                            _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(n_out)]

    def encode_fc_weights(self, W, stride, block, level):
        W = _f64(W)
        n_out, C, ho, wo = W.shape
        total = n_out * C * wo
        arr = (ctypes.c_void_p * total)()
        _check(lib.vr_encode_fc_weights(self.h, W.ctypes.data, n_out, C, ho, wo, stride, block, level, arr))
        sc = float(self.q[level])
        return [Plaintext(arr[i], self, level, sc) for i in range(total)]

    def fc(self, keys, Y, C, w_out, W_pt, bias, block, stream=None):
        bias = _f64(bias)
        n_out = bias.size
        arr = (ctypes.c_void_p * n_out)()
        _check(lib.vr_fc(self.h, keys.ek, _ptr_array(Y), C, w_out, _ptr_array(W_pt), bias.ctypes.data,
                         n_out, block, arr, _stream(stream)))
        return [Ciphertext(arr[i], self) for i in range(n_out)]

    # ------------------------------------------------------------ parity
    def ct_import(self, limbs, level, scale):
        a = np.ascontiguousarray(np.asarray(limbs, dtype=np.uint64))
        h = ctypes.c_void_p()
        _check(lib.vr_ct_import(self.h, a.ctypes.data, a.shape[0], level, float(scale), ctypes.byref(h)))
        return Ciphertext(h.value, self)

    def pt_import(self, limbs, level, scale):
        a = np.ascontiguousarray(np.asarray(limbs, dtype=np.uint64))
        h = ctypes.c_void_p()
        _check(lib.vr_pt_import(self.h, a.ctypes.data, level, float(scale), ctypes.byref(h)))
        return Plaintext(h.value, self, level, float(scale))

    def ntt_device(self, ptr, n_limbs, mod_index, inverse=False, stream=None):
        mi = np.ascontiguousarray(np.asarray(mod_index, dtype=np.uint32))
        _check(lib.vr_ntt(self.h, ptr, n_limbs, mi.ctypes.data, 1 if inverse else 0, _stream(stream)))


class Server:
    """Continuous-batching server over one context (vr_srv_*)."""

    def __init__(self, ctx, hbm_budget_bytes, max_batch=8):
        self.ctx = ctx
        self._keys = []
        self._models = {}
        h = ctypes.c_void_p()
        _check(lib.vr_srv_create(ctx.h, int(hbm_budget_bytes), int(max_batch), ctypes.byref(h)))
        self.h = h.value

    def close(self):
        if self.h:
            lib.vr_srv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def register_session(self, keys):
        sid = U64()
        _check(lib.vr_srv_register_session(self.h, keys.ek, ctypes.byref(sid)))
        self._keys.append(keys)   # keys outlive the server
        return sid.value

    def register_conv_model(self, C_in, h, w, pad, K, bias, stride, square=True):
        K = _f64(K)
        bias = _f64(bias)
        C_out, _, k, _ = K.shape
        mid = U32()
        _check(lib.vr_srv_register_conv_model(self.h, C_in, h, w, pad, K.ctypes.data, bias.ctypes.data,
                                              C_out, k, stride, 1 if square else 0, ctypes.byref(mid)))
        self._models[mid.value] = C_out * ((w + 2 * pad - k) // stride + 1)
        return mid.value

    def register_model(self, net):
        """A vr.CNN network (conv, x^2, FC); the network object is kept alive."""
        mid = U32()
        _check(lib.vr_srv_register_model(self.h, ctypes.byref(net.desc), ctypes.byref(mid)))
        self._models[mid.value] = net.outputs_per_set()
        self._nets = getattr(self, "_nets", []) + [net]
        return mid.value

    def submit(self, session, model, cols, n_images):
        t = U64()
        _check(lib.vr_srv_submit(self.h, session, model, _ptr_array(cols), len(cols), n_images,
                                 ctypes.byref(t)))
        return t.value

    def cancel(self, ticket):
        _check(lib.vr_srv_cancel(self.h, ticket))

    def poll(self, ticket, model, wait=True):
        """Output ciphertexts once done, else None."""
        cap = self._models[model]
        arr = (ctypes.c_void_p * cap)()
        n, ready = SZ(), ctypes.c_int()
        _check(lib.vr_srv_poll(self.h, ticket, 1 if wait else 0, arr, cap, ctypes.byref(n),
                               ctypes.byref(ready)))
        if not ready.value:
            return None
        return [Ciphertext(arr[i], self.ctx) for i in range(n.value)]

    def reset_stats(self):
        _check(lib.vr_srv_reset_stats(self.h))

    def stats(self):
        p50, p99, ips = DBL(), DBL(), DBL()
        done, waves, batched = U64(), U64(), U64()
        _check(lib.vr_srv_stats(self.h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(ips),
                                ctypes.byref(done), ctypes.byref(waves), ctypes.byref(batched)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "images_per_s": ips.value,
                "completed": done.value, "waves": waves.value, "batched": batched.value}


class CNN:
    """Network description (vr_cnn_desc): conv, optional x^2, optional FC."""

    def __init__(self, C_in, h, w, pad, K, bias, stride, square=True, fc_w=None, fc_bias=None,
                 fc_block=0):
        self.K, self.bias = _f64(K), _f64(bias)
        self.C_out, _, self.k, _ = self.K.shape
        self.C_in, self.h, self.w, self.pad, self.stride = C_in, h, w, pad, stride
        self.w_out = (w + 2 * pad - self.k) // stride + 1
        self.fc_w = list(fc_w) if fc_w is not None else None
        self.fc_bias = _f64(fc_bias) if fc_bias is not None else None
        self._fc_arr = _ptr_array(self.fc_w) if self.fc_w else None
        self.desc = vr_cnn_desc(C_in, h, w, pad, self.C_out, self.k, stride, self.K.ctypes.data,
                                self.bias.ctypes.data, 1 if square else 0,
                                ctypes.cast(self._fc_arr, ctypes.c_void_p) if self.fc_w else None,
                                self.fc_bias.ctypes.data if self.fc_w else None,
                                self.fc_bias.size if self.fc_w else 0, fc_block)

    def outputs_per_set(self):
        return self.fc_bias.size if self.fc_w else self.C_out * self.w_out

    def forward(self, ctx, keys, cols, n_sets=1, stream=None):
        n = n_sets * self.outputs_per_set()
        arr = (ctypes.c_void_p * n)()
        _check(lib.vr_cnn_forward(ctx.h, keys.ek, ctypes.byref(self.desc), _ptr_array(cols), n_sets, arr,
                                  _stream(stream)))
        return [Ciphertext(arr[i], ctx) for i in range(n)]


class Graph:
    """A network captured into a HIP graph (vr_graph_*)."""

    def __init__(self, ctx, keys, net, cols, n_sets=1):
        self.ctx, self.keys, self.net, self.n_sets = ctx, keys, net, n_sets
        h = ctypes.c_void_p()
        _check(lib.vr_graph_create(ctx.h, keys.ek, ctypes.byref(net.desc), _ptr_array(cols), n_sets,
                                   ctypes.byref(h)))
        self.h = h.value
        self.n_in = len(cols)

    def set_inputs(self, cols, stream=None):
        _check(lib.vr_graph_set_inputs(self.h, _ptr_array(cols), len(cols), _stream(stream)))

    def launch(self, stream=None):
        _check(lib.vr_graph_launch(self.h, _stream(stream)))

    def outputs(self):
        cap = self.n_sets * self.net.outputs_per_set()
        arr = (ctypes.c_void_p * cap)()
        n = SZ()
        _check(lib.vr_graph_outputs(self.h, arr, cap, ctypes.byref(n)))
        return [Ciphertext(arr[i], self.ctx) for i in range(n.value)]

    def close(self):
        if self.h:
            lib.vr_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Uneven batch of networks and products, run eagerly or as one HIP graph (vr_batch_*)."""

    def __init__(self, ctx, keys):
        self.ctx, self.keys = ctx, keys
        self._nets = []
        self._cap = []
        h = ctypes.c_void_p()
        _check(lib.vr_batch_create(ctx.h, keys.ek, ctypes.byref(h)))
        self.h = h.value

    def add_cnn(self, net, cols, n_sets=1):
        rid = U32()
        _check(lib.vr_batch_add_cnn(self.h, ctypes.byref(net.desc), _ptr_array(cols), n_sets, ctypes.byref(rid)))
        self._nets.append(net)          # the description's arrays must outlive the batch
        self._cap.append(n_sets * net.outputs_per_set())
        return rid.value

    def add_matmul(self, A, Bbar, m, n, p):
        rid = U32()
        _check(lib.vr_batch_add_matmul(self.h, _ptr_array(A), _ptr_array(Bbar), m, n, p, ctypes.byref(rid)))
        pp = 1
        while pp < min(m, p):
            pp <<= 1
        self._cap.append(pp)
        return rid.value

    def add_matmul_outer(self, A, B, m, n, p):
        rid = U32()
        _check(lib.vr_batch_add_matmul_outer(self.h, _ptr_array(A), _ptr_array(B), m, n, p,
                                             ctypes.byref(rid)))
        self._cap.append(self.ctx.outer_tiles(m, p)[2])
        return rid.value

    def run(self, stream=None):
        _check(lib.vr_batch_run(self.h, _stream(stream)))

    def capture(self):
        _check(lib.vr_batch_capture(self.h))

    def launch(self, stream=None):
        _check(lib.vr_batch_launch(self.h, _stream(stream)))

    def outputs(self, rid):
        cap = self._cap[rid]
        arr = (ctypes.c_void_p * cap)()
        n = SZ()
        _check(lib.vr_batch_outputs(self.h, rid, arr, cap, ctypes.byref(n)))
        return [Ciphertext(arr[i], self.ctx) for i in range(n.value)]

    def close(self):
        if self.h:
            lib.vr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
