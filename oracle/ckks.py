"""RNS-CKKS in the coefficient domain: the oracle's scheme layer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs CKKS through an HE library exposing KeyGen, Enc, Dec, Add, Mul,
cMul and a left rotation Rot(ct, l), with rescaling left implicit (section
"Fully Homomorphic Encryption" of the preliminaries).  It says nothing about
RNS limbs, NTTs, key switching or randomness; every such choice below is a
reading, named where it is made, so that two independent implementations
reach the same limbs:

  primes      largest q < 2^b with q = 1 mod 2N not taken yet, Q chain first
  roots       psi = g^((q-1)/2N) for the smallest g >= 2 with psi^N = -1
  security    sum of prime bit lengths <= 218 / 438 / 881 / 1740 for
              N = 2^13 / 2^14 / 2^15 / 2^16 (HE standard, ternary secret)
  randomness  ChaCha20 stream per (seed, purpose, object), the 256-bit seed
              being the key; fixed word positions per coefficient (no
              rejection), see ckks_oracle.c
  keys        hybrid key switching with dnum digits (Han & Ki, CT-RSA 2020),
              CRT-idempotent key form: b_j = -a_j s + e_j + [P]_{q_i} s' on the
              limbs of digit j
  ModUp       fast base conversion without correction, centred remainders;
              ModDown the same conversion of the P part, then (u - y) P^-1
  rotation    ModUp(c1), automorphism of every extended digit, inner product
              with the key of sigma_g(s), ModDown, plus sigma_g(c0)
  rescale     centred last limb, (c_i - [r]_{q_i}) * q_l^-1
  lazy ModDown  a product's relinearisation and its rescale, or a sum of
              scaled rotations and its rescale, end in one ModDown by P q_l:
              the operands stay P times a ciphertext over q_0..q_l, P
              (ExtCiphertext) and the centred conversion of their
              {q_l, p_0..p_{K-1}} limbs is divided out once
  encode      m_t = RHA((2*scale/N) Re sum_j z_j exp(-i pi g_j t / N)),
              g_j = 5^j mod 2N, via a 2N-point FFT; decode reads limb q_0
  constants   MulConst: RHA(c * dc) exactly as an integer; AddConst adds
              [RHA(c * scale)]_q to coefficient 0 of c_0

Parity status: every routine here is pinned by tests/test_oracle_*.py against
closed forms, brute force at tiny N (Python big integers), RFC 8439 vectors,
sympy primality, decryption invariants or FP64 plaintext layers.
"""
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from ._clib import lib, ptr, u64arr

# ----------------------------------------------------------------- parameters

_SECURITY = {13: 218, 14: 438, 15: 881, 16: 1740}


def security_bound(log_n):
    """Largest total modulus bit length for 128-bit classical security with a
    ternary secret (HE standard 2018 table; 2^16 conservatively 1740)."""
    return _SECURITY.get(log_n)


@dataclass
class Params:
    log_n: int
    q_bits: List[int]
    p_bits: List[int]
    dnum: int
    log2_scale: float
    sigma: float = 3.2
    allow_insecure: bool = False


PRESETS = {
    # A(16x16).B(16x16) matmul, N=2^13; q0 and p at 49 bits keep 218 bits.
    "C1": Params(13, [49, 40, 40, 40], [49], 4, 40.0),
    # the literal 60/40/40/40 + 60 chain: 240 bits, above the bound.
    "C1_literal": Params(13, [60, 40, 40, 40], [60], 4, 40.0, allow_insecure=True),
    # 28x28 conv layer at N=2^14, L=7.
    "C2": Params(14, [60] + [40] * 7, [60], 8, 40.0),
    # 128x128x3 CNN at N=2^16, L=24, dnum=3.
    "C3": Params(16, [60] + [50] * 24, [51] * 9, 3, 50.0),
}


def is_prime(n):
    return bool(lib.orc_is_prime(n))


def gen_primes(log_n, bits_list):
    """For each bit size in order: the largest prime q < 2^b, q = 1 mod 2N,
    not taken yet."""
    two_n = 1 << (log_n + 1)
    taken = []
    for b in bits_list:
        c = ((1 << b) - 1) // two_n * two_n + 1
        while c >= (1 << (b - 1)):
            if c not in taken and is_prime(c):
                break
            c -= two_n
        else:
            raise ValueError("no NTT prime of %d bits for N=2^%d" % (b, log_n))
        taken.append(c)
    return taken


def find_psi(q, log_n):
    """psi = g^((q-1)/2N) mod q for the smallest g >= 2 with psi^N = -1."""
    n = 1 << log_n
    assert (q - 1) % (2 * n) == 0
    g = 2
    while True:
        psi = pow(g, (q - 1) // (2 * n), q)
        if pow(psi, n, q) == q - 1:
            return psi
        g += 1


def cdt_table(sigma=3.2, tail=19):
    """T[k] = floor(2^63 F(k)), F(k) = sum_{|y|<=k} rho(y) / sum_{|y|<=tail} rho(y),
    rho(y) = exp(-y^2 / 2 sigma^2); T[tail] = 2^63.  60-digit arithmetic."""
    import mpmath
    with mpmath.workdps(60):
        s = mpmath.mpf(str(sigma))
        rho = [mpmath.exp(-mpmath.mpf(y * y) / (2 * s * s)) for y in range(tail + 1)]
        cum = []
        acc = mpmath.mpf(0)
        for k in range(tail + 1):
            acc += rho[k] if k == 0 else 2 * rho[k]
            cum.append(acc)
        total = cum[-1]
        t = [int(mpmath.floor(mpmath.mpf(2) ** 63 * cum[k] / total)) for k in range(tail)]
    return t + [1 << 63]


def rha(x):
    """Round half away from zero of a double, returned as an exact Python int."""
    t = math.trunc(x)
    if abs(x - t) >= 0.5:
        t += 1 if x > 0 else -1
    return int(t)


def rha_array(x):
    x = np.asarray(x, dtype=np.float64)
    t = np.trunc(x)
    return t + np.sign(x) * (np.abs(x - t) >= 0.5)


def pow2ceil(x):
    p = 1
    while p < x:
        p *= 2
    return p


# randomness purposes (nonce word 0)
PUR_SK, PUR_PK_A, PUR_PK_E, PUR_SWK_A, PUR_SWK_E, PUR_ENC_V, PUR_ENC_E0, PUR_ENC_E1 = range(1, 9)

# ------------------------------------------------------------------- objects


@dataclass
class Plaintext:
    m: np.ndarray          # [level+1, N] uint64, coefficient domain
    level: int
    scale: float


@dataclass
class Ciphertext:
    c: np.ndarray          # [ncomp, level+1, N] uint64, coefficient domain
    level: int
    scale: float

    @property
    def ncomp(self):
        return self.c.shape[0]


@dataclass
class ExtCiphertext:
    """P times a 2-component ciphertext, over q_0..q_level, p_0..p_{K-1}
    (coefficient domain): a key switch before its ModDown, on which linear
    operations continue until one ModDown by P q_level.  `scale` is the scale
    of the ciphertext it stands for (P is implicit)."""
    c: np.ndarray          # [2, level+1+K, N] uint64
    level: int
    scale: float


@dataclass
class SwitchingKey:
    """Digits j = 0..dnum-1; b[j], a[j] are [L+1+K, N] (q_0..q_L then p_0..p_{K-1})."""
    b: List[np.ndarray]
    a: List[np.ndarray]
    _ntt: Dict = field(default_factory=dict, repr=False)


@dataclass
class Keys:
    s: np.ndarray          # int64 ternary coefficients (secret: client side)
    pk_b: np.ndarray       # [L+1, N]
    pk_a: np.ndarray
    rlk: SwitchingKey
    rot: Dict[int, SwitchingKey]   # Galois element -> key


# ------------------------------------------------------------------- context


class Context:
    def __init__(self, params: Params):
        self.params = params
        self.log_n = params.log_n
        self.n = 1 << params.log_n
        self.slots = self.n // 2
        self.q = gen_primes(params.log_n, list(params.q_bits) + list(params.p_bits))
        self.p = self.q[len(params.q_bits):]
        self.q = self.q[:len(params.q_bits)]
        self.L = len(self.q) - 1
        self.K = len(self.p)
        self.dnum = params.dnum
        self.alpha = -(-(self.L + 1) // params.dnum)
        self.scale = 2.0 ** params.log2_scale
        bound = security_bound(params.log_n)
        total = sum(x.bit_length() for x in self.q + self.p)
        self.total_bits = total
        self.secure = bound is not None and total <= bound
        if not self.secure and not params.allow_insecure:
            raise ValueError("parameters exceed the 128-bit bound (%d bits)" % total)
        self.cdt = np.array(cdt_table(params.sigma), dtype=np.uint64)
        self._tables = {}
        # slot index j <-> Galois exponent g_j = 5^j mod 2N
        two_n = 2 * self.n
        self.gexp = np.zeros(self.slots, dtype=np.int64)
        g = 1
        for j in range(self.slots):
            self.gexp[j] = g
            g = g * 5 % two_n

    # ---------------------------------------------------------- limb helpers
    def _tab(self, q):
        if q not in self._tables:
            fwd = np.zeros(self.n, dtype=np.uint64)
            inv = np.zeros(self.n, dtype=np.uint64)
            lib.orc_ntt_tables(self.log_n, q, find_psi(q, self.log_n), ptr(fwd), ptr(inv))
            self._tables[q] = (fwd, inv)
        return self._tables[q]

    def ntt(self, a, q):
        out = u64arr(a).copy()
        lib.orc_ntt(ptr(out), self.log_n, q, ptr(self._tab(q)[0]))
        return out

    def intt(self, a, q):
        out = u64arr(a).copy()
        lib.orc_intt(ptr(out), self.log_n, q, ptr(self._tab(q)[1]))
        return out

    def polymul(self, a, b, q):
        """Negacyclic product of two limbs modulo q."""
        a, b = u64arr(a), u64arr(b)
        out = np.empty(self.n, dtype=np.uint64)
        scratch = np.empty(self.n, dtype=np.uint64)
        fwd, inv = self._tab(q)
        lib.orc_poly_mul(ptr(a), ptr(b), ptr(out), self.log_n, q, ptr(fwd), ptr(inv), ptr(scratch))
        return out

    @staticmethod
    def vadd(a, b, q):
        a, b = u64arr(a), u64arr(b)
        out = np.empty_like(a)
        lib.orc_vec_add(ptr(a), ptr(b), ptr(out), a.size, q)
        return out

    @staticmethod
    def vsub(a, b, q):
        a, b = u64arr(a), u64arr(b)
        out = np.empty_like(a)
        lib.orc_vec_sub(ptr(a), ptr(b), ptr(out), a.size, q)
        return out

    @staticmethod
    def vneg(a, q):
        a = u64arr(a)
        out = np.empty_like(a)
        lib.orc_vec_neg(ptr(a), ptr(out), a.size, q)
        return out

    @staticmethod
    def vmul(a, b, q):
        a, b = u64arr(a), u64arr(b)
        out = np.empty_like(a)
        lib.orc_vec_mul(ptr(a), ptr(b), ptr(out), a.size, q)
        return out

    @staticmethod
    def vscale(a, c, q):
        a = u64arr(a)
        out = np.empty_like(a)
        lib.orc_vec_mul_scalar(ptr(a), int(c) % q, ptr(out), a.size, q)
        return out

    @staticmethod
    def reduce_int(x, q):
        """[x]_q for an int64 coefficient vector."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
        out = np.empty(x.shape, dtype=np.uint64)
        lib.orc_vec_reduce_i64(ptr(x), ptr(out), x.size, q)
        return out

    def automorphism(self, a, g, q):
        a = u64arr(a)
        out = np.empty_like(a)
        lib.orc_automorphism(ptr(a), ptr(out), self.log_n, g, q)
        return out

    def base_convert(self, limbs, q_in, q_out):
        """Fast base conversion (no correction) of one polynomial's limbs."""
        src = u64arr(limbs).reshape(len(q_in), self.n)
        out = np.empty((len(q_out), self.n), dtype=np.uint64)
        qi, qo = u64arr(q_in), u64arr(q_out)
        lib.orc_base_convert(ptr(src), len(q_in), ptr(qi), ptr(out), len(q_out), ptr(qo), self.n)
        return out

    def moduli(self, level):
        return self.q[:level + 1]

    def ext_moduli(self, level):
        return self.q[:level + 1] + self.p

    def galois_element(self, step):
        """g = 5^(step mod S) mod 2N: left rotation by `step` slots."""
        return pow(5, step % self.slots, 2 * self.n)

    # ------------------------------------------------------------- sampling
    @staticmethod
    def seed_words(seed):
        """The 256-bit ChaCha20 key as four little-endian 64-bit words
        (a seed below 2^64 leaves the upper words zero)."""
        seed = int(seed)
        if not 0 <= seed < 1 << 256:
            raise ValueError("seed must be a 256-bit non-negative integer")
        return np.array([(seed >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(4)], dtype=np.uint64)

    def stream_words(self, seed, purpose, obj, first, count):
        out, key = np.empty(count, dtype=np.uint64), self.seed_words(seed)
        lib.orc_stream_words(ptr(key), purpose, obj, first, count, ptr(out))
        return out

    def sample_ternary(self, seed, purpose, obj):
        out, key = np.empty(self.n, dtype=np.int64), self.seed_words(seed)
        lib.orc_sample_ternary(ptr(key), purpose, obj, self.n, ptr(out))
        return out

    def sample_gauss(self, seed, purpose, obj):
        out, key = np.empty(self.n, dtype=np.int64), self.seed_words(seed)
        lib.orc_sample_gauss(ptr(key), purpose, obj, self.n, ptr(self.cdt), ptr(out))
        return out

    def sample_uniform(self, seed, purpose, obj, limb, q):
        out, key = np.empty(self.n, dtype=np.uint64), self.seed_words(seed)
        lib.orc_sample_uniform(ptr(key), purpose, obj, limb, self.log_n, q, ptr(out))
        return out

    # --------------------------------------------------------------- keygen
    def _int_poly_limbs(self, x, moduli):
        return np.stack([self.reduce_int(x, q) for q in moduli])

    def _ring_mul_int(self, limbs, x, moduli):
        """limb-wise negacyclic product of an RNS polynomial with an integer one."""
        return np.stack([self.polymul(limbs[i], self.reduce_int(x, q), q)
                         for i, q in enumerate(moduli)])

    def digit(self, j, level=None):
        """Q-limb indices of digit j at `level` (all of it at the top level)."""
        top = self.L if level is None else level
        lo, hi = j * self.alpha, min((j + 1) * self.alpha, self.L + 1)
        return [i for i in range(lo, hi) if i <= top]

    def n_digits(self, level):
        return -(-(level + 1) // self.alpha)

    def gen_switching_key(self, seed, s, s_prime_limbs, g):
        """Key from s' (limbs over q_0..q_L, p_0..p_{K-1}) to s; object id g*64 + j."""
        ext = self.q + self.p
        P = 1
        for pk in self.p:
            P *= pk
        bs, as_ = [], []
        for j in range(self.dnum):
            obj = g * 64 + j
            a = np.stack([self.sample_uniform(seed, PUR_SWK_A, obj, i, q) for i, q in enumerate(ext)])
            e = self.sample_gauss(seed, PUR_SWK_E, obj)
            b = np.empty_like(a)
            dj = set(self.digit(j))
            for i, q in enumerate(ext):
                v = self.vsub(self.reduce_int(e, q), self.polymul(a[i], self.reduce_int(s, q), q), q)
                if i in dj:   # Q limb of this digit: + [P]_{q_i} s'
                    v = self.vadd(v, self.vscale(s_prime_limbs[i], P % q, q), q)
                b[i] = v
            bs.append(b)
            as_.append(a)
        return SwitchingKey(bs, as_)

    def keygen(self, seed, rot_steps=()):
        ext = self.q + self.p
        s = self.sample_ternary(seed, PUR_SK, 0)
        pa = np.stack([self.sample_uniform(seed, PUR_PK_A, 0, i, q) for i, q in enumerate(self.q)])
        pe = self.sample_gauss(seed, PUR_PK_E, 0)
        pb = np.stack([self.vsub(self.reduce_int(pe, q), self.polymul(pa[i], self.reduce_int(s, q), q), q)
                       for i, q in enumerate(self.q)])
        s_limbs = self._int_poly_limbs(s, ext)
        s2 = np.stack([self.polymul(s_limbs[i], s_limbs[i], q) for i, q in enumerate(ext)])
        rlk = self.gen_switching_key(seed, s, s2, 0)
        rot = {}
        for r in rot_steps:
            g = self.galois_element(r)
            if g in rot or g == 1:
                continue
            sg = np.stack([self.automorphism(s_limbs[i], g, q) for i, q in enumerate(ext)])
            rot[g] = self.gen_switching_key(seed, s, sg, g)
        return Keys(s, pb, pa, rlk, rot)

    # -------------------------------------------------------- encode/decode
    def encode_int(self, z, scale, sub_log=0):
        """Integer coefficients m_t (int64) of the slot vector z (real, length <= S).
        sub_log > 0: z repeats with period S / 2^sub_log, so in exact arithmetic
        the polynomial lies in Z[X^(2^sub_log)]; the coefficients off that
        subring (rounding noise of the FFT) are set to zero before rounding."""
        z = np.zeros(self.slots) if z is None else np.asarray(z, dtype=np.float64)
        zz = np.zeros(self.slots)
        zz[:len(z)] = z
        w = np.zeros(2 * self.n, dtype=np.complex128)
        w[self.gexp] = zz
        f = np.fft.fft(w)[:self.n]
        re = f.real.copy()
        if sub_log:
            re[np.arange(self.n) % (1 << sub_log) != 0] = 0.0
        m = rha_array((2.0 * scale / self.n) * re)
        if np.any(np.abs(m) >= 2.0 ** 62):
            raise ValueError("encoded coefficient out of range")
        return m.astype(np.int64)

    def encode(self, z, level, scale, sub_log=0):
        m = self.encode_int(z, scale, sub_log)
        return Plaintext(self._int_poly_limbs(m, self.moduli(level)), level, float(scale))

    def decode(self, pt: Plaintext, n=None):
        q0 = self.q[0]
        c = pt.m[0].astype(np.int64)            # q_0 < 2^63
        cen = np.where(c > q0 // 2, c - q0, c).astype(np.float64)
        w = np.zeros(2 * self.n, dtype=np.float64)
        w[:self.n] = cen
        f = np.fft.fft(w)
        z = f.real[self.gexp] / pt.scale
        return z if n is None else z[:n]

    # ------------------------------------------------------ encrypt/decrypt
    def encrypt(self, keys: Keys, pt: Plaintext, seed, ct_id):
        lv = pt.level
        v = self.sample_ternary(seed, PUR_ENC_V, ct_id)
        e0 = self.sample_gauss(seed, PUR_ENC_E0, ct_id)
        e1 = self.sample_gauss(seed, PUR_ENC_E1, ct_id)
        c = np.empty((2, lv + 1, self.n), dtype=np.uint64)
        for i, q in enumerate(self.moduli(lv)):
            vq = self.reduce_int(v, q)
            c[0, i] = self.vadd(self.vadd(self.polymul(vq, keys.pk_b[i], q), self.reduce_int(e0, q), q),
                                pt.m[i], q)
            c[1, i] = self.vadd(self.polymul(vq, keys.pk_a[i], q), self.reduce_int(e1, q), q)
        return Ciphertext(c, lv, pt.scale)

    def decrypt(self, keys: Keys, ct: Ciphertext):
        m = np.empty((ct.level + 1, self.n), dtype=np.uint64)
        for i, q in enumerate(self.moduli(ct.level)):
            sq = self.reduce_int(keys.s, q)
            acc = ct.c[0, i]
            spow = sq
            for k in range(1, ct.ncomp):
                acc = self.vadd(acc, self.polymul(ct.c[k, i], spow, q), q)
                spow = self.polymul(spow, sq, q)
            m[i] = acc
        return Plaintext(m, ct.level, ct.scale)

    # ------------------------------------------------------------ basic ops
    @staticmethod
    def _check_pair(a, b):
        if a.level != b.level:
            raise ValueError("level mismatch")
        if a.scale != b.scale:
            raise ValueError("scale mismatch")

    def add(self, a: Ciphertext, b: Ciphertext):
        self._check_pair(a, b)
        nc = max(a.ncomp, b.ncomp)
        c = np.zeros((nc, a.level + 1, self.n), dtype=np.uint64)
        for k in range(nc):
            for i, q in enumerate(self.moduli(a.level)):
                x = a.c[k, i] if k < a.ncomp else np.zeros(self.n, np.uint64)
                y = b.c[k, i] if k < b.ncomp else np.zeros(self.n, np.uint64)
                c[k, i] = self.vadd(x, y, q)
        return Ciphertext(c, a.level, a.scale)

    def sub(self, a: Ciphertext, b: Ciphertext):
        self._check_pair(a, b)
        nc = max(a.ncomp, b.ncomp)
        c = np.zeros((nc, a.level + 1, self.n), dtype=np.uint64)
        for k in range(nc):
            for i, q in enumerate(self.moduli(a.level)):
                x = a.c[k, i] if k < a.ncomp else np.zeros(self.n, np.uint64)
                y = b.c[k, i] if k < b.ncomp else np.zeros(self.n, np.uint64)
                c[k, i] = self.vsub(x, y, q)
        return Ciphertext(c, a.level, a.scale)

    def mul_const(self, a: Ciphertext, value, const_scale):
        """cMul by a scalar: C = RHA(value * const_scale) (exact integer)."""
        C = rha(float(value) * float(const_scale))
        c = np.empty_like(a.c)
        for k in range(a.ncomp):
            for i, q in enumerate(self.moduli(a.level)):
                c[k, i] = self.vscale(a.c[k, i], C % q, q)
        return Ciphertext(c, a.level, a.scale * float(const_scale))

    def add_const(self, a: Ciphertext, value):
        C = rha(float(value) * a.scale)
        c = a.c.copy()
        for i, q in enumerate(self.moduli(a.level)):
            c[0, i, 0] = (int(c[0, i, 0]) + C % q) % q
        return Ciphertext(c, a.level, a.scale)

    def mul_plain(self, a: Ciphertext, pt: Plaintext):
        if pt.level < a.level:
            raise ValueError("plaintext level below ciphertext level")
        c = np.empty_like(a.c)
        for k in range(a.ncomp):
            for i, q in enumerate(self.moduli(a.level)):
                c[k, i] = self.polymul(a.c[k, i], pt.m[i], q)
        return Ciphertext(c, a.level, a.scale * pt.scale)

    def tensor(self, a: Ciphertext, b: Ciphertext):
        if a.level != b.level:
            raise ValueError("level mismatch")
        assert a.ncomp == 2 and b.ncomp == 2
        c = np.empty((3, a.level + 1, self.n), dtype=np.uint64)
        for i, q in enumerate(self.moduli(a.level)):
            c[0, i] = self.polymul(a.c[0, i], b.c[0, i], q)
            c[1, i] = self.vadd(self.polymul(a.c[0, i], b.c[1, i], q),
                                self.polymul(a.c[1, i], b.c[0, i], q), q)
            c[2, i] = self.polymul(a.c[1, i], b.c[1, i], q)
        return Ciphertext(c, a.level, a.scale * b.scale)

    def mod_drop(self, a: Ciphertext, level):
        if level > a.level:
            raise ValueError("cannot raise the level")
        return Ciphertext(a.c[:, :level + 1].copy(), level, a.scale)

    def rescale(self, a: Ciphertext):
        lv = a.level
        if lv == 0:
            raise ValueError("no limb left to rescale by")
        ql = self.q[lv]
        c = np.empty((a.ncomp, lv, self.n), dtype=np.uint64)
        for k in range(a.ncomp):
            for i in range(lv):
                out = np.empty(self.n, dtype=np.uint64)
                lib.orc_rescale_limb(ptr(u64arr(a.c[k, i])), ptr(u64arr(a.c[k, lv])), ptr(out),
                                     self.n, self.q[i], ql)
                c[k, i] = out
        return Ciphertext(c, lv - 1, a.scale / float(ql))

    # -------------------------------------------------------- key switching
    def mod_up(self, d, level, j):
        """Digit j of d (limbs q_0..q_level) extended to q_0..q_level, p_0..p_{K-1}."""
        dj = self.digit(j, level)
        ext = self.ext_moduli(level)
        targets = [e for e in range(len(ext)) if e not in dj]
        conv = self.base_convert(d[dj], [self.q[i] for i in dj], [ext[e] for e in targets])
        x = np.empty((len(ext), self.n), dtype=np.uint64)
        for i in dj:
            x[i] = d[i]
        for r, e in enumerate(targets):
            x[e] = conv[r]
        return x

    def _key_limb(self, key: SwitchingKey, j, which, e, level):
        """NTT of key digit j limb for extended index e at `level` (cached)."""
        idx = e if e <= level else self.L + 1 + (e - level - 1)
        ck = (j, which, idx)
        if ck not in key._ntt:
            arr = key.b[j] if which == 0 else key.a[j]
            key._ntt[ck] = self.ntt(arr[idx], (self.q + self.p)[idx])
        return key._ntt[ck]

    def inner_product(self, xs, key: SwitchingKey, level):
        """(u0, u1) = sum_j x^(j) * (b_j, a_j) over q_0..q_level, p_0..p_{K-1}."""
        ext = self.ext_moduli(level)
        u = np.empty((2, len(ext), self.n), dtype=np.uint64)
        for e, q in enumerate(ext):
            acc0 = np.zeros(self.n, dtype=np.uint64)
            acc1 = np.zeros(self.n, dtype=np.uint64)
            for j, x in enumerate(xs):
                X = self.ntt(x[e], q)   # products in the evaluation domain, summed there
                acc0 = self.vadd(acc0, self.vmul(X, self._key_limb(key, j, 0, e, level), q), q)
                acc1 = self.vadd(acc1, self.vmul(X, self._key_limb(key, j, 1, e, level), q), q)
            u[0, e] = self.intt(acc0, q)
            u[1, e] = self.intt(acc1, q)
        return u

    def mod_down(self, u, level):
        """(u_i - conv_P->q_i(u_P)) * P^-1 mod q_i for i <= level."""
        nq = level + 1
        y = self.base_convert(u[nq:], self.p, self.moduli(level))
        out = np.empty((nq, self.n), dtype=np.uint64)
        for i, q in enumerate(self.moduli(level)):
            P = 1
            for pk in self.p:
                P = P * pk % q
            out[i] = self.vscale(self.vsub(u[i], y[i], q), pow(P, q - 2, q), q)
        return out

    def key_switch(self, d, key: SwitchingKey, level, galois=None):
        xs = [self.mod_up(d, level, j) for j in range(self.n_digits(level))]
        if galois is not None:
            ext = self.ext_moduli(level)
            xs = [np.stack([self.automorphism(x[e], galois, q) for e, q in enumerate(ext)]) for x in xs]
        u = self.inner_product(xs, key, level)
        return self.mod_down(u[0], level), self.mod_down(u[1], level)

    def relinearize(self, a: Ciphertext, keys: Keys):
        if a.ncomp == 2:
            return a
        lv = a.level
        o0, o1 = self.key_switch(a.c[2], keys.rlk, lv)
        c = np.empty((2, lv + 1, self.n), dtype=np.uint64)
        for i, q in enumerate(self.moduli(lv)):
            c[0, i] = self.vadd(a.c[0, i], o0[i], q)
            c[1, i] = self.vadd(a.c[1, i], o1[i], q)
        return Ciphertext(c, lv, a.scale)

    def mul(self, a, b, keys):
        return self.relinearize(self.tensor(a, b), keys)

    # ------------------------------------------------ lazy ModDown (P basis)
    def p_mod(self, q):
        P = 1
        for pk in self.p:
            P = P * pk % q
        return P

    def lift(self, a: Ciphertext):
        """P a over q_0..q_l, P: P c_i on the Q limbs, zero on the special
        limbs (P vanishes there)."""
        assert a.ncomp == 2
        lv = a.level
        c = np.zeros((2, lv + 1 + self.K, self.n), dtype=np.uint64)
        for k in range(2):
            for i, q in enumerate(self.moduli(lv)):
                c[k, i] = self.vscale(a.c[k, i], self.p_mod(q), q)
        return ExtCiphertext(c, lv, a.scale)

    def rotate_ext(self, a: Ciphertext, step, keys: Keys):
        """Rotation without its ModDown: (u0 + P sigma_g(c0), u1) with (u0, u1)
        the key-switch sums of sigma_g(ModUp(c1)) -- mod_down_rescale of it is
        the rescaled rotation up to one rounding."""
        assert a.ncomp == 2
        g = self.galois_element(step)
        if g == 1:
            return self.lift(a)
        if g not in keys.rot:
            raise KeyError("no rotation key for step %d" % step)
        lv = a.level
        ext = self.ext_moduli(lv)
        xs = [self.mod_up(a.c[1], lv, j) for j in range(self.n_digits(lv))]
        xs = [np.stack([self.automorphism(x[e], g, q) for e, q in enumerate(ext)]) for x in xs]
        u = self.inner_product(xs, keys.rot[g], lv)
        for i, q in enumerate(self.moduli(lv)):
            u[0, i] = self.vadd(u[0, i], self.vscale(self.automorphism(a.c[0, i], g, q), self.p_mod(q), q), q)
        return ExtCiphertext(u, lv, a.scale)

    def rotate_many_ext(self, a, steps, keys):
        return [self.rotate_ext(a, r, keys) for r in steps]

    def mul_const_ext(self, e: ExtCiphertext, value, const_scale):
        """MulConst on every limb of the extended basis: C = RHA(value
        const_scale) reduced modulo each q_i and p_k."""
        C = rha(float(value) * float(const_scale))
        c = np.empty_like(e.c)
        for k in range(2):
            for i, q in enumerate(self.ext_moduli(e.level)):
                c[k, i] = self.vscale(e.c[k, i], C % q, q)
        return ExtCiphertext(c, e.level, e.scale * float(const_scale))

    def add_ext(self, a: ExtCiphertext, b: ExtCiphertext):
        if a.level != b.level:
            raise ValueError("level mismatch")
        if abs(a.scale - b.scale) > 1e-9 * a.scale:
            raise ValueError("scale mismatch")
        c = np.empty_like(a.c)
        for k in range(2):
            for i, q in enumerate(self.ext_moduli(a.level)):
                c[k, i] = self.vadd(a.c[k, i], b.c[k, i], q)
        return ExtCiphertext(c, a.level, a.scale)

    def add_const_ext(self, e: ExtCiphertext, value):
        """AddConst of P times the ciphertext: P [RHA(value scale)]_q added to
        coefficient 0 of c0 on the Q limbs."""
        C = rha(float(value) * e.scale)
        c = e.c.copy()
        for i, q in enumerate(self.moduli(e.level)):
            c[0, i, 0] = (int(c[0, i, 0]) + (C % q) * self.p_mod(q)) % q
        return ExtCiphertext(c, e.level, e.scale)

    def mod_down_rescale(self, e: ExtCiphertext):
        """ModDown by P q_l: each component v is divided by P q_l with the
        centred fast conversion ModDown uses, from the drop set {q_l, p_0..
        p_{K-1}} to q_0..q_{l-1}:
            out_i = (v_i - conv(v_D)_i) (P q_l)^-1 mod q_i,   i < l.
        Level l - 1, scale / q_l as for rescale.  Of a lifted ciphertext it is
        exactly the rescale."""
        lv = e.level
        if lv == 0:
            raise ValueError("no limb left to rescale by")
        nq = lv + 1
        drop = [self.q[lv]] + list(self.p)
        c = np.empty((2, lv, self.n), dtype=np.uint64)
        for comp in range(2):
            v = e.c[comp]
            vD = np.stack([v[lv]] + [v[nq + k] for k in range(self.K)])
            y = self.base_convert(vD, drop, self.q[:lv])
            for i in range(lv):
                q = self.q[i]
                inv = pow(self.p_mod(q) * self.q[lv] % q, q - 2, q)
                c[comp, i] = self.vscale(self.vsub(v[i], y[i], q), inv, q)
        return Ciphertext(c, lv - 1, e.scale / float(self.q[lv]))

    def relin_rescale(self, a: Ciphertext, keys: Keys):
        """Relinearisation and rescale as one ModDown by P q_l: with (u0, u1)
        the key-switch sums of c2 over q_0..q_l, p_0..p_{K-1}, the extended
        ciphertext u + P (c0, c1) goes through mod_down_rescale.  It equals
        rescale(relinearize(a)) up to a rounding difference of the division
        (not limb for limb)."""
        assert a.ncomp == 3
        lv = a.level
        if lv == 0:
            raise ValueError("no limb left to rescale by")
        xs = [self.mod_up(a.c[2], lv, j) for j in range(self.n_digits(lv))]
        u = self.inner_product(xs, keys.rlk, lv)
        lifted = self.lift(Ciphertext(a.c[:2], lv, a.scale))
        v = self.add_ext(ExtCiphertext(u, lv, a.scale), lifted)
        return self.mod_down_rescale(v)

    def rotate(self, a: Ciphertext, step, keys: Keys):
        """Left rotation of the slots by `step`."""
        assert a.ncomp == 2
        g = self.galois_element(step)
        if g == 1:
            return Ciphertext(a.c.copy(), a.level, a.scale)
        if g not in keys.rot:
            raise KeyError("no rotation key for step %d" % step)
        lv = a.level
        o0, o1 = self.key_switch(a.c[1], keys.rot[g], lv, galois=g)
        c = np.empty((2, lv + 1, self.n), dtype=np.uint64)
        for i, q in enumerate(self.moduli(lv)):
            c[0, i] = self.vadd(self.automorphism(a.c[0, i], g, q), o0[i], q)
            c[1, i] = o1[i]
        return Ciphertext(c, lv, a.scale)

    def rotate_many(self, a, steps, keys):
        """Hoisted rotations are bit-identical to single ones by construction."""
        return [self.rotate(a, r, keys) for r in steps]
