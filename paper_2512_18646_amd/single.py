"""The paper's single-ciphertext schedules on the library's per-operation
calls: the homomorphic matrix product (Algorithm 3, with RowShifter of
Algorithm 2 and SumColVec), SumForConv (Algorithm 1), Kernelspanner and the
homomorphic convolution (Algorithm 4), and the virtual rotation vRot
(Algorithm 5).  This is the prior method the column-wise encodings replace
when an image or matrix fits one ciphertext.

Every arithmetic step is one C-ABI call (vr_rotate, vr_mul_plain,
vr_mul_rescale, vr_rescale, vr_add, vr_mod_drop); this module only builds the
0/1 masks and
chooses the calls.  Layout: an r x c matrix is packed row-major into r c
slots and that block is repeated over the S slots (r c a power of two), so a
rotation of the ciphertext acts cyclically on every copy.  Masks are encoded
at scale q_l of the ciphertext's level and followed by a rescale, so they
keep the scale.

Schedule choices where the paper's listing is ambiguous:
  * RowShifter(ct.Bbar, p, idx) shifts Bbar by idx rows from the original
    ciphertext: Rot(ct, idx n) on the first m - idx rows, Rot(ct, n (idx - m +
    m mod p)) on the last idx rows, one rotation when p divides m, none at
    idx = 0; ct.A then drops one level so that every iteration's product is
    rescaled by the same prime.
  * SumColVec: rotate-and-sum left over the n columns, keep column 0, then
    rotate-and-sum right (2 log2 n rotations).
  * mask F[i][(i + idx) mod p]; Algorithm 4's offset mask (hth - a) mod k =
    (wth - b) mod k = 0 inside the valid region; the window sum rotates the
    column-summed partial for its row pass.
`encode` and `encrypt` hooks let a caller supply the plaintexts and fresh
ciphertexts (by default the library's own encoder and public-key encryption).
"""
import numpy as np


def _pow2(x):
    return x >= 1 and (x & (x - 1)) == 0


def tile(block, S):
    block = np.asarray(block, np.float64).reshape(-1)
    if S % block.size:
        raise ValueError("the packed block must divide the slot count")
    return np.tile(block, S // block.size)


def pack_a(A):
    """tau_a: A row-major."""
    return np.asarray(A, np.float64).reshape(-1)


def pack_bbar(B, m):
    """tau_b: row i of Bbar (m x n) is column i mod p of B."""
    B = np.asarray(B, np.float64)
    n, p = B.shape
    return np.stack([B[:, i % p] for i in range(m)]).reshape(-1)


class Ops:
    """The per-operation calls a schedule issues, with level alignment."""

    def __init__(self, ctx, keys, encode=None, encrypt=None, stream=None):
        self.ctx, self.keys, self.stream = ctx, keys, stream
        self.S = ctx.slots
        self._encode = encode or (lambda vec, level, scale: ctx.encode(vec, level, scale))
        self._encrypt = encrypt
        self.calls = 0

    def rot(self, ct, r):
        r %= self.S
        if r == 0:
            return ct
        self.calls += 1
        return self.ctx.rotate(self.keys, ct, r, stream=self.stream)

    def _level(self, a, b):
        lv = min(a.level, b.level)
        if a.level > lv:
            a = self.ctx.mod_drop(a, lv, stream=self.stream)
        if b.level > lv:
            b = self.ctx.mod_drop(b, lv, stream=self.stream)
        return a, b

    def add(self, a, b):
        a, b = self._level(a, b)
        self.calls += 1
        return self.ctx.add(a, b, stream=self.stream)

    def drop(self, ct, levels):
        return self.ctx.mod_drop(ct, ct.level - levels, stream=self.stream) if levels else ct

    def cmul(self, mask, ct):
        lv = ct.level
        pt = self._encode(np.asarray(mask, np.float64), lv, float(self.ctx.q[lv]))
        self.calls += 2
        return self.ctx.rescale(self.ctx.mul_plain(ct, pt, stream=self.stream), stream=self.stream)

    def mul(self, a, b):
        a, b = self._level(a, b)
        self.calls += 1
        return self.ctx.mul_rescale(self.keys, a, b, stream=self.stream)

    def enc(self, vec, like):
        if self._encrypt is None:
            raise ValueError("a fresh encryption needs the client's encrypt hook")
        return self._encrypt(np.asarray(vec, np.float64), like.level, like.scale)


def _rows_mask(m, n, rows, S):
    F = np.zeros((m, n))
    F[list(rows)] = 1.0
    return tile(F, S)


def row_shifter(ops, ct_B, m, n, p, idx):
    if idx == 0:
        return ct_B
    a, b = idx * n, n * (idx - m + m % p)
    if (a - b) % (m * n) == 0:
        return ops.rot(ct_B, a)
    upper = ops.cmul(_rows_mask(m, n, range(m - idx), ops.S), ops.rot(ct_B, a))
    lower = ops.cmul(_rows_mask(m, n, range(m - idx, m), ops.S), ops.rot(ct_B, b))
    return ops.add(upper, lower)


def sum_col_vec(ops, ct, m, n):
    t, s = ct, 1
    while s < n:
        t = ops.add(t, ops.rot(t, s))
        s <<= 1
    first = np.zeros((m, n))
    first[:, 0] = 1.0
    t = ops.cmul(tile(first, ops.S), t)
    s = 1
    while s < n:
        t = ops.add(t, ops.rot(t, -s))
        s <<= 1
    return t


def matmul(ops, ct_A, ct_B, m, n, p):
    """Algorithm 3: slot i n + j of the result holds (A B)[i][j], j < p."""
    if p > n or not _pow2(m * n) or not _pow2(n):
        raise ValueError("needs p <= n and powers of two m n and n")
    if m % p:
        ct_A = ops.drop(ct_A, 1)
    acc = None
    for idx in range(p):
        T = ops.mul(ct_A, row_shifter(ops, ct_B, m, n, p, idx))
        T = sum_col_vec(ops, T, m, n)
        F = np.zeros((m, n))
        F[np.arange(m), (np.arange(m) + idx) % p] = 1.0
        T = ops.cmul(tile(F, ops.S), T)
        if acc is None:
            acc = ops.enc(np.zeros(ops.S), like=T)
        acc = ops.add(acc, T)
    return acc


def window_sum(ops, ct, w, k):
    cols = ct
    for d in range(1, k):
        cols = ops.add(cols, ops.rot(ct, d))
    box = cols
    for d in range(1, k):
        box = ops.add(box, ops.rot(cols, d * w))
    return box


def sum_for_conv(ops, ct, h, w, k, k0):
    valid = np.zeros((h, w))
    valid[:h - k + 1, :w - k + 1] = 1.0
    t = ops.cmul(tile(valid, ops.S), window_sum(ops, ct, w, k))
    return ops.add(ops.enc(tile(k0 * valid, ops.S), like=t), t)


def kernelspanner(K, h, w):
    K = np.asarray(K, np.float64)
    k = K.shape[0]
    out = []
    for a in range(k):
        for b in range(k):
            P = np.zeros((h, w))
            for r in range(a, h - k + 1, k):
                for c in range(b, w - k + 1, k):
                    P[r:r + k, c:c + k] = K
            out.append(P)
    return out


def offset_mask(h, w, k, a, b):
    F = np.zeros((h, w))
    F[a:h - k + 1:k, b:w - k + 1:k] = 1.0
    return F


def conv(ops, ct_I, ct_S, h, w, k, k0):
    """Algorithm 4 with encrypted kernel matrices ct_S[a k + b]."""
    acc = None
    for a in range(k):
        for b in range(k):
            T = ops.mul(ct_I, ct_S[a * k + b])
            T = ops.cmul(tile(offset_mask(h, w, k, a, b), ops.S), window_sum(ops, T, w, k))
            if acc is None:
                bias = np.zeros((h, w))
                bias[:h - k + 1, :w - k + 1] = k0
                acc = ops.enc(tile(bias, ops.S), like=T)
            acc = ops.add(acc, T)
    return acc


def vrot(ops, ct, m, n, v, r):
    """Each row's first v slots rotated left by r within those v slots."""
    keep = np.zeros((m, n))
    keep[:, :v - r] = 1.0
    wrap = np.zeros((m, n))
    wrap[:, v - r:v] = 1.0
    return ops.add(ops.cmul(tile(keep, ops.S), ops.rot(ct, r)), ops.cmul(tile(wrap, ops.S), ops.rot(ct, r - v)))


def reform(ops, ct, h, w, k):
    """ReForm: the (h - k + 1) x (w - k + 1) outputs of a unit-stride
    convolution, top-left in the h x w block, packed row-major into the
    block's first slots (row r moves left by r (k - 1) under a mask of its
    destination)."""
    hp, wp = h - k + 1, w - k + 1
    acc = None
    for r in range(hp):
        dest = np.zeros(h * w)
        dest[r * wp:(r + 1) * wp] = 1.0
        t = ops.cmul(tile(dest, ops.S), ops.rot(ct, r * (k - 1)))
        acc = t if acc is None else ops.add(acc, t)
    return acc
