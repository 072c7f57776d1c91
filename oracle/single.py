"""The paper's single-ciphertext algorithms ("Technical Details"): the
tau_a / tau_b encodings, RowShifter (Algorithm 2) and the homomorphic matrix
product (Algorithm 3), SumForConv (Algorithm 1), Kernelspanner and the
homomorphic convolution (Algorithm 4), and the virtual rotation vRot
(Algorithm 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each algorithm is written once, in the paper's order of steps, against a small
operation interface, and evaluated two ways: on plain slot vectors
(`PlainOps`: Rot is a left cyclic shift of the S slots, cMult an elementwise
product with the mask, Mult an elementwise product, Enc the vector itself) and
on oracle ciphertexts (`HeOps`: the scheme of ckks.py; every cMult and Mult is
followed by a rescale, constants are encoded at scale q_l so the rescale
restores the scale).  Both count the operations they issue, for the paper's
operation-count tables (Tables 2 and 3).

Readings, where the paper is garbled or silent:
  layout      an r x c matrix is packed row-major into r c slots and that
              block is repeated over all S slots (r c a power of two), so a
              rotation of the real ciphertext acts cyclically on every copy,
              as the algorithms assume of a ciphertext the matrix fills.
  RowShifter  Algorithm 3 calls it on the original ct.Bbar in iteration idx,
              so it shifts Bbar by idx rows at once: rows i < m - idx come
              from Rot(ct, idx n) (row i + idx, which holds column
              (i + idx) mod p of B) and the last idx rows from
              Rot(ct, n (idx - m + m mod p)) (row i + idx - m + m mod p,
              holding the same column); two 0/1 row masks keep each part.
              The printed rotation amount has garbled parentheses.  When p
              divides m the two rotations coincide and one rotation is
              issued (the paper's remark on m mod p = 0); idx = 0 is the
              identity.
  SumColVec   (Han et al.) rotate-and-sum over the n columns of each row
              (log2 n rotations), keep column 0 (one cMult), rotate-and-sum
              rightwards to spread each row sum over its row (log2 n
              rotations): 2 log2 n Rot and Add, 1 cMult -- Table 2's Step 2
              with the n columns summed over in place of p.
  mask F      F[i][(i + idx) mod p] (the printed modulus n leaves C's m x p
              shape).
  SumForConv  the window sum is separable: the row pass rotates the
              column-summed partial, not ct.I (as printed, the two passes
              would add a row-plus-column cross, not the box sum the worked
              example states).  Standalone (Algorithm 1) it adds k0 and keeps
              every valid window, as the worked example shows; inside
              Algorithm 4 it is the bare window sum and Algorithm 4's offset
              mask F selects.  Rot by 0 is the identity and is not issued:
              2 (k - 1) rotations ("approximately 2k").
  Kernelspanner  P_(a,b) for offsets a, b < k: K tiled in k x k blocks whose
              top-left corners sit at (a + k t, b + k u), only blocks that fit
              in h x w (the printed h = w = 4, k = 2 example).
  Algorithm 4 mask  (hth - a) mod k = 0 and (wth - b) mod k = 0 for offset
              (a, b), with hth + k <= h and wth + k <= w (the printed pairing
              of i with wth is transposed against Kernelspanner); F is h x w.
              The result is the valid unit-stride cross-correlation plus k0
              at every valid position.
  vRot        rows of n slots, each holding a virtual ciphertext of v = h w
              values first: Rot(ct, r) masked to row positions j < v - r,
              plus Rot(ct, r - v) masked to v - r <= j < v (F2[m][j] read as
              F2[i][j]).  Positions past v come out zero.

Parity: pinned by tests/test_oracle_single.py against the paper's worked
examples (tests/golden/), plain brute force (A B, cross-correlation, cyclic
shifts) and the operation counts of Tables 2 and 3 under the readings above;
the encrypted runs against FP64.
"""
from collections import Counter

import numpy as np

from .ckks import Ciphertext, Context, Keys


def log2_exact(x):
    r = int(x).bit_length() - 1
    if x < 1 or (1 << r) != x:
        raise ValueError("%d is not a power of two" % x)
    return r


# ------------------------------------------------------------------ encodings

def tau_a(A):
    """tau_a: row-major A, entry k -> A[k // n][k mod n] for k < m n."""
    A = np.asarray(A, np.float64)
    m, n = A.shape
    return np.array([A[k // n, k % n] for k in range(m * n)])


def tau_b(B, m):
    """tau_b: B (n x p) transposed and tiled to m rows: entry k ->
    B[k mod n][(k // n) mod p] for k < m n (row i of Bbar is column i mod p)."""
    B = np.asarray(B, np.float64)
    n, p = B.shape
    return np.array([B[k % n, (k // n) % p] for k in range(m * n)])


def replicate(block, S):
    """The packed block repeated over all S slots (the layout reading)."""
    block = np.asarray(block, np.float64)
    if S % block.size:
        raise ValueError("the packed block must divide the slot count")
    return np.tile(block, S // block.size)


# ---------------------------------------------------------- operation sets

class PlainOps:
    """The algorithms on plain slot vectors."""

    def __init__(self, S):
        self.S = S
        self.count = Counter()

    def rot(self, x, r):
        if r % self.S == 0:
            return x
        self.count["Rot"] += 1
        return np.roll(x, -(r % self.S))

    def add(self, x, y):
        self.count["Add"] += 1
        return x + y

    def cmul(self, mask, x):
        self.count["cMult"] += 1
        return np.asarray(mask, np.float64) * x

    def mul(self, x, y):
        self.count["Mult"] += 1
        return x * y

    def enc(self, vec, like=None):
        return np.asarray(vec, np.float64).copy()

    def drop(self, x, levels):
        return x


class HeOps:
    """The algorithms on oracle ciphertexts.  cMult encodes its mask at scale
    q_l of the ciphertext's level and rescales; Mult is the tensor product
    followed by the fused relinearisation and rescale; Add drops the higher
    operand to the lower
    level (a level drop keeps the message); Enc encrypts a vector at a given
    ciphertext's level and scale (the third party's or client's encryption)."""

    def __init__(self, ctx: Context, keys: Keys, seed, first_id):
        self.ctx, self.keys = ctx, keys
        self.S = ctx.slots
        self.seed, self.next_id = seed, first_id
        self.count = Counter()

    def rot(self, ct, r):
        if r % self.S == 0:
            return ct
        self.count["Rot"] += 1
        return self.ctx.rotate(ct, r % self.S, self.keys)

    def _align(self, a, b):
        lv = min(a.level, b.level)
        if a.level > lv:
            a = self.ctx.mod_drop(a, lv)
        if b.level > lv:
            b = self.ctx.mod_drop(b, lv)
        return a, b

    def add(self, a, b):
        self.count["Add"] += 1
        a, b = self._align(a, b)
        return self.ctx.add(a, b)

    def drop(self, ct, levels):
        """A level drop (no operation of the paper's tables)."""
        return self.ctx.mod_drop(ct, ct.level - levels) if levels else ct

    def cmul(self, mask, ct):
        self.count["cMult"] += 1
        pt = self.ctx.encode(np.asarray(mask, np.float64), ct.level, float(self.ctx.q[ct.level]))
        return self.ctx.rescale(self.ctx.mul_plain(ct, pt))

    def mul(self, a, b):
        self.count["Mult"] += 1
        a, b = self._align(a, b)
        return self.ctx.relin_rescale(self.ctx.tensor(a, b), self.keys)

    def enc(self, vec, like=None, level=None):
        lv = like.level if like is not None else level
        scale = like.scale if like is not None else self.ctx.scale
        ct = self.ctx.encrypt(self.keys, self.ctx.encode(np.asarray(vec, np.float64), lv, scale),
                              self.seed, self.next_id)
        self.next_id += 1
        return ct


# -------------------------------------------------------------- Algorithm 2

def row_masks(m, n, S, rows):
    """0/1 mask of the packed m x n block keeping the given rows, replicated."""
    F = np.zeros((m, n))
    F[list(rows)] = 1.0
    return replicate(F.reshape(-1), S)


def row_shifter(ops, ct_B, m, n, p, idx):
    """Bbar shifted by idx rows: row i of the result holds column
    (i + idx) mod p of B (see the module's reading)."""
    if idx == 0:
        return ct_B
    r1 = idx * n
    r2 = n * (idx - m + m % p)
    if (r1 - r2) % (m * n) == 0:          # p | m: one rotation
        return ops.rot(ct_B, r1)
    T1 = ops.cmul(row_masks(m, n, ops.S, range(m - idx)), ops.rot(ct_B, r1))
    T2 = ops.cmul(row_masks(m, n, ops.S, range(m - idx, m)), ops.rot(ct_B, r2))
    return ops.add(T1, T2)


# -------------------------------------------------------------- Algorithm 3

def sum_col_vec(ops, ct, m, n):
    """Each row's sum over its n columns, in every column of the row."""
    t = ct
    step = 1
    while step < n:                       # left rotate-and-sum: row sum at column 0
        t = ops.add(t, ops.rot(t, step))
        step *= 2
    col0 = np.zeros((m, n))
    col0[:, 0] = 1.0
    t = ops.cmul(replicate(col0.reshape(-1), ops.S), t)
    step = 1
    while step < n:                       # right rotate-and-sum: spread it over the row
        t = ops.add(t, ops.rot(t, -step))
        step *= 2
    return t


def matmul(ops, ct_A, ct_B, m, n, p):
    """Algorithm 3: C (m x p) in the packed m x n layout, slot i n + j holding
    C[i][j] for j < p.  Needs p <= n and m n a power of two."""
    if p > n:
        raise ValueError("the product's p columns must fit the n-slot rows")
    log2_exact(m * n)
    log2_exact(n)
    # when RowShifter masks (p does not divide m), its shifted operands sit one
    # level below ct.Bbar: ct.A (and the unshifted ct.Bbar of idx = 0) meet
    # them there, so every iteration's product is rescaled by the same prime
    # and the accumulated terms carry the same scale
    if m % p:
        ct_A = ops.drop(ct_A, 1)
    acc = None
    for idx in range(p):
        T = row_shifter(ops, ct_B, m, n, p, idx)            # Step 1
        T = ops.mul(ct_A, T)
        T = sum_col_vec(ops, T, m, n)                       # Step 2
        F = np.zeros((m, n))                                # Step 3
        for i in range(m):
            F[i, (i + idx) % p] = 1.0
        T = ops.cmul(replicate(F.reshape(-1), ops.S), T)
        acc = ops.enc(np.zeros(ops.S), like=T) if acc is None else acc   # ct.C = Enc(0)
        acc = ops.add(acc, T)                               # Step 4
    return acc


def matmul_decode_layout(vec, m, n, p):
    """C from the packed m x n block (first copy)."""
    return np.asarray(vec[:m * n]).reshape(m, n)[:, :p]


# ------------------------------------------------------------ Algorithm 1

def window_sum(ops, ct, w, k):
    """Box sums of k x k windows anchored at their top-left slot: the column
    pass, then the row pass on the partial sums."""
    t = ct
    for pos in range(1, k):
        t = ops.add(t, ops.rot(ct, pos))
    u = t
    for pos in range(1, k):
        u = ops.add(u, ops.rot(t, pos * w))
    return u


def sum_for_conv(ops, ct, h, w, k, k0):
    """Algorithm 1 (standalone): k0 plus the k x k window sum at every valid
    window position of the h x w image, zero elsewhere (ct.I_s = Enc(k0 at
    the valid positions) is encrypted at the level and scale the masked sum
    reaches, so the two can be added)."""
    valid = np.zeros((h, w))
    valid[:h - k + 1, :w - k + 1] = 1.0
    t = window_sum(ops, ct, w, k)
    t = ops.cmul(replicate(valid.reshape(-1), ops.S), t)
    I_s = ops.enc(replicate((k0 * valid).reshape(-1), ops.S), like=t)
    return ops.add(I_s, t)


# ------------------------------------------------------------ Algorithm 4

def kernelspanner(K, h, w):
    """The k^2 matrices P_(a,b) (a, b < k), in the order a k + b."""
    K = np.asarray(K, np.float64)
    k = K.shape[0]
    out = []
    for a in range(k):
        for b in range(k):
            P = np.zeros((h, w))
            for r0 in range(a, h - k + 1, k):
                for c0 in range(b, w - k + 1, k):
                    P[r0:r0 + k, c0:c0 + k] = K
            out.append(P)
    return out


def conv_mask(h, w, k, a, b):
    F = np.zeros((h, w))
    for hth in range(h):
        for wth in range(w):
            if (hth - a) % k == 0 and (wth - b) % k == 0 and hth + k <= h and wth + k <= w:
                F[hth, wth] = 1.0
    return F


def conv(ops, ct_I, ct_S, h, w, k, k0):
    """Algorithm 4: ct_S[a k + b] encrypts Kernelspanner's P_(a,b) (encrypted
    weights, as the paper's third party prepares them).  Returns k0 plus the
    valid unit-stride cross-correlation at positions (r, c), r <= h - k,
    c <= w - k, of the packed h x w image."""
    acc = None
    for a in range(k):
        for b in range(k):
            T = ops.mul(ct_I, ct_S[a * k + b])                        # Step 1
            T = window_sum(ops, T, w, k)                               # Step 2
            T = ops.cmul(replicate(conv_mask(h, w, k, a, b).reshape(-1), ops.S), T)   # Step 3
            if acc is None:                                           # ct.I_s = Enc(k0 at valid positions)
                valid = np.zeros((h, w))
                valid[:h - k + 1, :w - k + 1] = k0
                acc = ops.enc(replicate(valid.reshape(-1), ops.S), like=T)
            acc = ops.add(acc, T)                                     # Step 4
    return acc


# ------------------------------------------------------------ Algorithm 5

def vrot(ops, ct, m, n, v, r):
    """Rotate each row's first v slots (a virtual ciphertext) left by r,
    cyclically within those v slots; the m x n block repeated over S."""
    if not 0 < r < v <= n:
        raise ValueError("need 0 < r < v <= n")
    F1 = np.zeros((m, n))
    F1[:, :v - r] = 1.0
    F2 = np.zeros((m, n))
    F2[:, v - r:v] = 1.0
    T1 = ops.cmul(replicate(F1.reshape(-1), ops.S), ops.rot(ct, r))
    T2 = ops.cmul(replicate(F2.reshape(-1), ops.S), ops.rot(ct, r - v))
    return ops.add(T1, T2)


def rotation_steps_matmul(m, n, p, S):
    """Rotation steps Algorithm 3 issues (as residues mod S)."""
    steps = set()
    for idx in range(1, p):
        steps.add((idx * n) % S)
        if (m % p) != 0:
            steps.add((n * (idx - m + m % p)) % S)
    t = 1
    while t < n:
        steps.add(t % S)
        steps.add((-t) % S)
        t *= 2
    steps.discard(0)
    return sorted(steps)


def rotation_steps_conv(w, k, S):
    steps = {pos % S for pos in range(1, k)} | {(pos * w) % S for pos in range(1, k)}
    steps.discard(0)
    return sorted(steps)


# ----------------------------------------------------------------- ReForm

def reform(ops, ct, h, w, k):
    """ReForm ("Homomorphic CNN Evaluation"): after a unit-stride k x k
    convolution the outputs occupy the top-left (h - k + 1) x (w - k + 1) of
    the h x w row-major block; ReForm packs them row-major into the first
    (h - k + 1)(w - k + 1) slots of the block: row r moves left by r (k - 1)
    slots and is kept by a mask of its destination -- h' - 1 rotations, h'
    cMult and h' - 1 Add for h' = h - k + 1 rows (the O(h) of the text)."""
    hp, wp = h - k + 1, w - k + 1
    acc = None
    for r in range(hp):
        F = np.zeros(h * w)
        F[r * wp:(r + 1) * wp] = 1.0
        t = ops.cmul(replicate(F, ops.S), ops.rot(ct, r * (k - 1)))
        acc = t if acc is None else ops.add(acc, t)
    return acc
