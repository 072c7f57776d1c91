"""Column-wise schedules of the oracle and their FP64 plaintext layers.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states the column-wise method in its abstract and contribution list
(an A(m x n).B(n x p) product with each operand held as n ciphertexts; an
h x w image held as w column ciphertexts of h slots) and, in "Secure
Inference", says that operands split over ciphertexts are multiplied pair-wise
and summed by linearity and that per-channel ciphertexts are summed.  It gives
no algorithm for the split forms, so the schedules below are readings built
from its single-ciphertext algorithms:

  matmul  column k of tau_a(A) (the A encoding of "Encoding Method for Matrix
          Multiplication") and column k of tau_b(B) are ciphertexts A_k and
          Bbar_k, replicated with periods M' = pow2(m) and P' = pow2(p); the
          revolver shift (RowShifter, which is one rotation when m mod p = 0,
          per "Homomorphic Matrix Multiplication") becomes Rot(Bbar_k, idx), and
          SumColVec becomes the sum over k:
              D_idx = RelinRescale(sum_k A_k * Rot(Bbar_k, idx)),
          slot i < m of D_idx holds C[i][(i + idx) mod P'].
  conv    the CNN convolution of "Convolutional Neural Networks" with stride s
          and zero padding pi; images are packed in blocks of H' = pow2(h+2pi)
          slots (virtual ciphertexts, B' = S/H' images per ciphertext); output
          column j' sums MulConst(Rot(col(c, s j'+v-pi), u), K[c'][c][u][v]) over
          c, u, v, adds the bias and rescales; slot b H' + s i' holds output
          row i' of image b.  The rotations' ModDown is deferred into the
          rescale (one ModDown by P q_l per output, see conv2d).
  matmul (outer-product form; the rotation-free alternative to the
          revolver above, built from the paper's observation that split
          operands are multiplied pair-wise and summed by linearity): C is
          tiled by R = S / P' rows per ciphertext (P' = pow2(p)); for tile t
          and inner index k the ciphertext A'_{t,k} holds A[t R + r][k] in
          every slot r P' + j with j < p (column k of A replicated across the
          row), and B'_k holds B[k][j] in slot r P' + j for every r (row k of
          B tiled down the rows).  Then
              C_t = RelinRescale(sum_k A'_{t,k} * B'_k),
          slot r P' + j of C_t holds C[t R + r][j]: n tensors and one
          relinearisation per tile, no rotation.
  square  RelinRescale(Tensor(Y, Y)).
  fc      Rescale(sum_{c',j'} MulPlain(Y(c',j'), pt_{o,c',j'})), then the
          SumColVec-style Z += Rot(Z, 2^t) over the H' block, then the bias.

RelinRescale(.) is the relinearisation and the rescale that follow every
ciphertext product, computed as one ModDown by P q_l (Context.relin_rescale):
one rounding instead of two, so its words differ from Rescale(Relin(.)) by a
few units of the coefficients while the decrypted values agree to within that
rounding.

Parity status: "parity unpinned by the paper" -- the paper gives no worked
example, figure or number for the split schedules; they are pinned only by the
FP64 plaintext layers below (and special cases: identity matrix, delta kernel,
constant image) to within 2^-20 normwise relative error.
"""
import math

import numpy as np

from .ckks import Context, Keys, pow2ceil, Plaintext

# ------------------------------------------------------------ FP64 layers


def ref_matmul(A, B):
    return np.asarray(A, np.float64) @ np.asarray(B, np.float64)


def ref_conv(X, K, bias, stride, pad):
    """out[b][c'][i'][j'] = bias[c'] + sum_{c,u,v} K[c'][c][u][v] Xpad[b][c][s i'+u][s j'+v]."""
    X = np.asarray(X, np.float64)
    B, C, h, w = X.shape
    Co, Ci, k, _ = K.shape
    Xp = np.zeros((B, C, h + 2 * pad, w + 2 * pad))
    Xp[:, :, pad:pad + h, pad:pad + w] = X
    ho = (h + 2 * pad - k) // stride + 1
    wo = (w + 2 * pad - k) // stride + 1
    out = np.zeros((B, Co, ho, wo))
    for co in range(Co):
        acc = np.full((B, ho, wo), float(bias[co]))
        for c in range(C):
            for u in range(k):
                for v in range(k):
                    acc += K[co, c, u, v] * Xp[:, c, u:u + stride * ho:stride, v:v + stride * wo:stride]
        out[:, co] = acc
    return out


def ref_fc(Y, W, bias):
    """logits[b][o] = bias[o] + sum W[o][c][i][j] Y[b][c][i][j] (NCHW flatten)."""
    Y = np.asarray(Y, np.float64)
    return Y.reshape(Y.shape[0], -1) @ W.reshape(W.shape[0], -1).T + bias[None, :]


def rel_error(y, ref):
    """max |y - ref| / max |ref| over the valid outputs of one layer."""
    y, ref = np.asarray(y, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))


# ------------------------------------------------------------- encodings


def image_block(h, pad):
    return pow2ceil(h + 2 * pad)


def image_column_slots(ctx: Context, X, c, j, pad):
    """Slot b H' + pad + i holds X[b][c][i][j]; zeros elsewhere."""
    B, C, h, w = X.shape
    Hp = image_block(h, pad)
    if B * Hp > ctx.slots:
        raise ValueError("too many images for one ciphertext")
    z = np.zeros(ctx.slots)
    for b in range(B):
        z[b * Hp + pad:b * Hp + pad + h] = X[b, c, :, j]
    return z


def encrypt_image_columns(ctx: Context, keys: Keys, X, pad, level, seed, first_ct_id):
    """Ciphertext (c, j) has id first_ct_id + c*w + j; returned in that order."""
    X = np.asarray(X, np.float64)
    B, C, h, w = X.shape
    out = []
    for c in range(C):
        for j in range(w):
            pt = ctx.encode(image_column_slots(ctx, X, c, j, pad), level, ctx.scale)
            out.append(ctx.encrypt(keys, pt, seed, first_ct_id + c * w + j))
    return out


def matrix_column_slots(ctx: Context, M, k, role, m, p):
    """role 0: column k of A, slot s -> A[s mod M'][k]; role 1: Bbar_k, slot
    s -> B[k][s mod P'] (zeros past m rows / p columns)."""
    M = np.asarray(M, np.float64)
    Mp, Pp = pow2ceil(m), pow2ceil(p)
    s = np.arange(ctx.slots)
    if role == 0:
        r = s % Mp
        return np.where(r < m, M[np.minimum(r, m - 1), k], 0.0)
    r = s % Pp
    return np.where(r < p, M[k, np.minimum(r, p - 1)], 0.0)


def encrypt_matrix_columns(ctx: Context, keys: Keys, M, role, m, p, level, seed, first_ct_id):
    M = np.asarray(M, np.float64)
    n = M.shape[1] if role == 0 else M.shape[0]
    return [ctx.encrypt(keys, ctx.encode(matrix_column_slots(ctx, M, k, role, m, p), level, ctx.scale),
                        seed, first_ct_id + k) for k in range(n)]


def outer_tiles(ctx: Context, m, p):
    """(P', R, T): column padding, rows per ciphertext and row tiles of the
    outer-product form."""
    Pp = pow2ceil(p)
    if Pp > ctx.slots:
        raise ValueError("p exceeds the slot count")
    R = ctx.slots // Pp
    return Pp, R, -(-m // R)


def matrix_outer_slots(ctx: Context, M, role, m, p, t, k):
    """role 2: A'_{t,k}, slot r P' + j -> A[t R + r][k] for j < p and
    t R + r < m; role 3: B'_k, slot r P' + j -> B[k][j] for j < p."""
    M = np.asarray(M, np.float64)
    Pp, R, _ = outer_tiles(ctx, m, p)
    s = np.arange(ctx.slots)
    r, j = s // Pp, s % Pp
    if role == 2:
        i = t * R + r
        return np.where((j < p) & (i < m), M[np.minimum(i, m - 1), k], 0.0)
    return np.where(j < p, M[k, np.minimum(j, p - 1)], 0.0)


def encrypt_matrix_outer(ctx: Context, keys: Keys, M, role, m, p, level, seed, first_ct_id):
    """role 2 (A, m x n): T n ciphertexts, A'_{t,k} at index t n + k; role 3
    (B, n x p): n ciphertexts B'_k.  Ciphertext i has id first_ct_id + i."""
    M = np.asarray(M, np.float64)
    _, _, T = outer_tiles(ctx, m, p)
    if role == 2:
        n = M.shape[1]
        idx = [(t, k) for t in range(T) for k in range(n)]
    else:
        idx = [(0, k) for k in range(M.shape[0])]
    return [ctx.encrypt(keys, ctx.encode(matrix_outer_slots(ctx, M, role, m, p, t, k), level, ctx.scale),
                        seed, first_ct_id + i) for i, (t, k) in enumerate(idx)]


# ------------------------------------------------------------- schedules


def matmul(ctx: Context, keys: Keys, A_cts, B_cts, m, n, p):
    """D_idx = RelinRescale(sum_k A_k * Rot(Bbar_k, idx)), idx < P'.  For
    m < p the paper multiplies the transposes, C^T = B^T A^T: the Bbar
    ciphertexts (slot s -> B[k][s mod P']) are exactly the A-role ciphertexts
    of B^T and the A ciphertexts (slot s -> A[s mod M'][k]) the Bbar-role
    ciphertexts of A^T, so the roles swap and slot i < p of D_idx holds
    C[(i + idx) mod M'][i] (M' ciphertexts)."""
    if m < p:
        return matmul(ctx, keys, B_cts, A_cts, p, n, m)
    Pp = pow2ceil(p)
    T = [None] * Pp
    for k in range(n):
        rots = [B_cts[k]] + ctx.rotate_many(B_cts[k], list(range(1, Pp)), keys)
        for idx in range(Pp):
            t = ctx.tensor(A_cts[k], rots[idx])
            T[idx] = t if T[idx] is None else ctx.add(T[idx], t)
    return [ctx.relin_rescale(T[idx], keys) for idx in range(Pp)]


def matmul_decode(ctx: Context, keys: Keys, D, m, p):
    if m < p:
        return matmul_decode(ctx, keys, D, p, m).T
    Pp = pow2ceil(p)
    C = np.full((m, p), np.nan)
    for idx in range(Pp):
        z = ctx.decode(ctx.decrypt(keys, D[idx]))
        for i in range(m):
            col = (i + idx) % Pp
            if col < p:
                C[i, col] = z[i]
    return C


def matmul_outer(ctx: Context, keys: Keys, A_cts, B_cts, m, n, p):
    """C_t = RelinRescale(sum_k Tensor(A'_{t,k}, B'_k)) for every row tile t."""
    _, _, T = outer_tiles(ctx, m, p)
    out = []
    for t in range(T):
        acc = None
        for k in range(n):
            x = ctx.tensor(A_cts[t * n + k], B_cts[k])
            acc = x if acc is None else ctx.add(acc, x)
        out.append(ctx.relin_rescale(acc, keys))
    return out


def matmul_outer_decode(ctx: Context, keys: Keys, D, m, p):
    Pp, R, T = outer_tiles(ctx, m, p)
    C = np.full((m, p), np.nan)
    for t in range(T):
        z = ctx.decode(ctx.decrypt(keys, D[t]))
        for r in range(R):
            i = t * R + r
            if i < m:
                C[i, :] = z[r * Pp:r * Pp + p]
    return C


def conv_out_size(h, pad, k, stride):
    return (h + 2 * pad - k) // stride + 1


def conv2d(ctx: Context, keys: Keys, cts, C_in, h, w, pad, K, bias, C_out, k, stride,
           only_cols=None, lazy=None):
    """All C_out * w_out outputs (index c' * w_out + j'), or, with only_cols,
    just the outputs of those output columns j' (same order, others None).

    lazy: the rotations stay P times a ciphertext over q_0..q_l, P
    (rotate_ext, the unrotated columns lifted), MulConst, Add and AddConst act
    there, and one ModDown by P q_l per output finishes every key switch of
    its sum and rescales it (mod_down_rescale).  lazy=False is the plain
    sequence Rot, MulConst, Add, AddConst, Rescale: the same message, rounded
    once per rotation instead of once per output.  Default: lazy when the
    kernel rotates (k > 1) and K <= level + 1 (the extended basis at most
    doubles the limbs), the rule the library applies."""
    K = np.asarray(K, np.float64)
    wo = conv_out_size(w, pad, k, stride)
    level = cts[0].level
    dc = float(ctx.q[level])
    if lazy is None:
        lazy = k > 1 and ctx.K <= level + 1
    mul_const = ctx.mul_const_ext if lazy else ctx.mul_const
    add = ctx.add_ext if lazy else ctx.add
    add_const = ctx.add_const_ext if lazy else ctx.add_const
    finish = ctx.mod_down_rescale if lazy else ctx.rescale
    rot = [[None] * w for _ in range(C_in)]

    def rotated(c, j):
        if rot[c][j] is None:
            ct = cts[c * w + j]
            if lazy:
                rot[c][j] = [ctx.lift(ct)] + ctx.rotate_many_ext(ct, list(range(1, k)), keys)
            else:
                rot[c][j] = [ct] + ctx.rotate_many(ct, list(range(1, k)), keys)
        return rot[c][j]

    out = []
    for co in range(C_out):
        for jo in range(wo):
            if only_cols is not None and jo not in only_cols:
                out.append(None)
                continue
            acc = None
            for c in range(C_in):
                for v in range(k):
                    jj = stride * jo + v - pad
                    if jj < 0 or jj >= w:
                        continue
                    for u in range(k):
                        t = mul_const(rotated(c, jj)[u], K[co, c, u, v], dc)
                        acc = t if acc is None else add(acc, t)
            acc = add_const(acc, float(bias[co]))
            out.append(finish(acc))
    return out


def conv_decode(ctx: Context, keys: Keys, Y, B, C_out, h, pad, k, stride, w):
    Hp = image_block(h, pad)
    ho, wo = conv_out_size(h, pad, k, stride), conv_out_size(w, pad, k, stride)
    out = np.zeros((B, C_out, ho, wo))
    for co in range(C_out):
        for jo in range(wo):
            z = ctx.decode(ctx.decrypt(keys, Y[co * wo + jo]))
            for b in range(B):
                out[b, co, :, jo] = z[b * Hp + stride * np.arange(ho)]
    return out


def square(ctx: Context, keys: Keys, ct):
    return ctx.relin_rescale(ctx.tensor(ct, ct), keys)


def fc_plaintexts(ctx: Context, W, C, ho, wo, stride, Hp, level):
    """pt[o][c*wo + j'] has slot b H' + s i' -> W[o][c][i'][j'] for i' < ho, every
    block b; encoded at scale (double) q_level.  The slot vector repeats with
    period H', so it is encoded in the subring Z[X^r], r = N / (2 H')."""
    W = np.asarray(W, np.float64).reshape(-1, C, ho, wo)
    nb = ctx.slots // Hp
    sub_log = (ctx.n // (2 * Hp)).bit_length() - 1
    pts = []
    for o in range(W.shape[0]):
        row = []
        for c in range(C):
            for jo in range(wo):
                z = np.zeros(ctx.slots)
                for b in range(nb):
                    z[b * Hp + stride * np.arange(ho)] = W[o, c, :, jo]
                row.append(ctx.encode(z, level, float(ctx.q[level]), sub_log))
        pts.append(row)
    return pts


def fc(ctx: Context, keys: Keys, Y, pts, bias, Hp):
    """Z_o = RotSum_Hp(Rescale(sum_i Y_i * pt_{o,i})) + bias_o.  Weights encoded
    below the inputs' level: the inputs are first dropped to it (a level drop
    keeps the message), so the layer runs at the weights' level."""
    out = []
    for o, row in enumerate(pts):
        acc = None
        for y, pt in zip(Y, row):
            if pt.level < y.level:
                y = ctx.mod_drop(y, pt.level)
            t = ctx.mul_plain(y, pt)
            acc = t if acc is None else ctx.add(acc, t)
        z = ctx.rescale(acc)
        step = 1
        while step < Hp:
            z = ctx.add(z, ctx.rotate(z, step, keys))
            step *= 2
        out.append(ctx.add_const(z, float(bias[o])))
    return out


def square_fc_lazy(ctx: Context, y_scale, p_scale, level):
    """Whether x^2 and the FC run with one relinearisation per FC output: the
    FC level l >= 2 and 2^10 times the tensors' weight-product scale
    y_scale^2 p_scale stays below Q_l / 2, checked in integers: with e the
    binary exponent of that scale (it is below 2^e) and b the total bit length
    of q_0..q_l (Q_l >= 2^(b - l - 1)), e + l + 12 <= b."""
    if level < 2:
        return False
    e = math.frexp(y_scale * y_scale * p_scale)[1]
    b = sum(int(q).bit_length() for q in ctx.q[:level + 1])
    return e + level + 12 <= b


def square_fc(ctx: Context, keys: Keys, Y, pts, bias, Hp):
    """x^2 then fc with lazy relinearisation (the paper's Mul of the
    activation, its relinearisation moved past the FC's linear sums): each
    input's tensor Tensor(Y_i, Y_i), taken on the FC level's limbs, is
    multiplied by the weight plaintexts and summed, and only the sums are
    relinearised:
        Z_o = RotSum_Hp(Rescale(RelinRescale(sum_i Tensor(Y_i, Y_i) pt_{o,i}))) + bias_o.
    One key switch per output instead of one per input; the decrypted
    result is that of fc(square(Y)) up to rounding.  Needs
    square_fc_lazy(Y scale, pt scale, level)."""
    level = min(Y[0].level, pts[0][0].level)
    if not square_fc_lazy(ctx, Y[0].scale, pts[0][0].scale, level):
        raise ValueError("no room for the unrelinearised FC products at this level")
    T = []
    for y in Y:
        yd = ctx.mod_drop(y, level) if y.level > level else y
        T.append(ctx.tensor(yd, yd))
    out = []
    for o, row in enumerate(pts):
        acc = None
        for t, pt in zip(T, row):
            p = ctx.mul_plain(t, pt)
            acc = p if acc is None else ctx.add(acc, p)
        z = ctx.rescale(ctx.relin_rescale(acc, keys))
        step = 1
        while step < Hp:
            z = ctx.add(z, ctx.rotate(z, step, keys))
            step *= 2
        out.append(ctx.add_const(z, float(bias[o])))
    return out


def fc_decode(ctx: Context, keys: Keys, Z, B, Hp):
    out = np.zeros((B, len(Z)))
    for o, z in enumerate(Z):
        v = ctx.decode(ctx.decrypt(keys, z))
        out[:, o] = v[np.arange(B) * Hp]
    return out


def fc_rotation_steps(Hp):
    steps, s = [], 1
    while s < Hp:
        steps.append(s)
        s *= 2
    return steps


# ------------------------------------------ deeper networks (Table 1 shape)

# The activations of the paper's CNN ("Neural Network Architecture", Table 1):
# coefficients of a0 + a1 x + a2 x^2 + a3 x^3.
ACT1 = (-0.00015120704, 0.4610149, 2.0225089, -1.4511951)
ACT2 = (-1.5650465, -0.9943767, 1.6794522, 0.5350255)


def poly_eval(ctx: Context, keys: Keys, ct, coeffs):
    """sum_i coeffs[i] x^i (degree d >= 1) by Horner's rule:
    t = MulConst(x, a_d) at constant scale q_l, rescaled, plus a_{d-1}; then
    for i = d-2 .. 0: t = RelinRescale(Tensor(t, x dropped to t's level))
    plus a_i.  Depth d; every addition is an AddConst at the running scale."""
    d = len(coeffs) - 1
    if d < 1:
        raise ValueError("degree must be at least 1")
    t = ctx.rescale(ctx.add_const(ctx.mul_const(ct, coeffs[d], float(ctx.q[ct.level])), coeffs[d - 1]))
    for i in range(d - 2, -1, -1):
        x = ctx.mod_drop(ct, t.level)
        t = ctx.add_const(ctx.relin_rescale(ctx.tensor(t, x), keys), coeffs[i])
    return t


def ref_poly(x, coeffs):
    return sum(c * np.asarray(x, np.float64) ** i for i, c in enumerate(coeffs))


def dense(ctx: Context, keys: Keys, Z, W, bias):
    """out_o = Rescale(sum_j MulConst(Z_j, W[o][j]) + AddConst(bias_o)): a
    fully connected layer on neuron ciphertexts (each holding its neuron's
    value at the same slots), e.g. the 64 -> 10 FC-2 of Table 1."""
    W = np.asarray(W, np.float64)
    dq = float(ctx.q[Z[0].level])
    out = []
    for o in range(W.shape[0]):
        acc = None
        for j, z in enumerate(Z):
            t = ctx.mul_const(z, W[o, j], dq)
            acc = t if acc is None else ctx.add(acc, t)
        out.append(ctx.rescale(ctx.add_const(acc, float(bias[o]))))
    return out


def deep_cnn(ctx: Context, keys: Keys, cts, C_in, h, w, pad, K, kb, stride, act1, fc_pts, fc_b, Hp, act2, W2, b2):
    """CONV -> ACT-1 -> FC-1 -> ACT-2 -> FC-2 (the layer sequence of Table 1)
    on column ciphertexts: the conv schedule, the polynomial activation on
    every conv output, the FC schedule to neuron ciphertexts (neuron o of
    image b at slot b Hp), the second activation on every neuron, and the
    dense FC-2."""
    Y = conv2d(ctx, keys, cts, C_in, h, w, pad, K, kb, K.shape[0], K.shape[2], stride)
    Y = [poly_eval(ctx, keys, y, act1) for y in Y]
    Z = fc(ctx, keys, Y, fc_pts, fc_b, Hp)
    Z = [poly_eval(ctx, keys, z, act2) for z in Z]
    return dense(ctx, keys, Z, W2, b2)


def ref_deep_cnn(X, K, kb, stride, pad, act1, W1, b1, act2, W2, b2):
    Y = ref_poly(ref_conv(X, K, kb, stride, pad), act1)
    Z = ref_poly(ref_fc(Y, W1, b1), act2)
    return Z @ np.asarray(W2, np.float64).T + np.asarray(b2, np.float64)[None, :]


# ------------------------------------------------ encrypted-weight layers

def conv2d_encw(ctx: Context, keys: Keys, cts, C_in, h, w, pad, Kct, bias_ct, C_out, k, stride):
    """The conv schedule with encrypted weights (the paper's usage model: the
    model provider encrypts the kernels and the cloud sees no weight in the
    clear).  Kct[((c' C_in + c) k + u) k + v] encrypts K[c'][c][u][v] in every
    slot at scale q_l; bias_ct[c'] encrypts the bias in every slot one level
    lower, at the scale the rescaled sum carries.  Each output is a sum of
    ct x ct products relinearised once (lazy relinearisation):
        Y(c', j') = RelinRescale(sum_{c,u,v} Tensor(Rot(col(c, s j'+v-pi), u),
                    Kct[c', c, u, v])) + bias_ct[c'].  One level."""
    wo = conv_out_size(w, pad, k, stride)
    rot = {}

    def rotated(c, j):
        if (c, j) not in rot:
            ct = cts[c * w + j]
            rot[(c, j)] = [ct] + ctx.rotate_many(ct, list(range(1, k)), keys)
        return rot[(c, j)]

    out = []
    for co in range(C_out):
        for jo in range(wo):
            acc = None
            for c in range(C_in):
                for v in range(k):
                    jj = stride * jo + v - pad
                    if jj < 0 or jj >= w:
                        continue
                    for u in range(k):
                        t = ctx.tensor(rotated(c, jj)[u], Kct[((co * C_in + c) * k + u) * k + v])
                        acc = t if acc is None else ctx.add(acc, t)
            out.append(ctx.add(ctx.relin_rescale(acc, keys), bias_ct[co]))
    return out


def encrypt_conv_weights(ctx: Context, keys: Keys, K, bias, level, x_scale, seed, first_ct_id):
    """The model provider's ciphertexts for conv2d_encw: every weight in every
    slot at scale q_level; every bias in every slot at level - 1 and the scale
    a rescaled product carries, (x_scale q_level) / q_level as a double."""
    K = np.asarray(K, np.float64)
    dq = float(ctx.q[level])
    kct = [ctx.encrypt(keys, ctx.encode(np.full(ctx.slots, wv), level, dq), seed, first_ct_id + i)
           for i, wv in enumerate(K.reshape(-1))]
    bscale = (x_scale * dq) / dq
    bct = [ctx.encrypt(keys, ctx.encode(np.full(ctx.slots, float(b)), level - 1, bscale), seed,
                       first_ct_id + K.size + i) for i, b in enumerate(bias)]
    return kct, bct


def fc_encw(ctx: Context, keys: Keys, Y, Wct, bias_ct, Hp):
    """FC with encrypted weights: Wct[o][i] encrypts the weight pattern of
    fc_plaintexts (scale q_l) and bias_ct[o] the bias in every slot one level
    lower at the scale the rescaled sum carries (see encrypt_fc_weights):
        Z_o = RotSum_Hp(RelinRescale(sum_i Tensor(Y_i, Wct[o][i]))) + bias_ct[o],
    one relinearisation per output (lazy)."""
    out = []
    for o, row in enumerate(Wct):
        acc = None
        for y, wct in zip(Y, row):
            t = ctx.tensor(y, wct)
            acc = t if acc is None else ctx.add(acc, t)
        z = ctx.relin_rescale(acc, keys)
        step = 1
        while step < Hp:
            z = ctx.add(z, ctx.rotate(z, step, keys))
            step *= 2
        out.append(ctx.add(z, bias_ct[o]))
    return out


def encrypt_fc_weights(ctx: Context, keys: Keys, W, bias, C, ho, wo, stride, Hp, level, y_scale, seed,
                       first_ct_id):
    """The model provider's ciphertexts for fc_encw: the weight patterns of
    fc_plaintexts encrypted at scale q_level, and each bias in every slot at
    level - 1 and scale (y_scale q_level) / q_level."""
    pts = fc_plaintexts(ctx, W, C, ho, wo, stride, Hp, level)
    dq = float(ctx.q[level])
    i = first_ct_id
    wct = []
    for row in pts:
        r = []
        for pt in row:
            r.append(ctx.encrypt(keys, pt, seed, i))
            i += 1
        wct.append(r)
    bct = []
    for b in bias:
        bct.append(ctx.encrypt(keys, ctx.encode(np.full(ctx.slots, float(b)), level - 1, (y_scale * dq) / dq),
                               seed, i))
        i += 1
    return wct, bct


# ------------------------------------- column-block packing of the product

def block_shape(ctx: Context, m, n, p):
    """(P', Mb, c, nb) of the column-block form: blocks of Mb = P' ceil((m +
    P' - 1) / P') slots (a multiple of P', at least m + P' - 1), c = the
    largest power of two with c Mb <= S and c <= pow2(n) columns per
    ciphertext, nb = ceil(n / c) ciphertexts per operand."""
    Pp = pow2ceil(p)
    Mb = Pp * -(-(m + Pp - 1) // Pp)
    if Mb > ctx.slots:
        raise ValueError("m + P' - 1 exceeds the slot count")
    c = 1
    while 2 * c * Mb <= ctx.slots and c < pow2ceil(n):
        c *= 2
    return Pp, Mb, c, -(-n // c)


def matrix_block_slots(ctx: Context, M, K, role, m, n, p):
    """Ciphertext K of the column-block form (NEXT to the column-split form:
    c columns per ciphertext instead of one).  role 4 (A): block j holds
    column K c + j of A in its first m slots; role 5 (Bbar): block j holds row
    K c + j of B, entry j' in every slot r with r mod P' = j' < p.  Zero past
    the n columns, past m rows / p columns and past the c blocks."""
    M = np.asarray(M, np.float64)
    Pp, Mb, c, nb = block_shape(ctx, m, n, p)
    z = np.zeros(ctx.slots)
    for j in range(c):
        col = K * c + j
        if col >= n:
            break
        base = j * Mb
        if role == 4:
            z[base:base + m] = M[:, col]
        else:
            r = np.arange(Mb)
            z[base:base + Mb] = np.where(r % Pp < p, M[col, np.minimum(r % Pp, p - 1)], 0.0)
    return z


def encrypt_matrix_blocks(ctx: Context, keys: Keys, M, role, m, n, p, level, seed, first_ct_id):
    nb = block_shape(ctx, m, n, p)[3]
    return [ctx.encrypt(keys, ctx.encode(matrix_block_slots(ctx, M, K, role, m, n, p), level, ctx.scale),
                        seed, first_ct_id + K) for K in range(nb)]


def matmul_block(ctx: Context, keys: Keys, A_cts, B_cts, m, n, p):
    """The column-split revolver on column blocks: D_idx =
    RelinRescale(sum_K A_K * Rot(Bbar_K, idx)) for idx < P' (the blocks'
    padding of P' - 1 slots past m keeps every rotated read inside its own
    block wherever A is non-zero, so no RowShifter fix-up is needed), then
    the c blocks are folded into block 0 by D += Rot(D, Mb 2^t), t < log2 c.
    Slot i < m of D_idx holds C[i][(i + idx) mod P'].  Needs m >= p."""
    if m < p:
        raise ValueError("the column-block form needs m >= p (multiply the transposes)")
    Pp, Mb, c, nb = block_shape(ctx, m, n, p)
    if len(A_cts) != nb or len(B_cts) != nb:
        raise ValueError("column-block operands need %d ciphertexts each" % nb)
    D = matmul(ctx, keys, A_cts, B_cts, m, nb, p)
    out = []
    for d in D:
        t = 1
        while t < c:
            d = ctx.add(d, ctx.rotate(d, Mb * t, keys))
            t *= 2
        out.append(d)
    return out


def block_rotation_steps(ctx: Context, m, n, p):
    Pp, Mb, c, nb = block_shape(ctx, m, n, p)
    steps = list(range(1, Pp))
    t = 1
    while t < c:
        steps.append(Mb * t)
        t *= 2
    return steps
