"""The layer schedules issued as one C-ABI call per HE operation.

This is the plain per-operation path the batched layer calls (vr_conv2d,
vr_square, vr_fc, vr_matmul) are measured against; it issues exactly the
operations of the schedules (rotations hoisted per input column, MulConst,
MulPlain, Add, AddConst, Rescale, Tensor, the fused Relinearise-Rescale,
Rotate) and therefore
reaches the same limbs.  Every arithmetic step runs in libvr.so.
"""


def pow2ceil(x):
    p = 1
    while p < x:
        p *= 2
    return p


def conv2d(ctx, keys, cols, C_in, h, w, pad, K, bias, stride, stream=None):
    C_out, _, k, _ = K.shape
    wo = (w + 2 * pad - k) // stride + 1
    level = cols[0].level
    dq = float(ctx.q[level])
    rot = [[None] * w for _ in range(C_in)]
    for c in range(C_in):
        for j in range(w):
            ct = cols[c * w + j]
            rot[c][j] = [ct] + (ctx.rotate_many(keys, ct, list(range(1, k)), stream=stream) if k > 1 else [])
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
                        t = ctx.mul_const(rot[c][jj][u], float(K[co, c, u, v]), dq, stream=stream)
                        acc = t if acc is None else ctx.add(acc, t, stream=stream)
            acc = ctx.add_const(acc, float(bias[co]), stream=stream)
            out.append(ctx.rescale(acc, stream=stream))
    return out


def square(ctx, keys, cts, stream=None):
    return [ctx.relin_rescale(keys, ctx.tensor(y, y, stream=stream), stream=stream) for y in cts]


def matmul(ctx, keys, A, Bbar, m, n, p, stream=None):
    if m < p:   # the transposed product on the same ciphertexts, roles swapped
        return matmul(ctx, keys, Bbar, A, p, n, m, stream=stream)
    Pp = pow2ceil(p)
    T = [None] * Pp
    for k in range(n):
        rots = [Bbar[k]] + (ctx.rotate_many(keys, Bbar[k], list(range(1, Pp)), stream=stream) if Pp > 1 else [])
        for idx in range(Pp):
            t = ctx.tensor(A[k], rots[idx], stream=stream)
            T[idx] = t if T[idx] is None else ctx.add(T[idx], t, stream=stream)
    return [ctx.relin_rescale(keys, T[idx], stream=stream) for idx in range(Pp)]


def fc(ctx, keys, Y, W_pt, bias, block, stream=None):
    """Z_o = RotSum over the block of Rescale(sum_i MulPlain(Y_i, pt[o][i])), plus
    bias[o]; W_pt is the flat list from encode_fc_weights ([o][i], i over the
    C_out * w_out inputs)."""
    per = len(Y)
    if per == 0 or len(W_pt) != len(bias) * per:
        raise ValueError("fc: %d weight plaintexts for %d outputs x %d inputs" % (len(W_pt), len(bias), per))
    # weights encoded below the inputs' level: drop the inputs to it first
    lv = W_pt[0].level
    if Y[0].level > lv:
        Y = [ctx.mod_drop(y, lv, stream=stream) for y in Y]
    out = []
    for o in range(len(bias)):
        acc = None
        for i, y in enumerate(Y):
            t = ctx.mul_plain(y, W_pt[o * per + i], stream=stream)
            acc = t if acc is None else ctx.add(acc, t, stream=stream)
        z = ctx.rescale(acc, stream=stream)
        step = 1
        while step < block:
            z = ctx.add(z, ctx.rotate(keys, z, step, stream=stream), stream=stream)
            step *= 2
        out.append(ctx.add_const(z, float(bias[o]), stream=stream))
    return out
