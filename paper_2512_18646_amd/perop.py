"""The layer schedules issued as one C-ABI call per HE operation.

This is the plain per-operation path the batched layer calls (vr_conv2d,
vr_square, vr_matmul) are measured against; it issues exactly the
operations of the schedules (rotations hoisted per input column, MulConst,
Add, AddConst, Rescale, Tensor, Relinearise) and therefore reaches the same
limbs.  Every arithmetic step runs in libvr.so.
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
    return [ctx.rescale(ctx.relinearize(keys, ctx.tensor(y, y, stream=stream), stream=stream), stream=stream)
            for y in cts]


def matmul(ctx, keys, A, Bbar, m, n, p, stream=None):
    Pp = pow2ceil(p)
    T = [None] * Pp
    for k in range(n):
        rots = [Bbar[k]] + (ctx.rotate_many(keys, Bbar[k], list(range(1, Pp)), stream=stream) if Pp > 1 else [])
        for idx in range(Pp):
            t = ctx.tensor(A[k], rots[idx], stream=stream)
            T[idx] = t if T[idx] is None else ctx.add(T[idx], t, stream=stream)
    return [ctx.rescale(ctx.relinearize(keys, T[idx], stream=stream), stream=stream) for idx in range(Pp)]
