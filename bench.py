#!/usr/bin/env python3
"""Throughput benchmark of column-wise encrypted CNN inference on one MI355X.

Workload (one step): the 3x128x128 network at N = 2^16 (L = 24 chain of
60 + 24x50-bit primes, 9 special primes of 51 bits, dnum 3) on one set of 128
images, each image channel held as 128 column ciphertexts (384 per set), the
ciphertexts entering at level 24 (the full chain): conv 3x3 stride 2 pad 1
with 8 filters (768 hoisted rotations, 13,752 MulConst), x^2 (512 tensor +
relinearisation + rescale), FC 8*64*64 -> 10 (5,120 MulPlain at the weights'
level 1, 80 rotations), as one whole-network call.  Inputs are encrypted
before the timed region and stay resident in HBM; the timed region is the
server-side evaluation only.

The JSON line adds the same step as one replayed HIP graph and as one C-ABI
call per HE operation, the network entering at level 3 (trimmed), the 28x28
conv layer at N = 2^14, the 16x16 matrix product at N = 2^13, HE rotations/s
at N = 2^16, serving and uneven batches, the live roofline of the step's
dominant kernel (HIP events around its launches inside the timed region) and
the CPU oracle timed on a bounded sample on one and on all host cores.
"""
import argparse
import collections
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "encrypted images/s, HE-rotations/s (N=2^16) batched vs per-op; p99 latency"


VALU_LANE_OPS = 256 * 64 * 2.4e9          # 256 CUs x 64 lanes per clock x 2.4 GHz
FP64_BFLY_OPS = 8                          # y*w, fma, *1/q, rint, fma, +e, X+T, X-T
NTT_PEAK_TBFLY = VALU_LANE_OPS / FP64_BFLY_OPS / 1e12


def ntt_roofline(prof_ms, calls, limbs, total_s, log_n, counter_name=None):
    """Roofline of the NTT class (the dominant kernel of the step).  One call
    transforms `limbs / calls` limbs (at N = 2^15 and 2^16 as two kernel
    launches, pass 0 and pass 1).  Algorithmic bytes: 16N per limb (each word
    read and written once); operations: N/2 log2 N butterflies per limb at
    FP64_BFLY_OPS lane operations each.  Both floors are computed per call and
    the larger one names the bound; `achieved` is against that bound's peak.
    `traffic`: HBM bytes per call from the FETCH_SIZE / WRITE_SIZE counter
    file in profiles/, while the kernel source is unchanged since it was
    measured (else null)."""
    if prof_ms <= 0 or calls == 0:
        return None
    n = 1 << log_n
    avg_s = prof_ms / calls / 1e3
    per_call = limbs / calls
    alg_bytes = 16 * n * per_call
    bfly = per_call * (n // 2) * log_n
    hbm_floor_s = alg_bytes / (HBM_PEAK_GBS * 1e9)
    alu_floor_s = bfly * FP64_BFLY_OPS / VALU_LANE_OPS
    traffic = None
    cnt = counter_file(counter_name, ("ntt.hip",)) if counter_name else None
    if cnt:
        traffic = round((cnt["read_bytes_per_limb"] + cnt["write_bytes_per_limb"]) * per_call)
    hbm_gbs = alg_bytes / avg_s / 1e9
    alu_t = bfly / avg_s / 1e12
    out = {"kernel": "ntt", "traffic": traffic, "traffic_unit": "bytes/call",
           "algorithmic_bytes_per_call": round(alg_bytes), "butterflies_per_call": round(bfly),
           "hbm_floor_us_per_call": round(hbm_floor_s * 1e6, 2), "alu_floor_us_per_call": round(alu_floor_s * 1e6, 2),
           "avg_call_us": round(avg_s * 1e6, 2), "calls": calls, "kernel_launches_per_call": 2 if log_n > 14 else 1,
           "limbs": limbs, "share_of_step": round(prof_ms / (total_s * 1e3), 3),
           "hbm_algorithmic_gbs": round(hbm_gbs, 1), "alu_tbutterfly_per_s": round(alu_t, 3),
           "alu_frac": round(alu_t / NTT_PEAK_TBFLY, 4)}
    if hbm_floor_s >= alu_floor_s:
        out.update({"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)})
    else:
        out.update({"bound": "alu", "achieved": round(alu_t, 3), "peak": round(NTT_PEAK_TBFLY, 3),
                    "unit": "Tbutterfly/s", "frac": round(alu_t / NTT_PEAK_TBFLY, 4)})
    if traffic:
        out["counter_gbs"] = round(traffic / avg_s / 1e9, 1)
        out["counter_frac"] = round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4)
    # the fixed key order of the contract first
    return {k: out[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")} | \
        {k: v for k, v in out.items() if k not in ("bound", "achieved", "peak", "unit", "frac", "traffic")}


def log_free(tag):
    import torch
    free, total = torch.cuda.mem_get_info()
    log("%s: %.1f of %.1f GiB free" % (tag, free / 2 ** 30, total / 2 ** 30))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if xs else None


def conv_setup(vr, level, sets, ntt_plan="auto"):
    import synthetic_inputs as SI
    W = SI.CONV_28
    ctx = vr.Context(14, [60] + [40] * 7, [60], 8, 40.0)
    if ntt_plan != "auto":
        ctx.set_tuning("ntt", ntt_plan)
    keys = ctx.keygen(1002, rot_steps=[1, 2, 3])
    _, K, bias = W.draw()
    cols = []
    for s in range(sets):
        X = SI.images(W.seed + 1000 * s, W.batch, W.channels, W.h, W.w)
        cols.append(ctx.encrypt_columns(keys, X, W.pad, level, 1002, 10000 * s))
    return W, ctx, keys, K, bias, cols


def decoded_gap(ctx, keys, got, ref):
    """max |decode(got) - decode(ref)| / max |decode(ref)| over paired
    ciphertexts: the per-operation path runs the plain conv (a ModDown per
    rotation) where the layer calls round once per output, so the two agree
    in their messages, not their limbs."""
    num = den = 0.0
    for a, b in zip(got, ref):
        da, db = ctx.decode(ctx.decrypt(keys, a)), ctx.decode(ctx.decrypt(keys, b))
        num = max(num, float(np.max(np.abs(da - db))))
        den = max(den, float(np.max(np.abs(db))))
    return num / den if den else num


def step_batched(ctx, keys, W, K, bias, cols):
    """All sets in one multi-set conv call, then x^2 over every output."""
    flat = [c for cs in cols for c in cs]
    y = ctx.conv2d_sets(keys, flat, len(cols), W.channels, W.h, W.w, W.pad, K, bias, W.stride)
    return ctx.square(keys, y)


def plain_conv_sq_fc(X, K, bias, stride, pad, Wfc, bfc):
    """FP64 plaintext network (conv, x^2, FC) for the decoded-error check."""
    B, C, h, w = X.shape
    Co, _, k, _ = K.shape
    Xp = np.pad(X, ((0, 0), (0, 0), (pad, pad), (pad, pad)))
    ho, wo = (h + 2 * pad - k) // stride + 1, (w + 2 * pad - k) // stride + 1
    Y = np.zeros((B, Co, ho, wo)) + bias[None, :, None, None]
    for u in range(k):
        for v in range(k):
            patch = Xp[:, :, u:u + stride * ho:stride, v:v + stride * wo:stride]
            Y += np.einsum("bchw,oc->bohw", patch, K[:, :, u, v])
    Y = Y ** 2
    return Y.reshape(B, -1) @ Wfc.reshape(Wfc.shape[0], -1).T + bfc[None, :]


def cnn128_bench(vr, level_in, sets, reps, graph=False):
    from paper_2512_18646_amd import perop
    """The 3x128x128 CNN (conv 3x3/2 pad 1 x8, x^2, FC 8*64*64 -> 10) at
    N = 2^16, L = 24 (60 + 24x50, P 9x51, dnum 3), 128 images per set (one
    set = 384 column ciphertexts), sets evaluated one after another."""
    import synthetic_inputs as SI
    W = SI.CNN_128
    ctx = vr.Context(16, [60] + [50] * 24, [51] * 9, 3, 50.0)
    Hp = 1 << (W.h + 2 * W.pad - 1).bit_length()
    steps = sorted(set(range(1, W.k)) | {1 << t for t in range(Hp.bit_length() - 1)})
    t = time.perf_counter()
    keys = ctx.keygen(1003, rot_steps=steps)
    X0, K, bias = W.draw()
    Wfc, bfc = W.draw_fc()
    Xs = [X0] + [SI.images(W.seed + 1000 * i, W.batch, W.channels, W.h, W.w) for i in range(1, sets)]
    cols = [ctx.encrypt_columns(keys, X, W.pad, level_in, 1003, 10000 * i) for i, X in enumerate(Xs)]
    wo = (W.w + 2 * W.pad - W.k) // W.stride + 1
    W_pt = ctx.encode_fc_weights(Wfc, W.stride, Hp, level_in - 2)
    sync()
    setup_s = time.perf_counter() - t

    def network(c):
        y = ctx.conv2d(keys, c, W.channels, W.h, W.w, W.pad, K, bias, W.stride)
        y2 = ctx.square(keys, y)
        del y
        return ctx.fc(keys, y2, W.c_out, wo, W_pt, bfc, Hp)

    z = network(cols[0])
    logits = np.zeros((W.batch, len(z)))
    for o, ct in enumerate(z):
        logits[:, o] = ctx.decode(ctx.decrypt(keys, ct))[np.arange(W.batch) * Hp]
    ref = plain_conv_sq_fc(X0, K, bias, W.stride, W.pad, Wfc, bfc)
    err = float(np.max(np.abs(logits - ref)) / np.max(np.abs(ref)))
    del z
    sync()
    lat = []
    t_all = time.perf_counter()
    for r in range(reps):
        for c in cols:
            t = time.perf_counter()
            z = network(c)
            sync()
            lat.append((time.perf_counter() - t) * 1e3)
            del z
    total = time.perf_counter() - t_all
    res = {"workload": "3x128x128 images, conv 3x3/2 pad 1 x8 + x^2 + FC 32768->10, N=2^16 L=24, "
                       "128 images per set", "level_in": level_in, "sets": sets, "reps": reps,
           "path": "three layer calls per set (conv, x^2, FC)",
           "images_per_s": round(W.batch * sets * reps / total, 2),
           "ms_per_set_p50": round(percentile(lat, 50), 2), "ms_per_set_p99": round(percentile(lat, 99), 2),
           "decoded_rel_error": err, "setup_s": round(setup_s, 1)}
    if graph:
        # every set in one whole-network call, and that call captured as one
        # HIP graph and replayed; limbs against the layer calls
        net = vr.CNN(W.channels, W.h, W.w, W.pad, K, bias, W.stride, square=True, fc_w=W_pt,
                     fc_bias=bfc, fc_block=Hp)
        flat = [c for cs in cols for c in cs]
        ref = network(cols[0])
        z = net.forward(ctx, keys, flat, n_sets=sets)
        sync()
        same = all(np.array_equal(z[i].export(), ref[i].export()) for i in range(len(ref)))
        del z
        t = time.perf_counter()
        for r in range(reps):
            z = net.forward(ctx, keys, flat, n_sets=sets)
            sync()
            del z
        res["network_call"] = {"images_per_s": round(W.batch * sets * reps / (time.perf_counter() - t), 2),
                               "identical": bool(same)}
        gr = vr.Graph(ctx, keys, net, flat, n_sets=sets)
        gr.launch()
        sync()
        glat = []
        t = time.perf_counter()
        for r in range(reps):
            t1 = time.perf_counter()
            gr.launch()
            sync()
            glat.append((time.perf_counter() - t1) * 1e3)
        g_total = time.perf_counter() - t
        gout = gr.outputs()
        same = all(np.array_equal(gout[i].export(), ref[i].export()) for i in range(len(ref)))
        res["graph"] = {"images_per_s": round(W.batch * sets * reps / g_total, 2),
                        "ms_per_replay_p50": round(percentile(glat, 50), 2), "identical": bool(same)}
        gr.close()
        # one C-ABI call per HE operation on the first set
        t = time.perf_counter()
        y = perop.square(ctx, keys, perop.conv2d(ctx, keys, cols[0], W.channels, W.h, W.w, W.pad, K, bias,
                                                 W.stride))
        zp = perop.fc(ctx, keys, y, W_pt, bfc, Hp)
        sync()
        t_op = time.perf_counter() - t
        res["per_op"] = {"images_per_s": round(W.batch / t_op, 2),
                         "message_rel_diff": decoded_gap(ctx, keys, zp, ref)}
        del gout, ref, y, zp
    reserved, _ = ctx.mem_info()
    res["device_gib_reserved"] = round(reserved / 2 ** 30, 1)
    return res


def uneven_bench(vr, n_req, level, reps, seed=4):
    """64 mixed requests at N = 2^16 (L = 24 chain, entering at `level`):
    products with m, n, p in 8..32 and 3x3/2 convolutions (8 filters, x^2)
    on 32x32 or 64x64 images, one full ciphertext set each.  Per-request calls
    versus one eager batch versus the batch captured as one HIP graph."""
    import synthetic_inputs as SI
    reqs = SI.uneven_requests(seed, n_req)
    ctx = vr.Context(16, [60] + [50] * 24, [51] * 9, 3, 50.0)
    max_p = max(1 << (min(r[1][0], r[1][2]) - 1).bit_length() for r in reqs if r[0] == "matmul")
    keys = ctx.keygen(1004, rot_steps=list(range(1, max(max_p, 3))))
    nets, items = {}, []
    images = 0
    for i, (kind, shape, rs) in enumerate(reqs):
        if kind == "matmul":
            m, n, p = shape
            A, B = SI.matmul_operands(rs, m, n, p)
            items.append(("matmul", ctx.encrypt_matrix_columns(keys, A, 0, m, p, level, 1004, (2 * i) << 20),
                          ctx.encrypt_matrix_columns(keys, B, 1, m, p, level, 1004, (2 * i + 1) << 20),
                          (m, n, p), (A, B)))
        else:
            side = shape
            if side not in nets:
                K, bias = SI.conv_weights(seed + side, 8, 1, 3, 0.05)
                nets[side] = vr.CNN(1, side, side, 1, K, bias, 2, square=True)
            hp = 1 << (side + 1).bit_length()
            B = ctx.slots // hp
            X = SI.images(rs, B, 1, side, side)
            items.append(("conv", ctx.encrypt_columns(keys, X, 1, level, 1004, (2 * i) << 20), side, B))
            images += B

    def per_request():
        outs = []
        for it in items:
            if it[0] == "matmul":
                m, n, p = it[3]
                outs.append(ctx.matmul(keys, it[1], it[2], m, n, p))
            else:
                outs.append(nets[it[2]].forward(ctx, keys, it[1]))
        return outs

    ref = per_request()
    sync()
    t = time.perf_counter()
    for _ in range(reps):
        per_request()
    sync()
    t_per = (time.perf_counter() - t) / reps
    batch = vr.Batch(ctx, keys)
    ids = [batch.add_matmul(it[1], it[2], *it[3]) if it[0] == "matmul" else batch.add_cnn(nets[it[2]], it[1])
           for it in items]
    batch.run()
    sync()
    t = time.perf_counter()
    for _ in range(reps):
        batch.run()
    sync()
    t_batch = (time.perf_counter() - t) / reps
    same_eager = all(np.array_equal(batch.outputs(ids[i])[0].export(), ref[i][0].export()) for i in (0, 1, 2, 3))
    batch.capture()
    batch.launch()
    sync()
    t = time.perf_counter()
    for _ in range(reps):
        batch.launch()
    sync()
    t_graph = (time.perf_counter() - t) / reps
    same_graph = all(np.array_equal(batch.outputs(ids[i])[-1].export(), ref[i][-1].export()) for i in range(len(ids)))
    # decoded check of the first product
    m, n, p = items[0][3]
    A, B = items[0][4]
    outs = batch.outputs(ids[0])
    Pp = len(outs)
    C = np.full((m, p), np.nan)
    for idx, ct in enumerate(outs):
        if m >= p:    # slot r: C[r][(r + idx) mod P']
            z = ctx.decode(ctx.decrypt(keys, ct), m)
            for r in range(m):
                if (r + idx) % Pp < p:
                    C[r, (r + idx) % Pp] = z[r]
        else:         # transposed product: slot i: C[(i + idx) mod M'][i]
            z = ctx.decode(ctx.decrypt(keys, ct), p)
            for i in range(p):
                if (i + idx) % Pp < m:
                    C[(i + idx) % Pp, i] = z[i]
    err = float(np.nanmax(np.abs(C - A @ B)) / np.max(np.abs(A @ B)))
    batch.close()
    n_mm = sum(1 for it in items if it[0] == "matmul")
    return {"workload": "%d requests: %d products (m, n, p in 8..32), %d 3x3/2 x8 + x^2 convolutions on "
                        "32x32 / 64x64 images (full sets), N=2^16 L=24 chain at level %d"
                        % (n_req, n_mm, n_req - n_mm, level),
            "requests_per_s": {"per_request": round(n_req / t_per, 1), "batch": round(n_req / t_batch, 1),
                               "graph": round(n_req / t_graph, 1)},
            "conv_images_per_s": {"per_request": round(images / t_per, 1), "batch": round(images / t_batch, 1),
                                  "graph": round(images / t_graph, 1)},
            "identical_to_per_request": bool(same_eager and same_graph), "product_rel_error": err}


def uneven_full_bench(vr, n_req, level, reps, seed=4):
    """The mixed batch at its full size ranges, N = 2^16 (L = 24 chain,
    entering at `level`): products with m, n, p uniform in 16..512 through the
    outer-product form (vr_matmul_outer: row tiles, no rotation) and 3x3/2
    convolutions (8 filters, x^2) on 32x32 .. 256x256 images (full ciphertext
    sets): one call per request, one eager uneven batch (vr_batch_*) and the
    batch captured as one HIP graph, with limb identity of sampled requests.
    Reports the rotations the column-split form would have needed
    (n (P' - 1) per product, transposed when p > m)."""
    import synthetic_inputs as SI
    reqs = SI.uneven_requests(seed, n_req, dim_range=(16, 512), sides=(32, 64, 128, 256))
    ctx = vr.Context(16, [60] + [50] * 24, [51] * 9, 3, 50.0)
    keys = ctx.keygen(1004, rot_steps=[1, 2])
    t0 = time.perf_counter()
    nets, items = {}, []
    images = rot_split = tensors = 0
    for i, (kind, shape, rs) in enumerate(reqs):
        if kind == "matmul":
            m, n, p = shape
            A, B = SI.matmul_operands(rs, m, n, p)
            items.append(("matmul", ctx.encrypt_matrix_columns(keys, A, 2, m, p, level, 1004, (2 * i) << 20),
                          ctx.encrypt_matrix_columns(keys, B, 3, m, p, level, 1004, (2 * i + 1) << 20),
                          (m, n, p), (A, B)))
            lo, hi = min(m, p), max(m, p)
            rot_split += n * ((1 << (lo - 1).bit_length()) - 1)
            tensors += ctx.outer_tiles(m, p)[2] * n
        else:
            side = shape
            if side not in nets:
                K, bias = SI.conv_weights(seed + side, 8, 1, 3, 0.05)
                nets[side] = vr.CNN(1, side, side, 1, K, bias, 2, square=True)
            hp = 1 << (side + 1).bit_length()
            B = ctx.slots // hp
            X = SI.images(rs, B, 1, side, side)
            items.append(("conv", ctx.encrypt_columns(keys, X, 1, level, 1004, (2 * i) << 20), side, B))
            images += B
    sync()
    setup_s = time.perf_counter() - t0

    def run():
        outs = []
        for it in items:
            if it[0] == "matmul":
                outs.append(ctx.matmul_outer(keys, it[1], it[2], *it[3]))
            else:
                outs.append(nets[it[2]].forward(ctx, keys, it[1]))
        return outs

    outs = run()
    sync()
    # decoded check of every product against FP64
    err = 0.0
    for it, o in zip(items, outs):
        if it[0] != "matmul":
            continue
        (m, n, p), (A, B) = it[3], it[4]
        Pp, R, T = ctx.outer_tiles(m, p)
        C = np.zeros((m, p))
        for t, ct in enumerate(o):
            z = ctx.decode(ctx.decrypt(keys, ct))
            rows = min(R, m - t * R)
            C[t * R:t * R + rows] = z[:rows * Pp].reshape(rows, Pp)[:, :p]
        err = max(err, float(np.max(np.abs(C - A @ B)) / np.max(np.abs(A @ B))))
    # requests whose limbs the batch and its graph must reproduce
    check = [0, 1, 2, 3, n_req // 2, n_req // 2 + 1, n_req - 2, n_req - 1]
    ref = {i: [c.export() for c in outs[i][:2]] for i in check}
    del outs
    t = time.perf_counter()
    for _ in range(reps):
        o = run()
        del o
    sync()
    t_run = (time.perf_counter() - t) / reps
    n_mm = sum(1 for it in items if it[0] == "matmul")
    # every request in one uneven batch (the batch references the callers'
    # input slabs, so the callers' handles are released once added), eager
    # and captured as one graph
    batch = vr.Batch(ctx, keys)
    ids = []
    for i, it in enumerate(items):
        ids.append(batch.add_matmul_outer(it[1], it[2], *it[3]) if it[0] == "matmul"
                   else batch.add_cnn(nets[it[2]], it[1]))
        items[i] = None
    items = None
    sync()

    def identical():
        return all(np.array_equal(batch.outputs(ids[i])[k].export(), ref[i][k])
                   for i in check for k in range(len(ref[i])))

    batch.run()
    sync()
    same_eager = identical()
    t = time.perf_counter()
    for _ in range(reps):
        batch.run()
    sync()
    t_batch = (time.perf_counter() - t) / reps
    batch.capture()
    batch.launch()
    sync()
    t = time.perf_counter()
    for _ in range(reps):
        batch.launch()
    sync()
    t_graph = (time.perf_counter() - t) / reps
    same_graph = identical()
    batch.close()
    reserved, _ = ctx.mem_info()
    return {"workload": "%d requests: %d products (m, n, p in 16..512, outer-product form), %d 3x3/2 x8 + x^2 "
                        "convolutions on 32x32 .. 256x256 images (full sets), N=2^16 L=24 chain at level %d"
                        % (n_req, n_mm, n_req - n_mm, level),
            "requests_per_s": {"per_request": round(n_req / t_run, 2), "batch": round(n_req / t_batch, 2),
                               "graph": round(n_req / t_graph, 2)},
            "ms_for_all": {"per_request": round(t_run * 1e3, 1), "batch": round(t_batch * 1e3, 1),
                           "graph": round(t_graph * 1e3, 1)},
            "conv_images_per_s": {"per_request": round(images / t_run, 1), "batch": round(images / t_batch, 1),
                                  "graph": round(images / t_graph, 1)},
            "identical_to_per_request": bool(same_eager and same_graph), "identity_checked_requests": check,
            "product_tensors": tensors, "column_split_rotations_avoided": rot_split,
            "products_max_rel_error": err, "setup_s": round(setup_s, 1),
            "device_gib_reserved": round(reserved / 2 ** 30, 1)}


def serving_n16_bench(vr, level=3, n_sessions=8, n_warm=20, n_meas=100, loads=(0.25, 0.5, 0.75, 0.9),
                      seed=5, max_batch=4):
    """Serving at N = 2^16 (L = 24 chain, requests entering at `level`): 8
    sessions with resident keys, Poisson arrivals of 28x28 (1 channel),
    64x64 and 128x128 (3 channels) requests in a 5:3:2 mix, each carrying
    b ~ U{1..B'} images, through the 3x3/2 x8 conv + x^2 + FC 8(s/2)^2 -> 10
    network adapted to the size.  Offered load swept as fractions of the
    saturating request rate measured first on a burst."""
    import synthetic_inputs as SI
    ctx = vr.Context(16, [60] + [50] * 24, [51] * 9, 3, 50.0)
    steps = [1, 2] + [1 << t for t in range(2, 8)]
    sessions = [ctx.keygen(2000 + i, rot_steps=steps) for i in range(n_sessions)]
    kinds = []
    for side, ch, frac in ((28, 1, 0.5), (64, 3, 0.3), (128, 3, 0.2)):
        K, bias = SI.conv_weights(seed + side, 8, ch, 3, 0.05)
        hp = 1 << (side + 1).bit_length()
        wo = (side + 2 - 3) // 2 + 1
        Wfc, bfc = SI.fc_weights(seed + 7 * side, 10, 8, wo, wo, 0.05)
        # the FC runs at level 1, or at level 3 when the requests enter high
        # enough: x^2 then goes into it unrelinearised (one key switch per FC
        # output) and the conv makes only the FC's limbs
        pts = ctx.encode_fc_weights(Wfc, 2, hp, 3 if level >= 4 else 1)
        net = vr.CNN(ch, side, side, 1, K, bias, 2, square=True, fc_w=pts, fc_bias=bfc, fc_block=hp)
        bmax = ctx.slots // hp
        cols = [ctx.encrypt_columns(keys, SI.images(seed + 31 * i + side, bmax, ch, side, side), 1, level,
                                    3000 + i, 100000 * side) for i, keys in enumerate(sessions)]
        kinds.append({"side": side, "net": net, "bmax": bmax, "cols": cols, "frac": frac})
    probs = np.array([k["frac"] for k in kinds])
    free, total = __import__("torch").cuda.mem_get_info()
    srv = vr.Server(ctx, int(total * 0.9), max_batch=max_batch)
    sids = [srv.register_session(k) for k in sessions]
    for k in kinds:
        k["mid"] = srv.register_model(k["net"])
    rng = np.random.default_rng(seed)

    def draw_request():
        ki = int(rng.choice(len(kinds), p=probs))
        si = int(rng.integers(n_sessions))
        k = kinds[ki]
        return ki, si, int(rng.integers(1, k["bmax"] + 1))

    def run(n, rate, tag=None):
        # results are collected once 256 newer requests are in flight, so a
        # long run holds a bounded number of outputs
        pending = collections.deque()
        t0 = time.perf_counter()
        due = t0
        for i in range(n):
            ki, si, b = draw_request()
            if rate:
                due += rng.exponential(1.0 / rate)
                delay = due - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            k = kinds[ki]
            pending.append((srv.submit(sids[si], k["mid"], k["cols"][si], b), k["mid"]))
            while len(pending) > 256:
                t, mid = pending.popleft()
                srv.poll(t, mid)
            if tag and (i + 1) % 500 == 0:
                log("%s: %d of %d requests submitted" % (tag, i + 1, n))
        while pending:
            t, mid = pending.popleft()
            srv.poll(t, mid)

    for k in kinds:                              # warm the cached constants of every network
        srv.poll(srv.submit(sids[0], k["mid"], k["cols"][0], 1), k["mid"])
    t0 = time.perf_counter()                     # saturation: a burst
    srv.reset_stats()
    n_burst = max(24, min(48, n_meas))
    run(n_burst, 0)
    burst_s = time.perf_counter() - t0
    sat = srv.stats()
    sat_req_s = n_burst / burst_s
    levels = []
    for load in loads:
        run(n_warm, load * sat_req_s)
        srv.reset_stats()
        run(n_meas, load * sat_req_s, "level %d, load %.2f" % (level, load))
        st = srv.stats()
        levels.append({"offered_load": load, "offered_req_per_s": round(load * sat_req_s, 2),
                       "images_per_s": round(st["images_per_s"], 1), "latency_ms_p50": round(st["p50_ms"], 2),
                       "latency_ms_p99": round(st["p99_ms"], 2),
                       "requests_per_wave": round(st["batched"] / max(st["waves"], 1), 2)})
    srv.close()
    return {"workload": "5:3:2 of 28x28x1 / 64x64x3 / 128x128x3 requests, b ~ U{1..B'} images each "
                        "(B' = 1024 / 256 / 128), conv 3x3/2 x8 + x^2 + FC -> 10, %d sessions, N=2^16 L=24 "
                        "chain at level %d, %d measured requests per load" % (n_sessions, level, n_meas),
            "saturation": {"req_per_s": round(sat_req_s, 2), "images_per_s": round(sat["images_per_s"], 1),
                           "latency_ms_p50": round(sat["p50_ms"], 2), "latency_ms_p99": round(sat["p99_ms"], 2),
                           "requests_per_wave": round(sat["batched"] / max(sat["waves"], 1), 2)},
            "loads": levels}


SERVE_MIX = (("28x28", 28, 0.5), ("64x64", 64, 0.3), ("128x128", 128, 0.2))


def serving_bench(vr, ctx, keys, n_req, load, level, seed=7):
    """Poisson arrivals of single-set requests with the 5:3:2 image-size mix
    (conv 4x4/2 x5 + x^2, one ciphertext set per request) through the
    continuous-batching server; latency is submit-to-completion."""
    import synthetic_inputs as SI
    _, K, bias = SI.CONV_28.draw()
    srv = vr.Server(ctx, 200 << 30, max_batch=4)
    sid = srv.register_session(keys)
    kinds = []
    for name, hw, _ in SERVE_MIX:
        mid = srv.register_conv_model(1, hw, hw, 0, K, bias, 2, square=True)
        B = ctx.slots // (1 << (hw - 1).bit_length())
        cols = ctx.encrypt_columns(keys, SI.images(seed + hw, B, 1, hw, hw), 0, level, 3000 + hw, 0)
        kinds.append((name, mid, cols, B))
    # service time of each kind alone (also warms the cached layer constants)
    alone_ms, alone_out = [], []
    for name, mid, cols, B in kinds:
        srv.poll(srv.submit(sid, mid, cols, B), mid)
        t = time.perf_counter()
        alone_out.append(srv.poll(srv.submit(sid, mid, cols, B), mid))
        alone_ms.append((time.perf_counter() - t) * 1e3)
    probs = np.array([p for _, _, p in SERVE_MIX])
    mean_ms = float(np.dot(probs, alone_ms))
    rate = load * 1e3 / mean_ms          # requests/s offered
    srv.close()
    srv = vr.Server(ctx, 200 << 30, max_batch=4)
    sid = srv.register_session(keys)
    for name, hw, _ in SERVE_MIX:
        srv.register_conv_model(1, hw, hw, 0, K, bias, 2, square=True)
    rng = np.random.default_rng(seed)
    which = rng.choice(len(kinds), size=n_req, p=probs)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    tickets = []
    t0 = time.perf_counter()
    due = t0
    for i in range(n_req):
        due += gaps[i]
        delay = due - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        name, mid, cols, B = kinds[which[i]]
        tickets.append((srv.submit(sid, mid, cols, B), which[i]))
    outs = {}
    for t, k in tickets:
        outs.setdefault(k, srv.poll(t, kinds[k][1]))
    st = srv.stats()
    srv.close()
    same = all(np.array_equal(outs[k][j].export(), alone_out[k][j].export())
               for k in outs for j in (0, len(outs[k]) - 1))
    return {"mix": "5:3:2 of 28x28 (256 img), 64x64 (128 img), 128x128 (64 img) per request, "
                   "N=2^14 L=7", "requests": n_req, "offered_load": load,
            "offered_req_per_s": round(rate, 2), "alone_ms": [round(x, 2) for x in alone_ms],
            "images_per_s": round(st["images_per_s"], 1), "latency_ms_p50": round(st["p50_ms"], 2),
            "latency_ms_p99": round(st["p99_ms"], 2), "waves": st["waves"],
            "requests_per_wave": round(st["batched"] / max(st["waves"], 1), 2),
            "identical_to_alone": bool(same)}


def sync():
    import torch
    torch.cuda.synchronize()


def rotations_bench(vr, level, n_ct, reps, ntt_plan="auto"):
    """HE rotations/s at N = 2^16: n_ct ciphertexts rotated by one step
    (ntt_plan: auto, or cand:i to pin the transform plan, e.g. for counter
    runs)."""
    ctx = vr.Context(16, [60] + [50] * 24, [51] * 9, 3, 50.0)
    if ntt_plan != "auto":
        ctx.set_tuning("ntt", ntt_plan)
    keys = ctx.keygen(1003, rot_steps=[1])
    z = np.random.default_rng(3).uniform(-1, 1, ctx.slots)
    cts = [ctx.encrypt(keys, ctx.encode(z, level), 1003, (3 << 20) + 64 * level + i) for i in range(n_ct)]
    out = {}
    ctx.rotate_batch(keys, cts, 1)
    sync()
    t = time.perf_counter()
    for _ in range(reps):
        r = ctx.rotate_batch(keys, cts, 1)
    sync()
    out["batched"] = n_ct * reps / (time.perf_counter() - t)
    ctx.rotate(keys, cts[0], 1)
    sync()
    t = time.perf_counter()
    for _ in range(reps):
        r1 = [ctx.rotate(keys, c, 1) for c in cts]
    sync()
    out["per_op"] = n_ct * reps / (time.perf_counter() - t)
    out["identical"] = bool(np.array_equal(r[0].export(), r1[0].export()))
    out["hbm_roofline"] = keyswitch_roofline(ctx, keys, cts, level, reps)
    out["base_convert"] = convert_compare(ctx, keys, cts, level, reps)
    return out


def keyswitch_roofline(ctx, keys, cts, level, reps):
    """HBM rooflines of the batched rotation's NTT and key-switch inner
    product, from the device time of every launch (HIP events):
    NTT: a limb moves 16N bytes (read and write once); with two passes
    (N = 2^16) the passes move 32N, the bytes HBM must carry.
    Inner product: a unit (ciphertext x extended limb) reads its beta digit
    limbs and writes two output limbs, 8N (beta + 2) bytes, plus the key's
    2 beta limbs of that extended limb, 16N beta, read once per batch."""
    n = ctx.n
    beta = -(-(level + 1) // ctx.alpha)
    res = {}
    cnt = counter_file("rotations_n16_hbm_counters.json", ("ntt.hip", "keyswitch.hip"))
    for cls in ("ntt", "ks_inner"):
        ctx.profile_start(cls, 1 << 14)
        for _ in range(reps):
            r = ctx.rotate_batch(keys, cts, 1)
            del r
        ms, la, un, _ = ctx.profile_stop()
        s_dev = ms / 1e3
        if cls == "ntt":
            moved = 32 * n * un if ctx.log_n > 14 else 16 * n * un
            alg = 16 * n * un
            res["ntt"] = {"launches_per_batch": la // reps, "limbs_per_batch": un // reps,
                          "us_per_batch": round(ms * 1e3 / reps, 1),
                          "pass_traffic_gbs": round(moved / s_dev / 1e9, 1),
                          "pass_traffic_frac_of_8000": round(moved / s_dev / 1e9 / HBM_PEAK_GBS, 4),
                          "algorithmic_gbs": round(alg / s_dev / 1e9, 1),
                          "algorithmic_frac_of_8000": round(alg / s_dev / 1e9 / HBM_PEAK_GBS, 4)}
            if cnt and level == 24 and len(cts) == 8:
                c = cnt["ntt_level24"]["bytes_per_limb"] * un / s_dev / 1e9
                res["ntt"]["counter_gbs"] = round(c, 1)
                res["ntt"]["counter_frac_of_8000"] = round(c / HBM_PEAK_GBS, 4)
        else:
            b = 8 * n * (beta + 2) * un + 16 * n * beta * un // len(cts)
            res["ks_inner"] = {"launches_per_batch": la // reps, "units_per_batch": un // reps,
                               "us_per_batch": round(ms * 1e3 / reps, 1),
                               "algorithmic_gbs": round(b / s_dev / 1e9, 1),
                               "algorithmic_frac_of_8000": round(b / s_dev / 1e9 / HBM_PEAK_GBS, 4)}
            k = cnt["ks_inner"].get(str(level)) if cnt else None
            if k and un // reps == k["units"]:
                c = (k["read_bytes_per_unit"] + k["write_bytes_per_unit"]) * un / s_dev / 1e9
                res["ks_inner"]["counter_gbs"] = round(c, 1)
                res["ks_inner"]["counter_frac_of_8000"] = round(c / HBM_PEAK_GBS, 4)
    return res


def counter_file(name, sources):
    """Counter-derived bytes per unit from profiles/, only while every kernel
    source it was measured on is byte-identical (else None)."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            cnt = json.load(f)
        for src in sources:
            with open(os.path.join(ROOT, "paper_2512_18646_amd", "csrc", src), "rb") as f:
                key = src.split(".")[0] + "_source_sha256_prefix"
                if not hashlib.sha256(f.read()).hexdigest().startswith(cnt[key]):
                    return None
        return cnt
    except (OSError, KeyError, ValueError):
        return None


def mfma_instructions(log_n, level, n_ct, alpha=9, K=9):
    """v_mfma_i32_16x16x32_i8 issued by one rotate_batch of n_ct ciphertexts
    (ModUp of every digit, ModDown of both halves)."""
    n16 = (1 << log_n) // 16
    nq, nxt = level + 1, level + 1 + K

    def conv(n_in, n_out, polys):
        return polys * n16 * ((n_out + 3) // 4) * 4 * ((n_in + 1 + 3) // 4)

    total = 0
    for j in range((nq + alpha - 1) // alpha):
        n_in = min(alpha, nq - j * alpha)
        total += conv(n_in, nxt - n_in, n_ct)
    return total + conv(K, nq, 2 * n_ct)


def convert_compare(ctx, keys, cts, level, reps):
    """Base-conversion device time per rotation with each kernel forced."""
    res = {}
    for mode in ("alu", "fp64", "mfma"):
        ctx.set_tuning("base_convert", mode)
        ctx.rotate_batch(keys, cts, 1)
        sync()
        ctx.profile_start("base_convert", 1 << 14)
        for _ in range(reps):
            ctx.rotate_batch(keys, cts, 1)
        ms, launches, _, _ = ctx.profile_stop()
        res[mode + "_us_per_rotation"] = round(ms * 1e3 / (reps * len(cts)), 2)
        if mode == "mfma":
            ops = mfma_instructions(16, level, len(cts)) * reps * 16 * 16 * 32 * 2
            tops = ops / (ms / 1e3) / 1e12
            res["mfma_int8_tops"] = round(tops, 1)
            res["mfma_util_of_5000_tops"] = round(tops / 5000.0, 4)
    ctx.set_tuning("base_convert", "auto")
    ctx.rotate_batch(keys, cts, 1)
    sync()
    res["autotuned"] = sorted(set(line.split(": ")[1] for line in ctx.tuning_report().splitlines()
                                  if ": " in line))
    return res


def cnn128_setup(vr, level_in, sets, fc_level=3, ntt_plan="auto"):
    """The 3x128x128 network at N = 2^16 (60 + 24x50, P 9x51, dnum 3): keys,
    `sets` encrypted 128-image sets (384 column ciphertexts each) entering at
    level_in, and the network (conv 3x3/2 pad 1 x8, x^2, FC 8*64*64 -> 10 with
    its weights encoded at fc_level, the level the FC runs at: at 3 the
    network call takes the x^2 tensors into the FC unrelinearised and
    relinearises the ten sums)."""
    import synthetic_inputs as SI
    W = SI.CNN_128
    ctx = vr.Context(16, [60] + [50] * 24, [51] * 9, 3, 50.0)
    if ntt_plan != "auto":
        ctx.set_tuning("ntt", ntt_plan)
    Hp = 1 << (W.h + 2 * W.pad - 1).bit_length()
    steps = sorted(set(range(1, W.k)) | {1 << t for t in range(Hp.bit_length() - 1)})
    keys = ctx.keygen(1003, rot_steps=steps)
    X0, K, bias = W.draw()
    Wfc, bfc = W.draw_fc()
    Xs = [X0] + [SI.images(W.seed + 1000 * i, W.batch, W.channels, W.h, W.w) for i in range(1, sets)]
    cols = [ctx.encrypt_columns(keys, X, W.pad, level_in, 1003, 10000 * i) for i, X in enumerate(Xs)]
    fc_level = min(fc_level, level_in - 1)
    W_pt = ctx.encode_fc_weights(Wfc, W.stride, Hp, fc_level)
    net = vr.CNN(W.channels, W.h, W.w, W.pad, K, bias, W.stride, square=True, fc_w=W_pt, fc_bias=bfc,
                 fc_block=Hp)
    return {"W": W, "ctx": ctx, "keys": keys, "X0": X0, "K": K, "bias": bias, "Wfc": Wfc, "bfc": bfc,
            "W_pt": W_pt, "Hp": Hp, "cols": cols, "net": net, "fc_level": fc_level}


def cnn128_logit_error(C, z):
    """Decoded logits of set 0 against the FP64 plaintext network."""
    W, ctx, keys = C["W"], C["ctx"], C["keys"]
    logits = np.zeros((W.batch, len(z)))
    for o, ct in enumerate(z):
        logits[:, o] = ctx.decode(ctx.decrypt(keys, ct))[np.arange(W.batch) * C["Hp"]]
    ref = plain_conv_sq_fc(C["X0"], C["K"], C["bias"], W.stride, W.pad, C["Wfc"], C["bfc"])
    return float(np.max(np.abs(logits - ref)) / np.max(np.abs(ref)))


def headline_extras(vr, perop, C, args, ref, images):
    """The headline step as one replayed HIP graph (limbs against the
    whole-network call) and as one C-ABI call per HE operation on the first
    set (the plain conv schedule: its decoded logits against FP64)."""
    ctx, keys, net, W = C["ctx"], C["keys"], C["net"], C["W"]
    flat = [c for cs in C["cols"] for c in cs]
    res = {}
    ctx.trim()
    gr = vr.Graph(ctx, keys, net, flat, n_sets=len(C["cols"]))
    gr.launch()
    sync()
    glat = []
    t = time.perf_counter()
    for _ in range(max(2, args.steps // 4)):
        t1 = time.perf_counter()
        gr.launch()
        sync()
        glat.append((time.perf_counter() - t1) * 1e3)
    g_total = time.perf_counter() - t
    gout = gr.outputs()
    res["graph"] = {"images_per_s": round(images * len(glat) / g_total, 2),
                    "ms_per_step_p50": round(percentile(glat, 50), 2),
                    "identical": bool(all(np.array_equal(gout[i].export(), ref[i]) for i in range(len(ref))))}
    del gout
    gr.close()
    ctx.trim()
    t = time.perf_counter()
    y = perop.square(ctx, keys, perop.conv2d(ctx, keys, C["cols"][0], W.channels, W.h, W.w, W.pad, C["K"],
                                             C["bias"], W.stride))
    zp = perop.fc(ctx, keys, y, C["W_pt"], C["bfc"], C["Hp"])
    sync()
    t_op = time.perf_counter() - t
    res["per_op"] = {"images_per_s": round(W.batch / t_op, 2),
                     "decoded_rel_error": cnn128_logit_error(C, zp)}
    del y, zp
    return res


def matmul16_bench(vr, perop, reps=20):
    """The 16x16 by 16x16 encrypted product at N = 2^13 (49 + 3x40, P 49,
    dnum 4): 16 + 16 column ciphertexts at level 3, one vr_matmul call per
    product (240 rotations hoisted over 16 ModUps, 256 tensors, 16
    relinearisations); latency p50/p99 over `reps` calls, the per-op path, and
    the decoded error against FP64."""
    import synthetic_inputs as SI
    seed, m, n, p = SI.MATMUL_16
    ctx = vr.Context(13, [49, 40, 40, 40], [49], 4, 40.0)
    keys = ctx.keygen(1001, rot_steps=list(range(1, 16)))
    A, B = SI.matmul_operands(seed, m, n, p)
    Ac = ctx.encrypt_matrix_columns(keys, A, 0, m, p, 3, 1001, 0)
    Bc = ctx.encrypt_matrix_columns(keys, B, 1, m, p, 3, 1001, 1 << 20)
    D = ctx.matmul(keys, Ac, Bc, m, n, p)
    sync()
    lat = []
    for _ in range(reps):
        t = time.perf_counter()
        D = ctx.matmul(keys, Ac, Bc, m, n, p)
        sync()
        lat.append((time.perf_counter() - t) * 1e3)
    C = np.full((m, p), np.nan)
    for idx, ct in enumerate(D):
        z = ctx.decode(ctx.decrypt(keys, ct), m)
        for i in range(m):
            C[i, (i + idx) % 16] = z[i]
    err = float(np.max(np.abs(C - A @ B)) / np.max(np.abs(A @ B)))
    t = time.perf_counter()
    Dp = perop.matmul(ctx, keys, Ac, Bc, m, n, p)
    sync()
    t_op = (time.perf_counter() - t) * 1e3
    same = all(np.array_equal(x.export(), y.export()) for x, y in zip(D, Dp))
    return {"workload": "A(16x16) B(16x16), 16 + 16 column ciphertexts, N=2^13 (49+3x40, P 49, dnum 4), level 3",
            "latency_ms_p50": round(percentile(lat, 50), 3), "latency_ms_p99": round(percentile(lat, 99), 3),
            "per_op_ms": round(t_op, 2), "per_op_identical": bool(same), "decoded_rel_error": err}


def conv28_bench(vr, perop, args):
    """The 28x28 conv + x^2 layer at N = 2^14, L = 7 on 4 sets of 256 images
    per step (multi-set conv call + batched x^2), its graph replay, the per-op
    path on one set, and the live roofline of its NTT class."""
    W, ctx, keys, K, bias, cols = conv_setup(vr, 7, 4, args.ntt_plan)
    images = W.batch * len(cols)
    for _ in range(2):
        step_batched(ctx, keys, W, K, bias, cols)
    sync()
    steps = max(5, args.steps // 2)
    ctx.profile_start("ntt", 1 << 18)
    sync()
    t = time.perf_counter()
    for _ in range(steps):
        y = step_batched(ctx, keys, W, K, bias, cols)
        del y
    sync()
    total = time.perf_counter() - t
    ms, la, un, _ = ctx.profile_stop()
    res = {"workload": "conv 28x28 4x4/2 x5 + x^2, 4 sets of 256 images per step, N=2^14 L=7 (60+7x40, P 60, "
                       "dnum 8)", "images_per_s": round(images * steps / total, 2),
           "ms_per_step": round(total / steps * 1e3, 3),
           "roofline_ntt": ntt_roofline(ms, la, un, total, 14, "ntt_hbm_counters.json")}
    net = vr.CNN(W.channels, W.h, W.w, W.pad, K, bias, W.stride, square=True)
    flat = [c for cs in cols for c in cs]
    gr = vr.Graph(ctx, keys, net, flat, n_sets=len(cols))
    gr.launch()
    sync()
    t = time.perf_counter()
    for _ in range(steps):
        gr.launch()
    sync()
    g_total = time.perf_counter() - t
    ref = step_batched(ctx, keys, W, K, bias, cols[:1])
    gout = gr.outputs()
    res["graph"] = {"images_per_s": round(images * steps / g_total, 2),
                    "identical": bool(all(np.array_equal(gout[i].export(), ref[i].export()) for i in range(len(ref))))}
    gr.close()
    del gout
    t = time.perf_counter()
    ys = perop.square(ctx, keys, perop.conv2d(ctx, keys, cols[0], W.channels, W.h, W.w, W.pad, K, bias, W.stride))
    sync()
    t_op = time.perf_counter() - t
    res["per_op"] = {"images_per_s": round(W.batch / t_op, 2),
                     "message_rel_diff": decoded_gap(ctx, keys, ys, ref)}
    res["batched_over_per_op"] = round(res["images_per_s"] / res["per_op"]["images_per_s"], 2)
    return res


# ------------------------------------------------------------ CPU oracle leg
#
# The oracle runs in a child process that never loads the GPU runtime, so it
# can fork worker processes for the all-core run.

def host_info():
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": ncpu, "cpu_count": os.cpu_count(), "model": model}


_ORC = {}


def _orc_c3_sample(_=None):
    """One sample of every operation class of the C3 network step, on the
    oracle (keys and inputs prepared before the fork): seconds per class."""
    o, ok, cts = _ORC["o"], _ORC["ok"], _ORC["cts"]
    t = {}
    t0 = time.perf_counter()
    r1 = o.rotate_ext(cts[24], 1, ok)
    t["rot24"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    acc = None
    dq = float(o.q[24])
    for r in range(6):
        x = o.mul_const_ext(r1, 0.01 * (r + 1), dq)
        acc = x if acc is None else o.add_ext(acc, x)
    t["mulconst_add24"] = (time.perf_counter() - t0) / 6
    t0 = time.perf_counter()
    y = o.mod_down_rescale(o.add_const_ext(acc, 0.5))
    t["addconst_rescale24"] = time.perf_counter() - t0
    # x^2 into the FC at level 3 (square_fc): tensor on the FC's limbs, the
    # weight products on 3 components, one relinearisation per output
    t0 = time.perf_counter()
    y3 = o.mod_drop(y, 3)
    T = o.tensor(y3, y3)
    t["tensor3"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    acc = None
    for r in range(6):
        x = o.mul_plain(T, _ORC["pt3"])
        acc = x if acc is None else o.add(acc, x)
    t["mulplain_add3"] = (time.perf_counter() - t0) / 6
    t0 = time.perf_counter()
    z = o.rescale(o.relin_rescale(acc, ok))
    t["relin_rescale3"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.add(z, o.rotate(z, 1, ok))
    t["rot_add1"] = time.perf_counter() - t0
    return t


# operation counts of one 128-image set of the C3 network entering at level 24
# (FC weights at level 3: x^2 relinearised once per FC output)
C3_OPS = {"rot24": 768, "mulconst_add24": 13752, "addconst_rescale24": 512, "tensor3": 512,
          "mulplain_add3": 5120, "relin_rescale3": 10, "rot_add1": 80}


def cpu_oracle_child():
    """Runs in a fresh process: the oracle's C3 network step (single core and
    on every host core), C1 whole, the C2 sample, NTT per limb.  Prints JSON."""
    import multiprocessing as mp
    from oracle import Context as OC, PRESETS
    from oracle import layers as Ly
    import synthetic_inputs as SI
    res = {"host": host_info()}
    # C3 at level 24 (keys, one input ciphertext at level 24, one FC weight
    # plaintext at level 3)
    t0 = time.perf_counter()
    o = OC(PRESETS["C3"])
    ok = o.keygen(1003, rot_steps=[1])
    z = np.random.default_rng(3).uniform(0, 1, o.slots)
    _ORC.update(o=o, ok=ok, cts={24: o.encrypt(ok, o.encode(z, 24, o.scale), 1003, 0)},
                pt3=o.encode(z * 0.01, 3, float(o.q[3])))
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    one = _orc_c3_sample()
    t_one = time.perf_counter() - t0
    s_set = sum(C3_OPS[k] * one[k] for k in C3_OPS)
    cores = max(1, min(16, res["host"]["nproc"] or 1))
    ctxmp = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctxmp.Pool(cores) as pool:
        samples = pool.map(_orc_c3_sample, range(cores))
    t_all = time.perf_counter() - t0
    # all-core throughput: cores samples in t_all seconds, each sample standing
    # for sample_weight of a set
    s_set_sample = sum(C3_OPS[k] * one[k] for k in C3_OPS)
    w_sample = t_one / s_set_sample            # fraction of a set one sample represents
    sets_per_s_all = cores * w_sample / t_all
    res["c3_level24"] = {
        "single_core_images_per_s": round(128 / s_set, 5),
        "all_core_images_per_s": round(128 * sets_per_s_all, 5), "cores": cores,
        "seconds_per_op_single_core": {k: round(v, 4) for k, v in one.items()},
        "op_counts_per_set": C3_OPS, "extrapolated": True,
        "sample": "one of each operation class of the 128-image C3 set at level 24 (1 rotation kept in the "
                  "extended basis at level 24, 6 MulConst+Add there, AddConst + ModDown by P q_l, one x^2 "
                  "tensor on the FC's level-3 limbs, 6 MulPlain+Add of 3-component tensors at level 3, one "
                  "relinearise-rescale + rescale, "
                  "rotate+add at level 1), %.1f s on one core, scaled by the set's operation counts; all-core: "
                  "the same sample on %d processes at once (%.1f s wall)" % (t_one, cores, t_all),
        "setup_s": round(setup, 1)}
    del samples
    # C1 whole: 16x16 product at N = 2^13
    oc = OC(PRESETS["C1"])
    okc = oc.keygen(1001, rot_steps=list(range(1, 16)))
    seed, m, n, p = SI.MATMUL_16
    A, B = SI.matmul_operands(seed, m, n, p)
    Ac = Ly.encrypt_matrix_columns(oc, okc, A, 0, m, p, 3, 1001, 0)
    Bc = Ly.encrypt_matrix_columns(oc, okc, B, 1, m, p, 3, 1001, 1 << 20)
    t0 = time.perf_counter()
    Ly.matmul(oc, okc, Ac, Bc, m, n, p)
    res["c1_matmul16"] = {"seconds": round(time.perf_counter() - t0, 3), "cores": 1,
                          "sample": "the whole product (240 rotations, 256 tensors, 16 relinearisations)"}
    # NTT of one limb
    ntt = {}
    for name, pre in (("2^13", "C1"), ("2^14", "C2"), ("2^16", "C3")):
        oo = oc if pre == "C1" else (o if pre == "C3" else OC(PRESETS[pre]))
        q = oo.q[1]
        a = np.random.default_rng(9).integers(0, q, oo.n, dtype=np.uint64)
        reps = 40 if pre != "C3" else 10
        t0 = time.perf_counter()
        for _ in range(reps):
            oo.ntt(a, q)
        ntt[name] = {"us_per_limb": round((time.perf_counter() - t0) / reps * 1e6, 1), "cores": 1}
    res["ntt_per_limb"] = ntt
    res["c2_conv28"] = cpu_baseline(7, out_cols=(0, 6, 12))
    res["c2_conv28"]["value"] = round(res["c2_conv28"]["value"], 4)
    print(json.dumps(res), flush=True)


def cpu_oracle_leg(timeout=900):
    """The oracle legs in a child process (see cpu_oracle_child)."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-oracle-child"], capture_output=True,
                       text=True, timeout=timeout, cwd=ROOT)
    if r.returncode != 0:
        raise RuntimeError("oracle child failed: " + r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_rotations_n16(counts=((24, 2), (3, 4))):
    """The oracle's one-slot rotation at N = 2^16 (60 + 24x50, P 9x51, dnum 3)
    on one host core: `count` rotations per level, timed after key
    generation and encryption (which are not timed)."""
    from oracle import Context as OC, PRESETS
    o = OC(PRESETS["C3"])
    ok = o.keygen(1003, rot_steps=[1])
    z = np.random.default_rng(3).uniform(-1, 1, o.slots)
    res = {}
    for lv, count in counts:
        cts = [o.encrypt(ok, o.encode(z, lv, o.scale), 1003, (3 << 20) + 64 * lv + i) for i in range(count)]
        t = time.perf_counter()
        for c in cts:
            o.rotate(c, 1, ok)
        dt = time.perf_counter() - t
        res["level%d" % lv] = {"rotations_per_s": round(count / dt, 4), "sample": "%d rotations" % count,
                               "seconds": round(dt, 1)}
    res["cores"] = 1
    return res


def cpu_baseline(level, out_cols=(0, 3, 6, 9, 12)):
    """The oracle on a bounded sample of the same layer: every operation the
    output columns j' in out_cols need (their input columns rotated by 1..3,
    5 filters of 16 MulConst + AddConst + Rescale each, then x^2 of the
    outputs), timed per operation class and scaled by the layer's operation
    counts (84 rotations, 13 output columns) to images/s."""
    import synthetic_inputs as SI
    from oracle import Context, PRESETS
    from oracle import layers as Ly
    W = SI.CONV_28
    o = Context(PRESETS["C2"])
    ok = o.keygen(1002, rot_steps=[1, 2, 3])
    X, K, bias = W.draw()
    in_cols = sorted({W.stride * jo + v - W.pad for jo in out_cols for v in range(W.k)
                      if 0 <= W.stride * jo + v - W.pad < W.w})
    cols = {j: o.encrypt(ok, o.encode(Ly.image_column_slots(o, X, 0, j, W.pad), level, o.scale), 1002, j)
            for j in in_cols}
    t0 = time.perf_counter()
    rots = {j: [c] + o.rotate_many(c, [1, 2, 3], ok) for j, c in cols.items()}
    n_rot = 3 * len(in_cols)
    t_rot = (time.perf_counter() - t0) / n_rot
    t0 = time.perf_counter()
    dq = float(o.q[level])
    for jo in out_cols:
        for co in range(W.c_out):
            acc = None
            for v in range(W.k):
                j = W.stride * jo + v - W.pad
                if not 0 <= j < W.w:
                    continue
                for u in range(W.k):
                    t = o.mul_const(rots[j][u], K[co, 0, u, v], dq)
                    acc = t if acc is None else o.add(acc, t)
            Ly.square(o, ok, o.rescale(o.add_const(acc, float(bias[co]))))
    t_col = (time.perf_counter() - t0) / len(out_cols)
    wo = Ly.conv_out_size(W.w, W.pad, W.k, W.stride)
    t_layer = 84 * t_rot + wo * t_col
    return {"value": W.batch / t_layer, "unit": "images/s", "cores": 1, "kind": "oracle",
            "sample": "output columns %s of one 256-image set (%d rotations, %d MulConst, %d rescales, "
                      "%d x^2) timed at level %d, scaled to the layer's 84 rotations and %d output "
                      "columns; measured %.1f s" % (list(out_cols), n_rot, 80 * len(out_cols),
                                                    5 * len(out_cols), 5 * len(out_cols), level, wo,
                                                    n_rot * t_rot + len(out_cols) * t_col)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sets", type=int, default=1, help="128-image ciphertext sets per step")
    ap.add_argument("--level", type=int, default=24, help="level of the fresh ciphertexts (24 = full chain)")
    ap.add_argument("--profile-class", default="ntt")
    ap.add_argument("--no-extra", action="store_true", help="only the headline step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cnn", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration; its timed bandwidth goes into the JSON line as copy_probe)")
    ap.add_argument("--cnn-sets", type=int, default=2)
    ap.add_argument("--serve-requests", type=int, default=60)
    ap.add_argument("--serve-n16-requests", type=int, default=100,
                    help="measured requests per offered load in the N=2^16 serving leg at level 3")
    ap.add_argument("--serve-n16-requests-24", type=int, default=50,
                    help="measured requests per offered load in the N=2^16 serving leg at level 24")
    ap.add_argument("--serve-n16-levels", default="3,24",
                    help="levels of the N=2^16 serving legs (comma list of 3 and 24)")
    ap.add_argument("--serve-load", default="0.8,2.0",
                    help="offered loads, as fractions of the one-request-at-a-time service rate")
    ap.add_argument("--ntt-plan", default="auto",
                    help="NTT pass plan of the N=2^14 leg: auto (autotuned), fixed, or cand:i")
    ap.add_argument("--ntt-plan-n16", default="auto",
                    help="NTT pass plan of the N=2^16 legs: auto or cand:i (pins the plan, e.g. for counter "
                         "runs)")
    ap.add_argument("--rotations-only", action="store_true",
                    help="only the N=2^16 rotation leg (for profiling its kernels)")
    ap.add_argument("--breakdown", action="store_true",
                    help="one extra headline step per kernel class, reporting its device time per step")
    ap.add_argument("--legs", default="all",
                    help="extra legs to run after the headline: all, or a comma list of trimmed, conv28, "
                         "matmul16, rotations, serving, serving16 (the N=2^16 serving legs only), uneven, cpu")
    ap.add_argument("--cpu-oracle-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    legs = set(args.legs.split(",")) if args.legs != "all" else \
        {"trimmed", "conv28", "matmul16", "rotations", "serving", "uneven", "cpu"}
    if args.no_extra:
        legs = set()
    if args.no_cnn:
        legs.discard("trimmed")
    if args.no_serve:
        legs.discard("serving")
    if args.no_uneven:
        legs.discard("uneven")
    if args.no_cpu_baseline:
        legs.discard("cpu")
    if args.cpu_oracle_child:
        cpu_oracle_child()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X "
              "(sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    from paper_2512_18646_amd import vr, perop
    copy_probe = None
    if args.copy_probe:
        # a plain 1 GiB device copy, cold then warm: the HBM counters' scale;
        # then ten more, timed: the copy bandwidth the NTT passes compare with
        import torch
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        sync()
        t = time.perf_counter()
        for _ in range(10):
            dst.copy_(src)
        sync()
        dt = (time.perf_counter() - t) / 10
        copy_probe = {"bytes_moved": 2 << 30, "us_per_copy": round(dt * 1e6, 1),
                      "tb_per_s": round((2 << 30) / dt / 1e12, 3)}
        log("copy probe: 1 GiB in %.1f us, %.2f TB/s moved" % (dt * 1e6, (2 << 30) / dt / 1e12))
        del src, dst
    if args.rotations_only:
        out = {"rotations_per_s_n16": {"level24": rotations_bench(vr, 24, 8, args.steps, args.ntt_plan_n16),
                                       "level3": rotations_bench(vr, 3, 32, args.steps, args.ntt_plan_n16)}}
        print(json.dumps(out), flush=True)
        return

    # ------------------------------------------------ headline: C3 network
    log("setup: keys and %d set(s) of 128 3x128x128 images at level %d, N=2^16" % (args.sets, args.level))
    t0 = time.perf_counter()
    C = cnn128_setup(vr, args.level, args.sets, ntt_plan=args.ntt_plan_n16)
    ctx, keys, net, W = C["ctx"], C["keys"], C["net"], C["W"]
    flat = [c for cs in C["cols"] for c in cs]
    images = W.batch * args.sets
    sync()
    setup_s = time.perf_counter() - t0

    def step():
        return net.forward(ctx, keys, flat, n_sets=args.sets)

    z = step()
    sync()
    err = cnn128_logit_error(C, z[:W.fc_out])
    ref = [c.export() for c in z[:W.fc_out]]
    del z
    for i in range(args.warmup):
        z = step()
        sync()
        del z
        log("warmup %d done" % i)
    lat = []
    ctx.profile_start(args.profile_class, 1 << 20)
    sync()
    t_all = time.perf_counter()
    for i in range(args.steps):
        t = time.perf_counter()
        z = step()
        sync()
        lat.append((time.perf_counter() - t) * 1e3)
        del z
    sync()
    total = time.perf_counter() - t_all
    prof_ms, prof_calls, prof_units, dropped = ctx.profile_stop()
    log("timed %d steps: %.2f ms/step" % (args.steps, total / args.steps * 1e3))
    value = images * args.steps / total
    roofline = None
    if args.profile_class == "ntt":
        roofline = ntt_roofline(prof_ms, prof_calls, prof_units, total, 16, "ntt_n16_cnn128_hbm_counters.json")
        if roofline:
            roofline["dropped"] = dropped
    out = {"metric": METRIC, "value": round(value, 2), "unit": "images/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic",
           "config": {"workload": "3x128x128 images, conv 3x3/2 pad 1 x8 + x^2 + FC 32768->10, N=2^16 "
                                  "(60+24x50, P 9x51, dnum 3), ciphertexts entering at level %d, %d x 128 "
                                  "images per step" % (args.level, args.sets),
                      "images_per_step": images, "level_in": args.level, "fc_level": C["fc_level"],
                      "path": "whole-network call (vr_cnn_forward); x^2 relinearised once per FC output "
                              "when the FC level has room (fc_level >= 3 here)"},
           "latency_ms_p50": round(percentile(lat, 50), 3), "latency_ms_p99": round(percentile(lat, 99), 3),
           "roofline": roofline, "decoded_rel_error": err, "setup_s": round(setup_s, 1)}
    out["autotuned"] = ctx.tuning_report().splitlines()
    if copy_probe:
        out["copy_probe"] = copy_probe

    if args.breakdown:
        bd = {}
        for cls in ("ntt", "ks_inner", "base_convert", "lincomb", "moddown", "tensor"):
            ctx.profile_start(cls, 1 << 20)
            z = step()
            ms, la, un, _ = ctx.profile_stop()
            del z
            bd[cls] = {"ms": round(ms, 3), "launches": la, "units": un}
        out["breakdown_per_step"] = bd

    if not args.no_extra and not args.no_graph:
        log("headline as a graph and per-op")
        out.update(headline_extras(vr, perop, C, args, ref, images))
        out["batched_over_per_op"] = round(value / out["per_op"]["images_per_s"], 2)
    reserved, _ = ctx.mem_info()
    out["device_gib_reserved"] = round(reserved / 2 ** 30, 1)
    del C, ctx, keys, net, flat
    import gc
    gc.collect()

    if "trimmed" in legs:
        log("cnn128 at level 3 (trimmed)")
        log_free("before this leg")
        out["cnn128_trimmed_n16"] = cnn128_bench(vr, 3, args.cnn_sets, 2, graph=True)
        gc.collect()

    if "conv28" in legs:
        log("28x28 conv layer at N=2^14")
        log_free("before this leg")
        out["conv28_n14"] = conv28_bench(vr, perop, args)
        gc.collect()
    if "matmul16" in legs:
        log("16x16 matmul at N=2^13")
        out["matmul16_n13"] = matmul16_bench(vr, perop)
        gc.collect()
    if "rotations" in legs:
        log("rotations at N=2^16")
        log_free("before this leg")
        out["rotations_per_s_n16"] = {"level24": rotations_bench(vr, 24, 8, 3),
                                      "level3": rotations_bench(vr, 3, 32, 3)}
        for v in out["rotations_per_s_n16"].values():
            v["batched"], v["per_op"] = round(v["batched"], 1), round(v["per_op"], 1)
        gc.collect()

    if "serving" in legs:
        log("serving (Poisson arrivals, image-size mix) at N=2^14")
        W2, ctx2, keys2, K2, bias2, _ = conv_setup(vr, 7, 0, args.ntt_plan)
        out["serving"] = [serving_bench(vr, ctx2, keys2, args.serve_requests, float(x), 7)
                          for x in args.serve_load.split(",")]
        del ctx2, keys2
        gc.collect()
    if "serving" in legs or "serving16" in legs:
        s_levels = [int(x) for x in args.serve_n16_levels.split(",")]
        if 3 in s_levels:
            log("serving at N=2^16, level 3")
            log_free("before this leg")
            out["serving_n16"] = serving_n16_bench(vr, level=3, n_meas=args.serve_n16_requests)
            gc.collect()
        if 24 in s_levels:
            log("serving at N=2^16, level 24")
            log_free("before this leg")
            out["serving_n16_level24"] = serving_n16_bench(vr, level=24, n_sessions=4, n_warm=10,
                                                           n_meas=args.serve_n16_requests_24, loads=(0.5, 0.9))
            gc.collect()

    if "uneven" in legs:
        log("uneven batch at N=2^16")
        log_free("before this leg")
        out["uneven_batch_n16"] = uneven_bench(vr, 64, 3, 2)
        gc.collect()
        log("uneven batch at full size ranges (outer-product products)")
        log_free("before this leg")
        out["uneven_full_n16"] = uneven_full_bench(vr, 64, 3, 2)
        gc.collect()

    if "cpu" in legs:
        log("cpu baseline (oracle, child process)")
        cpu = cpu_oracle_leg()
        c3 = cpu["c3_level24"]
        out["cpu_baseline"] = {"value": c3["all_core_images_per_s"], "unit": "images/s", "cores": c3["cores"],
                               "kind": "oracle", "sample": c3["sample"],
                               "single_core_value": c3["single_core_images_per_s"], "host": cpu["host"],
                               "extrapolated": True, "c3_level24": c3, "c1_matmul16": cpu["c1_matmul16"],
                               "ntt_per_limb": cpu["ntt_per_limb"], "c2_conv28": cpu["c2_conv28"]}
        log("cpu baseline: oracle rotations at N=2^16")
        out["cpu_baseline"]["rotations_n16"] = cpu_rotations_n16()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
