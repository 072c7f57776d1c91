"""GPU parity of the column-wise layers (matmul, conv, x^2, FC) against the
oracle, limb for limb, plus the decoded FP64 bar (2^-20 normwise relative,
max |y - ref| / max |ref|), batched-versus-per-op identity, and the
full-size workloads on sampled output columns."""
import numpy as np
import pytest

import synthetic_inputs as SI
from oracle import layers as Ly
from oracle import Params, PRESETS, Context as OracleContext
from tests.gpu_helpers import pair, to_gpu, assert_same, gpu_ctx, SEED_KEYS

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -20


def gpu_matmul_decode(g, gk, D, m, p):
    Pp = len(D)
    C = np.full((m, p), np.nan)
    for idx, ct in enumerate(D):
        z = g.decode(g.decrypt(gk, ct), m)
        for i in range(m):
            if (i + idx) % Pp < p:
                C[i, (i + idx) % Pp] = z[i]
    return C


def gpu_conv_decode(g, gk, Y, B, C_out, h, pad, k, stride, w):
    Hp = Ly.image_block(h, pad)
    ho, wo = Ly.conv_out_size(h, pad, k, stride), Ly.conv_out_size(w, pad, k, stride)
    out = np.zeros((B, C_out, ho, wo))
    for co in range(C_out):
        for jo in range(wo):
            z = g.decode(g.decrypt(gk, Y[co * wo + jo]))
            for b in range(B):
                out[b, co, :, jo] = z[b * Hp + stride * np.arange(ho)]
    return out


@pytest.fixture(scope="module")
def c1mm():
    return pair("C1", rot_steps=tuple(range(1, 16)))


def test_matmul_16x16_bit_exact(c1mm):
    o, ok, g, gk = c1mm
    seed, m, n, p = SI.MATMUL_16
    A, B = SI.matmul_operands(seed, m, n, p)
    Ac = Ly.encrypt_matrix_columns(o, ok, A, 0, m, p, 3, 1001, 0)
    Bc = Ly.encrypt_matrix_columns(o, ok, B, 1, m, p, 3, 1001, 100)
    D = Ly.matmul(o, ok, Ac, Bc, m, n, p)
    gD = g.matmul(gk, [to_gpu(g, c) for c in Ac], [to_gpu(g, c) for c in Bc], m, n, p)
    assert len(gD) == len(D) == 16
    for i, (x, y) in enumerate(zip(gD, D)):
        assert_same(x, y, "C[%d]" % i)
    assert Ly.rel_error(gpu_matmul_decode(g, gk, gD, m, p), A @ B) < EPS


def test_matmul_gpu_encrypt_end_to_end(c1mm):
    """GPU encode/encrypt of the columns, GPU product, GPU decrypt/decode."""
    o, ok, g, gk = c1mm
    seed, m, n, p = SI.MATMUL_16
    A, B = SI.matmul_operands(seed, m, n, p)
    gA = g.encrypt_matrix_columns(gk, A, 0, m, p, 3, 1001, 0)
    gB = g.encrypt_matrix_columns(gk, B, 1, m, p, 3, 1001, 100)
    gD = g.matmul(gk, gA, gB, m, n, p)
    assert gD[0].level == 2
    assert Ly.rel_error(gpu_matmul_decode(g, gk, gD, m, p), A @ B) < EPS


def test_matmul_m_below_p_bit_exact(c1mm):
    """m < p: the transposed product on the same ciphertexts, roles swapped
    (M' = 8 outputs, slot i < p of C[idx] holding (A B)[(i + idx) mod 8][i]),
    limb for limb against the oracle, per-op identical, decoded against FP64."""
    o, ok, g, gk = c1mm
    m, n, p = 5, 4, 13
    rng = np.random.default_rng(14)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    Ac = Ly.encrypt_matrix_columns(o, ok, A, 0, m, p, 3, 8, 0)
    Bc = Ly.encrypt_matrix_columns(o, ok, B, 1, m, p, 3, 8, 100)
    D = Ly.matmul(o, ok, Ac, Bc, m, n, p)
    gA, gB = [to_gpu(g, c) for c in Ac], [to_gpu(g, c) for c in Bc]
    gD = g.matmul(gk, gA, gB, m, n, p)
    assert len(gD) == len(D) == 8
    for i, (x, y) in enumerate(zip(gD, D)):
        assert_same(x, y, "C[%d]" % i)
    from paper_2512_18646_amd import perop
    for i, (x, y) in enumerate(zip(perop.matmul(g, gk, gA, gB, m, n, p), D)):
        assert_same(x, y, "per-op C[%d]" % i)
    got = np.full((m, p), np.nan)
    for idx, ct in enumerate(gD):
        z = g.decode(g.decrypt(gk, ct), p)
        for i in range(p):
            if (i + idx) % 8 < m:
                got[(i + idx) % 8, i] = z[i]
    assert Ly.rel_error(got, A @ B) < EPS


def test_matmul_ragged_identity_and_per_op(c1mm):
    o, ok, g, gk = c1mm
    m, n, p = 12, 5, 5
    A = np.random.default_rng(2).uniform(-1, 1, (m, n))
    Ac = Ly.encrypt_matrix_columns(o, ok, A, 0, m, p, 3, 7, 0)
    Bc = Ly.encrypt_matrix_columns(o, ok, np.eye(n), 1, m, p, 3, 7, 100)
    D = Ly.matmul(o, ok, Ac, Bc, m, n, p)
    gA, gB = [to_gpu(g, c) for c in Ac], [to_gpu(g, c) for c in Bc]
    gD = g.matmul(gk, gA, gB, m, n, p)
    for i, (x, y) in enumerate(zip(gD, D)):
        assert_same(x, y, "C[%d]" % i)
    from paper_2512_18646_amd import perop
    for i, (x, y) in enumerate(zip(perop.matmul(g, gk, gA, gB, m, n, p), D)):
        assert_same(x, y, "per-op C[%d]" % i)
    assert Ly.rel_error(gpu_matmul_decode(g, gk, gD, m, p), A) < EPS


def gpu_outer_decode(g, gk, D, m, p):
    Pp, R, T = g.outer_tiles(m, p)
    assert len(D) == T
    C = np.full((m, p), np.nan)
    for t, ct in enumerate(D):
        z = g.decode(g.decrypt(gk, ct))
        for r in range(R):
            if t * R + r < m:
                C[t * R + r] = z[r * Pp:r * Pp + p]
    return C


def test_matmul_outer_bit_exact_ragged_tiles(c1mm):
    """Outer-product product at N = 2^13 (S = 4096): m = 300, n = 5, p = 20
    gives P' = 32, R = 128, three row tiles (the last one ragged); oracle
    ciphertexts in, every limb of every tile against the oracle, decoded
    against FP64."""
    o, ok, g, gk = c1mm
    m, n, p = 300, 5, 20
    rng = np.random.default_rng(61)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    Ac = Ly.encrypt_matrix_outer(o, ok, A, 2, m, p, 3, 1001, 0)
    Bc = Ly.encrypt_matrix_outer(o, ok, B, 3, m, p, 3, 1001, 500)
    D = Ly.matmul_outer(o, ok, Ac, Bc, m, n, p)
    gD = g.matmul_outer(gk, [to_gpu(g, c) for c in Ac], [to_gpu(g, c) for c in Bc], m, n, p)
    assert len(gD) == len(D) == 3
    for i, (x, y) in enumerate(zip(gD, D)):
        assert_same(x, y, "C[%d]" % i)
    assert Ly.rel_error(gpu_outer_decode(g, gk, gD, m, p), A @ B) < EPS


def test_matmul_outer_gpu_encrypt_end_to_end(c1mm):
    """GPU encode/encrypt of the outer-product operands (roles 2 and 3), GPU
    product, GPU decrypt/decode against FP64: m = 200, n = 40, p = 100 (P' =
    128, R = 32, seven tiles), m = 1 with p = 1, and p = S (one row per tile)."""
    o, ok, g, gk = c1mm
    rng = np.random.default_rng(62)
    for m, n, p in ((200, 40, 100), (1, 3, 1), (3, 2, g.slots)):
        A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
        gA = g.encrypt_matrix_columns(gk, A, 2, m, p, 3, 7, 0)
        gB = g.encrypt_matrix_columns(gk, B, 3, m, p, 3, 7, 100000)
        assert len(gA) == g.outer_tiles(m, p)[2] * n and len(gB) == n
        C = gpu_outer_decode(g, gk, g.matmul_outer(gk, gA, gB, m, n, p), m, p)
        assert not np.any(np.isnan(C))
        assert Ly.rel_error(C, A @ B) < EPS, (m, n, p)


def test_matmul_outer_errors(c1mm):
    from paper_2512_18646_amd import vr
    o, ok, g, gk = c1mm
    A = g.encrypt_matrix_columns(gk, np.ones((4, 2)), 2, 4, 3, 3, 1, 0)
    B = g.encrypt_matrix_columns(gk, np.ones((2, 3)), 3, 4, 3, 2, 1, 50)
    with pytest.raises(vr.VRError) as e:
        g.matmul_outer(gk, A, B, 4, 2, 3)
    assert e.value.code == vr.VR_ELEVEL
    with pytest.raises(vr.VRError) as e:
        g.encrypt_matrix_columns(gk, np.ones((2, 2 * g.slots)), 3, 4, 2 * g.slots, 3, 1, 0)
    assert e.value.code == vr.VR_EINVAL


def test_matmul_rejects_operands_at_different_levels(c1mm):
    from paper_2512_18646_amd import vr
    o, ok, g, gk = c1mm
    A = g.encrypt_matrix_columns(gk, np.ones((4, 3)), 0, 4, 8, 3, 1, 0)
    B = g.encrypt_matrix_columns(gk, np.ones((3, 8)), 1, 4, 8, 2, 1, 10)
    with pytest.raises(vr.VRError) as e:
        g.matmul(gk, A, B, 4, 3, 8)
    assert e.value.code == vr.VR_ELEVEL


@pytest.fixture(scope="module")
def small_cnn():
    """N = 2^10 on the 49/40/40/40 chain: rotations for conv (1, 2) and FC blocks."""
    return pair("C1", rot_steps=(1, 2, 4, 8), log_n=10)


def test_conv_square_fc_bit_exact_small(small_cnn):
    o, ok, g, gk = small_cnn
    B, Ci, h, w, Co, k, s, pad = 8, 2, 10, 9, 3, 3, 2, 1
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (B, Ci, h, w))
    K = rng.normal(0, 0.1, (Co, Ci, k, k))
    bias = rng.normal(0, 0.1, Co)
    cts = Ly.encrypt_image_columns(o, ok, X, pad, 3, 3, 0)
    gcts = [to_gpu(g, c) for c in cts]
    Y = Ly.conv2d(o, ok, cts, Ci, h, w, pad, K, bias, Co, k, s)
    gY = g.conv2d(gk, gcts, Ci, h, w, pad, K, bias, s)
    for i, (x, y) in enumerate(zip(gY, Y)):
        assert_same(x, y, "conv %d" % i)
    # the per-operation path issues the plain sequence (a ModDown per rotation)
    from paper_2512_18646_amd import perop
    Yp = Ly.conv2d(o, ok, cts, Ci, h, w, pad, K, bias, Co, k, s, lazy=False)
    for i, (x, y) in enumerate(zip(perop.conv2d(g, gk, gcts, Ci, h, w, pad, K, bias, s), Yp)):
        assert_same(x, y, "per-op conv %d" % i)
    Y2 = [Ly.square(o, ok, y) for y in Y]
    gY2 = g.square(gk, gY)
    for i, (x, y) in enumerate(zip(gY2, Y2)):
        assert_same(x, y, "square %d" % i)
    ref = Ly.ref_conv(X, K, bias, s, pad)
    got = gpu_conv_decode(g, gk, gY2, B, Co, h, pad, k, s, w)
    assert Ly.rel_error(got, ref ** 2) < EPS
    Hp = Ly.image_block(h, pad)
    ho, wo = ref.shape[2], ref.shape[3]
    W = rng.normal(0, 0.05, (4, Co, ho, wo))
    fb = rng.normal(0, 0.05, 4)
    pts = Ly.fc_plaintexts(o, W, Co, ho, wo, s, Hp, Y2[0].level)
    Z = Ly.fc(o, ok, Y2, pts, fb, Hp)
    gpts = [g.pt_import(pt.m, pt.level, pt.scale) for row in pts for pt in row]
    gZ = g.fc(gk, gY2, Co, wo, gpts, fb, Hp)
    for i, (x, y) in enumerate(zip(gZ, Z)):
        assert_same(x, y, "fc %d" % i)
    # weights one level below the inputs (conv outputs at level 2, weights at
    # level 1): the FC reads the inputs' first two limbs only
    pts1 = Ly.fc_plaintexts(o, W, Co, ho, wo, s, Hp, 1)
    Z1 = Ly.fc(o, ok, Y, pts1, fb, Hp)
    gZ1 = g.fc(gk, gY, Co, wo, [g.pt_import(pt.m, pt.level, pt.scale) for row in pts1 for pt in row], fb, Hp)
    assert gZ1[0].level == 0
    for i, (x, y) in enumerate(zip(gZ1, Z1)):
        assert_same(x, y, "fc below the input level %d" % i)
    # GPU-encoded weights: decoded logits still within the bar, and the
    # compact weight copies (runs of N / (2 H') equal words kept once) give the
    # same words as the full limbs
    gpts2 = g.encode_fc_weights(W, s, Hp, Y2[0].level)
    assert o.n // (2 * Hp) > 1
    gZ2 = g.fc(gk, gY2, Co, wo, gpts2, fb, Hp)
    g.set_tuning("fc_compact", "off")
    try:
        gZ3 = g.fc(gk, gY2, Co, wo, gpts2, fb, Hp)
    finally:
        g.set_tuning("fc_compact", "on")
    for i, (x, y) in enumerate(zip(gZ2, gZ3)):
        assert x.meta == y.meta and np.array_equal(x.export(), y.export()), "compact fc %d" % i
    logits = np.zeros((B, 4))
    for oi, z in enumerate(gZ2):
        logits[:, oi] = g.decode(g.decrypt(gk, z))[np.arange(B) * Hp]
    assert Ly.rel_error(logits, Ly.ref_fc(ref ** 2, W, fb)) < EPS


def test_conv_edge_shapes(small_cnn):
    """k = 1 (no rotation), stride 1 with padding, one image, ragged block."""
    o, ok, g, gk = small_cnn
    rng = np.random.default_rng(4)
    for (B, Ci, h, w, Co, k, s, pad) in [(1, 1, 5, 4, 2, 1, 1, 0), (3, 1, 7, 6, 1, 3, 1, 1),
                                         (2, 2, 12, 5, 2, 2, 2, 0)]:
        X = rng.uniform(0, 1, (B, Ci, h, w))
        K = rng.normal(0, 0.1, (Co, Ci, k, k))
        bias = rng.normal(0, 0.1, Co)
        cts = Ly.encrypt_image_columns(o, ok, X, pad, 2, 5, 0)
        Y = Ly.conv2d(o, ok, cts, Ci, h, w, pad, K, bias, Co, k, s)
        gY = g.conv2d(gk, [to_gpu(g, c) for c in cts], Ci, h, w, pad, K, bias, s)
        for i, (x, y) in enumerate(zip(gY, Y)):
            assert_same(x, y, "conv %s %d" % ((B, Ci, h, w, Co, k, s, pad), i))


@pytest.mark.parametrize("level", [2, 7])
def test_conv28_full_size_sampled(level):
    """The 28x28 conv layer at N = 2^14, L = 7 on a full set of 256 images:
    GPU layer on every column, oracle on output columns 0, 6 and 12."""
    W = SI.CONV_28
    o, ok, g, gk = pair("C2", rot_steps=(1, 2, 3))
    X, K, bias = W.draw()
    cts = Ly.encrypt_image_columns(o, ok, X, W.pad, level, 2002, 0)
    gY = g.conv2d(gk, [to_gpu(g, c) for c in cts], 1, W.h, W.w, W.pad, K, bias, W.stride)
    cols = {0, 6, 12}
    Y = Ly.conv2d(o, ok, cts, 1, W.h, W.w, W.pad, K, bias, W.c_out, W.k, W.stride, only_cols=cols)
    wo = Ly.conv_out_size(W.w, W.pad, W.k, W.stride)
    assert len(gY) == W.c_out * wo == 65
    checked = 0
    for i, y in enumerate(Y):
        if y is not None:
            assert_same(gY[i], y, "conv28 out %d" % i)
            checked += 1
    assert checked == 15
    gY2 = g.square(gk, gY)
    i0 = 0 * wo + 6
    assert_same(gY2[i0], Ly.square(o, ok, Y[i0]), "square")
    ref = Ly.ref_conv(X, K, bias, W.stride, W.pad)
    got = gpu_conv_decode(g, gk, gY2, W.batch, W.c_out, W.h, W.pad, W.k, W.stride, W.w)
    assert Ly.rel_error(got, ref ** 2) < EPS


def test_conv28_gpu_only_end_to_end():
    """GPU encryption of the columns, GPU conv + x^2, GPU decryption: FP64 bar."""
    W = SI.CONV_28
    o, ok, g, gk = pair("C2", rot_steps=(1, 2, 3))
    X, K, bias = W.draw()
    gcts = g.encrypt_columns(gk, X, W.pad, 7, 2002, 0)
    gY2 = g.square(gk, g.conv2d(gk, gcts, 1, W.h, W.w, W.pad, K, bias, W.stride))
    ref = Ly.ref_conv(X, K, bias, W.stride, W.pad)
    got = gpu_conv_decode(g, gk, gY2, W.batch, W.c_out, W.h, W.pad, W.k, W.stride, W.w)
    assert gY2[0].level == 5
    assert Ly.rel_error(got, ref ** 2) < EPS


def test_cnn128_trimmed_sampled():
    """The 3x128x128 network at N = 2^16 (L = 24 chain, dnum 3, 9-prime
    digits) on one 128-image set entering at level 3: GPU conv on all 384
    columns, oracle on output column 0 of every filter (inputs 0 and 1 of each
    channel encrypted by the oracle), x^2 of one output, then the GPU FC on
    the whole set against the FP64 network."""
    W = SI.CNN_128
    o, ok, g, gk = pair("C3", rot_steps=(1, 2))
    X, K, bias = W.draw()
    Hp = Ly.image_block(W.h, W.pad)
    gcols = g.encrypt_columns(gk, X, W.pad, 3, 3003, 0)
    ocols = [None] * (W.channels * W.w)
    for c in range(W.channels):
        for j in (0, 1, 2, 3):
            slots = Ly.image_column_slots(o, X, c, j, W.pad)
            ocols[c * W.w + j] = o.encrypt(ok, o.encode(slots, 3, o.scale), 3003, c * W.w + j)
            gcols[c * W.w + j] = to_gpu(g, ocols[c * W.w + j])
    gY = g.conv2d(gk, gcols, W.channels, W.h, W.w, W.pad, K, bias, W.stride)
    wo = Ly.conv_out_size(W.w, W.pad, W.k, W.stride)
    assert len(gY) == W.c_out * wo == 512
    # output column 0 (its left neighbour is padding) and the interior column
    # 1 (input columns 1, 2, 3 at offsets 0, 1, 2)
    Y = Ly.conv2d(o, ok, ocols, W.channels, W.h, W.w, W.pad, K, bias, W.c_out, W.k, W.stride,
                  only_cols={0, 1})
    for co in range(W.c_out):
        for jo in (0, 1):
            assert_same(gY[co * wo + jo], Y[co * wo + jo], "cnn128 conv out (%d, %d)" % (co, jo))
    gY2 = g.square(gk, gY)
    assert_same(gY2[3 * wo], Ly.square(o, ok, Y[3 * wo]), "cnn128 square")
    Wfc, bfc = W.draw_fc()
    gk.add_rotations(SEED_KEYS, [1 << t for t in range(2, Hp.bit_length() - 1)])   # FC rotate-and-sum
    pts = g.encode_fc_weights(Wfc, W.stride, Hp, gY2[0].meta[1])
    gZ = g.fc(gk, gY2, W.c_out, wo, pts, bfc, Hp)
    logits = np.zeros((W.batch, W.fc_out))
    for oi, z in enumerate(gZ):
        logits[:, oi] = g.decode(g.decrypt(gk, z))[np.arange(W.batch) * Hp]
    ref = Ly.ref_fc(Ly.ref_conv(X, K, bias, W.stride, W.pad) ** 2, Wfc, bfc)
    assert gZ[0].meta[1] == 0
    assert Ly.rel_error(logits, ref) < EPS


@pytest.mark.timeout(400)
def test_cnn128_full_level_chunked_key_switching():
    """The 3x128x128 conv and x^2 entering at level 24 (the whole L = 24
    chain, three digits of nine primes), with the layer calls' key switching
    forced into chunks of two ciphertexts: every filter of output column 0
    and the square of one of them, limb for limb against the oracle (inputs
    0 and 1 of each channel encrypted by the oracle, the rest by the GPU),
    and the squared layer decoded against FP64."""
    W = SI.CNN_128
    o, ok, g, gk = pair("C3", rot_steps=(1, 2))
    X, K, bias = W.draw()
    lv = 24
    gcols = g.encrypt_columns(gk, X, W.pad, lv, 3004, 0)
    ocols = [None] * (W.channels * W.w)
    for c in range(W.channels):
        for j in (0, 1):
            slots = Ly.image_column_slots(o, X, c, j, W.pad)
            ocols[c * W.w + j] = o.encrypt(ok, o.encode(slots, lv, o.scale), 3004, c * W.w + j)
            gcols[c * W.w + j] = to_gpu(g, ocols[c * W.w + j])
    wo = Ly.conv_out_size(W.w, W.pad, W.k, W.stride)
    g.set_tuning("switch_chunk", "2")
    try:
        gY = g.conv2d(gk, gcols, W.channels, W.h, W.w, W.pad, K, bias, W.stride)
        gY2 = g.square(gk, gY)
    finally:
        g.set_tuning("switch_chunk", "0")
    assert gY[0].level == lv - 1 and gY2[0].level == lv - 2
    Y = Ly.conv2d(o, ok, ocols, W.channels, W.h, W.w, W.pad, K, bias, W.c_out, W.k, W.stride,
                  only_cols={0})
    for co in range(W.c_out):
        assert_same(gY[co * wo], Y[co * wo], "level-24 conv out (%d, 0)" % co)
    assert_same(gY2[5 * wo], Ly.square(o, ok, Y[5 * wo]), "level-24 square")
    ref = Ly.ref_conv(X, K, bias, W.stride, W.pad) ** 2
    Hp = Ly.image_block(W.h, W.pad)
    got = np.zeros((W.batch, 2, (W.h + 2 * W.pad - W.k) // W.stride + 1))
    for i, co in enumerate((0, 7)):
        z = g.decode(g.decrypt(gk, gY2[co * wo + 9]))
        for b in range(W.batch):
            got[b, i] = z[b * Hp + W.stride * np.arange(got.shape[2])]
    assert Ly.rel_error(got, ref[:, [0, 7]][:, :, :, 9]) < EPS


def test_cnn128_network_level24_pruned_equals_full():
    """The headline network (3x128x128, conv 3x3/2 pad 1 x8, x^2, FC 32768 ->
    10 with its weights at level 3) entering at level 24: the network call,
    whose conv makes only the 4 limbs the FC reads (its weighted sums as
    int8 matrix-core products) and whose FC reads the compact weight copies,
    gives the same words as with every conv limb made and dropped after, the
    sums as FP64 and 64-bit integer products and the full weight limbs read
    (conv_prune, lincomb_mfma, lincomb_wide and fc_compact off), and its
    logits decode to the FP64 network."""
    from paper_2512_18646_amd import vr
    W = SI.CNN_128
    Hp = Ly.image_block(W.h, W.pad)
    steps = sorted(set(range(1, W.k)) | {1 << t for t in range(Hp.bit_length() - 1)})
    g = gpu_ctx(PRESETS["C3"])
    gk = g.keygen(1003, rot_steps=steps)
    X, K, bias = W.draw()
    Wfc, bfc = W.draw_fc()
    cols = g.encrypt_columns(gk, X, W.pad, 24, 3005, 0)
    pts = g.encode_fc_weights(Wfc, W.stride, Hp, 3)
    net = vr.CNN(W.channels, W.h, W.w, W.pad, K, bias, W.stride, square=True, fc_w=pts, fc_bias=bfc,
                 fc_block=Hp)
    out = net.forward(g, gk, cols)
    knobs = ("conv_prune", "fc_compact", "lincomb_wide", "lincomb_mfma")
    for kn in knobs:
        g.set_tuning(kn, "off")
    try:
        full = net.forward(g, gk, cols)
    finally:
        for kn in knobs:
            g.set_tuning(kn, "on")
    assert len(out) == len(full) == W.fc_out
    for i, (a, b) in enumerate(zip(out, full)):
        assert a.meta == b.meta and a.meta[1] == 1, i
        assert np.array_equal(a.export(), b.export()), "logit ciphertext %d" % i
    logits = np.zeros((W.batch, W.fc_out))
    for oi, z in enumerate(out):
        logits[:, oi] = g.decode(g.decrypt(gk, z))[np.arange(W.batch) * Hp]
    ref = Ly.ref_fc(Ly.ref_conv(X, K, bias, W.stride, W.pad) ** 2, Wfc, bfc)
    assert Ly.rel_error(logits, ref) < EPS


def test_matmul_block_bit_exact_and_planner(c1mm):
    """Column-block form at N = 2^13 (S = 4096): m = 12, n = 40, p = 5 gives
    blocks of 24 slots, 64 columns per ciphertext, one ciphertext per
    operand; limb for limb against the oracle (operands encrypted by the
    oracle), GPU-encrypted end to end against FP64; the planner's choices."""
    o, ok, g, gk = c1mm
    m, n, p = 12, 40, 5
    Pp, Mb, c, nb = Ly.block_shape(o, m, n, p)
    assert g.block_shape(m, n, p) == (Pp, Mb, c, nb) == (8, 24, 64, 1)
    steps = Ly.block_rotation_steps(o, m, n, p)
    ok2 = o.keygen(1001, rot_steps=steps)
    gk2 = g.keygen(1001, rot_steps=steps)
    rng = np.random.default_rng(19)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    Ac = Ly.encrypt_matrix_blocks(o, ok2, A, 4, m, n, p, 3, 9, 0)
    Bc = Ly.encrypt_matrix_blocks(o, ok2, B, 5, m, n, p, 3, 9, 100)
    D = Ly.matmul_block(o, ok2, Ac, Bc, m, n, p)
    gD = g.matmul_block(gk2, [to_gpu(g, x) for x in Ac], [to_gpu(g, x) for x in Bc], m, n, p)
    for i, (x, y) in enumerate(zip(gD, D)):
        assert_same(x, y, "block C[%d]" % i)
    gA = g.encrypt_matrix_columns(gk2, A, 4, m, p, 3, 9, 1000)
    gB = g.encrypt_matrix_columns(gk2, B, 5, m, p, 3, 9, 2000)
    assert len(gA) == len(gB) == nb
    assert Ly.rel_error(gpu_matmul_decode(g, gk2, g.matmul_block(gk2, gA, gB, m, n, p), m, p), A @ B) < EPS
    # planner: the outer form wins on device work (one tile, one key switch
    # for 16 x 16 x 16); a client limit below its upload (32 ciphertexts)
    # leaves the block form, which needs fewer key switches than the
    # column-split one; the transposed flag for m < p
    form, cost = g.matmul_plan(16, 16, 16, 3)
    assert form == "outer" and cost["outer"]["client_cts"] == 32 and cost["outer"]["key_switches"] == 1
    assert cost["column_block"]["key_switches"] < cost["column_split"]["key_switches"]
    form, cost = g.matmul_plan(16, 16, 16, 3, max_client_cts=4)
    assert form == "column_block" and cost["column_block"]["client_cts"] == 2
    form, cost = g.matmul_plan(512, 512, 512, 3)
    assert form == "outer"
    form2, _ = g.matmul_plan(512, 512, 512, 3, max_client_cts=cost["column_block"]["client_cts"])
    assert form2 in ("column_block", "column_split")
    _, cost = g.matmul_plan(5, 8, 13, 3)
    assert cost["column_split"]["transposed"] == 1 and cost["outer"]["transposed"] == 0
