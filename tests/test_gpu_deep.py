"""GPU parity of the deeper network of the paper's Table 1 shape (CONV ->
cubic ACT-1 -> FC -> cubic ACT-2 -> dense FC-2) and of its two new layer
calls (vr_poly_eval, vr_dense): limb for limb against the oracle, decoded
logits against the FP64 network."""
import numpy as np
import pytest

from oracle import Context as OracleContext, Params
from oracle import layers as Ly
from tests.gpu_helpers import gpu_ctx, to_gpu, assert_same

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -20


@pytest.fixture(scope="module")
def deep():
    p = Params(10, [60] + [40] * 9, [60], 10, 40.0, allow_insecure=True)
    Hp = Ly.image_block(28, 0)
    steps = [1, 2] + Ly.fc_rotation_steps(Hp)
    o = OracleContext(p)
    ok = o.keygen(11, rot_steps=steps)
    g = gpu_ctx(p)
    gk = g.keygen(11, rot_steps=steps)
    return o, ok, g, gk, Hp


def test_poly_eval_and_dense_bit_exact(deep):
    o, ok, g, gk, Hp = deep
    rng = np.random.default_rng(41)
    Z = rng.uniform(-1, 1, (5, o.slots))
    cts = [o.encrypt(ok, o.encode(z, 6, o.scale), 11, 100 + j) for j, z in enumerate(Z)]
    gcts = [to_gpu(g, c) for c in cts]
    for coeffs in (Ly.ACT1, Ly.ACT2, (0.5, -2.0), (0.1, 0.2, 0.3, 0.4, 0.5)):
        ref = [Ly.poly_eval(o, ok, c, coeffs) for c in cts]
        got = g.poly_eval(gk, gcts, coeffs)
        for i, (x, y) in enumerate(zip(got, ref)):
            assert_same(x, y, "poly %s out %d" % (coeffs, i))
    W, b = rng.normal(0, 0.3, (3, 5)), rng.normal(0, 0.3, 3)
    ref = Ly.dense(o, ok, cts, W, b)
    got = g.dense(gcts, W, b)
    for i, (x, y) in enumerate(zip(got, ref)):
        assert_same(x, y, "dense out %d" % i)


def test_deep_cnn_table1_shape_bit_exact(deep):
    o, ok, g, gk, Hp = deep
    B, h, w, k, Co = 4, 28, 28, 3, 4
    rng = np.random.default_rng(11)
    X = rng.uniform(0, 1, (B, 1, h, w))
    K, kb = rng.normal(0, 0.1, (Co, 1, k, k)), rng.normal(0, 0.1, Co)
    ho = wo = h - k + 1
    W1, b1 = rng.normal(0, 0.01, (6, Co, ho, wo)), rng.normal(0, 0.05, 6)
    W2, b2 = rng.normal(0, 0.3, (3, 6)), rng.normal(0, 0.3, 3)
    cts = Ly.encrypt_image_columns(o, ok, X, 0, 9, 11, 0)
    pts = Ly.fc_plaintexts(o, W1, Co, ho, wo, 1, Hp, 5)
    ref = Ly.deep_cnn(o, ok, cts, 1, h, w, 0, K, kb, 1, Ly.ACT1, pts, b1, Hp, Ly.ACT2, W2, b2)
    Y = g.conv2d(gk, [to_gpu(g, c) for c in cts], 1, h, w, 0, K, kb, 1)
    Y = g.poly_eval(gk, Y, Ly.ACT1)
    gpts = [g.pt_import(pt.m, pt.level, pt.scale) for row in pts for pt in row]
    Z = g.fc(gk, Y, Co, wo, gpts, b1, Hp)
    Z = g.poly_eval(gk, Z, Ly.ACT2)
    out = g.dense(Z, W2, b2)
    for i, (x, y) in enumerate(zip(out, ref)):
        assert_same(x, y, "deep network logit %d" % i)
    logits = np.zeros((B, 3))
    for oi, z in enumerate(out):
        logits[:, oi] = g.decode(g.decrypt(gk, z))[np.arange(B) * Hp]
    expect = Ly.ref_deep_cnn(X, K, kb, 1, 0, Ly.ACT1, W1, b1, Ly.ACT2, W2, b2)
    assert Ly.rel_error(logits, expect) < EPS


def test_encrypted_weight_conv_and_fc_bit_exact():
    """Encrypted-weight conv and FC (ct x ct products, one lazy
    relinearisation per output, bias ciphertexts added after the rescale):
    limb for limb against the oracle, decoded against FP64."""
    from tests.gpu_helpers import pair
    o, ok, g, gk = pair("C1", rot_steps=(1, 2, 4, 8), log_n=10)
    B, Ci, h, w, Co, k, s, pad = 8, 2, 10, 9, 3, 3, 2, 1
    rng = np.random.default_rng(15)
    X = rng.uniform(0, 1, (B, Ci, h, w))
    K, bias = rng.normal(0, 0.1, (Co, Ci, k, k)), rng.normal(0, 0.1, Co)
    cts = Ly.encrypt_image_columns(o, ok, X, pad, 3, 15, 0)
    kct, bct = Ly.encrypt_conv_weights(o, ok, K, bias, 3, cts[0].scale, 16, 0)
    Y = Ly.conv2d_encw(o, ok, cts, Ci, h, w, pad, kct, bct, Co, k, s)
    gY = g.conv2d_encw(gk, [to_gpu(g, c) for c in cts], Ci, h, w, pad, [to_gpu(g, c) for c in kct],
                       [to_gpu(g, c) for c in bct], Co, k, s)
    for i, (x, y) in enumerate(zip(gY, Y)):
        assert_same(x, y, "encrypted-weight conv %d" % i)
    Hp = Ly.image_block(h, pad)
    ref = Ly.ref_conv(X, K, bias, s, pad)
    ho, wo = ref.shape[2], ref.shape[3]
    W, fb = rng.normal(0, 0.05, (4, Co, ho, wo)), rng.normal(0, 0.05, 4)
    wct, fbct = Ly.encrypt_fc_weights(o, ok, W, fb, Co, ho, wo, s, Hp, 2, Y[0].scale, 17, 0)
    Z = Ly.fc_encw(o, ok, Y, wct, fbct, Hp)
    gZ = g.fc_encw(gk, gY, [to_gpu(g, c) for row in wct for c in row], [to_gpu(g, c) for c in fbct], Hp)
    for i, (x, y) in enumerate(zip(gZ, Z)):
        assert_same(x, y, "encrypted-weight fc %d" % i)
    logits = np.zeros((B, 4))
    for oi, z in enumerate(gZ):
        logits[:, oi] = g.decode(g.decrypt(gk, z))[np.arange(B) * Hp]
    assert Ly.rel_error(logits, Ly.ref_fc(ref, W, fb)) < EPS
