"""The whole-network call and its HIP-graph capture: identical limbs to the
per-layer calls, on every replay, with eager work and synchronisations
between replays and after new inputs are copied in."""
import numpy as np
import pytest

from oracle import layers as Ly
from tests.gpu_helpers import pair

pytestmark = pytest.mark.gpu

B, CI, H, W_, CO, K_, S_, PAD = 8, 2, 10, 9, 3, 3, 2, 1


@pytest.fixture(scope="module")
def net():
    from paper_2512_18646_amd import vr
    o, ok, g, gk = pair("C1", rot_steps=(1, 2, 4, 8), log_n=10)
    rng = np.random.default_rng(51)
    K = rng.normal(0, 0.1, (CO, CI, K_, K_))
    bias = rng.normal(0, 0.1, CO)
    Hp = Ly.image_block(H, PAD)
    wo = Ly.conv_out_size(W_, PAD, K_, S_)
    ho = Ly.conv_out_size(H, PAD, K_, S_)
    Wfc = rng.normal(0, 0.05, (4, CO, ho, wo))
    fb = rng.normal(0, 0.05, 4)
    pts = g.encode_fc_weights(Wfc, S_, Hp, 1)
    full = vr.CNN(CI, H, W_, PAD, K, bias, S_, square=True, fc_w=pts, fc_bias=fb, fc_block=Hp)
    conv_sq = vr.CNN(CI, H, W_, PAD, K, bias, S_, square=True)
    sets = [g.encrypt_columns(gk, rng.uniform(0, 1, (B, CI, H, W_)), PAD, 3, 61, 100 * i)
            for i in range(4)]
    return g, gk, full, conv_sq, sets, (K, bias, Wfc, fb, pts, Hp, wo)


def layers_ref(g, gk, cols, params, fc=True):
    K, bias, Wfc, fb, pts, Hp, wo = params
    y = g.square(gk, g.conv2d(gk, cols, CI, H, W_, PAD, K, bias, S_))
    return g.fc(gk, y, CO, wo, pts, fb, Hp) if fc else y


def limbs(cts):
    return [c.export() for c in cts]


def check(got, ref, what):
    assert len(got) == len(ref), what
    for i, (a, b) in enumerate(zip(got, ref)):
        assert a.meta == b.meta, (what, i)
        assert np.array_equal(a.export(), b.export()), "%s: output %d differs" % (what, i)


def test_cnn_forward_matches_layer_calls(net):
    g, gk, full, conv_sq, sets, params = net
    out = full.forward(g, gk, sets[0] + sets[1], n_sets=2)
    check(out[:4], layers_ref(g, gk, sets[0], params), "set 0")
    check(out[4:], layers_ref(g, gk, sets[1], params), "set 1")
    # the FC weights' compact copies (N / (2 H') = 32 words per run) against
    # the full limbs
    g.set_tuning("fc_compact", "off")
    try:
        check(out, full.forward(g, gk, sets[0] + sets[1], n_sets=2), "full weight limbs")
    finally:
        g.set_tuning("fc_compact", "on")
    out2 = conv_sq.forward(g, gk, sets[2], n_sets=1)
    check(out2, layers_ref(g, gk, sets[2], params, fc=False), "conv + x^2")


def test_graph_replays_match_eager(net):
    from paper_2512_18646_amd import vr
    g, gk, full, conv_sq, sets, params = net
    ref01 = [layers_ref(g, gk, sets[i], params) for i in (0, 1)]
    ref23 = [layers_ref(g, gk, sets[i], params) for i in (2, 3)]
    gr = vr.Graph(g, gk, full, sets[0] + sets[1], n_sets=2)
    for rep in range(3):
        gr.launch()
        out = gr.outputs()
        check(out[:4], ref01[0], "replay %d set 0" % rep)
        check(out[4:], ref01[1], "replay %d set 1" % rep)
        layers_ref(g, gk, sets[3], params)          # eager work between replays
    gr.set_inputs(sets[2] + sets[3])
    for rep in range(2):
        gr.launch()
        out = gr.outputs()
        check(out[:4], ref23[0], "new inputs replay %d set 0" % rep)
        check(out[4:], ref23[1], "new inputs replay %d set 1" % rep)
        conv_sq.forward(g, gk, sets[0])[0].export()
    kept = limbs(out)
    gr.close()
    assert all(np.array_equal(a, b.export()) for a, b in zip(kept, out))   # handles outlive the graph
    g2 = vr.Graph(g, gk, conv_sq, sets[1])
    ref = layers_ref(g, gk, sets[1], params, fc=False)
    for rep in range(3):
        g2.launch()
        check(g2.outputs(), ref, "conv + x^2 graph replay %d" % rep)
    g2.close()


@pytest.mark.parametrize("fc_level,lv", [(3, 5), (1, 5), (3, 7)])
def test_network_square_fc_lazy_relinearisation(fc_level, lv):
    """FC weights at a level with room for the unrelinearised products (3):
    the network call fuses x^2 into the FC, one relinearisation per output,
    limb for limb the oracle's square_fc after its (lazy) conv, also as a
    replayed graph; the conv then makes only the FC level's limbs of its
    outputs (entering at 7, 4 of the 7 limbs), identical to making every
    limb and dropping them after (conv_prune off); at level 1 the network
    keeps the per-layer form.  All decode to the FP64 network."""
    from paper_2512_18646_amd import vr
    from tests.gpu_helpers import to_gpu, assert_same
    o, ok, g, gk = pair("C2", rot_steps=(1, 2, 4, 8), log_n=10)
    B, Ci, h, w, Co, k, s, pad = 4, 2, 10, 9, 3, 3, 2, 1
    rng = np.random.default_rng(52)
    X = rng.uniform(0, 1, (B, Ci, h, w))
    K = rng.normal(0, 0.1, (Co, Ci, k, k))
    bias = rng.normal(0, 0.1, Co)
    Hp = Ly.image_block(h, pad)
    ref = Ly.ref_conv(X, K, bias, s, pad)
    ho, wo = ref.shape[2], ref.shape[3]
    W = rng.normal(0, 0.05, (4, Co, ho, wo))
    fb = rng.normal(0, 0.05, 4)
    cts = Ly.encrypt_image_columns(o, ok, X, pad, lv, 3, 0)
    Y = Ly.conv2d(o, ok, cts, Ci, h, w, pad, K, bias, Co, k, s)
    pts = Ly.fc_plaintexts(o, W, Co, ho, wo, s, Hp, fc_level)
    lazy = Ly.square_fc_lazy(o, Y[0].scale, pts[0][0].scale, min(Y[0].level, fc_level))
    assert lazy == (fc_level == 3)
    if lazy:
        Z = Ly.square_fc(o, ok, Y, pts, fb, Hp)
    else:
        Z = Ly.fc(o, ok, [Ly.square(o, ok, y) for y in Y], pts, fb, Hp)
    gpts = [g.pt_import(pt.m, pt.level, pt.scale) for row in pts for pt in row]
    net = vr.CNN(Ci, h, w, pad, K, bias, s, square=True, fc_w=gpts, fc_bias=fb, fc_block=Hp)
    gcts = [to_gpu(g, c) for c in cts]
    out = net.forward(g, gk, gcts, n_sets=1)
    for i, (a, b) in enumerate(zip(out, Z)):
        assert_same(a, b, "network output %d (fc level %d, entering at %d)" % (i, fc_level, lv))
    g.set_tuning("conv_prune", "off")
    try:
        full = net.forward(g, gk, gcts, n_sets=1)
    finally:
        g.set_tuning("conv_prune", "on")
    for i, (a, b) in enumerate(zip(full, Z)):
        assert_same(a, b, "network output %d, every conv limb" % i)
    gr = vr.Graph(g, gk, net, gcts, n_sets=1)
    for rep in range(2):
        gr.launch()
        for i, (a, b) in enumerate(zip(gr.outputs(), Z)):
            assert_same(a, b, "graph replay %d output %d" % (rep, i))
    gr.close()
    logits = np.zeros((B, 4))
    for oi, z in enumerate(out):
        logits[:, oi] = g.decode(g.decrypt(gk, z))[np.arange(B) * Hp]
    assert Ly.rel_error(logits, Ly.ref_fc(ref ** 2, W, fb)) < 2.0 ** -20


def test_per_op_network_matches_layer_calls(net):
    """The network as one C-ABI call per HE operation (conv: hoisted
    rotations, MulConst, Add, AddConst, Rescale; x^2: Tensor, the fused
    relinearise-rescale; FC: MulPlain, Add, Rescale, rotations, AddConst)
    decrypts to the layer calls' messages (their conv rounds once per output;
    the plain per-op conv is pinned limb for limb in the layer tests)."""
    from paper_2512_18646_amd import perop
    g, gk, full, conv_sq, sets, params = net
    K, bias, Wfc, fb, pts, Hp, wo = params
    y = perop.square(g, gk, perop.conv2d(g, gk, sets[3], CI, H, W_, PAD, K, bias, S_))
    got, ref = perop.fc(g, gk, y, pts, fb, Hp), layers_ref(g, gk, sets[3], params)
    # the layer calls defer the conv rotations' ModDown into the rescale
    # (one rounding per output instead of one per rotation): same messages
    assert len(got) == len(ref)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert a.meta == b.meta, i
        da, db = g.decode(g.decrypt(gk, a)), g.decode(g.decrypt(gk, b))
        assert np.max(np.abs(da - db)) < 1e-6 * max(1.0, np.max(np.abs(db))), i
