"""Multi-set conv and the continuous-batching server: a request's output limbs
are the same whether it is evaluated alone, in a batched multi-set call or in
a server wave mixed with other requests, sessions and models; admission by
memory, cancellation and level errors."""
import numpy as np
import pytest

from oracle import layers as Ly
from tests.gpu_helpers import pair, to_gpu, assert_same

pytestmark = pytest.mark.gpu

SHAPE = dict(B=8, Ci=2, h=10, w=9, k=3, s=2, pad=1)


@pytest.fixture(scope="module")
def small():
    return pair("C1", rot_steps=(1, 2, 4, 8), log_n=10)


def draw(rng, co=3):
    S = SHAPE
    X = rng.uniform(0, 1, (S["B"], S["Ci"], S["h"], S["w"]))
    K = rng.normal(0, 0.1, (co, S["Ci"], S["k"], S["k"]))
    bias = rng.normal(0, 0.1, co)
    return X, K, bias


def same_limbs(a, b, what):
    assert a.meta == b.meta, what
    assert np.array_equal(a.export(), b.export()), what


def test_conv2d_sets_matches_single_set_calls(small):
    o, ok, g, gk = small
    S = SHAPE
    rng = np.random.default_rng(11)
    _, K, bias = draw(rng)
    sets = [g.encrypt_columns(gk, rng.uniform(0, 1, (S["B"], S["Ci"], S["h"], S["w"])), S["pad"], 3,
                              77, 100 * i) for i in range(3)]
    flat = [c for st in sets for c in st]
    Y = g.conv2d_sets(gk, flat, 3, S["Ci"], S["h"], S["w"], S["pad"], K, bias, S["s"])
    per = len(Y) // 3
    for i, st in enumerate(sets):
        one = g.conv2d(gk, st, S["Ci"], S["h"], S["w"], S["pad"], K, bias, S["s"])
        assert len(one) == per
        for j in range(per):
            same_limbs(Y[i * per + j], one[j], "set %d out %d" % (i, j))
    # one set against the oracle
    X, _, _ = draw(np.random.default_rng(12))
    cts = Ly.encrypt_image_columns(o, ok, X, S["pad"], 3, 5, 0)
    ref = Ly.conv2d(o, ok, cts, S["Ci"], S["h"], S["w"], S["pad"], K, bias, 3, S["k"], S["s"])
    gc = [to_gpu(g, c) for c in cts]
    Y2 = g.conv2d_sets(gk, flat[:S["Ci"] * S["w"]] + gc, 2, S["Ci"], S["h"], S["w"], S["pad"], K,
                       bias, S["s"])
    for j in range(per):
        assert_same(Y2[per + j], ref[j], "oracle set out %d" % j)


def alone(g, keys, cols, K, bias, square):
    S = SHAPE
    y = g.conv2d(keys, cols, S["Ci"], S["h"], S["w"], S["pad"], K, bias, S["s"])
    return g.square(keys, y) if square else y


def test_server_mixed_requests_identical_to_alone(small):
    from paper_2512_18646_amd import vr
    o, ok, g, gk = small
    S = SHAPE
    gk2 = g.keygen(2024, rot_steps=[1, 2])
    rng = np.random.default_rng(21)
    _, K1, b1 = draw(rng, 3)
    _, K2, b2 = draw(rng, 2)
    srv = vr.Server(g, 8 << 30, max_batch=4)
    s1, s2 = srv.register_session(gk), srv.register_session(gk2)
    m1 = srv.register_conv_model(S["Ci"], S["h"], S["w"], S["pad"], K1, b1, S["s"], square=True)
    m2 = srv.register_conv_model(S["Ci"], S["h"], S["w"], S["pad"], K2, b2, S["s"], square=False)
    plan = [(s1, gk, m1, K1, b1, True)] * 5 + [(s2, gk2, m1, K1, b1, True)] * 2 + \
           [(s1, gk, m2, K2, b2, False)] * 3
    order = np.random.default_rng(5).permutation(len(plan))
    # the first request carries the oracle's encryption, to anchor the served limbs
    X0 = rng.uniform(0, 1, (S["B"], S["Ci"], S["h"], S["w"]))
    ocols = Ly.encrypt_image_columns(o, ok, X0, S["pad"], 3, 800, 0)
    batch = [(s1, gk, m1, K1, b1, True, [to_gpu(g, c) for c in ocols])]
    for n, i in enumerate(order):
        sess, keys, model, K, bias, sq = plan[i]
        X = rng.uniform(0, 1, (S["B"], S["Ci"], S["h"], S["w"]))
        batch.append((sess, keys, model, K, bias, sq, g.encrypt_columns(keys, X, S["pad"], 3, 900 + n, 0)))
    # submitted in a burst, so that later requests queue behind the first waves
    reqs = [(srv.submit(sess, model, cols, S["B"]), keys, model, K, bias, sq, cols)
            for sess, keys, model, K, bias, sq, cols in batch]
    outs = [srv.poll(r[0], r[2]) for r in reqs]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["batched"] == len(reqs)
    assert st["waves"] < len(reqs), st          # some waves held several requests
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    for (t, keys, model, K, bias, sq, cols), got in zip(reqs, outs):
        ref = alone(g, keys, cols, K, bias, sq)
        assert len(got) == len(ref)
        for j, (a, b) in enumerate(zip(got, ref)):
            same_limbs(a, b, "ticket %d out %d" % (t, j))
    Y = Ly.conv2d(o, ok, ocols, S["Ci"], S["h"], S["w"], S["pad"], K1, b1, 3, S["k"], S["s"])
    for j, y in enumerate(Y):
        assert_same(outs[0][j], Ly.square(o, ok, y), "served vs oracle %d" % j)


def test_server_admission_cancel_and_levels(small):
    from paper_2512_18646_amd import vr
    o, ok, g, gk = small
    S = SHAPE
    rng = np.random.default_rng(31)
    X, K, bias = draw(rng)
    with pytest.raises(vr.VRError) as e:
        vr.Server(g, 1 << 16).register_session(gk)     # keys alone exceed the budget
    assert e.value.code == vr.VR_EBUSY
    tight = vr.Server(g, 12 << 20)
    sid = tight.register_session(gk)
    mid = tight.register_conv_model(S["Ci"], S["h"], S["w"], S["pad"], K, bias, S["s"])
    cols = g.encrypt_columns(gk, X, S["pad"], 3, 1, 0)
    with pytest.raises(vr.VRError) as e:
        tight.submit(sid, mid, cols, S["B"])           # the request can never fit
    assert e.value.code == vr.VR_EBUSY
    tight.close()

    srv = vr.Server(g, 8 << 30, max_batch=2)
    sid = srv.register_session(gk)
    mid = srv.register_conv_model(S["Ci"], S["h"], S["w"], S["pad"], K, bias, S["s"])
    low = g.encrypt_columns(gk, X, S["pad"], 1, 2, 0)
    with pytest.raises(vr.VRError) as e:
        srv.submit(sid, mid, low, S["B"])              # conv + x^2 needs two levels
    assert e.value.code == vr.VR_ELEVEL
    with pytest.raises(vr.VRError) as e:
        srv.submit(sid, mid, cols[:-1], S["B"])
    assert e.value.code == vr.VR_EINVAL
    tickets = [srv.submit(sid, mid, cols, S["B"]) for _ in range(8)]
    try:
        srv.cancel(tickets[-1])
        cancelled = True
    except vr.VRError as err:                         # it had already started
        assert err.code == vr.VR_EINVAL
        cancelled = False
    ref = alone(g, gk, cols, K, bias, True)
    for t in tickets[:-1]:
        for a, b in zip(srv.poll(t, mid), ref):
            same_limbs(a, b, "ticket %d" % t)
    if cancelled:
        with pytest.raises(vr.VRError) as e:
            srv.poll(tickets[-1], mid)
        assert e.value.code == vr.VR_ECANCELED
    else:
        srv.poll(tickets[-1], mid)
    with pytest.raises(vr.VRError):
        srv.poll(tickets[0], mid)                      # ticket already consumed
    srv.close()


def test_caching_allocator_steady_state(small):
    """Repeated identical layer calls reuse cached blocks: nothing new is
    reserved after the first call, freed outputs return their bytes, and trim
    hands every free block back."""
    o, ok, g, gk = small
    S = SHAPE
    X, K, bias = draw(np.random.default_rng(41))
    cols = g.encrypt_columns(gk, X, S["pad"], 3, 3, 0)
    reserved, used = [], []
    for _ in range(3):
        y = alone(g, gk, cols, K, bias, True)
        y[0].export()                                  # synchronises
        reserved.append(g.mem_info()[0])
        del y
        used.append(g.mem_info()[1])
    # the first call also caches the layer's constants (weights, term lists)
    assert reserved[1] == reserved[2] == reserved[0], reserved
    assert used[0] == used[1] == used[2], used
    g.trim()
    r, u = g.mem_info()
    assert r == u == used[0]


def test_chunked_key_switching_identical(small):
    """Layers key-switch in chunks when the scratch would exceed its budget;
    forcing tiny chunks gives the same limbs."""
    o, ok, g, gk = small
    S = SHAPE
    X, K, bias = draw(np.random.default_rng(61))
    cols = g.encrypt_columns(gk, X, S["pad"], 3, 6, 0)
    ref = alone(g, gk, cols, K, bias, True)
    g.set_tuning("switch_chunk", "4")
    try:
        got = alone(g, gk, cols, K, bias, True)
    finally:
        g.set_tuning("switch_chunk", "0")
    for j, (a, b) in enumerate(zip(got, ref)):
        same_limbs(a, b, "chunked out %d" % j)


def test_server_full_network_model(small):
    """A registered conv + x^2 + FC network: served results identical to the
    whole-network call on each request alone."""
    from paper_2512_18646_amd import vr
    o, ok, g, gk = small
    S = SHAPE
    rng = np.random.default_rng(81)
    _, K, bias = draw(rng)
    Hp = Ly.image_block(S["h"], S["pad"])
    wo = Ly.conv_out_size(S["w"], S["pad"], S["k"], S["s"])
    ho = Ly.conv_out_size(S["h"], S["pad"], S["k"], S["s"])
    pts = g.encode_fc_weights(rng.normal(0, 0.05, (4, 3, ho, wo)), S["s"], Hp, 1)
    net = vr.CNN(S["Ci"], S["h"], S["w"], S["pad"], K, bias, S["s"], square=True, fc_w=pts,
                 fc_bias=rng.normal(0, 0.05, 4), fc_block=Hp)
    srv = vr.Server(g, 8 << 30, max_batch=4)
    sid = srv.register_session(gk)
    mid = srv.register_model(net)
    inputs = [g.encrypt_columns(gk, rng.uniform(0, 1, (S["B"], S["Ci"], S["h"], S["w"])), S["pad"], 3,
                                400 + i, 0) for i in range(5)]
    tickets = [srv.submit(sid, mid, c, S["B"]) for c in inputs]
    outs = [srv.poll(t, mid) for t in tickets]
    low = g.encrypt_columns(gk, rng.uniform(0, 1, (S["B"], S["Ci"], S["h"], S["w"])), S["pad"], 2, 499, 0)
    with pytest.raises(vr.VRError) as e:
        srv.submit(sid, mid, low, S["B"])             # conv, x^2 and FC need three levels
    assert e.value.code == vr.VR_ELEVEL
    srv.close()
    for i, (c, got) in enumerate(zip(inputs, outs)):
        ref = net.forward(g, gk, c)
        assert len(got) == len(ref) == 4
        for j, (a, b) in enumerate(zip(got, ref)):
            same_limbs(a, b, "request %d logit %d" % (i, j))


def test_server_lazy_fc_pruned_waves_identical_to_alone():
    """Requests entering at level 7 of the C2 chain with FC weights at level 3
    (x^2 relinearised once per FC output, the conv pruned to the FC's four
    limbs), from two sessions with their own keys: every served result is
    identical to the whole-network call on that request alone."""
    from paper_2512_18646_amd import vr
    o, ok, g, gk = pair("C2", rot_steps=(1, 2, 4, 8), log_n=10)
    gk2 = g.keygen(77, rot_steps=[1, 2, 4, 8])
    S = SHAPE
    rng = np.random.default_rng(82)
    _, K, bias = draw(rng)
    Hp = Ly.image_block(S["h"], S["pad"])
    wo = Ly.conv_out_size(S["w"], S["pad"], S["k"], S["s"])
    ho = Ly.conv_out_size(S["h"], S["pad"], S["k"], S["s"])
    pts = g.encode_fc_weights(rng.normal(0, 0.05, (4, 3, ho, wo)), S["s"], Hp, 3)
    net = vr.CNN(S["Ci"], S["h"], S["w"], S["pad"], K, bias, S["s"], square=True, fc_w=pts,
                 fc_bias=rng.normal(0, 0.05, 4), fc_block=Hp)
    srv = vr.Server(g, 8 << 30, max_batch=4)
    sids = [srv.register_session(gk), srv.register_session(gk2)]
    mid = srv.register_model(net)
    keys = [gk, gk2]
    inputs = [g.encrypt_columns(keys[i % 2], rng.uniform(0, 1, (S["B"], S["Ci"], S["h"], S["w"])), S["pad"], 7,
                                600 + i, 0) for i in range(6)]
    tickets = [srv.submit(sids[i % 2], mid, c, S["B"]) for i, c in enumerate(inputs)]
    outs = [srv.poll(t, mid) for t in tickets]
    srv.close()
    for i, (c, got) in enumerate(zip(inputs, outs)):
        ref = net.forward(g, keys[i % 2], c)
        assert len(got) == len(ref) == 4
        for j, (a, b) in enumerate(zip(got, ref)):
            assert a.meta[1] == 1, (i, j)
            same_limbs(a, b, "request %d logit %d" % (i, j))


@pytest.mark.timeout(300)
def test_server_n16_identical_to_alone_and_oracle():
    """Serving at N = 2^16 (the L = 24 chain, dnum 3) at level 3: requests of
    two sessions and two models submitted in one burst; every served output
    has the limbs of the same request evaluated alone, and the first request
    (the oracle's encryption) matches the oracle's conv + x^2 limb for limb."""
    from paper_2512_18646_amd import vr
    o, ok, g, gk = pair("C3", rot_steps=(1, 2))
    gk2 = g.keygen(2025, rot_steps=[1, 2])
    B, Ci, h, w, k, s, pad = 64, 1, 8, 8, 3, 2, 1
    rng = np.random.default_rng(41)
    K1, b1 = rng.normal(0, 0.05, (2, Ci, k, k)), rng.normal(0, 0.05, 2)
    K2, b2 = rng.normal(0, 0.05, (3, Ci, k, k)), rng.normal(0, 0.05, 3)
    srv = vr.Server(g, 64 << 30, max_batch=4)
    s1, s2 = srv.register_session(gk), srv.register_session(gk2)
    m1 = srv.register_conv_model(Ci, h, w, pad, K1, b1, s, square=True)
    m2 = srv.register_conv_model(Ci, h, w, pad, K2, b2, s, square=False)
    X0 = rng.uniform(0, 1, (B, Ci, h, w))
    ocols = Ly.encrypt_image_columns(o, ok, X0, pad, 3, 4100, 0)
    batch = [(s1, gk, m1, K1, b1, True, [to_gpu(g, c) for c in ocols])]
    plan = [(s1, gk, m1, K1, b1, True)] * 3 + [(s2, gk2, m1, K1, b1, True)] * 2 + \
           [(s1, gk, m2, K2, b2, False)] * 2
    for n, (sess, keys, model, K, bias, sq) in enumerate(plan):
        X = rng.uniform(0, 1, (B, Ci, h, w))
        batch.append((sess, keys, model, K, bias, sq, g.encrypt_columns(keys, X, pad, 3, 4200 + n, 0)))
    reqs = [(srv.submit(sess, model, cols, B), keys, model, K, bias, sq, cols)
            for sess, keys, model, K, bias, sq, cols in batch]
    outs = [srv.poll(r[0], r[2]) for r in reqs]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    for (t, keys, model, K, bias, sq, cols), got in zip(reqs, outs):
        y = g.conv2d(keys, cols, Ci, h, w, pad, K, bias, s)
        ref = g.square(keys, y) if sq else y
        assert len(got) == len(ref)
        for j, (a, b) in enumerate(zip(got, ref)):
            same_limbs(a, b, "N=2^16 ticket %d out %d" % (t, j))
    Y = Ly.conv2d(o, ok, ocols, Ci, h, w, pad, K1, b1, 2, k, s)
    for j, y in enumerate(Y):
        assert_same(outs[0][j], Ly.square(o, ok, y), "N=2^16 served vs oracle %d" % j)
