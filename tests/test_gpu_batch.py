"""Uneven batches (vr_batch_*): products of different shapes sharing rotation
keys, networks merged into multi-set evaluations, run eagerly and as one
captured graph -- every request's limbs identical to its own call, on every
replay."""
import numpy as np
import pytest

from oracle import layers as Ly
from tests.gpu_helpers import pair, to_gpu, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return pair("C1", rot_steps=tuple(range(1, 16)), log_n=10)


def same(a_list, b_list, what):
    assert len(a_list) == len(b_list), what
    for i, (a, b) in enumerate(zip(a_list, b_list)):
        assert a.meta == b.meta, (what, i)
        assert np.array_equal(a.export(), b.export()), "%s: output %d differs" % (what, i)


def test_uneven_batch_eager_and_graph(ctx):
    from paper_2512_18646_amd import vr
    o, ok, g, gk = ctx
    rng = np.random.default_rng(71)
    mm = []
    for i, (m, n, p) in enumerate([(8, 6, 8), (16, 5, 4), (8, 8, 3), (16, 3, 16), (3, 4, 12)]):
        A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
        if i == 0:   # the oracle's encryption, to anchor the batched limbs
            Ac = [to_gpu(g, c) for c in Ly.encrypt_matrix_columns(o, ok, A, 0, m, p, 3, 81, 0)]
            Bc = [to_gpu(g, c) for c in Ly.encrypt_matrix_columns(o, ok, B, 1, m, p, 3, 81, 100)]
        else:
            Ac = g.encrypt_matrix_columns(gk, A, 0, m, p, 3, 82 + i, 0)
            Bc = g.encrypt_matrix_columns(gk, B, 1, m, p, 3, 82 + i, 100)
        mm.append((A, B, Ac, Bc, m, n, p))
    K1, b1 = rng.normal(0, 0.1, (3, 2, 3, 3)), rng.normal(0, 0.1, 3)
    K2, b2 = rng.normal(0, 0.1, (2, 1, 2, 2)), rng.normal(0, 0.1, 2)
    net1 = vr.CNN(2, 10, 9, 1, K1, b1, 2, square=True)
    net2 = vr.CNN(1, 7, 6, 0, K2, b2, 1, square=False)
    def cols(seed, X, pad):
        return g.encrypt_columns(gk, X, pad, 3, seed, 0)

    nets = [(net1, cols(90, rng.uniform(0, 1, (8, 2, 10, 9)), 1), 1),
            (net1, cols(95, rng.uniform(0, 1, (8, 2, 10, 9)), 1) + cols(96, rng.uniform(0, 1, (8, 2, 10, 9)), 1), 2),
            (net2, cols(99, rng.uniform(0, 1, (4, 1, 7, 6)), 0), 1)]
    b = vr.Batch(g, gk)
    ids, refs = [], []
    for A, B, Ac, Bc, m, n, p in mm:
        ids.append(b.add_matmul(Ac, Bc, m, n, p))
        refs.append(g.matmul(gk, Ac, Bc, m, n, p))
    for net, flat, sets in nets:
        ids.append(b.add_cnn(net, flat, sets))
        refs.append(net.forward(g, gk, flat, sets))
    b.run()
    for i, r in zip(ids, refs):
        same(b.outputs(i), r, "eager request %d" % i)
    # the anchored product against the oracle
    A, B, Ac, Bc, m, n, p = mm[0]
    D = Ly.matmul(o, ok, Ly.encrypt_matrix_columns(o, ok, A, 0, m, p, 3, 81, 0),
                  Ly.encrypt_matrix_columns(o, ok, B, 1, m, p, 3, 81, 100), m, n, p)
    for j, (x, y) in enumerate(zip(b.outputs(ids[0]), D)):
        assert_same(x, y, "batched product %d" % j)
    b.capture()
    for rep in range(3):
        b.launch()
        for i, r in zip(ids, refs):
            same(b.outputs(i), r, "replay %d request %d" % (rep, i))
        net2.forward(g, gk, nets[2][1])[0].export()     # eager work between replays
    b.close()


def test_uneven_batch_outer_products(ctx):
    """Outer-product products in a batch (ragged row tiles, two shapes at one
    level) beside a column-split product and a network: every request's
    limbs identical to its own call, eagerly and on three graph replays with
    eager work between them; the first outer product against the oracle."""
    from paper_2512_18646_amd import vr
    o, ok, g, gk = ctx
    rng = np.random.default_rng(72)
    reqs = []
    for i, (m, n, p) in enumerate([(40, 5, 12), (9, 7, 100), (3, 2, 3)]):
        A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
        if i == 0:
            Ac = [to_gpu(g, c) for c in Ly.encrypt_matrix_outer(o, ok, A, 2, m, p, 3, 91, 0)]
            Bc = [to_gpu(g, c) for c in Ly.encrypt_matrix_outer(o, ok, B, 3, m, p, 3, 91, 1000)]
        else:
            Ac = g.encrypt_matrix_columns(gk, A, 2, m, p, 3, 92 + i, 0)
            Bc = g.encrypt_matrix_columns(gk, B, 3, m, p, 3, 92 + i, 1000)
        reqs.append((A, B, Ac, Bc, m, n, p))
    A2, B2 = rng.uniform(-1, 1, (8, 4)), rng.uniform(-1, 1, (4, 8))
    Ac2 = g.encrypt_matrix_columns(gk, A2, 0, 8, 8, 3, 97, 0)
    Bc2 = g.encrypt_matrix_columns(gk, B2, 1, 8, 8, 3, 97, 100)
    K, bias = rng.normal(0, 0.1, (2, 1, 3, 3)), rng.normal(0, 0.1, 2)
    net = vr.CNN(1, 8, 8, 1, K, bias, 2, square=True)
    cols = g.encrypt_columns(gk, rng.uniform(0, 1, (8, 1, 8, 8)), 1, 3, 98, 0)
    b = vr.Batch(g, gk)
    ids, refs = [], []
    for A, B, Ac, Bc, m, n, p in reqs:
        ids.append(b.add_matmul_outer(Ac, Bc, m, n, p))
        refs.append(g.matmul_outer(gk, Ac, Bc, m, n, p))
    ids.append(b.add_matmul(Ac2, Bc2, 8, 4, 8))
    refs.append(g.matmul(gk, Ac2, Bc2, 8, 4, 8))
    ids.append(b.add_cnn(net, cols))
    refs.append(net.forward(g, gk, cols))
    b.run()
    for i, r in zip(ids, refs):
        same(b.outputs(i), r, "eager request %d" % i)
    A, B, _, _, m, n, p = reqs[0]
    D = Ly.matmul_outer(o, ok, Ly.encrypt_matrix_outer(o, ok, A, 2, m, p, 3, 91, 0),
                        Ly.encrypt_matrix_outer(o, ok, B, 3, m, p, 3, 91, 1000), m, n, p)
    assert len(D) == len(b.outputs(ids[0])) == 2
    for j, (x, y) in enumerate(zip(b.outputs(ids[0]), D)):
        assert_same(x, y, "batched outer product tile %d" % j)
    b.capture()
    for rep in range(3):
        b.launch()
        for i, r in zip(ids, refs):
            same(b.outputs(i), r, "replay %d request %d" % (rep, i))
        net.forward(g, gk, cols)[0].export()     # eager work between replays
    b.close()


@pytest.mark.parametrize("chunk", [1, 3, 7])
def test_products_with_chunked_key_switching(ctx, chunk):
    """Column-split products whose Bbar columns are key-switched in chunks
    of `chunk` ciphertexts (chunk boundaries inside requests and between
    requests of different P'): every request's limbs identical to the
    unchunked call, the first one against the oracle."""
    from paper_2512_18646_amd import vr
    o, ok, g, gk = ctx
    rng = np.random.default_rng(73)
    shapes = [(16, 5, 16), (8, 6, 8), (16, 3, 4), (8, 4, 3)]
    mm = []
    for i, (m, n, p) in enumerate(shapes):
        A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
        Ac = [to_gpu(g, c) for c in Ly.encrypt_matrix_columns(o, ok, A, 0, m, p, 3, 110 + i, 0)]
        Bc = [to_gpu(g, c) for c in Ly.encrypt_matrix_columns(o, ok, B, 1, m, p, 3, 110 + i, 100)]
        mm.append((A, B, Ac, Bc, m, n, p))
    g.set_tuning("switch_chunk", "0")
    refs = [g.matmul(gk, Ac, Bc, m, n, p) for A, B, Ac, Bc, m, n, p in mm]
    try:
        g.set_tuning("switch_chunk", str(chunk))
        b = vr.Batch(g, gk)
        ids = [b.add_matmul(Ac, Bc, m, n, p) for A, B, Ac, Bc, m, n, p in mm]
        b.run()
        for i, r in zip(ids, refs):
            same(b.outputs(i), r, "chunk %d request %d" % (chunk, i))
        A, B, Ac, Bc, m, n, p = mm[0]
        alone = g.matmul(gk, Ac, Bc, m, n, p)
        same(alone, refs[0], "chunk %d single product" % chunk)
        b.close()
    finally:
        g.set_tuning("switch_chunk", "0")
    A, B, _, _, m, n, p = mm[0]
    D = Ly.matmul(o, ok, Ly.encrypt_matrix_columns(o, ok, A, 0, m, p, 3, 110, 0),
                  Ly.encrypt_matrix_columns(o, ok, B, 1, m, p, 3, 110, 100), m, n, p)
    for j, (x, y) in enumerate(zip(refs[0], D)):
        assert_same(x, y, "product %d" % j)
