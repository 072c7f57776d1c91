"""GPU parity of the paper's single-ciphertext schedules (Algorithms 1-5) run
through the library's per-operation calls: limb for limb against the oracle
on the same inputs, masks and fresh encryptions, and end to end (GPU
encoding and encryption) against FP64."""
import numpy as np
import pytest

from oracle import Context as OracleContext, Params
from oracle import single as OS
from tests.gpu_helpers import gpu_ctx, to_gpu, assert_same

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -20
SEED = 5


@pytest.fixture(scope="module")
def ctx8():
    p = Params(8, [60, 40, 40, 40, 40, 40], [60], 6, 40.0, allow_insecure=True)
    o = OracleContext(p)
    steps = sorted(set(OS.rotation_steps_matmul(8, 4, 3, o.slots)) | set(OS.rotation_steps_matmul(8, 4, 4, o.slots)) |
                   set(OS.rotation_steps_conv(8, 3, o.slots)) | {5, 5 - 12} | {2 * r for r in range(1, 6)})
    steps = sorted({s % o.slots for s in steps})
    ok = o.keygen(SEED, rot_steps=steps)
    g = gpu_ctx(p)
    gk = g.keygen(SEED, rot_steps=steps)
    return o, ok, g, gk


def hooks(o, ok, g, first_id):
    """The oracle's plaintexts and fresh encryptions, imported, in the order
    the schedule asks for them (the oracle run draws the same ids)."""
    nxt = [first_id]

    def encode(vec, level, scale):
        pt = o.encode(vec, level, scale)
        return g.pt_import(pt.m, pt.level, pt.scale)

    def encrypt(vec, level, scale):
        ct = o.encrypt(ok, o.encode(vec, level, scale), SEED, nxt[0])
        nxt[0] += 1
        return to_gpu(g, ct)
    return encode, encrypt


@pytest.mark.parametrize("m,n,p", [(8, 4, 3), (8, 4, 4)])
def test_single_matmul_bit_exact(ctx8, m, n, p):
    from paper_2512_18646_amd import single as GS
    o, ok, g, gk = ctx8
    rng = np.random.default_rng(31 + p)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    ops = OS.HeOps(o, ok, SEED, 100)
    ctA = ops.enc(OS.replicate(OS.tau_a(A), o.slots), level=5)
    ctB = ops.enc(OS.replicate(OS.tau_b(B, m), o.slots), level=5)
    ref = OS.matmul(ops, ctA, ctB, m, n, p)
    enc, encr = hooks(o, ok, g, 102)
    gops = GS.Ops(g, gk, encode=enc, encrypt=encr)
    got = GS.matmul(gops, to_gpu(g, ctA), to_gpu(g, ctB), m, n, p)
    assert_same(got, ref, "Algorithm 3 (%d, %d, %d)" % (m, n, p))
    C = g.decode(g.decrypt(gk, got))[:m * n].reshape(m, n)[:, :p]
    assert np.max(np.abs(C - A @ B)) / np.max(np.abs(A @ B)) < EPS


def test_single_conv_and_sumforconv_bit_exact(ctx8):
    from paper_2512_18646_amd import single as GS
    o, ok, g, gk = ctx8
    h = w = 8
    k = 3
    rng = np.random.default_rng(32)
    I, K, k0 = rng.uniform(0, 1, (h, w)), rng.normal(0, 0.1, (k, k)), 0.05
    ops = OS.HeOps(o, ok, SEED, 300)
    ctI = ops.enc(OS.replicate(I.reshape(-1), o.slots), level=5)
    ctS = [ops.enc(OS.replicate(P.reshape(-1), o.slots), level=5) for P in OS.kernelspanner(K, h, w)]
    ref = OS.conv(ops, ctI, ctS, h, w, k, k0)
    enc, encr = hooks(o, ok, g, 300 + 1 + k * k)
    gops = GS.Ops(g, gk, encode=enc, encrypt=encr)
    assert all(np.array_equal(a, b) for a, b in zip(GS.kernelspanner(K, h, w), OS.kernelspanner(K, h, w)))
    got = GS.conv(gops, to_gpu(g, ctI), [to_gpu(g, c) for c in ctS], h, w, k, k0)
    assert_same(got, ref, "Algorithm 4")
    # standalone SumForConv (Algorithm 1) on the image
    ops2 = OS.HeOps(o, ok, SEED, 400)
    ref2 = OS.sum_for_conv(ops2, ctI, h, w, k, k0)
    enc, encr = hooks(o, ok, g, 400)
    got2 = GS.sum_for_conv(GS.Ops(g, gk, encode=enc, encrypt=encr), to_gpu(g, ctI), h, w, k, k0)
    assert_same(got2, ref2, "Algorithm 1")


def test_single_vrot_bit_exact(ctx8):
    from paper_2512_18646_amd import single as GS
    o, ok, g, gk = ctx8
    m, n, v, r = 4, 16, 12, 5
    X = np.random.default_rng(33).uniform(-1, 1, (m, n))
    ops = OS.HeOps(o, ok, SEED, 500)
    ct = ops.enc(OS.replicate(X.reshape(-1), o.slots), level=3)
    ref = OS.vrot(ops, ct, m, n, v, r)
    enc, _ = hooks(o, ok, g, 501)
    got = GS.vrot(GS.Ops(g, gk, encode=enc), to_gpu(g, ct), m, n, v, r)
    assert_same(got, ref, "Algorithm 5")
    z = g.decode(g.decrypt(gk, got))[:m * n].reshape(m, n)
    expect = np.zeros((m, n))
    for i in range(m):
        expect[i, :v] = np.roll(X[i, :v], -r)
    assert np.max(np.abs(z - expect)) < 1e-6


def test_single_matmul_gpu_only_end_to_end(ctx8):
    """GPU encoding of masks, GPU encryption of the operands and the zero
    accumulator: decoded product against FP64."""
    from paper_2512_18646_amd import single as GS
    o, ok, g, gk = ctx8
    m, n, p = 8, 4, 3
    rng = np.random.default_rng(34)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    ids = [900]

    def encrypt(vec, level, scale):
        ids[0] += 1
        return g.encrypt(gk, g.encode(vec, level, scale), 77, ids[0])
    ctA = encrypt(GS.tile(GS.pack_a(A), g.slots), 5, g.scale)
    ctB = encrypt(GS.tile(GS.pack_bbar(B, m), g.slots), 5, g.scale)
    got = GS.matmul(GS.Ops(g, gk, encrypt=encrypt), ctA, ctB, m, n, p)
    C = g.decode(g.decrypt(gk, got))[:m * n].reshape(m, n)[:, :p]
    assert np.max(np.abs(C - A @ B)) / np.max(np.abs(A @ B)) < EPS


def test_single_reform_bit_exact(ctx8):
    from paper_2512_18646_amd import single as GS
    o, ok, g, gk = ctx8
    h, w, k = 8, 8, 3
    X = np.random.default_rng(35).uniform(-1, 1, (h, w))
    ops = OS.HeOps(o, ok, SEED, 600)
    ct = ops.enc(OS.replicate(X.reshape(-1), o.slots), level=3)
    ref = OS.reform(ops, ct, h, w, k)
    enc, _ = hooks(o, ok, g, 601)
    got = GS.reform(GS.Ops(g, gk, encode=enc), to_gpu(g, ct), h, w, k)
    assert_same(got, ref, "ReForm")
    z = g.decode(g.decrypt(gk, got))[:h * w]
    hp, wp = h - k + 1, w - k + 1
    assert np.max(np.abs(z[:hp * wp] - X[:hp, :wp].reshape(-1))) < 1e-6
