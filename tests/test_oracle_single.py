"""Pins of the oracle's single-ciphertext algorithms (the paper's Technical
Details): the printed worked examples (tests/golden/), brute force on plain
slot vectors (A B, valid cross-correlation, cyclic shifts), the operation
counts of Tables 2 and 3, and the encrypted runs against FP64."""
import os

import numpy as np
import pytest

from oracle import Context, Params
from oracle import single as Sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = 2.0 ** -20


def _blocks(name):
    """Named blocks of token rows from a golden file."""
    out, cur = [], None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            toks = line.split()
            if len(toks) == 1 and toks[0].isalpha() and toks[0].isupper():
                cur = (toks[0], [])
                out.append(cur)
            else:
                cur[1].append(toks)
    return out


# ------------------------------------------------------------ worked examples

def test_kernelspanner_printed_example():
    vals = {"k1": 1.0, "k2": 2.0, "k3": 3.0, "k4": 4.0, "k0": 5.0, "0": 0.0}
    blocks = _blocks("kernelspanner_h4w4k2.txt")
    printed = [np.array([[vals[t] for t in row] for row in rows]) for name, rows in blocks if name == "P"]
    bias = [np.array([[vals[t] for t in row] for row in rows]) for name, rows in blocks if name == "BIAS"][0]
    got = Sg.kernelspanner(np.array([[1.0, 2.0], [3.0, 4.0]]), 4, 4)
    assert len(got) == len(printed) == 4
    for P in printed:    # the printed order differs from a k + b: match as a set
        assert sum(np.array_equal(P, G) for G in got) == 1
    valid = np.zeros((4, 4))
    valid[:3, :3] = 5.0
    assert np.array_equal(bias, valid)


def test_tau_b_and_rowshifter_printed_example():
    m, n, p = 5, 3, 3
    blocks = dict(_blocks("tau_b_rowshifter_m5n3p3.txt"))
    B = np.array([[10.0 * (r + 1) + (c + 1) for c in range(p)] for r in range(n)])   # bKC -> 10 K + C

    def sym(t):
        return 10.0 * int(t[1]) + int(t[2])
    bbar = np.array([[sym(t) for t in row] for row in blocks["BBAR"]])
    shifted = np.array([[sym(t) for t in row] for row in blocks["SHIFTED"]])
    assert np.array_equal(Sg.tau_b(B, m).reshape(m, n), bbar)
    S = 64   # m n = 15 is not a power of two: one copy in the first 15 slots, rotations within it
    ops = Sg.PlainOps(m * n)
    got = Sg.row_shifter(ops, Sg.tau_b(B, m), m, n, p, 1)
    assert np.array_equal(got.reshape(m, n), shifted)
    assert ops.count["Rot"] == 2 and ops.count["cMult"] == 2 and ops.count["Add"] == 1
    assert S


def test_sumforconv_printed_example():
    z = np.array([[10.0 * p + q for q in range(1, 5)] for p in range(1, 5)])
    s = lambda i, j: sum(z[pp - 1, qq - 1] for pp in range(i, i + 3) for qq in range(j, j + 3))
    block = dict(_blocks("sumforconv_n4f4k3.txt"))["S"]
    expect = np.array([[s(int(t[1]), int(t[2])) if t != "0" else 0.0 for t in row] for row in block])
    S = 64
    ops = Sg.PlainOps(S)
    got = Sg.sum_for_conv(ops, Sg.replicate(z.reshape(-1), S), 4, 4, 3, 0.0)
    assert np.array_equal(got[:16].reshape(4, 4), expect)
    assert np.array_equal(got, Sg.replicate(expect.reshape(-1), S))
    # about 2k additions, one cMult and 2k rotations (Rot by 0 not issued)
    assert ops.count["Rot"] == 4 and ops.count["cMult"] == 1 and ops.count["Add"] == 5


# ------------------------------------------------------- plain brute force

@pytest.mark.parametrize("m,n,p", [(8, 4, 3), (8, 4, 4), (4, 8, 3), (16, 2, 2), (2, 4, 2), (8, 8, 5)])
def test_rowshifter_rows_hold_shifted_columns(m, n, p):
    S = 4 * m * n
    rng = np.random.default_rng(m * 100 + n * 10 + p)
    B = rng.integers(-9, 10, (n, p)).astype(float)
    Bbar = Sg.replicate(Sg.tau_b(B, m), S)
    for idx in range(p):
        ops = Sg.PlainOps(S)
        R = Sg.row_shifter(ops, Bbar, m, n, p, idx)[:m * n].reshape(m, n)
        for i in range(m):
            assert np.array_equal(R[i], B[:, (i + idx) % p])
        rot = 0 if idx == 0 else (1 if m % p == 0 else 2)
        assert ops.count["Rot"] == rot


@pytest.mark.parametrize("m,n,p", [(8, 4, 3), (8, 4, 4), (4, 8, 3), (16, 2, 2), (2, 4, 2), (8, 8, 5)])
def test_matmul_plain_equals_product_and_table2_counts(m, n, p):
    S = 2 * m * n
    rng = np.random.default_rng(7 * m + n + p)
    A = rng.integers(-9, 10, (m, n)).astype(float)
    B = rng.integers(-9, 10, (n, p)).astype(float)
    ops = Sg.PlainOps(S)
    C = Sg.matmul(ops, Sg.replicate(Sg.tau_a(A), S), Sg.replicate(Sg.tau_b(B, m), S), m, n, p)
    block = C[:m * n].reshape(m, n)
    assert np.array_equal(block[:, :p], A @ B)
    assert not block[:, p:].any()
    assert np.array_equal(C, Sg.replicate(block.reshape(-1), S))
    # Table 2 per iteration, SumColVec over the n columns: Step 1 one Mult and
    # RowShifter's 2 Rot, 2 cMult, 1 Add (one Rot when p | m, none at idx 0);
    # Step 2 2 log2 n Rot and Add, 1 cMult; Step 3 1 cMult; Step 4 1 Add
    L = Sg.log2_exact(n)
    rs = [(0, 0, 0)] + [((1, 0, 0) if m % p == 0 else (2, 2, 1))] * (p - 1)
    assert ops.count["Mult"] == p
    assert ops.count["Rot"] == sum(r for r, _, _ in rs) + p * 2 * L
    assert ops.count["cMult"] == sum(c for _, c, _ in rs) + p * 2
    assert ops.count["Add"] == sum(a for _, _, a in rs) + p * (2 * L + 1)


@pytest.mark.parametrize("h,w,k", [(4, 4, 2), (8, 8, 3), (4, 8, 3), (8, 4, 2), (8, 8, 5)])
def test_conv_plain_equals_cross_correlation_and_table3_counts(h, w, k):
    S = 2 * h * w
    rng = np.random.default_rng(h * 10 + w + k)
    I = rng.integers(0, 10, (h, w)).astype(float)
    K = rng.integers(-5, 6, (k, k)).astype(float)
    k0 = 7.0
    ops = Sg.PlainOps(S)
    P = [Sg.replicate(M.reshape(-1), S) for M in Sg.kernelspanner(K, h, w)]
    out = Sg.conv(ops, Sg.replicate(I.reshape(-1), S), P, h, w, k, k0)
    block = out[:h * w].reshape(h, w)
    ref = np.zeros((h, w))
    for r in range(h - k + 1):
        for c in range(w - k + 1):
            ref[r, c] = k0 + sum(K[u, v] * I[r + u, c + v] for u in range(k) for v in range(k))
    assert np.array_equal(block, ref)
    # Table 3 per kernel offset: Step 1 one Mult; Step 2 the window sum,
    # 2 (k - 1) Rot and Add; Step 3 one cMult; Step 4 one Add
    kk = k * k
    assert ops.count["Mult"] == kk and ops.count["cMult"] == kk
    assert ops.count["Rot"] == kk * 2 * (k - 1) and ops.count["Add"] == kk * (2 * (k - 1) + 1)


def test_kernelspanner_covers_every_window_once():
    """Every valid window anchor is the anchor of exactly one offset's mask."""
    for h, w, k in [(4, 4, 2), (8, 8, 3), (7, 5, 3)]:
        tot = sum(Sg.conv_mask(h, w, k, a, b) for a in range(k) for b in range(k))
        valid = np.zeros((h, w))
        valid[:h - k + 1, :w - k + 1] = 1
        assert np.array_equal(tot, valid)


@pytest.mark.parametrize("m,n,v,r", [(4, 16, 12, 5), (8, 8, 8, 1), (2, 32, 20, 19)])
def test_vrot_rotates_each_virtual_block(m, n, v, r):
    S = 2 * m * n
    rng = np.random.default_rng(v + r)
    X = np.zeros((m, n))
    X[:, :v] = rng.integers(1, 100, (m, v))
    X[:, v:] = rng.integers(1, 100, (m, n - v))    # junk past each virtual block
    ops = Sg.PlainOps(S)
    got = Sg.vrot(ops, Sg.replicate(X.reshape(-1), S), m, n, v, r)[:m * n].reshape(m, n)
    for i in range(m):
        assert np.array_equal(got[i, :v], np.roll(X[i, :v], -r))
        assert not got[i, v:].any()
    assert ops.count["Rot"] == 2 and ops.count["cMult"] == 2 and ops.count["Add"] == 1


# ------------------------------------------------------------ encrypted runs

@pytest.fixture(scope="module")
def ctx8():
    ctx = Context(Params(8, [60, 40, 40, 40, 40, 40], [60], 6, 40.0, allow_insecure=True))
    steps = sorted(set(Sg.rotation_steps_matmul(8, 4, 3, ctx.slots)) |
                   set(Sg.rotation_steps_conv(8, 3, ctx.slots)))
    return ctx, ctx.keygen(5, rot_steps=steps)


def test_matmul_encrypted_against_fp64(ctx8):
    ctx, keys = ctx8
    m, n, p = 8, 4, 3
    rng = np.random.default_rng(21)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    ops = Sg.HeOps(ctx, keys, 5, 1000)
    ctA = ops.enc(Sg.replicate(Sg.tau_a(A), ctx.slots), level=5)
    ctB = ops.enc(Sg.replicate(Sg.tau_b(B, m), ctx.slots), level=5)
    C = Sg.matmul(ops, ctA, ctB, m, n, p)
    assert C.level == 1
    got = Sg.matmul_decode_layout(ctx.decode(ctx.decrypt(keys, C)), m, n, p)
    ref = A @ B
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < EPS


def test_conv_encrypted_weights_against_fp64(ctx8):
    ctx, keys = ctx8
    h = w = 8
    k = 3
    rng = np.random.default_rng(22)
    I = rng.uniform(0, 1, (h, w))
    K = rng.normal(0, 0.1, (k, k))
    k0 = 0.05
    ops = Sg.HeOps(ctx, keys, 5, 2000)
    ctI = ops.enc(Sg.replicate(I.reshape(-1), ctx.slots), level=5)
    ctS = [ops.enc(Sg.replicate(P.reshape(-1), ctx.slots), level=5) for P in Sg.kernelspanner(K, h, w)]
    out = Sg.conv(ops, ctI, ctS, h, w, k, k0)
    got = np.asarray(ctx.decode(ctx.decrypt(keys, out)))[:h * w].reshape(h, w)
    ref = np.zeros((h, w))
    for r in range(h - k + 1):
        for c in range(w - k + 1):
            ref[r, c] = k0 + np.sum(K * I[r:r + k, c:c + k])
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < EPS


@pytest.mark.parametrize("h,w,k", [(3, 3, 2), (8, 8, 3), (4, 8, 2), (8, 4, 3)])
def test_reform_packs_the_valid_region(h, w, k):
    """The printed 3 x 3 -> 2 x 2 example and larger shapes: the valid region
    row-major in the first h' w' slots, zero after it, junk elsewhere in the
    input ignored; h' - 1 rotations, h' cMult, h' - 1 Add."""
    blk = h * w
    S = 4 * blk if blk & (blk - 1) == 0 else blk    # the printed 3 x 3 fills its ciphertext
    rng = np.random.default_rng(h + w + k)
    J = rng.integers(1, 100, (h, w)).astype(float)     # valid region plus junk outside it
    x = J.reshape(-1)
    ops = Sg.PlainOps(S)
    hp, wp = h - k + 1, w - k + 1
    got = Sg.reform(ops, Sg.replicate(x, S), h, w, k)[:blk]
    assert np.array_equal(got[:hp * wp], J[:hp, :wp].reshape(-1))
    assert not got[hp * wp:].any()
    assert ops.count["Rot"] == hp - 1 and ops.count["cMult"] == hp and ops.count["Add"] == hp - 1
