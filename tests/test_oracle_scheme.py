"""Pins of the oracle's CKKS scheme and column-wise schedules: closed forms of
the encoder, decryption invariants, key-switching noise, rotation identities,
and the schedules against FP64 plaintext layers (matmul, convolution, x^2,
FC) including their special cases."""
import numpy as np
import pytest

from oracle import Context, Params, PRESETS, Ciphertext
from oracle import layers as Ly
from oracle.ckks import rha

EPS = 2.0 ** -20


def small_ctx(log_n=8, q_bits=(60, 40, 40, 40), p_bits=(60,), dnum=4, log2_scale=40.0):
    return Context(Params(log_n, list(q_bits), list(p_bits), dnum, log2_scale, allow_insecure=True))


# ------------------------------------------------------------------ encoder

def test_encode_constant_closed_form():
    ctx = small_ctx()
    for c in (0.75, -0.3, 1.0):
        m = ctx.encode_int(np.full(ctx.slots, c), ctx.scale)
        assert m[0] == rha(c * ctx.scale)
        assert np.all(m[1:] == 0)


def test_encode_single_slot_closed_form():
    """z = e_j: m_t = RHA((2 scale / N) cos(pi g_j t / N))."""
    ctx = small_ctx(log_n=6)
    j = 3
    z = np.zeros(ctx.slots)
    z[j] = 1.0
    m = ctx.encode_int(z, ctx.scale)
    t = np.arange(ctx.n)
    want = 2 * ctx.scale / ctx.n * np.cos(np.pi * ctx.gexp[j] * t / ctx.n)
    assert np.max(np.abs(m - want)) <= 0.5 + 1e-3


def test_encode_periodic_vector_lies_in_subring():
    """A slot vector with period H' is fixed by the Galois element 5^H', of
    order r = S / H' modulo 2N, whose fixed ring is Z[X^r]: the brute-force
    coefficients (2 scale / N) sum_j z_j cos(pi g_j t / N) vanish for t not a
    multiple of r, and the subring encoding equals their rounding everywhere
    and decodes to z."""
    ctx = small_ctx(log_n=7)
    S, Hp = ctx.slots, 8
    r = S // Hp
    z = np.tile(np.random.default_rng(4).uniform(-1, 1, Hp), r)
    t = np.arange(ctx.n)
    want = np.array([2 * ctx.scale / ctx.n * sum(z[j] * np.cos(np.pi * ctx.gexp[j] * tt / ctx.n)
                                                  for j in range(S)) for tt in t])
    assert np.max(np.abs(want[t % r != 0])) < 1e-2
    m = ctx.encode_int(z, ctx.scale, sub_log=r.bit_length() - 1)
    assert np.all(m[t % r != 0] == 0)
    assert np.array_equal(m, np.array([rha(x) for x in want]))
    assert np.array_equal(m[t % r == 0], ctx.encode_int(z, ctx.scale)[t % r == 0])
    pt = ctx.encode(z, 1, ctx.scale, sub_log=r.bit_length() - 1)
    assert np.max(np.abs(ctx.decode(pt) - z)) < 2.0 ** -30


def test_decode_encode_roundtrip():
    ctx = Context(PRESETS["C2"])
    z = np.random.default_rng(0).uniform(-1, 1, ctx.slots)
    pt = ctx.encode(z, 2, ctx.scale)
    assert np.max(np.abs(ctx.decode(pt) - z)) < 2.0 ** -(40 - 10)


def test_automorphism_5_rotates_slots_left():
    ctx = small_ctx(log_n=7)
    z = np.random.default_rng(1).uniform(-1, 1, ctx.slots)
    pt = ctx.encode(z, 0, ctx.scale)
    q = ctx.q[0]
    pt.m[0] = ctx.automorphism(pt.m[0], 5, q)
    assert np.max(np.abs(ctx.decode(pt) - np.roll(z, -1))) < 1e-9
    # 5 has order S modulo 2N: rotation by S is the identity element
    assert ctx.galois_element(ctx.slots) == 1


# ---------------------------------------------------------- encrypt / decrypt

@pytest.mark.parametrize("name", ["C1", "C2"])
def test_decrypt_encrypt_noise(name):
    ctx = Context(PRESETS[name])
    keys = ctx.keygen(1000 + 1)
    z = np.random.default_rng(2).uniform(-1, 1, ctx.slots)
    ct = ctx.encrypt(keys, ctx.encode(z, ctx.L, ctx.scale), 77, 0)
    err = np.max(np.abs(ctx.decode(ctx.decrypt(keys, ct)) - z))
    assert err < 2.0 ** -21
    # the public key is an encryption of zero: b + a s is small
    q = ctx.q[1]
    bas = ctx.vadd(keys.pk_b[1], ctx.polymul(keys.pk_a[1], ctx.reduce_int(keys.s, q), q), q)
    cen = np.where(bas > q // 2, bas.astype(np.float64) - q, bas.astype(np.float64))
    assert np.abs(cen).max() <= 19


def test_encrypt_is_deterministic_in_seed_and_id():
    ctx = small_ctx()
    keys = ctx.keygen(3)
    pt = ctx.encode(np.ones(4), 2, ctx.scale)
    a = ctx.encrypt(keys, pt, 5, 1)
    b = ctx.encrypt(keys, pt, 5, 1)
    c = ctx.encrypt(keys, pt, 5, 2)
    assert np.array_equal(a.c, b.c) and not np.array_equal(a.c, c.c)


def test_key_switch_noise_bound():
    """decrypt(KS(d)) - d s' is small for s' = s^2 (relinearisation key)."""
    ctx = Context(PRESETS["C1"])
    keys = ctx.keygen(9)
    rng = np.random.default_rng(3)
    lv = ctx.L
    d = np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.moduli(lv)])
    o0, o1 = ctx.key_switch(d, keys.rlk, lv)
    for i, q in enumerate(ctx.moduli(lv)):
        s = ctx.reduce_int(keys.s, q)
        got = ctx.vadd(o0[i], ctx.polymul(o1[i], s, q), q)
        want = ctx.polymul(d[i], ctx.polymul(s, s, q), q)
        e = ctx.vsub(got, want, q).astype(np.float64)
        e = np.where(e > q // 2, e - q, e)
        assert np.abs(e).max() < 2.0 ** 16


def test_relin_rescale_decrypts_the_product():
    """x y through the fused relinearise-and-rescale decodes to the FP64
    product at the scale of a rescale, with no more error than the two-step
    form."""
    ctx = Context(PRESETS["C1"])
    keys = ctx.keygen(21)
    rng = np.random.default_rng(22)
    x, y = rng.uniform(-1, 1, ctx.slots), rng.uniform(-1, 1, ctx.slots)
    cx = ctx.encrypt(keys, ctx.encode(x, ctx.L, ctx.scale), 3, 0)
    cy = ctx.encrypt(keys, ctx.encode(y, ctx.L, ctx.scale), 3, 1)
    T = ctx.tensor(cx, cy)
    f = ctx.relin_rescale(T, keys)
    r = ctx.rescale(ctx.relinearize(T, keys))
    assert f.level == ctx.L - 1 and f.scale == r.scale
    ef = np.max(np.abs(ctx.decode(ctx.decrypt(keys, f)) - x * y))
    er = np.max(np.abs(ctx.decode(ctx.decrypt(keys, r)) - x * y))
    assert ef < EPS and ef < 2 * er + 1e-12


def test_lazy_rotation_decrypts():
    """A rotation kept in the extended basis and rescaled by the ModDown by
    P q_l decrypts to the rotated message at the rescaled scale."""
    ctx = small_ctx(log_n=8)
    keys = ctx.keygen(23, rot_steps=[5])
    z = np.random.default_rng(24).uniform(-1, 1, ctx.slots)
    ct = ctx.encrypt(keys, ctx.encode(z, 3, ctx.scale), 1, 0)
    dq = float(ctx.q[3])
    e = ctx.add_const_ext(ctx.mul_const_ext(ctx.rotate_ext(ct, 5, keys), 0.5, dq), 0.25)
    y = ctx.mod_down_rescale(e)
    assert y.level == 2 and y.scale == ctx.scale
    assert np.max(np.abs(ctx.decode(ctx.decrypt(keys, y)) - (0.5 * np.roll(z, -5) + 0.25))) < 1e-7


# ----------------------------------------------------------------- rotations

def test_rotation_invariants():
    ctx = small_ctx(log_n=8)
    keys = ctx.keygen(4, rot_steps=[1, 2, 3, 5])
    z = np.random.default_rng(4).uniform(-1, 1, ctx.slots)
    ct = ctx.encrypt(keys, ctx.encode(z, 3, ctx.scale), 1, 0)
    r12 = ctx.rotate(ctx.rotate(ct, 1, keys), 2, keys)
    r3 = ctx.rotate(ct, 3, keys)
    d12 = ctx.decode(ctx.decrypt(keys, r12))
    d3 = ctx.decode(ctx.decrypt(keys, r3))
    assert np.max(np.abs(d3 - np.roll(z, -3))) < 1e-6
    assert np.max(np.abs(d12 - d3)) < 1e-6
    assert np.array_equal(ctx.rotate(ct, ctx.slots, keys).c, ct.c)
    with pytest.raises(KeyError):
        ctx.rotate(ct, 4, keys)
    hoisted = ctx.rotate_many(ct, [1, 5], keys)
    assert np.array_equal(hoisted[1].c, ctx.rotate(ct, 5, keys).c)


def test_add_level_and_scale_checks():
    ctx = small_ctx()
    keys = ctx.keygen(1)
    a = ctx.encrypt(keys, ctx.encode([1.0], 3, ctx.scale), 1, 0)
    b = ctx.encrypt(keys, ctx.encode([1.0], 2, ctx.scale), 1, 1)
    with pytest.raises(ValueError):
        ctx.add(a, b)
    c = Ciphertext(a.c, a.level, a.scale * 2)
    with pytest.raises(ValueError):
        ctx.add(a, c)


def test_mul_const_add_const_rescale():
    ctx = small_ctx(log_n=9)
    keys = ctx.keygen(2)
    z = np.random.default_rng(5).uniform(-1, 1, ctx.slots)
    ct = ctx.encrypt(keys, ctx.encode(z, 3, ctx.scale), 1, 0)
    y = ctx.rescale(ctx.add_const(ctx.mul_const(ct, -0.37, float(ctx.q[3])), 0.25))
    assert y.level == 2 and y.scale == ctx.scale
    assert np.max(np.abs(ctx.decode(ctx.decrypt(keys, y)) - (-0.37 * z + 0.25))) < 1e-7


# ------------------------------------------------------- schedules vs FP64

@pytest.fixture(scope="module")
def ctx10():
    ctx = small_ctx(log_n=10, q_bits=(49, 40, 40, 40), p_bits=(49,), dnum=4)
    keys = ctx.keygen(1001, rot_steps=list(range(1, 16)) + [32, 64, 128])
    return ctx, keys


def test_matmul_schedule_random(ctx10):
    ctx, keys = ctx10
    m, n, p = 16, 16, 16
    rng = np.random.default_rng(1)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    Ac = Ly.encrypt_matrix_columns(ctx, keys, A, 0, m, p, 3, 1, 0)
    Bc = Ly.encrypt_matrix_columns(ctx, keys, B, 1, m, p, 3, 1, 100)
    D = Ly.matmul(ctx, keys, Ac, Bc, m, n, p)
    assert len(D) == 16 and D[0].level == 2
    C = Ly.matmul_decode(ctx, keys, D, m, p)
    assert Ly.rel_error(C, A @ B) < EPS


def test_matmul_schedule_m_below_p(ctx10):
    """m < p through the transposed schedule, decoded against FP64."""
    ctx, keys = ctx10
    m, n, p = 5, 4, 13
    rng = np.random.default_rng(13)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    D = Ly.matmul(ctx, keys, Ly.encrypt_matrix_columns(ctx, keys, A, 0, m, p, 3, 4, 0),
                  Ly.encrypt_matrix_columns(ctx, keys, B, 1, m, p, 3, 4, 100), m, n, p)
    assert len(D) == Ly.pow2ceil(m)
    got = Ly.matmul_decode(ctx, keys, D, m, p)
    assert not np.isnan(got).any()
    assert Ly.rel_error(got, A @ B) < EPS


def test_matmul_schedule_identity_and_ragged(ctx10):
    """B = I gives C = A; m=12 > p=5 pads to M'=16, P'=8 (ragged tail)."""
    ctx, keys = ctx10
    m, n, p = 12, 5, 5
    rng = np.random.default_rng(2)
    A = rng.uniform(-1, 1, (m, n))
    Ac = Ly.encrypt_matrix_columns(ctx, keys, A, 0, m, p, 3, 2, 0)
    Bc = Ly.encrypt_matrix_columns(ctx, keys, np.eye(n), 1, m, p, 3, 2, 100)
    D = Ly.matmul(ctx, keys, Ac, Bc, m, n, p)
    assert len(D) == 8
    C = Ly.matmul_decode(ctx, keys, D, m, p)
    assert not np.any(np.isnan(C))
    assert Ly.rel_error(C, A) < EPS


def test_matmul_column_slot_layout_brute_force():
    """The column-split encodings on plain slot vectors: with rotation as a
    left cyclic shift of the slots (pinned by the automorphism test above),
    D_idx = sum_k A_k * Rot(Bbar_k, idx) holds C[i][(i + idx) mod P'] in slot
    i (exact on small integers), and zero there when that column is past p;
    brute force over ragged shapes, every entry of A B reached once."""
    ctx = small_ctx(log_n=6)   # 32 slots
    rng = np.random.default_rng(11)
    for m, n, p in ((4, 3, 3), (12, 5, 5), (8, 2, 8), (16, 3, 1), (32, 2, 32)):
        A = rng.integers(-9, 10, (m, n)).astype(float)
        B = rng.integers(-9, 10, (n, p)).astype(float)
        C = A @ B
        Pp = Ly.pow2ceil(p)
        seen = np.zeros((m, p), int)
        for idx in range(Pp):
            D = sum(Ly.matrix_column_slots(ctx, A, k, 0, m, p) * np.roll(Ly.matrix_column_slots(ctx, B, k, 1, m, p), -idx)
                    for k in range(n))
            for i in range(m):
                col = (i + idx) % Pp
                if col < p:
                    assert D[i] == C[i, col]
                    seen[i, col] += 1
                else:
                    assert D[i] == 0.0
        assert (seen == 1).all()


def test_matmul_transposed_slot_layout_brute_force():
    """m < p: the same ciphertexts with their roles swapped (Bbar_k as the
    A role, A_k rotated) give C^T = B^T A^T: sum_k Bbar_k * Rot(A_k, idx)
    holds C[(i + idx) mod M'][i] in slot i < p, zero where that row is past
    m; every entry of A B reached once (plain slot vectors, small integers)."""
    ctx = small_ctx(log_n=6)   # 32 slots
    rng = np.random.default_rng(12)
    for m, n, p in ((3, 4, 4), (5, 2, 12), (1, 3, 16), (7, 3, 32)):
        A = rng.integers(-9, 10, (m, n)).astype(float)
        B = rng.integers(-9, 10, (n, p)).astype(float)
        C = A @ B
        Mp = Ly.pow2ceil(m)
        seen = np.zeros((m, p), int)
        for idx in range(Mp):
            D = sum(Ly.matrix_column_slots(ctx, B, k, 1, m, p) * np.roll(Ly.matrix_column_slots(ctx, A, k, 0, m, p), -idx)
                    for k in range(n))
            for i in range(p):
                row = (i + idx) % Mp
                if row < m:
                    assert D[i] == C[row, i]
                    seen[row, i] += 1
                else:
                    assert D[i] == 0.0
        assert (seen == 1).all()


def test_conv_column_slot_layout_brute_force():
    """The conv's column encoding on plain slot vectors: Y(c', j') = bias +
    sum_{c,u,v} K[c'][c][u][v] Rot(col(c, s j' + v - pad), u), with rotation
    a left cyclic shift, holds output row i' of image b in slot b H' + s i';
    checked exactly (small integers) against cross-correlation with zero
    padding written out as loops, for several strides, pads and a full slot
    vector (the last image block wraps around)."""
    ctx = small_ctx(log_n=6)   # 32 slots
    rng = np.random.default_rng(12)
    for B, C_in, h, w, pad, k, stride, C_out in ((4, 2, 5, 5, 1, 3, 2, 2), (2, 1, 6, 7, 0, 4, 2, 3),
                                                 (3, 2, 4, 4, 2, 2, 1, 1), (4, 1, 8, 3, 0, 3, 3, 2)):
        X = rng.integers(-5, 6, (B, C_in, h, w)).astype(float)
        K = rng.integers(-3, 4, (C_out, C_in, k, k)).astype(float)
        bias = rng.integers(-4, 5, C_out).astype(float)
        Hp = Ly.image_block(h, pad)
        assert B * Hp <= ctx.slots
        ho, wo = (h + 2 * pad - k) // stride + 1, (w + 2 * pad - k) // stride + 1
        for co in range(C_out):
            for jo in range(wo):
                Y = np.full(ctx.slots, bias[co])
                for c in range(C_in):
                    for v in range(k):
                        jj = stride * jo + v - pad
                        if 0 <= jj < w:
                            col = Ly.image_column_slots(ctx, X, c, jj, pad)
                            for u in range(k):
                                Y = Y + K[co, c, u, v] * np.roll(col, -u)
                for b in range(B):
                    for io in range(ho):
                        want = bias[co]
                        for c in range(C_in):
                            for u in range(k):
                                for v in range(k):
                                    i, j = stride * io + u - pad, stride * jo + v - pad
                                    if 0 <= i < h and 0 <= j < w:
                                        want += K[co, c, u, v] * X[b, c, i, j]
                        assert Y[b * Hp + stride * io] == want


def test_fc_slot_layout_and_block_sum_brute_force():
    """FC on plain slot vectors: the weight plaintexts (decoded and rounded;
    small integer weights) times the conv-output layout, with arbitrary junk
    in every slot that holds no output row, summed over the ciphertexts and
    then Z += Rot(Z, 2^t) for 2^t < H', hold bias-free FC output o of image b
    in slot b H', exactly against the dot product written out as loops."""
    ctx = small_ctx(log_n=6)   # 32 slots
    rng = np.random.default_rng(13)
    for B, C, ho, wo, stride, Hp, n_out in ((4, 2, 3, 2, 2, 8, 3), (2, 1, 5, 3, 3, 16, 2), (8, 3, 2, 2, 2, 4, 2)):
        assert B * Hp <= ctx.slots and stride * (ho - 1) < Hp
        Yv = rng.integers(-5, 6, (B, C, ho, wo)).astype(float)
        W = rng.integers(-3, 4, (n_out, C, ho, wo)).astype(float)
        pts = Ly.fc_plaintexts(ctx, W.reshape(n_out, -1), C, ho, wo, stride, Hp, 3)
        wslots = [[np.rint(ctx.decode(pt).real) for pt in row] for row in pts]
        cts = []
        for c in range(C):
            for jo in range(wo):
                z = rng.integers(-50, 51, ctx.slots).astype(float)   # junk outside the output rows
                for b in range(B):
                    z[b * Hp + stride * np.arange(ho)] = Yv[b, c, :, jo]
                cts.append(z)
        for o in range(n_out):
            Z = sum(y * wv for y, wv in zip(cts, wslots[o]))
            step = 1
            while step < Hp:
                Z = Z + np.roll(Z, -step)
                step *= 2
            for b in range(B):
                want = 0.0
                for c in range(C):
                    for i in range(ho):
                        for j in range(wo):
                            want += W[o, c, i, j] * Yv[b, c, i, j]
                assert Z[b * Hp] == want


def test_matmul_outer_slot_layout_brute_force():
    """The outer-product encodings on plain slot vectors: sum_k A'_{t,k} * B'_k
    (element-wise, exact on small integers) is tile t of A B, slot r P' + j
    = C[t R + r][j], zeros elsewhere; brute force over ragged shapes with
    several tiles (m not a multiple of R, p not a power of two)."""
    ctx = small_ctx(log_n=6)   # 32 slots
    rng = np.random.default_rng(5)
    for m, n, p in ((5, 3, 3), (13, 4, 5), (2, 7, 8), (33, 2, 1)):
        A = rng.integers(-9, 10, (m, n)).astype(float)
        B = rng.integers(-9, 10, (n, p)).astype(float)
        C = A @ B
        Pp, R, T = Ly.outer_tiles(ctx, m, p)
        assert Pp * R == ctx.slots and T == -(-m // R)
        seen = np.zeros((m, p), bool)
        for t in range(T):
            acc = sum(Ly.matrix_outer_slots(ctx, A, 2, m, p, t, k) * Ly.matrix_outer_slots(ctx, B, 3, m, p, 0, k)
                      for k in range(n))
            for s in range(ctx.slots):
                i, j = t * R + s // Pp, s % Pp
                if i < m and j < p:
                    assert acc[s] == C[i, j]
                    seen[i, j] = True
                else:
                    assert acc[s] == 0.0
        assert seen.all()


def test_matmul_outer_schedule_random_and_identity(ctx10):
    """Encrypted outer-product product against FP64 (two row tiles with a
    ragged last one at N = 2^10: S = 512, P' = 64, R = 8, m = 12), and A = I
    giving C = B; n tensors and one relinearisation per tile, no rotation."""
    ctx, keys = ctx10
    rng = np.random.default_rng(3)
    m, n, p = 12, 7, 40
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    Ac = Ly.encrypt_matrix_outer(ctx, keys, A, 2, m, p, 3, 3, 0)
    Bc = Ly.encrypt_matrix_outer(ctx, keys, B, 3, m, p, 3, 3, 1000)
    assert len(Ac) == 2 * n and len(Bc) == n
    D = Ly.matmul_outer(ctx, keys, Ac, Bc, m, n, p)
    assert len(D) == 2 and D[0].level == 2
    C = Ly.matmul_outer_decode(ctx, keys, D, m, p)
    assert not np.any(np.isnan(C))
    assert Ly.rel_error(C, A @ B) < EPS
    m2 = n2 = 6
    B2 = rng.uniform(-1, 1, (n2, p))
    Ac = Ly.encrypt_matrix_outer(ctx, keys, np.eye(m2), 2, m2, p, 3, 4, 0)
    Bc = Ly.encrypt_matrix_outer(ctx, keys, B2, 3, m2, p, 3, 4, 1000)
    C = Ly.matmul_outer_decode(ctx, keys, Ly.matmul_outer(ctx, keys, Ac, Bc, m2, n2, p), m2, p)
    assert Ly.rel_error(C, B2) < EPS


def test_conv_schedule_random_square_fc(ctx10):
    ctx, keys = ctx10
    B, Ci, h, w, Co, k, s, pad = 8, 2, 10, 9, 3, 3, 2, 1
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (B, Ci, h, w))
    K = rng.normal(0, 0.1, (Co, Ci, k, k))
    bias = rng.normal(0, 0.1, Co)
    cts = Ly.encrypt_image_columns(ctx, keys, X, pad, 3, 3, 0)
    Y = Ly.conv2d(ctx, keys, cts, Ci, h, w, pad, K, bias, Co, k, s)
    ref = Ly.ref_conv(X, K, bias, s, pad)
    got = Ly.conv_decode(ctx, keys, Y, B, Co, h, pad, k, s, w)
    assert Ly.rel_error(got, ref) < EPS
    Y2 = [Ly.square(ctx, keys, y) for y in Y]
    got2 = Ly.conv_decode(ctx, keys, Y2, B, Co, h, pad, k, s, w)
    assert Ly.rel_error(got2, ref ** 2) < EPS
    Hp = Ly.image_block(h, pad)
    ho, wo = ref.shape[2], ref.shape[3]
    W = rng.normal(0, 0.05, (4, Co, ho, wo))
    fb = rng.normal(0, 0.05, 4)
    pts = Ly.fc_plaintexts(ctx, W, Co, ho, wo, s, Hp, Y2[0].level)
    Z = Ly.fc(ctx, keys, Y2, pts, fb, Hp)
    logits = Ly.fc_decode(ctx, keys, Z, B, Hp)
    assert Ly.rel_error(logits, Ly.ref_fc(ref ** 2, W, fb)) < EPS
    # weights one level below the inputs (conv outputs at level 2, weights at
    # level 1): the layer runs at the weights' level and still decodes to the
    # FP64 FC of the conv outputs
    assert Y[0].level == 2
    pts1 = Ly.fc_plaintexts(ctx, W, Co, ho, wo, s, Hp, 1)
    Z1 = Ly.fc(ctx, keys, Y, pts1, fb, Hp)
    assert Z1[0].level == 0
    assert Ly.rel_error(Ly.fc_decode(ctx, keys, Z1, B, Hp), Ly.ref_fc(ref, W, fb)) < EPS


def test_square_fc_lazy_relinearisation_against_fp64():
    """x^2 and FC with one relinearisation per FC output decode to the FP64
    FC of the squared conv outputs, as the per-layer form does; the rule
    refuses levels without room for the unrelinearised products."""
    ctx = small_ctx(log_n=10, q_bits=(49, 40, 40, 40, 40, 40), p_bits=(49,), dnum=6)
    keys = ctx.keygen(1002, rot_steps=list(range(1, 3)) + [2 ** i for i in range(2, 8)])
    B, Ci, h, w, Co, k, s, pad = 4, 2, 10, 9, 3, 3, 2, 1
    rng = np.random.default_rng(30)
    X = rng.uniform(0, 1, (B, Ci, h, w))
    K = rng.normal(0, 0.1, (Co, Ci, k, k))
    bias = rng.normal(0, 0.1, Co)
    cts = Ly.encrypt_image_columns(ctx, keys, X, pad, 5, 3, 0)
    Y = Ly.conv2d(ctx, keys, cts, Ci, h, w, pad, K, bias, Co, k, s)
    assert Y[0].level == 4
    ref = Ly.ref_conv(X, K, bias, s, pad)
    Hp = Ly.image_block(h, pad)
    ho, wo = ref.shape[2], ref.shape[3]
    W = rng.normal(0, 0.05, (4, Co, ho, wo))
    fb = rng.normal(0, 0.05, 4)
    pts = Ly.fc_plaintexts(ctx, W, Co, ho, wo, s, Hp, 3)
    assert Ly.square_fc_lazy(ctx, Y[0].scale, pts[0][0].scale, 3)
    assert not Ly.square_fc_lazy(ctx, Y[0].scale, pts[0][0].scale, 2)
    assert not Ly.square_fc_lazy(ctx, Y[0].scale, pts[0][0].scale, 1)
    Z = Ly.square_fc(ctx, keys, Y, pts, fb, Hp)
    assert Z[0].level == 1
    want = Ly.ref_fc(ref ** 2, W, fb)
    lazy = Ly.fc_decode(ctx, keys, Z, B, Hp)
    assert Ly.rel_error(lazy, want) < EPS
    plain = Ly.fc_decode(ctx, keys, Ly.fc(ctx, keys, [Ly.square(ctx, keys, y) for y in Y], pts, fb, Hp), B, Hp)
    assert Ly.rel_error(plain, want) < EPS
    with pytest.raises(ValueError):
        Ly.square_fc(ctx, keys, Y, Ly.fc_plaintexts(ctx, W, Co, ho, wo, s, Hp, 2), fb, Hp)


def test_conv_special_cases(ctx10):
    """A delta kernel returns the strided, shifted image; a constant image
    returns the constant times the kernel sum (interior outputs)."""
    ctx, keys = ctx10
    B, h, w, k, s = 4, 12, 12, 3, 2
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (B, 1, h, w))
    K = np.zeros((1, 1, k, k))
    K[0, 0, 1, 2] = 1.0
    cts = Ly.encrypt_image_columns(ctx, keys, X, 0, 2, 4, 0)
    Y = Ly.conv2d(ctx, keys, cts, 1, h, w, 0, K, np.zeros(1), 1, k, s)
    got = Ly.conv_decode(ctx, keys, Y, B, 1, h, 0, k, s, w)
    ho = (h - k) // s + 1
    want = X[:, :, 1:1 + s * ho:s, 2:2 + s * ho:s]
    assert np.max(np.abs(got - want)) < 1e-6
    Xc = np.full((B, 1, h, w), 0.6)
    K2 = rng.normal(0, 0.1, (1, 1, k, k))
    cts = Ly.encrypt_image_columns(ctx, keys, Xc, 0, 2, 5, 0)
    Y = Ly.conv2d(ctx, keys, cts, 1, h, w, 0, K2, np.zeros(1), 1, k, s)
    got = Ly.conv_decode(ctx, keys, Y, B, 1, h, 0, k, s, w)
    assert np.max(np.abs(got - 0.6 * K2.sum())) < 1e-6


# --------------------------------------------- deeper networks (Table 1)

def test_poly_eval_horner_against_fp64_and_depth():
    """Horner evaluation of the Table 1 activations: depth equal to the
    degree, decoded against the FP64 polynomial; degree 1 is one MulConst."""
    ctx = small_ctx(log_n=9, q_bits=(60, 40, 40, 40, 40), p_bits=(60,), dnum=5)
    keys = ctx.keygen(8)
    z = np.random.default_rng(9).uniform(-1, 1, ctx.slots)
    ct = ctx.encrypt(keys, ctx.encode(z, 4, ctx.scale), 8, 0)
    for coeffs in (Ly.ACT1, Ly.ACT2, (0.5, -2.0)):
        y = Ly.poly_eval(ctx, keys, ct, coeffs)
        assert y.level == 4 - (len(coeffs) - 1)
        got = ctx.decode(ctx.decrypt(keys, y))
        assert Ly.rel_error(got, Ly.ref_poly(z, coeffs)) < EPS


def test_dense_layer_against_fp64():
    ctx = small_ctx(log_n=9)
    keys = ctx.keygen(10)
    rng = np.random.default_rng(10)
    Z = rng.uniform(-1, 1, (5, ctx.slots))
    W, b = rng.normal(0, 0.3, (3, 5)), rng.normal(0, 0.3, 3)
    cts = [ctx.encrypt(keys, ctx.encode(z, 3, ctx.scale), 10, j) for j, z in enumerate(Z)]
    out = Ly.dense(ctx, keys, cts, W, b)
    got = np.stack([ctx.decode(ctx.decrypt(keys, c)) for c in out])
    assert Ly.rel_error(got, W @ Z + b[:, None]) < EPS


def test_deep_cnn_table1_shape_against_fp64():
    """CONV 3x3 (4 kernels, stride 1) -> ACT-1 -> FC -> ACT-2 -> FC-2 with the
    paper's activations on 28 x 28 images (FC-1 narrowed to 6 neurons and
    FC-2 to 3 outputs to keep the oracle fast), decoded logits against the
    FP64 network."""
    ctx = small_ctx(log_n=10, q_bits=(60,) + (40,) * 9, p_bits=(60,), dnum=10)
    B, h, w, k, Co = 4, 28, 28, 3, 4
    Hp = Ly.image_block(h, 0)
    keys = ctx.keygen(11, rot_steps=[1, 2] + Ly.fc_rotation_steps(Hp))
    rng = np.random.default_rng(11)
    X = rng.uniform(0, 1, (B, 1, h, w))
    K, kb = rng.normal(0, 0.1, (Co, 1, k, k)), rng.normal(0, 0.1, Co)
    ho = wo = h - k + 1
    W1, b1 = rng.normal(0, 0.01, (6, Co, ho, wo)), rng.normal(0, 0.05, 6)
    W2, b2 = rng.normal(0, 0.3, (3, 6)), rng.normal(0, 0.3, 3)
    cts = Ly.encrypt_image_columns(ctx, keys, X, 0, 9, 11, 0)
    pts = Ly.fc_plaintexts(ctx, W1, Co, ho, wo, 1, Hp, 5)
    out = Ly.deep_cnn(ctx, keys, cts, 1, h, w, 0, K, kb, 1, Ly.ACT1, pts, b1, Hp, Ly.ACT2, W2, b2)
    assert out[0].level == 0
    got = Ly.fc_decode(ctx, keys, out, B, Hp)
    ref = Ly.ref_deep_cnn(X, K, kb, 1, 0, Ly.ACT1, W1, b1, Ly.ACT2, W2, b2)
    assert Ly.rel_error(got, ref) < EPS


# ------------------------------------------------ encrypted-weight mode

def test_encrypted_weight_conv_and_fc_against_fp64(ctx10):
    """Conv and FC with encrypted weights (ct x ct products, one lazy
    relinearisation per output) decode to the FP64 layers; with the same
    weights the conv output decodes like the plaintext-weight schedule."""
    ctx, keys = ctx10
    B, Ci, h, w, Co, k, s, pad = 8, 2, 10, 9, 3, 3, 2, 1
    rng = np.random.default_rng(15)
    X = rng.uniform(0, 1, (B, Ci, h, w))
    K, bias = rng.normal(0, 0.1, (Co, Ci, k, k)), rng.normal(0, 0.1, Co)
    cts = Ly.encrypt_image_columns(ctx, keys, X, pad, 3, 15, 0)
    kct, bct = Ly.encrypt_conv_weights(ctx, keys, K, bias, 3, cts[0].scale, 16, 0)
    Y = Ly.conv2d_encw(ctx, keys, cts, Ci, h, w, pad, kct, bct, Co, k, s)
    assert Y[0].level == 2 and Y[0].ncomp == 2
    ref = Ly.ref_conv(X, K, bias, s, pad)
    got = Ly.conv_decode(ctx, keys, Y, B, Co, h, pad, k, s, w)
    assert Ly.rel_error(got, ref) < EPS
    Hp = Ly.image_block(h, pad)
    ho, wo = ref.shape[2], ref.shape[3]
    W, fb = rng.normal(0, 0.05, (4, Co, ho, wo)), rng.normal(0, 0.05, 4)
    wct, fbct = Ly.encrypt_fc_weights(ctx, keys, W, fb, Co, ho, wo, s, Hp, 2, Y[0].scale, 17, 0)
    Z = Ly.fc_encw(ctx, keys, Y, wct, fbct, Hp)
    logits = Ly.fc_decode(ctx, keys, Z, B, Hp)
    assert Ly.rel_error(logits, Ly.ref_fc(ref, W, fb)) < EPS


# --------------------------------------------------- column-block form

def test_matmul_block_slot_layout_brute_force():
    """Column blocks on plain slot vectors: sum_K A_K * Rot(Bbar_K, idx), then
    the fold over the c blocks, holds C[i][(i + idx) mod P'] in slot i < m
    (zero where that column is past p), exact on small integers, every entry
    reached once; ragged shapes with several ciphertexts per operand."""
    ctx = small_ctx(log_n=7)   # 64 slots
    rng = np.random.default_rng(17)
    for m, n, p in ((4, 3, 3), (5, 9, 4), (8, 20, 2), (12, 5, 5), (3, 17, 1)):
        A = rng.integers(-9, 10, (m, n)).astype(float)
        B = rng.integers(-9, 10, (n, p)).astype(float)
        C = A @ B
        Pp, Mb, c, nb = Ly.block_shape(ctx, m, n, p)
        assert Mb >= m + Pp - 1 and Mb % Pp == 0 and c * Mb <= ctx.slots and nb * c >= n
        seen = np.zeros((m, p), int)
        for idx in range(Pp):
            D = sum(Ly.matrix_block_slots(ctx, A, K, 4, m, n, p) *
                    np.roll(Ly.matrix_block_slots(ctx, B, K, 5, m, n, p), -idx) for K in range(nb))
            t = 1
            while t < c:
                D = D + np.roll(D, -Mb * t)
                t *= 2
            for i in range(m):
                col = (i + idx) % Pp
                if col < p:
                    assert D[i] == C[i, col]
                    seen[i, col] += 1
                else:
                    assert D[i] == 0.0
        assert (seen == 1).all()


def test_matmul_block_schedule_against_fp64(ctx10):
    ctx, keys = ctx10
    m, n, p = 12, 20, 5
    rng = np.random.default_rng(18)
    A, B = rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (n, p))
    Pp, Mb, c, nb = Ly.block_shape(ctx, m, n, p)
    k2 = ctx.keygen(1001, rot_steps=Ly.block_rotation_steps(ctx, m, n, p))
    D = Ly.matmul_block(ctx, k2, Ly.encrypt_matrix_blocks(ctx, k2, A, 4, m, n, p, 3, 5, 0),
                        Ly.encrypt_matrix_blocks(ctx, k2, B, 5, m, n, p, 3, 5, 100), m, n, p)
    assert len(D) == Pp and nb == 2 and c == 16   # two ciphertexts per operand, the second ragged
    got = Ly.matmul_decode(ctx, k2, D, m, p)
    assert Ly.rel_error(got, A @ B) < EPS
