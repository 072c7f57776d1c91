"""Pins of the oracle's arithmetic primitives against things other than itself:
sympy primality, RFC 8439 vectors, schoolbook negacyclic products, Horner
evaluation, Python big-integer CRT, exact rounding, and sampler statistics."""
import os
import random

import numpy as np
import pytest
import sympy

from oracle import Context, Params, PRESETS, Ciphertext, gen_primes, find_psi, cdt_table, security_bound
from oracle._clib import lib, ptr
from oracle.ckks import rha, rha_array

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ primes

@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C1_literal"])
def test_prime_chain_definition(name):
    p = PRESETS[name]
    n2 = 1 << (p.log_n + 1)
    bits = list(p.q_bits) + list(p.p_bits)
    primes = gen_primes(p.log_n, bits)
    assert len(set(primes)) == len(primes)
    for k, (q, b) in enumerate(zip(primes, bits)):
        assert sympy.isprime(q)
        assert q % n2 == 1
        assert q.bit_length() == b
        # nothing larger below 2^b qualifies unless an earlier entry took it
        c = q + n2
        while c < (1 << b):
            assert (not sympy.isprime(c)) or c in primes[:k]
            c += n2


def test_security_bound():
    assert Context(PRESETS["C1"]).secure
    assert Context(PRESETS["C2"]).secure
    assert Context(PRESETS["C3"]).secure
    lit = PRESETS["C1_literal"]
    assert not Context(lit).secure
    with pytest.raises(ValueError):
        Context(Params(lit.log_n, lit.q_bits, lit.p_bits, lit.dnum, lit.log2_scale))
    assert security_bound(13) == 218 and security_bound(16) == 1740


@pytest.mark.parametrize("log_n", [4, 13, 16])
def test_psi_is_primitive_2n_root(log_n):
    for q in gen_primes(16, [60, 50, 51, 40]):
        psi = find_psi(q, log_n)
        n = 1 << log_n
        assert pow(psi, n, q) == q - 1
        assert pow(psi, 2 * n, q) == 1


# ---------------------------------------------------------- scalar arithmetic

def test_mulmod_edges():
    rnd = random.Random(1)
    for q in gen_primes(16, [60, 50, 40]):
        vals = [0, 1, 2, q - 1, q - 2, q // 2, q // 2 + 1] + [rnd.randrange(q) for _ in range(50)]
        for a in vals:
            for b in vals[:10]:
                assert lib.orc_mulmod(a, b, q) == a * b % q
        for x in [0, 1, -1, q, -q, 2 ** 62, -(2 ** 62), -(2 ** 63)]:
            assert lib.orc_reduce_i64(x, q) == x % q


def test_rha_half_away_from_zero():
    assert [rha(x) for x in (0.5, -0.5, 1.5, -1.5, 2.4999, -2.5000001)] == [1, -1, 2, -2, 2, -3]
    big = float(2 ** 52 + 1)
    assert rha(big) == 2 ** 52 + 1          # floor(x + 0.5) would give 2^52 + 2
    assert list(rha_array([0.5, -0.5, big])) == [1.0, -1.0, big]


# --------------------------------------------------------------------- NTT

def _schoolbook_negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += a[i] * b[j]
            else:
                out[k - n] -= a[i] * b[j]
    return [x % q for x in out]


def _brev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2)


@pytest.mark.parametrize("log_n", [3, 4, 5, 6])
def test_polymul_equals_schoolbook(log_n):
    rnd = random.Random(log_n)
    P = Params(log_n, [60, 40], [51], 1, 30.0, allow_insecure=True)
    ctx = Context(P)
    for q in ctx.q + ctx.p + gen_primes(16, [50]):
        a = [rnd.randrange(q) for _ in range(ctx.n)]
        b = [rnd.randrange(q) for _ in range(ctx.n)]
        got = ctx.polymul(np.array(a, np.uint64), np.array(b, np.uint64), q)
        assert [int(x) for x in got] == _schoolbook_negacyclic(a, b, q)


@pytest.mark.parametrize("log_n", [3, 6])
def test_ntt_order_is_bitreversed_evaluation(log_n):
    """Output i equals the Horner value of a at psi^(2 brev(i) + 1)."""
    rnd = random.Random(7)
    ctx = Context(Params(log_n, [50], [51], 1, 30.0, allow_insecure=True))
    q = ctx.q[0]
    psi = find_psi(q, log_n)
    a = [rnd.randrange(q) for _ in range(ctx.n)]
    got = [int(x) for x in ctx.ntt(np.array(a, np.uint64), q)]
    for i in range(ctx.n):
        x = pow(psi, 2 * _brev(i, log_n) + 1, q)
        acc = 0
        for c in reversed(a):
            acc = (acc * x + c) % q
        assert got[i] == acc
    back = ctx.intt(np.array(got, np.uint64), q)
    assert [int(v) for v in back] == a


def test_ntt_roundtrip_full_size():
    ctx = Context(PRESETS["C2"])
    rng = np.random.default_rng(3)
    for q in (ctx.q[0], ctx.q[3], ctx.p[0]):
        a = rng.integers(0, q, ctx.n, dtype=np.uint64)
        assert np.array_equal(ctx.intt(ctx.ntt(a, q), q), a)


# ------------------------------------------------------------------ ChaCha20

def _golden_chacha():
    d = {}
    for line in open(os.path.join(GOLDEN, "rfc8439_chacha20.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            d[k] = [int(x, 16) for x in v]
    return d


def test_chacha_quarter_round_rfc8439():
    g = _golden_chacha()
    s = np.array(g["quarter_in"], dtype=np.uint32)
    lib.orc_chacha_quarter(ptr(s))
    assert [int(x) for x in s] == g["quarter_out"]


def test_chacha_block_rfc8439():
    g = _golden_chacha()
    key = np.array(g["block_key"], dtype=np.uint32)
    nonce = np.array(g["block_nonce"], dtype=np.uint32)
    out = np.zeros(16, dtype=np.uint32)
    lib.orc_chacha20_block(ptr(key), g["block_counter"][0], ptr(nonce), ptr(out))
    assert [int(x) for x in out] == g["block_out"]


def test_stream_word_layout():
    """word w = little-endian bytes 8w..8w+7 of the keystream (block w // 8)."""
    ctx = Context(PRESETS["C1"])
    seed, pur, obj = 0x1122334455667788, 6, 0x0000000a0000000b
    words = ctx.stream_words(seed, pur, obj, 0, 24)
    key = np.array([seed & 0xffffffff, seed >> 32, 0, 0, 0, 0, 0, 0], dtype=np.uint32)
    nonce = np.array([pur, obj & 0xffffffff, obj >> 32], dtype=np.uint32)
    for blk in range(3):
        out = np.zeros(16, dtype=np.uint32)
        lib.orc_chacha20_block(ptr(key), blk, ptr(nonce), ptr(out))
        for j in range(8):
            assert int(words[blk * 8 + j]) == int(out[2 * j]) | (int(out[2 * j + 1]) << 32)
    assert np.array_equal(ctx.stream_words(seed, pur, obj, 5, 10), words[5:15])


# ------------------------------------------------------------------ samplers

def test_uniform_sampler_192bit_product():
    ctx = Context(PRESETS["C3"])
    q = ctx.p[2]
    limb = 3
    got = ctx.sample_uniform(9, 4, 70, limb, q)
    w = ctx.stream_words(9, 4, 70, 2 * limb * ctx.n, 2 * ctx.n)
    for t in list(range(64)) + [ctx.n - 1]:
        W = int(w[2 * t]) | (int(w[2 * t + 1]) << 64)
        assert int(got[t]) == (W * q) >> 128
    assert got.max() < q
    assert abs(float(got.astype(np.float64).mean()) / q - 0.5) < 0.01


def test_ternary_sampler_frequencies():
    ctx = Context(PRESETS["C3"])
    s = ctx.sample_ternary(5, 1, 0)
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == [-1, 0, 1]
    assert np.all(np.abs(counts / s.size - 1 / 3) < 0.01)


def test_cdt_table_properties():
    t = cdt_table(3.2)
    assert len(t) == 20 and t[-1] == 1 << 63
    assert all(a < b for a, b in zip(t, t[1:]))
    rho = np.exp(-np.arange(20) ** 2 / (2 * 3.2 ** 2))
    z = rho[0] + 2 * rho[1:].sum()
    assert abs(t[0] / 2.0 ** 63 - rho[0] / z) < 1e-12
    assert abs(t[5] / 2.0 ** 63 - (rho[0] + 2 * rho[1:6].sum()) / z) < 1e-12


def test_gaussian_sampler_statistics():
    ctx = Context(PRESETS["C3"])
    e = np.concatenate([ctx.sample_gauss(11, 3, k) for k in range(4)]).astype(np.float64)
    assert abs(e.mean()) < 0.05
    assert abs(e.var() / 3.2 ** 2 - 1) < 0.03
    assert np.abs(e).max() <= 19
    assert abs(np.mean(e > 0) - np.mean(e < 0)) < 0.01


# ------------------------------------------------------------ base conversion

def _crt(residues, moduli):
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M, M


@pytest.mark.parametrize("alpha", [1, 3, 9])
def test_base_conversion_is_lift_plus_small_multiple(alpha):
    """conv(x) = X + e Q_D exactly, |e| <= alpha/2, for X the centred CRT lift."""
    ctx = Context(Params(3, [50] * 9, [51] * 9, 1, 30.0, allow_insecure=True))
    rng = np.random.default_rng(alpha)
    qin = ctx.q[:alpha]
    qout = ctx.p + ctx.q[alpha:]
    x = np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in qin])
    out = ctx.base_convert(x, qin, qout)
    for t in range(ctx.n):
        X, Q = _crt([x[i, t] for i in range(alpha)], qin)
        if X > Q // 2:
            X -= Q
        es = set()
        for o, to in enumerate(qout):
            # find the e with out = X + e Q mod t_o among |e| <= alpha/2 + 1
            cand = [e for e in range(-alpha, alpha + 1) if (X + e * Q - int(out[o, t])) % to == 0]
            assert len(cand) == 1
            es.add(cand[0])
        assert len(es) == 1
        assert abs(es.pop()) <= alpha / 2 + 0.5


# ------------------------------------------------------------------- rescale

def test_rescale_is_rounded_division():
    ctx = Context(Params(3, [60, 50, 50, 50], [51], 4, 30.0, allow_insecure=True))
    rng = np.random.default_rng(4)
    from oracle import Ciphertext
    lv = 3
    c = np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.q])
                  for _ in range(2)])
    out = ctx.rescale(Ciphertext(c, lv, 2.0 ** 60))
    for k in range(2):
        for t in range(ctx.n):
            X, Q = _crt([c[k, i, t] for i in range(lv + 1)], ctx.q)
            ql = ctx.q[lv]
            # round(X / q_l) with X taken modulo Q: the rescaled value modulo Q/q_l
            Y = (2 * X + ql) // (2 * ql)
            for i in range(lv):
                assert int(out.c[k, i, t]) == Y % ctx.q[i]
    assert out.scale == 2.0 ** 60 / ctx.q[lv]


def test_mod_down_is_division_by_p():
    """ModDown returns round(U / P) up to +-K/2 (centred base conversion)."""
    ctx = Context(Params(3, [60, 50, 50], [51, 51, 51], 1, 30.0, allow_insecure=True))
    rng = np.random.default_rng(8)
    lv = 2
    ext = ctx.ext_moduli(lv)
    u = np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ext])
    out = ctx.mod_down(u, lv)
    P = 1
    for p in ctx.p:
        P *= p
    Qm = 1
    for q in ctx.q:
        Qm *= q
    for t in range(ctx.n):
        U, M = _crt([u[i, t] for i in range(len(ext))], ext)
        Y, _ = _crt([out[i, t] for i in range(lv + 1)], ctx.q)
        diff = (Y - (2 * U + P) // (2 * P)) % Qm
        if diff > Qm // 2:
            diff -= Qm
        assert abs(diff) <= ctx.K / 2 + 1


@pytest.mark.parametrize("p_bits,dnum", [((51, 51, 51), 1), ((51,), 3)])
def test_relin_rescale_is_one_rounded_division(p_bits, dnum):
    """Relinearisation and rescale as one ModDown by P q_l agree, coefficient
    by coefficient over q_0..q_{l-1}, with Rescale(Relin(.)) to within the two
    roundings (|diff| <= K/2 + 2): a dropped P c term or a division by the
    wrong prime moves the result by about q_l or P."""
    ctx = Context(Params(3, [60, 50, 50, 50], list(p_bits), dnum, 30.0, allow_insecure=True))
    keys = ctx.keygen(12)
    rng = np.random.default_rng(9)
    lv = 3
    c = np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.moduli(lv)])
                  for _ in range(3)])
    a = Ciphertext(c, lv, 2.0 ** 60)
    fused = ctx.relin_rescale(a, keys)
    ref = ctx.rescale(ctx.relinearize(a, keys))
    assert fused.level == ref.level == lv - 1 and fused.scale == ref.scale
    Qm = 1
    for q in ctx.q[:lv]:
        Qm *= q
    for comp in range(2):
        for t in range(ctx.n):
            X, _ = _crt([fused.c[comp, i, t] for i in range(lv)], ctx.q[:lv])
            Y, _ = _crt([ref.c[comp, i, t] for i in range(lv)], ctx.q[:lv])
            diff = (X - Y) % Qm
            if diff > Qm // 2:
                diff -= Qm
            assert abs(diff) <= ctx.K / 2 + 2
    # the fused form is not the unfused one limb for limb on random words
    assert not np.array_equal(fused.c, ref.c)
    with pytest.raises(ValueError):
        ctx.relin_rescale(Ciphertext(c[:, :1], 0, 1.0), keys)


def _crt_diff(x, y, moduli):
    M = 1
    for q in moduli:
        M *= q
    X, _ = _crt(x, moduli)
    Y, _ = _crt(y, moduli)
    d = (X - Y) % M
    return d - M if d > M // 2 else d


def test_lazy_moddown_of_lifted_ops_is_the_plain_rescale():
    """On P times a ciphertext (lift), MulConst, Add and AddConst in the
    extended basis followed by the ModDown by P q_l give exactly the rescale
    of the same operations on the ciphertext: the conversion of
    (P c_l, 0, ..., 0) is P [c_l] with no overflow term."""
    ctx = Context(Params(4, [60, 50, 50, 50], [51, 51, 51], 1, 30.0, allow_insecure=True))
    keys = ctx.keygen(14)
    rng = np.random.default_rng(15)
    lv = 3
    mk = lambda: Ciphertext(np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64)
                                                for q in ctx.moduli(lv)]) for _ in range(2)]), lv, 2.0 ** 30)
    a, b = mk(), mk()
    dq = float(ctx.q[lv])
    plain = ctx.add_const(ctx.add(ctx.mul_const(a, 0.37, dq), ctx.mul_const(b, -1.25, dq)), 0.5)
    ext = ctx.add_const_ext(ctx.add_ext(ctx.mul_const_ext(ctx.lift(a), 0.37, dq),
                                        ctx.mul_const_ext(ctx.lift(b), -1.25, dq)), 0.5)
    got, want = ctx.mod_down_rescale(ext), ctx.rescale(plain)
    assert got.level == want.level and got.scale == want.scale
    assert np.array_equal(got.c, want.c)
    # the special limbs of a lift are zero, its Q limbs P c
    la = ctx.lift(a)
    assert not la.c[:, lv + 1:].any()
    q = ctx.q[1]
    assert int(la.c[0, 1, 3]) == int(a.c[0, 1, 3]) * ctx.p[0] * ctx.p[1] * ctx.p[2] % q


def test_lazy_rotation_sum_within_the_roundings():
    """sum_t w_t Rot(a, r_t) rescaled once through the extended basis stays
    within the roundings of the plain form: each plain rotation's ModDown
    error (<= K/2 + 1) is scaled by |C_t| / q_l, the lazy form rounds once."""
    ctx = Context(Params(4, [60, 50, 50, 50], [51, 51, 51], 1, 30.0, allow_insecure=True))
    steps = [1, 3]
    keys = ctx.keygen(16, rot_steps=steps)
    rng = np.random.default_rng(17)
    lv = 3
    a = Ciphertext(np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.moduli(lv)])
                             for _ in range(2)]), lv, 2.0 ** 30)
    dq = float(ctx.q[lv])
    ws = [0.75, -0.5, 0.25]
    plain = ctx.mul_const(a, ws[0], dq)
    ext = ctx.mul_const_ext(ctx.lift(a), ws[0], dq)
    for w, r in zip(ws[1:], steps):
        plain = ctx.add(plain, ctx.mul_const(ctx.rotate(a, r, keys), w, dq))
        ext = ctx.add_ext(ext, ctx.mul_const_ext(ctx.rotate_ext(a, r, keys), w, dq))
    got, want = ctx.mod_down_rescale(ext), ctx.rescale(plain)
    bound = sum(abs(w) for w in ws[1:]) * (ctx.K / 2 + 1) + ctx.K / 2 + 2
    for comp in range(2):
        for t in range(ctx.n):
            d = _crt_diff(got.c[comp, :, t], want.c[comp, :, t], ctx.q[:lv])
            assert abs(d) <= bound
    # one rotation alone: ModDown by P q_l of (u0 + P sigma(c0), u1)
    one = ctx.mod_down_rescale(ctx.rotate_ext(a, 3, keys))
    ref = ctx.rescale(ctx.rotate(a, 3, keys))
    for t in range(ctx.n):
        assert abs(_crt_diff(one.c[0, :, t], ref.c[0, :, t], ctx.q[:lv])) <= ctx.K / 2 + 2
    # step 0 is the lift
    assert np.array_equal(ctx.rotate_ext(a, 0, keys).c, ctx.lift(a).c)


# -------------------------------------------------------------- automorphism

def test_automorphism_is_ring_homomorphism():
    ctx = Context(Params(5, [50], [51], 1, 30.0, allow_insecure=True))
    q = ctx.q[0]
    rng = np.random.default_rng(5)
    a = rng.integers(0, q, ctx.n, dtype=np.uint64)
    b = rng.integers(0, q, ctx.n, dtype=np.uint64)
    g, h = 5, 2 * ctx.n - 1
    lhs = ctx.automorphism(ctx.automorphism(a, h, q), g, q)
    assert np.array_equal(lhs, ctx.automorphism(a, g * h % (2 * ctx.n), q))
    assert np.array_equal(ctx.automorphism(ctx.polymul(a, b, q), g, q),
                          ctx.polymul(ctx.automorphism(a, g, q), ctx.automorphism(b, g, q), q))
    # X -> X^g sends X to X^g
    x = np.zeros(ctx.n, np.uint64)
    x[1] = 1
    y = ctx.automorphism(x, g, q)
    assert int(y[g]) == 1 and int(y.sum()) == 1


# ------------------------------------------------- add, sub and level drop

def _lift(ct_c, k, t, moduli):
    return _crt([ct_c[k, i, t] for i in range(len(moduli))], moduli)


def test_add_sub_are_big_integer_add_sub():
    """Add and Sub act limb-wise; through the CRT they must be addition and
    subtraction of the lifted integers modulo Q (a missing third component
    counts as zero).  Residues include 0 and q - 1."""
    from oracle import Ciphertext
    ctx = Context(Params(3, [60, 50, 50, 40], [51], 4, 30.0, allow_insecure=True))
    rng = np.random.default_rng(11)
    lv = 3
    qs = ctx.q[:lv + 1]

    def rand_ct(ncomp):
        c = np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in qs])
                      for _ in range(ncomp)])
        for k in range(ncomp):
            for i, q in enumerate(qs):
                c[k, i, 0], c[k, i, 1] = 0, q - 1
        return Ciphertext(c, lv, 2.0 ** 30)

    a, b3 = rand_ct(2), rand_ct(3)
    s_ab, d_ab, d_ba = ctx.add(a, b3), ctx.sub(a, b3), ctx.sub(b3, a)
    assert s_ab.ncomp == d_ab.ncomp == d_ba.ncomp == 3
    for k in range(3):
        for t in range(ctx.n):
            X, Q = _lift(a.c, k, t, qs) if k < 2 else (0, None)
            Y, Q = _lift(b3.c, k, t, qs)
            assert _lift(s_ab.c, k, t, qs)[0] == (X + Y) % Q
            assert _lift(d_ab.c, k, t, qs)[0] == (X - Y) % Q
            assert _lift(d_ba.c, k, t, qs)[0] == (Y - X) % Q


def test_mod_drop_keeps_the_decrypted_message():
    """Dropping to level l' keeps the residues mod q_0..q_l': the decryption
    at l' is the same small integer polynomial (message plus noise) as at l,
    so its centred lift mod Q_l' equals the centred lift mod Q_l."""
    ctx = Context(Params(5, [60, 40, 40, 40, 40], [60], 5, 30.0, allow_insecure=True))
    keys = ctx.keygen(21)
    z = np.random.default_rng(12).uniform(-1, 1, ctx.slots)
    ct = ctx.encrypt(keys, ctx.encode(z, 4, ctx.scale), 21, 3)

    def centred(pt, level):
        out = []
        for t in range(ctx.n):
            X, Q = _crt([pt.m[i, t] for i in range(level + 1)], ctx.q[:level + 1])
            out.append(X - Q if X > Q // 2 else X)
        return out

    full = centred(ctx.decrypt(keys, ct), 4)
    assert max(abs(v) for v in full) > 2 ** 20          # a real message, not noise
    for lv in (3, 1, 0):
        d = ctx.mod_drop(ct, lv)
        assert d.level == lv and d.scale == ct.scale and d.c.shape == (2, lv + 1, ctx.n)
        assert centred(ctx.decrypt(keys, d), lv) == full
    with pytest.raises(ValueError):
        ctx.mod_drop(ctx.mod_drop(ct, 1), 2)


def test_stream_key_is_the_256_bit_seed():
    """All 32 key bytes come from the seed: the key words are the seed's
    little-endian 32-bit words, so seeds that differ only above bit 64 give
    different streams, and a seed below 2^64 keys with 24 zero bytes."""
    ctx = Context(PRESETS["C1"])
    pur, obj = 3, 77
    nonce = np.array([pur, obj, 0], dtype=np.uint32)
    for seed in (0x1122334455667788, (0xdeadbeef << 200) | (7 << 64) | 5, (1 << 256) - 1):
        words = ctx.stream_words(seed, pur, obj, 0, 8)
        key = np.array([(seed >> (32 * i)) & 0xffffffff for i in range(8)], dtype=np.uint32)
        out = np.zeros(16, dtype=np.uint32)
        lib.orc_chacha20_block(ptr(key), 0, ptr(nonce), ptr(out))
        assert [int(w) for w in words] == [int(out[2 * j]) | (int(out[2 * j + 1]) << 32) for j in range(8)]
    a = ctx.stream_words(5, pur, obj, 0, 8)
    b = ctx.stream_words(5 | (1 << 192), pur, obj, 0, 8)
    assert not np.array_equal(a, b)
    with pytest.raises(ValueError):
        ctx.stream_words(1 << 256, pur, obj, 0, 8)
