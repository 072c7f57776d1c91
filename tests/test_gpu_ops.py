"""GPU parity of every RNS-CKKS primitive against the oracle, limb for limb.

Inputs are oracle ciphertexts imported through vr_ct_import (coefficient
domain), outputs are exported through vr_ct_export; both sides hold keys from
the same seed.  Bar: bit-exact on every limb (integer arithmetic)."""
import numpy as np
import pytest

from oracle import Params, PRESETS, Context as OracleContext
from tests.gpu_helpers import pair, to_gpu, assert_same, gpu_ctx

pytestmark = pytest.mark.gpu


def test_moduli_match_oracle():
    for name in ("C1", "C2", "C3"):
        o = OracleContext(PRESETS[name])
        g = gpu_ctx(PRESETS[name])
        assert g.q == o.q and g.p == o.p, name
        assert g.secure


@pytest.mark.parametrize("log_n", [6, 13, 14, 15, 16])
def test_ntt_matches_oracle(log_n):
    p = Params(log_n, [60, 50, 40], [51], 1, 30.0, allow_insecure=True)
    check_ntt(OracleContext(p), gpu_ctx(p), log_n)


@pytest.mark.parametrize("log_n", [13, 14, 15, 16])
def test_ntt_every_candidate_plan(log_n):
    """Each pass plan the autotuner may pick gives the exact transform (both
    the FP64 path, 40/50/51-bit moduli, and the integer path, 60-bit)."""
    from paper_2512_18646_amd import vr
    p = Params(log_n, [60, 50, 40], [51], 1, 30.0, allow_insecure=True)
    o, g = OracleContext(p), gpu_ctx(p)
    tried = 0
    while True:
        g.set_tuning("ntt", "cand:%d" % tried)
        try:
            check_ntt(o, g, log_n, reps=1)
        except vr.VRError as e:
            assert e.code == vr.VR_EINVAL and tried >= 1
            break
        tried += 1
    g.set_tuning("ntt", "auto")
    check_ntt(o, g, log_n, reps=1)
    assert "ntt N=2^%d forward" % log_n in g.tuning_report()


@pytest.mark.parametrize("log_n", [13, 14, 16])
def test_ntt_every_plan_reduction_bands(log_n):
    """FP64 moduli in each band of the reduction schedule (45 and 49 bits:
    forward every four stages; 45: inverse every four, 49: every two) under
    every plan, with rows of extreme balanced inputs (all (q-1)/2, all
    (q+1)/2, alternating)."""
    from paper_2512_18646_amd import vr
    p = Params(log_n, [49, 45, 40], [45], 1, 30.0, allow_insecure=True)
    o, g = OracleContext(p), gpu_ctx(p)
    tried = 0
    while True:
        g.set_tuning("ntt", "cand:%d" % tried)
        try:
            check_ntt(o, g, log_n, reps=2)
        except vr.VRError as e:
            assert e.code == vr.VR_EINVAL and tried >= 1
            break
        tried += 1


@pytest.mark.parametrize("log_n", [13, 14])
def test_ntt_every_plan_many_limbs(log_n):
    """600 limbs in one launch (more than one per CU, so persistent plans walk
    several limbs per workgroup): sampled limbs, including ones a workgroup
    reaches on a later iteration, against the oracle, and the exact round
    trip for all, under every plan."""
    import torch
    from paper_2512_18646_amd import vr
    p = Params(log_n, [60, 50, 40], [51], 1, 30.0, allow_insecure=True)
    o, g = OracleContext(p), gpu_ctx(p)
    mods = o.q + o.p
    count = 600
    rng = np.random.default_rng(100 + log_n)
    host = np.stack([rng.integers(0, mods[i % 4], o.n, dtype=np.uint64) for i in range(count)])
    mi = [i % 4 for i in range(count)]
    sample = [0, 1, 255, 256, 257, 300, 511, 512, 513, 599]
    tried = 0
    while True:
        g.set_tuning("ntt", "cand:%d" % tried)
        dev = torch.from_numpy(host.view(np.int64).copy()).cuda()
        try:
            g.ntt_device(dev.data_ptr(), count, mi)
        except vr.VRError as e:
            assert e.code == vr.VR_EINVAL and tried >= 1
            break
        torch.cuda.synchronize()
        fwd = dev.cpu().numpy().view(np.uint64)
        for r in sample:
            assert np.array_equal(fwd[r], o.ntt(host[r], mods[mi[r]])), (tried, r)
        g.ntt_device(dev.data_ptr(), count, mi, inverse=True)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy().view(np.uint64), host), tried
        tried += 1


def check_ntt(o, g, log_n, reps=3):
    import torch
    mods = o.q + o.p
    rng = np.random.default_rng(log_n)
    host = np.stack([rng.integers(0, mods[i % 4], o.n, dtype=np.uint64) for i in range(4 * reps)])
    host[0, :8] = [0, 1, mods[0] - 1, 2, 3, mods[0] - 2, 0, 1]
    # largest balanced magnitudes: (q-1)/2 and (q+1)/2 = -(q-1)/2
    half = [(int(q) - 1) // 2 for q in mods[:4]]
    host[1] = half[1]
    host[2] = half[2] + 1
    host[3, 0::2] = half[3]
    host[3, 1::2] = half[3] + 1
    mi = [i % 4 for i in range(4 * reps)]
    dev = torch.from_numpy(host.view(np.int64).copy()).cuda()
    g.ntt_device(dev.data_ptr(), 4 * reps, mi)
    torch.cuda.synchronize()
    fwd = dev.cpu().numpy().view(np.uint64)
    for r in range(4 * reps):
        assert np.array_equal(fwd[r], o.ntt(host[r], mods[mi[r]])), r
    g.ntt_device(dev.data_ptr(), 4 * reps, mi, inverse=True)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy().view(np.uint64), host)


def test_secret_and_public_key_match():
    o, ok, g, gk = pair("C1")
    assert np.array_equal(gk.secret_coeffs().astype(np.int64), ok.s)
    # the public key shows through an encryption of an imported plaintext
    pt = o.encode(np.linspace(-1, 1, 100), 3, o.scale)
    gpt = g.pt_import(pt.m, 3, pt.scale)
    assert_same(g.encrypt(gk, gpt, 77, 5), o.encrypt(ok, pt, 77, 5), "encrypt")


@pytest.mark.parametrize("name,level", [("C1", 3), ("C1", 0), ("C2", 7)])
def test_encrypt_decrypt_match(name, level):
    o, ok, g, gk = pair(name)
    z = np.random.default_rng(1).uniform(-1, 1, o.slots)
    pt = o.encode(z, level, o.scale)
    ct = o.encrypt(ok, pt, 3, 11)
    gct = g.encrypt(gk, g.pt_import(pt.m, level, pt.scale), 3, 11)
    assert_same(gct, ct, "encrypt")
    gpt = g.decrypt(gk, gct)
    assert np.array_equal(gpt.export(), o.decrypt(ok, ct).m)
    assert np.max(np.abs(g.decode(gpt) - z)) < 2.0 ** -20


def test_encode_within_one_of_oracle():
    for name in ("C1", "C3"):
        o, ok, g, gk = pair(name)
        z = np.random.default_rng(2).uniform(-1, 1, o.slots)
        gpt = g.encode(z, 1)
        mo = o.encode(z, 1, o.scale).m
        mg = gpt.export()
        q = np.array(o.q[:2], dtype=np.uint64)[:, None]
        d = (mg.astype(np.int64) - mo.astype(np.int64))
        d = np.where(d > (q // 2).astype(np.int64), d - q.astype(np.int64), d)
        d = np.where(d < -(q // 2).astype(np.int64), d + q.astype(np.int64), d)
        assert np.abs(d).max() <= 1, name
        assert np.max(np.abs(g.decode(gpt) - z)) < 2.0 ** -30


@pytest.fixture(scope="module")
def c1():
    return pair("C1", rot_steps=(1, 2, 3, 5, -1, 4096 - 3))


def _fresh(o, ok, seed, level=3, n=None):
    z = np.random.default_rng(seed).uniform(-1, 1, n or o.slots)
    return o.encrypt(ok, o.encode(z, level, o.scale), 5, seed)


def test_add_sub_match(c1):
    o, ok, g, gk = c1
    a, b = _fresh(o, ok, 1), _fresh(o, ok, 2)
    assert_same(g.add(to_gpu(g, a), to_gpu(g, b)), o.add(a, b), "add")
    assert_same(g.sub(to_gpu(g, a), to_gpu(g, b)), o.sub(a, b), "sub")


@pytest.mark.parametrize("c", [0.37, -0.9, 0.0, 1e-3])
def test_mul_const_add_const_match(c1, c):
    o, ok, g, gk = c1
    a = _fresh(o, ok, 3)
    dq = float(o.q[3])
    assert_same(g.mul_const(to_gpu(g, a), c, dq), o.mul_const(a, c, dq), "mul_const")
    assert_same(g.add_const(to_gpu(g, a), c), o.add_const(a, c), "add_const")
    # constants beyond 2^63 (c * scale at the product scale)
    big = o.mul_const(a, 0.5, dq)
    assert_same(g.add_const(to_gpu(g, big), -0.7), o.add_const(big, -0.7), "add_const big")


def test_mul_plain_tensor_relin_match(c1):
    o, ok, g, gk = c1
    a, b = _fresh(o, ok, 4), _fresh(o, ok, 5)
    pt = o.encode(np.random.default_rng(9).uniform(-1, 1, o.slots), 3, float(o.q[3]))
    gpt = g.pt_import(pt.m, 3, pt.scale)
    assert_same(g.mul_plain(to_gpu(g, a), gpt), o.mul_plain(a, pt), "mul_plain")
    t = o.tensor(a, b)
    gt = g.tensor(to_gpu(g, a), to_gpu(g, b))
    assert_same(gt, t, "tensor")
    assert_same(g.relinearize(gk, gt), o.relinearize(t, ok), "relin")
    assert_same(g.mul(gk, to_gpu(g, a), to_gpu(g, b)), o.mul(a, b, ok), "mul")


@pytest.mark.parametrize("level", [3, 2, 1])
def test_rescale_and_mod_drop_match(c1, level):
    o, ok, g, gk = c1
    a = _fresh(o, ok, 6, level=level)
    assert_same(g.rescale(to_gpu(g, a)), o.rescale(a), "rescale")
    t = o.tensor(a, a)
    assert_same(g.rescale(to_gpu(g, t)), o.rescale(t), "rescale 3 comps")
    assert_same(g.mod_drop(to_gpu(g, a), 0), o.mod_drop(a, 0), "mod_drop")


@pytest.mark.parametrize("level", [3, 0])
def test_rotate_match(c1, level):
    o, ok, g, gk = c1
    a = _fresh(o, ok, 7, level=level)
    ga = to_gpu(g, a)
    for step in (1, 5, -1, 4096 - 3, 0):
        assert_same(g.rotate(gk, ga, step), o.rotate(a, step, ok), "rotate %d" % step)
    many = g.rotate_many(gk, ga, [1, 2, 3, 0])
    for st, m in zip([1, 2, 3, 0], many):
        assert_same(m, o.rotate(a, st, ok), "hoisted %d" % st)


@pytest.mark.parametrize("name", ["C1", "C2", "C3"])
def test_switching_keys_match(name):
    """Relinearisation and rotation keys, limb for limb (coefficient domain)."""
    o, ok, g, gk = pair(name, rot_steps=(1, 3))
    keys = [(0, ok.rlk)] + [(gal, k) for gal, k in sorted(ok.rot.items())]
    for gal, key in keys:
        got = gk.switching_key(gal)
        for j in range(o.dnum):
            for comp, want in ((0, key.b[j]), (1, key.a[j])):
                if not np.array_equal(got[j, comp], want):
                    limbs = sorted({int(l) for l, _ in np.argwhere(got[j, comp] != want)})
                    raise AssertionError("%s key g=%d digit %d comp %d differs on limbs %s"
                                         % (name, gal, j, comp, limbs[:10]))


def test_rotation_decrypts_on_gpu():
    o, ok, g, gk = pair("C2", rot_steps=(1, 3))
    z = np.random.default_rng(4).uniform(-1, 1, o.slots)
    ct = g.encrypt(gk, g.encode(z, 7), 1, 2)
    for st in (1, 3):
        d = g.decode(g.decrypt(gk, g.rotate(gk, ct, st)))
        assert np.max(np.abs(d - np.roll(z, -st))) < 2.0 ** -20, st


@pytest.mark.parametrize("mode", ["alu", "mfma", "fp64", "split", "auto"])
@pytest.mark.parametrize("name,level", [("C2", 2), ("C2", 7), ("C3", 3), ("C3", 24), ("C3", 20)])
def test_keyswitch_match_other_chains(name, level, mode):
    """Rotation and relinearisation with 60-bit q_0 / special primes (C2) and
    9-prime digits with a short last digit (C3 at levels 3 and 20; digit 0
    holds the 60-bit q_0, split in halves by the FP64 kernel, and q_0 is a
    target of the other digits and of ModDown, taking the integer form), with
    the base conversions on the vector ALU, in FP64, on the INT8 matrix cores,
    split (FP64 for the targets after q_0, the ALU kernel for q_0) and as the
    autotuner picks (its first call runs every kernel); one-limb digits (C2)
    convert inside the NTT's first load whatever the mode."""
    o, ok, g, gk = pair(name, rot_steps=(1, 3))
    z = np.random.default_rng(level).uniform(-1, 1, o.slots)
    a = o.encrypt(ok, o.encode(z, level, o.scale), 9, level)
    ga = to_gpu(g, a)
    g.set_tuning("base_convert", mode)
    try:
        assert_same(g.rotate(gk, ga, 1), o.rotate(a, 1, ok), "%s rotate l=%d %s" % (name, level, mode))
        many = g.rotate_many(gk, ga, [3, 1])
        assert_same(many[0], o.rotate(a, 3, ok), "%s hoisted 3 %s" % (name, mode))
        t = o.tensor(a, a)
        assert_same(g.relinearize(gk, to_gpu(g, t)), o.relinearize(t, ok), "%s relin %s" % (name, mode))
        assert_same(g.relin_rescale(gk, to_gpu(g, t)), o.relin_rescale(t, ok),
                    "%s relin-rescale l=%d %s" % (name, level, mode))
        if mode == "auto" and name == "C3":   # one-limb digits (C2) convert inside the NTT
            rep = g.tuning_report()
            assert "modup l%d d0" % level in rep and "untimed" not in rep.split("modup l%d d0" % level)[1].split("\n")[0]
    finally:
        g.set_tuning("base_convert", "auto")


@pytest.mark.parametrize("plan", ["auto", "cand:0"])
@pytest.mark.parametrize("name,level", [("C1", 3), ("C2", 7), ("C2", 1)])
def test_finish_in_transform_and_separate_match(name, level, plan):
    """ModDown's (U - Y) P^-1 (+ the Galois-mapped c_0 of a rotation) and
    rescale's (c - r) q_l^-1 run in the forward transform's last round under
    the whole-limb plan the autotuner keeps at N = 2^13 and 2^14, and in their
    own kernels under a plan without a whole-limb pass (cand:0): both against
    the oracle."""
    o, ok, g, gk = pair(name, rot_steps=(1, 3))
    z = np.random.default_rng(40 + level).uniform(-1, 1, o.slots)
    a = o.encrypt(ok, o.encode(z, level, o.scale), 11, level)
    ga = to_gpu(g, a)
    g.set_tuning("ntt", plan)
    try:
        assert_same(g.rotate(gk, ga, 1), o.rotate(a, 1, ok), "%s rotate %s" % (name, plan))
        many = g.rotate_many(gk, ga, [3, 1])
        assert_same(many[0], o.rotate(a, 3, ok), "%s hoisted 3 %s" % (name, plan))
        t = o.tensor(a, a)
        assert_same(g.relinearize(gk, to_gpu(g, t)), o.relinearize(t, ok), "%s relin %s" % (name, plan))
        assert_same(g.relin_rescale(gk, to_gpu(g, t)), o.relin_rescale(t, ok), "%s relin-rescale %s" % (name, plan))
        assert_same(g.rescale(ga), o.rescale(a), "%s rescale %s" % (name, plan))
        assert_same(g.rescale(to_gpu(g, t)), o.rescale(t), "%s rescale 3 comps %s" % (name, plan))
    finally:
        g.set_tuning("ntt", "auto")


def test_finish_every_plan_n16():
    """At N = 2^16 (C3, level 3: 50-bit Q limbs and 51-bit special primes)
    under every candidate plan: the compile-time two-pass plans run ModDown's
    and rescale's finish in the forward transform's last pass, the others in
    their own kernels; rotation, hoisted rotation, relinearisation and
    rescale against the oracle."""
    from paper_2512_18646_amd import vr
    o, ok, g, gk = pair("C3", rot_steps=(1, 3))
    z = np.random.default_rng(44).uniform(-1, 1, o.slots)
    a = o.encrypt(ok, o.encode(z, 3, o.scale), 12, 3)
    t = o.tensor(a, a)
    want = [o.rotate(a, 1, ok), o.rotate(a, 3, ok), o.relinearize(t, ok), o.rescale(a), o.rescale(t),
            o.relin_rescale(t, ok)]
    ga, gt = to_gpu(g, a), to_gpu(g, t)
    tried = 0
    try:
        while True:
            g.set_tuning("ntt", "cand:%d" % tried)
            try:
                got = g.rotate(gk, ga, 1)
            except vr.VRError as e:
                assert e.code == vr.VR_EINVAL and tried >= 1
                break
            assert_same(got, want[0], "rotate cand:%d" % tried)
            assert_same(g.rotate_many(gk, ga, [3, 1])[0], want[1], "hoisted 3 cand:%d" % tried)
            assert_same(g.relinearize(gk, gt), want[2], "relin cand:%d" % tried)
            assert_same(g.rescale(ga), want[3], "rescale cand:%d" % tried)
            assert_same(g.rescale(gt), want[4], "rescale 3 comps cand:%d" % tried)
            assert_same(g.relin_rescale(gk, gt), want[5], "relin-rescale cand:%d" % tried)
            tried += 1
    finally:
        g.set_tuning("ntt", "auto")
    assert tried >= 4


def test_relin_rescale_product_and_errors(c1):
    """vr_mul_rescale is the tensor then the fused ModDown by P q_l (against the
    oracle word for word, and decoded against FP64); a level-0 or 2-component
    input is refused."""
    from paper_2512_18646_amd import vr
    o, ok, g, gk = c1
    rng = np.random.default_rng(46)
    x, y = rng.uniform(-1, 1, o.slots), rng.uniform(-1, 1, o.slots)
    a = o.encrypt(ok, o.encode(x, o.L, o.scale), 13, 0)
    b = o.encrypt(ok, o.encode(y, o.L, o.scale), 13, 1)
    got = g.mul_rescale(gk, to_gpu(g, a), to_gpu(g, b))
    assert_same(got, o.relin_rescale(o.tensor(a, b), ok), "mul-rescale")
    assert np.max(np.abs(g.decode(g.decrypt(gk, got)) - x * y)) < 2.0 ** -20
    with pytest.raises(vr.VRError) as e:
        g.relin_rescale(gk, to_gpu(g, a))
    assert e.value.code == vr.VR_EINVAL
    t0 = o.tensor(o.mod_drop(a, 0), o.mod_drop(b, 0))
    with pytest.raises(vr.VRError) as e:
        g.relin_rescale(gk, to_gpu(g, t0))
    assert e.value.code == vr.VR_ELEVEL


def test_error_paths(c1):
    from paper_2512_18646_amd import vr
    o, ok, g, gk = c1
    a = to_gpu(g, _fresh(o, ok, 8, level=3))
    b = to_gpu(g, _fresh(o, ok, 9, level=2))
    with pytest.raises(vr.VRError) as e:
        g.add(a, b)
    assert e.value.code == vr.VR_ELEVEL
    c = g.mul_const(a, 1.0, 2.0)
    with pytest.raises(vr.VRError) as e:
        g.add(a, c)
    assert e.value.code == vr.VR_ESCALE
    with pytest.raises(vr.VRError) as e:
        g.rotate(gk, a, 7)
    assert e.value.code == vr.VR_ENOKEY
    z = to_gpu(g, _fresh(o, ok, 10, level=0))
    with pytest.raises(vr.VRError) as e:
        g.rescale(z)
    assert e.value.code == vr.VR_ELEVEL
