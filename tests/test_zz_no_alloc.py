"""vr_rotate_noalloc: the rotation with every key-switching intermediate in
the library's fixed device array, on caller-owned device limbs.  Two calls in
a row (the second on a smaller input, at a lower level) must give the limbs
of vr_rotate on the same ciphertexts; a level whose tables are not built yet
is refused without allocating."""
import numpy as np
import pytest

from oracle import PRESETS
from tests.gpu_helpers import gpu_ctx

pytestmark = pytest.mark.gpu


def _dev(torch, limbs):
    return torch.from_numpy(np.ascontiguousarray(limbs).view(np.int64)).cuda()


def _rotate_noalloc(g, keys, ct, step, torch):
    """Coefficient limbs of ct -> device, to the evaluation domain (vr_ntt),
    vr_rotate_noalloc into a second device buffer, back to coefficients."""
    nc, lv, _ = ct.meta
    mods = list(range(lv + 1)) * 2
    src = _dev(torch, ct.export())
    dst = torch.full_like(src, -1)
    torch.cuda.synchronize()
    g.ntt_device(src.data_ptr(), len(mods), mods)
    torch.cuda.synchronize()
    g.rotate_noalloc(keys, src.data_ptr(), lv, step, dst.data_ptr(), stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    g.ntt_device(dst.data_ptr(), len(mods), mods, inverse=True)
    torch.cuda.synchronize()
    return dst.cpu().numpy().view(np.uint64).reshape(2, lv + 1, g.n)


@pytest.mark.parametrize("name,log_n,levels", [("C1", 10, (3, 1)), ("C3", 16, (24, 3))])
def test_rotate_noalloc_matches_rotate(name, log_n, levels):
    import torch
    from paper_2512_18646_amd import vr
    p = PRESETS[name]
    if log_n != p.log_n:
        from oracle import Params
        p = Params(log_n, p.q_bits, p.p_bits, p.dnum, p.log2_scale, allow_insecure=True)
    g = gpu_ctx(p)
    keys = g.keygen(3300, rot_steps=[1, 5])
    z = np.random.default_rng(33).uniform(-1, 1, g.slots)
    for call, (lv, step) in enumerate(zip(levels, (1, 5))):
        ct = g.encrypt(keys, g.encode(z, lv), 3300, call)
        ref = g.rotate(keys, ct, step)      # also builds this level's plans and tables
        got = _rotate_noalloc(g, keys, ct, step, torch)
        assert np.array_equal(got, ref.export()), "%s call %d (level %d, step %d)" % (name, call, lv, step)
    # step 0 is a copy
    ct = g.encrypt(keys, g.encode(z, levels[1]), 3300, 9)
    assert np.array_equal(_rotate_noalloc(g, keys, ct, 0, torch), ct.export())


def test_rotate_noalloc_refuses_unprepared_level_and_missing_key():
    import torch
    from paper_2512_18646_amd import vr
    g = gpu_ctx(PRESETS["C3"])
    keys = g.keygen(3301, rot_steps=[1])
    z = np.random.default_rng(34).uniform(-1, 1, g.slots)
    ct = g.encrypt(keys, g.encode(z, 11), 3301, 0)
    with pytest.raises(vr.VRError) as e:
        _rotate_noalloc(g, keys, ct, 1, torch)      # no rotation at level 11 yet: tables missing
    assert e.value.code == vr.VR_EINVAL
    with pytest.raises(vr.VRError) as e:
        _rotate_noalloc(g, keys, ct, 3, torch)      # no key for step 3
    assert e.value.code == vr.VR_ENOKEY
    ref = g.rotate(keys, ct, 1)
    assert np.array_equal(_rotate_noalloc(g, keys, ct, 1, torch), ref.export())
