"""Shared helpers for the GPU parity tests: build one oracle context and one
GPU context per parameter set, with keys from the same seed."""
import functools

import numpy as np

from oracle import Context as OracleContext, Params, PRESETS

SEED_KEYS = 1000


def gpu_ctx(params):
    from paper_2512_18646_amd import vr
    return vr.Context.from_params(params)


@functools.lru_cache(maxsize=None)
def pair(name, rot_steps=(), log_n=None):
    """(oracle ctx, oracle keys, gpu ctx, gpu keys) for a preset (optionally at a smaller N)."""
    p = PRESETS[name]
    if log_n is not None:
        p = Params(log_n, p.q_bits, p.p_bits, p.dnum, p.log2_scale, allow_insecure=True)
    o = OracleContext(p)
    ok = o.keygen(SEED_KEYS, rot_steps=list(rot_steps))
    g = gpu_ctx(p)
    gk = g.keygen(SEED_KEYS, rot_steps=list(rot_steps))
    return o, ok, g, gk


def to_gpu(g, ct):
    return g.ct_import(ct.c, ct.level, ct.scale)


def assert_same(gct, oct_, what=""):
    got = gct.export()
    nc, lv, sc = gct.meta
    assert (nc, lv) == (oct_.ncomp, oct_.level), what
    assert sc == oct_.scale, what
    if not np.array_equal(got, oct_.c):
        bad = np.argwhere(got != oct_.c)
        where = sorted({(int(k), int(l)) for k, l, _ in bad})
        raise AssertionError("%s: %d limb words differ, first at %s; (component, limb) pairs %s"
                             % (what, len(bad), bad[0], where[:12]))
