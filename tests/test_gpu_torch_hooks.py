"""The boundary's PyTorch plumbing: device memory from PyTorch's caching
allocator through vr_context_set_allocator, and PyTorch streams passed to the
evaluation calls; limbs identical to the built-in allocator on the context's
stream, and the memory back in PyTorch's pool once the handles are gone."""
import gc

import numpy as np
import pytest

from oracle import layers as Ly
from tests.gpu_helpers import pair, to_gpu

pytestmark = pytest.mark.gpu


def _conv_square(g, gk, gcts, K, bias, stream=None):
    y = g.conv2d(gk, gcts, 2, 10, 9, 1, K, bias, 2, stream=stream)
    return g.square(gk, y, stream=stream)


def test_torch_allocator_and_streams_give_the_same_limbs():
    import torch
    o, ok, g, gk = pair("C1", rot_steps=(1, 2), log_n=10)
    rng = np.random.default_rng(60)
    X = rng.uniform(0, 1, (4, 2, 10, 9))
    K = rng.normal(0, 0.1, (3, 2, 3, 3))
    bias = rng.normal(0, 0.1, 3)
    cts = Ly.encrypt_image_columns(o, ok, X, 1, 3, 3, 0)
    gcts = [to_gpu(g, c) for c in cts]
    ref = [c.export() for c in _conv_square(g, gk, gcts, K, bias)]
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    g.use_torch_allocator()
    try:
        # on a PyTorch stream, memory from PyTorch's pool
        s = torch.cuda.Stream()
        out = _conv_square(g, gk, gcts, K, bias, stream=s)
        s.synchronize()
        assert torch.cuda.memory_allocated() > base
        assert all(np.array_equal(a.export(), b) for a, b in zip(out, ref))
        r1 = g.rotate(gk, gcts[0], 1, stream=s)
        s.synchronize()
        want = g.rotate(gk, gcts[0], 1)
        assert np.array_equal(r1.export(), want.export())
        del out, r1, want
        gc.collect()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        g.use_builtin_allocator()
    # the built-in allocator again, on the context's stream
    again = _conv_square(g, gk, gcts, K, bias)
    assert all(np.array_equal(a.export(), b) for a, b in zip(again, ref))
