"""Seeded synthetic inputs shaped like the paper's workloads.

Both the oracle tests and the GPU path draw their plaintext inputs (matrices,
images, weights) from here, so that the two sides see the same numbers.  This
module holds none of the method's arithmetic: only numpy PCG64 draws with the
shapes and value ranges of the workloads (pixels in [0, 1] like the paper's
normalised 28x28 grayscale digits, entries uniform in [-1, 1] for matrices,
normal weights).  The paper's own dataset and trained weights are not used.
"""
from dataclasses import dataclass

import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def matmul_operands(seed, m, n, p):
    """A (m x n), B (n x p), entries uniform in [-1, 1]."""
    g = rng(seed)
    return g.uniform(-1.0, 1.0, (m, n)), g.uniform(-1.0, 1.0, (n, p))


def images(seed, batch, channels, h, w, quantise=False):
    """Pixels uniform in [0, 1]; optionally rounded to k/255 like 8-bit pixels."""
    x = rng(seed).uniform(0.0, 1.0, (batch, channels, h, w))
    return np.round(x * 255.0) / 255.0 if quantise else x


def conv_weights(seed, c_out, c_in, k, std):
    """Kernel K[c_out][c_in][k][k] and bias[c_out], both N(0, std^2)."""
    g = rng(seed)
    return g.normal(0.0, std, (c_out, c_in, k, k)), g.normal(0.0, std, c_out)


def fc_weights(seed, n_out, c, h, w, std):
    """W[n_out][c][h][w] and bias[n_out], both N(0, std^2)."""
    g = rng(seed)
    return g.normal(0.0, std, (n_out, c, h, w)), g.normal(0.0, std, n_out)


@dataclass
class ConvWorkload:
    name: str
    batch: int
    channels: int
    h: int
    w: int
    c_out: int
    k: int
    stride: int
    pad: int
    std: float
    seed: int
    fc_out: int = 0
    fc_std: float = 0.0

    def draw(self, batch=None):
        b = self.batch if batch is None else batch
        X = images(self.seed, b, self.channels, self.h, self.w)
        K, bias = conv_weights(self.seed + 100, self.c_out, self.channels, self.k, self.std)
        return X, K, bias

    def draw_fc(self):
        ho = (self.h + 2 * self.pad - self.k) // self.stride + 1
        wo = (self.w + 2 * self.pad - self.k) // self.stride + 1
        return fc_weights(self.seed + 200, self.fc_out, self.c_out, ho, wo, self.fc_std)


# 28x28 single-channel images, one full ciphertext set (256 images in 32-slot
# blocks at N=2^14), 5 filters 4x4 stride 2 no padding, weights N(0, 0.1^2).
CONV_28 = ConvWorkload("conv28", 256, 1, 28, 28, 5, 4, 2, 0, 0.1, 2)

# 3x128x128 images, 128 per set (256-slot blocks at N=2^16), 8 filters 3x3
# stride 2 pad 1, FC 8*64*64 -> 10, weights N(0, 0.05^2).
CNN_128 = ConvWorkload("cnn128", 128, 3, 128, 128, 8, 3, 2, 1, 0.05, 3, fc_out=10, fc_std=0.05)

# 16x16 by 16x16 matrices, entries uniform in [-1, 1].
MATMUL_16 = (1, 16, 16, 16)   # seed, m, n, p


def uneven_requests(seed, count, dim_range=(8, 32), sides=(32, 64)):
    """A mixed batch: even indices are products with m, n, p uniform integers
    in dim_range, odd indices are one-channel convolutions (3x3, 8 filters,
    stride 2, pad 1, then x^2) on images of a side drawn from `sides`, with a
    full ciphertext set of images; weights N(0, 0.05^2)."""
    g = rng(seed)
    reqs = []
    for i in range(count):
        if i % 2 == 0:
            m, n, p = (int(v) for v in g.integers(dim_range[0], dim_range[1] + 1, 3))
            reqs.append(("matmul", (m, n, p), int(g.integers(1 << 30))))
        else:
            side = int(g.choice(sides))
            reqs.append(("conv", side, int(g.integers(1 << 30))))
    return reqs
