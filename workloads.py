"""Seeded synthetic workloads shared by the tests and the benchmark.

This module only draws random numbers and shapes and converts inputs to their
stored dtype; it holds none of the GEMM or scheduling arithmetic.  Both the
oracle side and the device side of a test receive the arrays made here.

Workloads (stand-ins for the paper's evaluation corpus, which is a random
log-sample of GEMM shapes with m, n, k in [128, 8192] and is not available as
a list):

* ``plain_f32``: M=384 N=384 K=1024 FP32, A and B iid uniform[-1, 1] from seed
  0 (128x128 tiles give 9 tiles: the quantisation case), plus an
  integer-valued variant with entries in {-2..2}.
* ``bf16_sweep``: 1000 shapes, M, N, K log-uniform in [128, 8192]; the first
  half rounded to multiples of 128, the second half given random +1..127
  offsets; A, B iid N(0, 1) in bf16.
* ``ladder``: M=N=K in {1024, 4096, 8192} and M=128 N=K=8192, N(0, 1) inputs.
* ``grouped``: 64 problems with N=4096 K=2048 and M drawn from a Zipf(1.2)
  law over the integers [16, 4096].
* ``autograd``: bf16 2048x2048x8192 and 256x4096x4096.
"""
from __future__ import annotations

import math

import numpy as np

LADDER_SHAPES = [(1024, 1024, 1024), (4096, 4096, 4096), (8192, 8192, 8192), (128, 8192, 8192)]
AUTOGRAD_SHAPES = [(2048, 2048, 8192), (256, 4096, 4096)]


def rng(seed: int = 0) -> np.random.Generator:
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- shapes

def sweep_shapes(n: int = 1000, seed: int = 0, lo: int = 128, hi: int = 8192):
    """Log-uniform GEMM shapes: first half multiples of 128, second half with
    random +1..127 offsets above a multiple of 128."""
    g = rng(seed)
    d = np.exp(g.uniform(math.log(lo), math.log(hi), size=(n, 3)))
    half = n // 2
    out = []
    for i in range(n):
        if i < half:
            v = np.maximum(np.rint(d[i] / 128.0), 1) * 128
        else:
            v = np.floor(d[i] / 128.0) * 128 + g.integers(1, 128, size=3)
        out.append(tuple(int(x) for x in v))
    return out


def zipf_ms(G: int = 64, lo: int = 16, hi: int = 4096, s: float = 1.2, seed: int = 0):
    """G integers from P(m) proportional to m**-s on [lo, hi], by inverse CDF."""
    m = np.arange(lo, hi + 1, dtype=np.float64)
    w = m ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng(seed).random(G)
    idx = np.searchsorted(cdf, u, side="left")
    return [int(m[i]) for i in idx]


# ---------------------------------------------------------------- matrices

def uniform_f32(g: np.random.Generator, shape, lo=-1.0, hi=1.0) -> np.ndarray:
    return g.uniform(lo, hi, size=shape).astype(np.float32)


def normal_f32(g: np.random.Generator, shape) -> np.ndarray:
    return g.standard_normal(size=shape, dtype=np.float32)


def integer_f32(g: np.random.Generator, shape, lo=-2, hi=2) -> np.ndarray:
    return g.integers(lo, hi + 1, size=shape).astype(np.float32)


def to_stored(x_f32: np.ndarray, dtype: str) -> np.ndarray:
    """Stored representation of float32 data: float32 values for "f32", the
    uint16 bit patterns of the round-to-nearest-even conversion for "bf16" and
    "f16" (torch's CPU conversion)."""
    import torch
    x = np.ascontiguousarray(x_f32, dtype=np.float32)
    if dtype == "f32":
        return x
    t = torch.from_numpy(x)
    if dtype == "bf16":
        return t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16).copy()
    if dtype == "f16":
        return t.to(torch.float16).view(torch.int16).numpy().view(np.uint16).copy()
    raise ValueError(dtype)


def plain_f32(seed: int = 0, integer: bool = False, M: int = 384, N: int = 384, K: int = 1024):
    """The FP32 quantisation-case GEMM inputs (A then B from one generator)."""
    g = rng(seed)
    if integer:
        return integer_f32(g, (M, K)), integer_f32(g, (K, N))
    return uniform_f32(g, (M, K)), uniform_f32(g, (K, N))


def normal_pair(M: int, N: int, K: int, seed: int = 0):
    g = rng(seed)
    return normal_f32(g, (M, K)), normal_f32(g, (K, N))
