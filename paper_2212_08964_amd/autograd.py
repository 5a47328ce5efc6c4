"""Differentiable Stream-K GEMM: C = A @ B with a hand-written backward.

Both gradient products go through the same library and decomposition:
  dA = dC @ B^T   (B^T is a column-major view of B: both operands K-contiguous)
  dB = A^T @ dC   (A^T is a column-major view of A, dC row-major: both operands
                   contiguous along M and N, read with the LDS transpose path)
No operand is copied or transposed in memory.
"""
from __future__ import annotations

import torch

from . import skgemm


class SkGemmFunction(torch.autograd.Function):
    """C = A @ B on the GPU through skgemm (forward and backward)."""

    @staticmethod
    def forward(ctx, A, B, policy="auto", out_dtype=None):
        ctx.save_for_backward(A, B)
        ctx.policy = policy
        ctx.out_dtype = out_dtype
        return skgemm.matmul(A, B, policy=policy, out_dtype=out_dtype)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        if dC.dtype != A.dtype:
            dC = dC.to(A.dtype)
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = skgemm.matmul(dC, B.t(), policy=ctx.policy, out_dtype=A.dtype if A.dtype != torch.float8_e4m3fn
                               else torch.float32)
        if ctx.needs_input_grad[1]:
            dB = skgemm.matmul(A.t(), dC, policy=ctx.policy, out_dtype=B.dtype if B.dtype != torch.float8_e4m3fn
                               else torch.float32)
        return dA, dB, None, None


def skgemm_matmul(A, B, policy="auto", out_dtype=None):
    """Autograd-aware A @ B through the Stream-K library."""
    return SkGemmFunction.apply(A, B, policy, out_dtype)
