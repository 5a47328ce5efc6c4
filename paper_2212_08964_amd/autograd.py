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


class GraphedStep:
    """One training step's three products, C = A @ B, dA = dC @ B^T and
    dB = A^T @ dC, for fixed tensors, captured once in a HIP graph and then
    replayed with no host work per product (the autograd and Python costs of
    a small step are paid once, at capture).  The caller updates A, B and dC
    in place between replays; C, dA and dB are the graph's own outputs,
    overwritten by every replay.

    The products run on a stream of this object's own: it is warmed up there
    before capture, so the fix-up workspace for that stream exists beforehand
    and the graph holds only the GEMM launches."""

    def __init__(self, A, B, dC, policy="auto"):
        if A.dim() != 2 or B.dim() != 2 or dC.shape != (A.shape[0], B.shape[1]) or A.shape[1] != B.shape[0]:
            raise ValueError("GraphedStep needs A (M x K), B (K x N) and dC (M x N)")
        self.A, self.B, self.dC, self.policy = A, B, dC, policy
        self.C = torch.empty((A.shape[0], B.shape[1]), dtype=A.dtype, device=A.device)
        self.dA = torch.empty_like(A)
        self.dB = torch.empty_like(B)
        self.stream = torch.cuda.Stream(device=A.device)
        self.stream.wait_stream(torch.cuda.current_stream(A.device))
        with torch.cuda.stream(self.stream):
            for _ in range(2):
                self._products()
        torch.cuda.current_stream(A.device).wait_stream(self.stream)
        torch.cuda.synchronize(A.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._products()

    def _products(self):
        skgemm.matmul(self.A, self.B, out=self.C, policy=self.policy)
        skgemm.matmul(self.dC, self.B.t(), out=self.dA, policy=self.policy)
        skgemm.matmul(self.A.t(), self.dC, out=self.dB, policy=self.policy)

    def replay(self):
        """Run the captured step on the current stream's order; returns (C, dA, dB)."""
        self.graph.replay()
        return self.C, self.dA, self.dB
