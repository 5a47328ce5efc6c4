"""Hand-written backward of the Stream-K GEMM against the oracle's gradient.

The oracle gradient (dA = dC B^T, dB = A^T dC in FP64 of the stored inputs)
is pinned against FP64 central differences on the CPU (test_oracle_gemm).
Here the GPU gradients must match it: FP32 inputs within 1e-5, BF16 inputs
with BF16 gradients within 1e-2 (relative Frobenius).  A finite-difference
check through the GPU's FP32 forward closes the loop at 64^3.
"""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import to_f64
from oracle import gemm as og

pytestmark = pytest.mark.gpu


def fn():
    from paper_2212_08964_amd.autograd import skgemm_matmul
    return skgemm_matmul


def _run(M, N, K, dtype, policy="auto", seed=0):
    a, b = W.normal_pair(M, N, K, seed=seed)
    dc = W.normal_f32(W.rng(seed + 100), (M, N))
    A = torch.from_numpy(a).to(dtype).cuda().requires_grad_(True)
    B = torch.from_numpy(b).to(dtype).cuda().requires_grad_(True)
    dC = torch.from_numpy(dc).to(dtype).cuda()
    C = fn()(A, B, policy)
    C.backward(dC)
    torch.cuda.synchronize()
    return A, B, dC, C


@pytest.mark.parametrize("policy", ["auto", "sk", "dp"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (300, 200, 500), (256, 1024, 512), (33, 65, 129)])
def test_backward_f32(shape, policy):
    M, N, K = shape
    A, B, dC, C = _run(M, N, K, torch.float32, policy)
    dA_ref, dB_ref = og.gemm_grad(to_f64(A.detach()), to_f64(B.detach()), to_f64(dC))
    assert og.rel_frobenius(to_f64(C.detach()), og.gemm_f64(to_f64(A.detach()), to_f64(B.detach()))) <= 1e-5
    assert og.rel_frobenius(to_f64(A.grad), dA_ref) <= 1e-5
    assert og.rel_frobenius(to_f64(B.grad), dB_ref) <= 1e-5


@pytest.mark.parametrize("shape", [(256, 4096, 4096), (2048, 2048, 8192)])
def test_backward_bf16_benchmark_shapes(shape):
    M, N, K = shape
    A, B, dC, C = _run(M, N, K, torch.bfloat16, "auto", seed=1)
    a, b, dc = to_f64(A.detach()), to_f64(B.detach()), to_f64(dC)
    rows_m = np.array([0, 1, M // 2, M - 1])
    rows_k = np.array([0, 7, K // 3, K - 1])
    assert og.rel_frobenius(to_f64(C.detach()[torch.from_numpy(rows_m).cuda()]), og.gemm_rows_f64(a, b, rows_m)) <= 1e-2
    # dA = dC B^T (rows of dA), dB = A^T dC (rows of dB = columns of A)
    dA_rows = og.gemm_rows_f64(dc, np.ascontiguousarray(b.T), rows_m)
    dB_rows = og.gemm_rows_f64(np.ascontiguousarray(a.T), dc, rows_k)
    assert og.rel_frobenius(to_f64(A.grad[torch.from_numpy(rows_m).cuda()]), dA_rows) <= 1e-2
    assert og.rel_frobenius(to_f64(B.grad[torch.from_numpy(rows_k).cuda()]), dB_rows) <= 1e-2


def test_finite_differences_through_gpu_forward():
    """L(A) = <dC, A B> is linear in A: central differences of the GPU FP32
    forward equal dL/dA up to FP32 rounding of L."""
    M = N = K = 64
    A, B, dC, _ = _run(M, N, K, torch.float32, "sk", seed=3)
    from paper_2212_08964_amd import skgemm
    h = 0.5
    for i, k in [(0, 0), (5, 40), (63, 63), (31, 2)]:
        Ap = A.detach().clone()
        Am = A.detach().clone()
        Ap[i, k] += h
        Am[i, k] -= h
        Lp = float((dC.double() * skgemm.matmul(Ap, B.detach(), policy="sk").double()).sum())
        Lm = float((dC.double() * skgemm.matmul(Am, B.detach(), policy="sk").double()).sum())
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - float(A.grad[i, k])) <= 1e-3 * max(1.0, abs(fd))


@pytest.mark.parametrize("shape", [(256, 512, 1024), (300, 200, 700)])
def test_graphed_step_replays_match_eager(shape):
    """The graph-captured step (C = A B, dA = dC B^T, dB = A^T dC): every
    replay, with eager work on the default stream between replays, equals the
    eager products bitwise (same plans, same kernels), also after the inputs
    are updated in place; and the products match the FP64 oracle."""
    from paper_2212_08964_amd import skgemm
    from paper_2212_08964_amd.autograd import GraphedStep
    M, N, K = shape
    g = W.rng(M + N)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(W.normal_f32(g, (M, K))).to(torch.bfloat16).to(dev)
    B = torch.from_numpy(W.normal_f32(g, (K, N))).to(torch.bfloat16).to(dev)
    dC = torch.from_numpy(W.normal_f32(g, (M, N))).to(torch.bfloat16).to(dev)
    step = GraphedStep(A, B, dC)

    def eager():
        return (skgemm.matmul(A, B), skgemm.matmul(dC, B.t()), skgemm.matmul(A.t(), dC))

    noise = torch.randn((512, 512), device=dev).to(torch.bfloat16)
    for r in range(4):
        if r == 2:      # new inputs, in place
            A.copy_(torch.from_numpy(W.normal_f32(g, (M, K))).to(torch.bfloat16))
            dC.copy_(torch.from_numpy(W.normal_f32(g, (M, N))).to(torch.bfloat16))
        skgemm.matmul(noise, noise)
        C, dA, dB = step.replay()
        torch.cuda.synchronize()
        ref = eager()
        torch.cuda.synchronize()
        for got, want in zip((C, dA, dB), ref):
            assert torch.equal(got, want), r
    a, b, dc = to_f64(A), to_f64(B), to_f64(dC)
    assert og.rel_frobenius(to_f64(C), og.gemm_f64(a, b)) <= 1e-2
    assert og.rel_frobenius(to_f64(dA), og.gemm_f64(dc, b.T.copy())) <= 1e-2
    assert og.rel_frobenius(to_f64(dB), og.gemm_f64(a.T.copy(), dc)) <= 1e-2
