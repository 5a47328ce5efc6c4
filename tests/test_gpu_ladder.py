"""Precision ladder at full size: FP16 and FP8 (per-tensor scales) GEMMs at
M=N=K in {1024, 4096, 8192} and the skinny 128 x 8192 x 8192, automatic
policy, FP32 accumulation and FP32 output, on sampled rows against the FP64
oracle.

FP16 must be within 1e-2 relative Frobenius error of the FP64 GEMM of its
stored inputs.  FP8 reports two errors: against the FP64 GEMM of the
dequantised inputs (the kernel's own error, bound 5e-5: gfx950's FP8 MFMA
sums its products at about 16 significant bits before the FP32 accumulate)
and against the FP64 GEMM of the unquantised inputs (the total error,
including quantisation, bound 6e-2).  The measured errors are printed.
"""
import numpy as np
import pytest
import torch

from helpers import to_f64
from oracle import gemm as og

pytestmark = pytest.mark.gpu

SHAPES = [(1024, 1024, 1024), (4096, 4096, 4096), (8192, 8192, 8192), (128, 8192, 8192)]


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def _inputs(M, N, K):
    g = torch.Generator(device="cpu").manual_seed(M * 7 + K)
    A = torch.randn((M, K), generator=g, dtype=torch.float32)
    B = torch.randn((K, N), generator=g, dtype=torch.float32)
    return A, B


def _rows(M):
    r = np.random.default_rng(M).choice(M, size=min(M, 12), replace=False)
    return np.unique(np.concatenate([r, [0, M - 1]]))


@pytest.mark.parametrize("shape", SHAPES)
def test_ladder_f16(shape):
    M, N, K = shape
    A, B = _inputs(M, N, K)
    Ad = A.to(torch.float16).cuda()
    Bd = B.to(torch.float16).cuda()
    C = sk().matmul(Ad, Bd, out_dtype=torch.float32)
    rows = _rows(M)
    got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = og.gemm_rows_f64(to_f64(Ad), to_f64(Bd), rows)
    err = og.rel_frobenius(got, ref)
    print(f"ladder f16 {M}x{N}x{K}: rel-Frobenius {err:.3e} on {rows.size} rows", flush=True)
    assert err <= 1e-2


@pytest.mark.parametrize("shape", SHAPES)
def test_ladder_fp8(shape):
    M, N, K = shape
    A, B = _inputs(M, N, K)
    C, (qa, sa), (qb, sb) = sk().matmul_fp8(A.cuda(), B.cuda())
    rows = _rows(M)
    got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
    dqa = to_f64(qa) * sa.item()
    dqb = to_f64(qb) * sb.item()
    kernel_err = og.rel_frobenius(got, og.gemm_rows_f64(dqa, dqb, rows))
    total_err = og.rel_frobenius(got, og.gemm_rows_f64(A.numpy(), B.numpy(), rows))
    print(f"ladder fp8 {M}x{N}x{K}: kernel error {kernel_err:.3e}, total error {total_err:.3e} "
          f"on {rows.size} rows", flush=True)
    assert kernel_err <= 5e-5
    assert total_err <= 6e-2
