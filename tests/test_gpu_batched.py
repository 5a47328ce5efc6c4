"""Strided batched Stream-K GEMM (one persistent launch over batch equal
problems) through the C ABI: every problem against the FP64 oracle, integer
inputs bit-exact under split plans, the schedule trace against the grouped
enumerator of the equal problems, column-major C and beta."""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import oracle_grouped_plan_for, records_to_schedule, to_f64
from oracle import gemm as og
from oracle import grouped as GR

pytestmark = pytest.mark.gpu


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def dev():
    return torch.device("cuda:0")


@pytest.mark.parametrize("shape", [(8, 300, 500, 700), (32, 128, 256, 2048), (3, 1000, 130, 77), (5, 1, 7, 9),
                                   (64, 64, 64, 512)])
@pytest.mark.parametrize("policy", ["auto", "sk", "dp"])
def test_batched_parity(shape, policy):
    batch, M, N, K = shape
    g = W.rng(batch + M)
    A = torch.from_numpy(W.normal_f32(g, (batch, M, K))).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(W.normal_f32(g, (batch, K, N))).to(torch.bfloat16).to(dev())
    C = sk().batched_matmul(A, B, policy=policy, out_dtype=torch.float32)
    torch.cuda.synchronize()
    for i in range(batch):
        ref = og.gemm_f64(to_f64(A[i]), to_f64(B[i]))
        assert og.rel_frobenius(to_f64(C[i]), ref) <= 1e-5, (i, policy)


@pytest.mark.parametrize("g_", [0, 2, 5])
def test_batched_integer_exact_and_trace(g_):
    """Integer inputs: bit-exact under the split plans; the trace equals the
    grouped enumerator's schedule of the equal problems."""
    batch, M, N, K = 6, 384, 256, 1024
    gen = W.rng(9)
    a = np.stack([W.integer_f32(gen, (M, K)) for _ in range(batch)])
    b = np.stack([W.integer_f32(gen, (K, N)) for _ in range(batch)])
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    tile = (128, 128, 64, 4)
    plan = sk().BatchedPlan(batch, M, N, K, ta=sk().BF16, tc=sk().F32, policy="sk", tile=tile)
    t = plan.info()["t"]
    force = g_ * t
    plan = sk().BatchedPlan(batch, M, N, K, ta=sk().BF16, tc=sk().F32, policy="sk", force_g=force, tile=tile)
    info = plan.info()
    tr = torch.full((plan.trace_capacity() * 8,), -7, dtype=torch.int32, device=dev())
    C = sk().batched_matmul(A, B, policy="sk", force_g=force, tile=tile, out_dtype=torch.float32, trace=tr)
    torch.cuda.synchronize()
    for i in range(batch):
        assert np.array_equal(to_f64(C[i]), og.gemm_f64(a[i].astype(np.float64), b[i].astype(np.float64))), i
    recs = [tuple(int(v) for v in r) for r in tr.cpu().numpy().reshape(-1, 8) if r[0] != -7]
    got = records_to_schedule(recs, info["grid"])
    ref = oracle_grouped_plan_for([(M, N, K)] * batch, info, plan.model_constants(), "sk", force_g=force)
    assert got == GR.enumerate_grouped_schedule(ref)
    if g_ >= 2:
        assert info["coop_s"] == g_


def test_batched_strided_views_beta_and_col_major_c():
    """Operands as strided views of larger buffers (batch stride beyond the
    matrix), C column-major with beta != 0."""
    batch, M, N, K = 4, 200, 300, 256
    g = W.rng(2)
    Abuf = torch.from_numpy(W.normal_f32(g, (batch, M + 3, K))).to(torch.bfloat16).to(dev())
    Bbuf = torch.from_numpy(W.normal_f32(g, (batch, N, K))).to(torch.bfloat16).to(dev())
    A = Abuf[:, :M, :]                          # row-major, batch stride (M + 3) * K
    B = Bbuf.transpose(1, 2)                    # column-major B
    C0 = torch.from_numpy(W.normal_f32(g, (batch, N, M))).to(dev())
    C = C0.clone().transpose(1, 2)              # column-major C
    sk().batched_matmul(A, B, C, alpha=0.5, beta=2.0, policy="sk")
    torch.cuda.synchronize()
    for i in range(batch):
        ref = og.gemm_f64(to_f64(A[i]), to_f64(B[i]), 0.5, 2.0, to_f64(C0[i].t()))
        assert og.rel_frobenius(to_f64(C[i]), ref) <= 1e-5, i
