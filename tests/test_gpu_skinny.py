"""The skinny 64x256x64 16-bit tile (problems of at most 64 rows) against the
float64 oracle through the C ABI: parity for every policy and both B layouts,
integer inputs bit-exact under forced grids, and the schedule trace equal to
the enumerator's."""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import oracle_plan_for, records_to_schedule, to_f64
from oracle import gemm as og
from oracle import schedule as S

pytestmark = pytest.mark.gpu

SKINNY = (64, 256, 64)
TOL_OUT32 = 1e-5
TOL_16 = 1e-2


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def dev():
    return torch.device("cuda:0")


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("shape", [(1, 1000, 3000), (7, 257, 129), (16, 4096, 2048), (33, 700, 1500), (64, 2048, 4096),
                                   (64, 256, 64), (40, 5000, 77)])
@pytest.mark.parametrize("b_col", [False, True])
def test_skinny_parity(dtype, shape, b_col):
    M, N, K = shape
    a, b = W.normal_pair(M, N, K, seed=M + N + K)
    A = torch.from_numpy(a).to(dtype).to(dev())
    B = torch.from_numpy(b).to(dtype).to(dev())
    if b_col:
        B = B.t().contiguous().t()
    ref = og.gemm_f64(to_f64(A), to_f64(B))
    for pol in ("auto", "dp", "sk"):
        C32 = sk().matmul(A, B, policy=pol, out_dtype=torch.float32, tile=SKINNY)
        C16 = sk().matmul(A, B, policy=pol, tile=SKINNY)
        torch.cuda.synchronize()
        assert og.rel_frobenius(to_f64(C32), ref) <= TOL_OUT32, (pol, "f32 out")
        assert og.rel_frobenius(to_f64(C16), ref) <= TOL_16, (pol, "16-bit out")


def test_skinny_is_the_automatic_choice_for_short_problems():
    A = torch.randn((16, 4096), device=dev()).to(torch.bfloat16)
    B = torch.randn((4096, 8192), device=dev()).to(torch.bfloat16)
    info = sk().get_plan(16, 8192, 4096, sk().ROW_MAJOR, sk().ROW_MAJOR, sk().ROW_MAJOR, sk().BF16,
                         sk().BF16).info()
    assert info["tile"] == (64, 256, 64, 4)
    C = sk().matmul(A, B)
    torch.cuda.synchronize()
    assert og.rel_frobenius(to_f64(C), og.gemm_f64(to_f64(A), to_f64(B))) <= TOL_16


@pytest.mark.parametrize("b_col", [False, True])
def test_skinny_integer_exact_every_grid(b_col):
    M, N, K = 50, 1300, 3000
    g = W.rng(4)
    A = torch.from_numpy(W.integer_f32(g, (M, K))).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(W.integer_f32(g, (K, N))).to(torch.bfloat16).to(dev())
    if b_col:
        B = B.t().contiguous().t()
    ref = og.gemm_f64(to_f64(A), to_f64(B))
    for pol in ["auto", "paper", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"]:
        for fg in ([0] if pol != "sk" else [0, 1, 5, 6, 47, 200, 400]):
            try:
                C = sk().matmul(A, B, policy=pol, force_g=fg, out_dtype=torch.float32, tile=SKINNY)
            except sk().SkgemmError as e:
                assert fg > 0 and e.status == sk().ERR_CAPACITY, (pol, fg, e)
                continue
            torch.cuda.synchronize()
            assert np.array_equal(to_f64(C), ref), (pol, fg)


@pytest.mark.parametrize("policy,g", [("sk", 0), ("sk", 23), ("dp", 0), ("auto", 0)])
def test_skinny_trace_matches_enumerator(policy, g):
    M, N, K = 60, 3000, 2500
    a, b = W.normal_pair(M, N, K, seed=1)
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    plan = sk().Plan(M, N, K, ta=sk().BF16, tc=sk().F32, policy=policy, force_g=g, tile=SKINNY)
    info = plan.info()
    assert info["tile"] == (64, 256, 64, 4)
    tr = torch.full((plan.trace_capacity() * 8,), -7, dtype=torch.int32, device=dev())
    C = sk().matmul(A, B, policy=policy, force_g=g, tile=SKINNY, out_dtype=torch.float32, trace=tr)
    torch.cuda.synchronize()
    recs = [tuple(int(v) for v in r) for r in tr.cpu().numpy().reshape(-1, 8) if r[0] != -7]
    ref = oracle_plan_for(info, plan.model_constants(), policy, force_g=g)
    assert records_to_schedule(recs, info["grid"]) == S.enumerate_schedule(ref)
    assert og.rel_frobenius(to_f64(C), og.gemm_f64(to_f64(A), to_f64(B))) <= TOL_OUT32


TALL = (256, 64, 64)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("shape", [(1000, 1, 3000), (257, 7, 129), (4096, 16, 2048), (700, 33, 1500), (2048, 64, 4096),
                                   (5000, 40, 77)])
@pytest.mark.parametrize("a_col", [False, True])
def test_tall_parity(dtype, shape, a_col):
    """The tall 256x64x64 tile (K-contiguous B: column-major) for every policy
    and both A layouts."""
    M, N, K = shape
    a, b = W.normal_pair(M, N, K, seed=M + N + K)
    A = torch.from_numpy(a).to(dtype).to(dev())
    B = torch.from_numpy(b).to(dtype).to(dev()).t().contiguous().t()
    if a_col:
        A = A.t().contiguous().t()
    ref = og.gemm_f64(to_f64(A), to_f64(B))
    for pol in ("auto", "dp", "sk"):
        C32 = sk().matmul(A, B, policy=pol, out_dtype=torch.float32, tile=TALL)
        C16 = sk().matmul(A, B, policy=pol, tile=TALL)
        torch.cuda.synchronize()
        assert og.rel_frobenius(to_f64(C32), ref) <= TOL_OUT32, (pol, "f32 out")
        assert og.rel_frobenius(to_f64(C16), ref) <= TOL_16, (pol, "16-bit out")


def test_tall_integer_exact_every_grid_and_trace():
    M, N, K = 1300, 50, 3000
    g = W.rng(8)
    A = torch.from_numpy(W.integer_f32(g, (M, K))).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(W.integer_f32(g, (K, N))).to(torch.bfloat16).to(dev()).t().contiguous().t()
    ref = og.gemm_f64(to_f64(A), to_f64(B))
    for pol in ["auto", "paper", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"]:
        for fg in ([0] if pol != "sk" else [0, 1, 5, 6, 47, 200, 400]):
            try:
                C = sk().matmul(A, B, policy=pol, force_g=fg, out_dtype=torch.float32, tile=TALL)
            except sk().SkgemmError as e:
                assert fg > 0 and e.status == sk().ERR_CAPACITY, (pol, fg, e)
                continue
            torch.cuda.synchronize()
            assert np.array_equal(to_f64(C), ref), (pol, fg)
    plan = sk().Plan(M, N, K, lb=sk().COL_MAJOR, ta=sk().BF16, tc=sk().F32, policy="sk", force_g=23, tile=TALL)
    info = plan.info()
    assert info["tile"] == (256, 64, 64, 4)
    tr = torch.full((plan.trace_capacity() * 8,), -7, dtype=torch.int32, device=dev())
    sk().matmul(A, B, policy="sk", force_g=23, tile=TALL, out_dtype=torch.float32, trace=tr)
    torch.cuda.synchronize()
    recs = [tuple(int(v) for v in r) for r in tr.cpu().numpy().reshape(-1, 8) if r[0] != -7]
    ref_plan = oracle_plan_for(info, plan.model_constants(), "sk", force_g=23)
    assert records_to_schedule(recs, info["grid"]) == S.enumerate_schedule(ref_plan)
