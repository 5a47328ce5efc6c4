"""skgemm_run_noalloc (the entry point for callers that cannot allocate)
against skgemm_run with a caller-owned workspace, through the C ABI: the same
plan gives bitwise the same C; two calls in a row, the second on a smaller
problem; a data-parallel plan (no workspace); a plan beyond the array's
64 MiB is refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle import gemm as og
from helpers import to_f64

pytestmark = pytest.mark.gpu


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def _pair(M, N, K, seed):
    a, b = W.normal_pair(M, N, K, seed=seed)
    return (torch.from_numpy(a).to(torch.bfloat16).cuda(), torch.from_numpy(b).to(torch.bfloat16).cuda())


def _both(plan, A, B, M, N, K):
    """C from skgemm_run (fresh zeroed workspace) and from skgemm_run_noalloc."""
    L = sk().lib()
    stream = torch.cuda.current_stream().cuda_stream
    nws = plan.workspace_size()
    ws = torch.zeros(max(nws, 256), dtype=torch.uint8, device="cuda")
    C1 = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    C2 = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    st = L.skgemm_run(plan.handle, A.data_ptr(), K, B.data_ptr(), N, C1.data_ptr(), N, 1.0, 0.0, None, None,
                      ws.data_ptr() if nws else None, nws, stream)
    assert st == sk().OK
    st = L.skgemm_run_noalloc(plan.handle, A.data_ptr(), K, B.data_ptr(), N, C2.data_ptr(), N, 1.0, 0.0, None,
                              None, stream)
    assert st == sk().OK, sk().status_string(st)
    torch.cuda.synchronize()
    return C1, C2


@pytest.mark.parametrize("policy,fixup", [("sk", "auto"), ("sk", "owner"), ("auto", "auto"),
                                          ("2tile_sk_dp", "owner")])
def test_noalloc_equals_run_two_calls_second_smaller(policy, fixup):
    cases = [(1536, 1280, 4096, 1), (384, 640, 1000, 2)]     # second call: a smaller problem
    for (M, N, K, seed) in cases:
        A, B = _pair(M, N, K, seed)
        # the small tile: any grid up to the capacity fits the array
        plan = sk().Plan(M, N, K, ta=sk().BF16, tc=sk().F32, policy=policy, fixup=fixup, tile=(128, 128, 64, 4))
        assert plan.workspace_size() <= 64 << 20
        C1, C2 = _both(plan, A, B, M, N, K)
        assert torch.equal(C1, C2), (M, N, K, policy)
        assert og.rel_frobenius(to_f64(C2), og.gemm_f64(to_f64(A), to_f64(B))) <= 1e-5


def test_noalloc_data_parallel_and_repeat():
    M, N, K = 512, 768, 640
    A, B = _pair(M, N, K, 3)
    plan = sk().Plan(M, N, K, ta=sk().BF16, tc=sk().F32, policy="dp")
    assert plan.workspace_size() == 0
    C1, C2 = _both(plan, A, B, M, N, K)
    assert torch.equal(C1, C2)
    # the same split plan many times on the shared array (flags self-clean)
    plan = sk().Plan(M, N, K, ta=sk().BF16, tc=sk().F32, policy="sk", tile=(128, 128, 64, 4))
    first = None
    for _ in range(20):
        C1, C2 = _both(plan, A, B, M, N, K)
        assert torch.equal(C1, C2)
        first = C2 if first is None else first
        assert torch.equal(C2, first)


def test_noalloc_refuses_plans_beyond_its_array():
    # 256 Stream-K workgroups with 256x256 FP32 partial tiles: 64 MiB of partials + flags
    p = sk().Plan(256 * 16, 256 * 16, 8192, ta=sk().BF16, tc=sk().F32, policy="sk", force_g=256,
                  tile=(256, 256, 64))
    assert p.workspace_size() > 64 << 20
    L = sk().lib()
    st = L.skgemm_run_noalloc(p.handle, 1 << 40, 8192, 1 << 40, 4096, 1 << 40, 4096, 1.0, 0.0, None, None, None)
    assert st == sk().ERR_WORKSPACE
