"""GPU parity of the FP64 Stream-K GEMM (FP64 in, accumulation, fix-up and out)
against the FP64 oracle.

Both sides accumulate in binary64 in different orders, so the bound per
element is the standard one for a length-K dot product,
|C - C_ref| <= gamma_K * (|A| |B|), gamma_K = K u / (1 - K u), u = 2^-53; the
relative Frobenius error is checked against 1e-12 as well.  Integer-valued
inputs are exact in FP64 and must match bit for bit under every policy and
grid.  The schedule trace must equal the oracle's enumerator.
"""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import oracle_plan_for, records_to_schedule
from oracle import gemm as og
from oracle import schedule as S

pytestmark = pytest.mark.gpu

POLICIES = ["auto", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"]
SHAPES = [(64, 64, 16), (1000, 700, 900), (1, 1, 1), (65, 129, 17), (384, 384, 1024), (2048, 512, 4096),
          (7, 300, 5000), (130, 2, 64)]
U64 = 2.0 ** -53
# the two FP64 tiles (the planner picks one per problem; tests pin each)
TILES = [(64, 64, 16), (128, 128, 16)]


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def dev():
    return torch.device("cuda:0")


def _inputs(M, N, K, seed):
    g = W.rng(seed)
    return g.standard_normal((M, K)), g.standard_normal((K, N))


def _reference(a, b, K):
    """The oracle's product and the elementwise rounding bound of a K-term sum."""
    gamma = K * U64 / (1 - K * U64)
    return og.gemm_f64(a, b), gamma * (np.abs(a) @ np.abs(b)) + 1e-300


def _check(C, ref_bound):
    ref, bound = ref_bound
    got = C.cpu().numpy()
    assert og.rel_frobenius(got, ref) <= 1e-12
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("shape", SHAPES)
def test_f64_parity_every_policy(shape, tile):
    M, N, K = shape
    a, b = _inputs(M, N, K, seed=M + N + K)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    rb = _reference(a, b, K)
    for pol in POLICIES:
        C = sk().matmul(A, B, policy=pol, tile=tile)
        torch.cuda.synchronize()
        assert C.dtype == torch.float64
        _check(C, rb)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("g", [1, 3, 16, 100, 176, 352, 500])
def test_f64_integer_exact_forced_grids(g, tile):
    M, N, K = 1000, 700, 900
    rng = W.rng(11)
    a = rng.integers(-2, 3, (M, K)).astype(np.float64)
    b = rng.integers(-2, 3, (K, N)).astype(np.float64)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    try:
        C = sk().matmul(A, B, policy="sk", force_g=g, tile=tile)
    except sk().SkgemmError as e:
        assert e.status == sk().ERR_CAPACITY
        pytest.skip("grid larger than the co-resident capacity of this GPU")
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), og.gemm_f64(a, b))


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("layouts", ["nn", "nt", "tn", "tt"])
@pytest.mark.parametrize("c_col", [False, True])
def test_f64_layouts(layouts, c_col, tile):
    M, N, K = 333, 517, 290
    a, b = _inputs(M, N, K, seed=5)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    if layouts[0] == "t":
        A = A.t().contiguous().t()
    if layouts[1] == "t":
        B = B.t().contiguous().t()
    out = torch.empty((N, M), dtype=torch.float64, device=dev()).t() if c_col else \
        torch.empty((M, N), dtype=torch.float64, device=dev())
    rb = _reference(a, b, K)
    for pol in ("auto", "sk", "dp"):
        C = sk().matmul(A, B, out=out, policy=pol, tile=tile)
        torch.cuda.synchronize()
        _check(C, rb)


def test_f64_alpha_beta_and_nan_c():
    M, N, K = 260, 300, 500
    a, b = _inputs(M, N, K, seed=6)
    c0 = W.rng(7).standard_normal((M, N))
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    ref = og.gemm_f64(a, b, 0.5, -2.0, c0)
    for pol in ("sk", "dp", "auto"):
        C = torch.from_numpy(c0).to(dev())
        sk().matmul(A, B, out=C, alpha=0.5, beta=-2.0, policy=pol)
        torch.cuda.synchronize()
        assert og.rel_frobenius(C.cpu().numpy(), ref) <= 1e-12, pol
        Cn = torch.full((M, N), float("nan"), dtype=torch.float64, device=dev())
        sk().matmul(A, B, out=Cn, policy=pol)
        torch.cuda.synchronize()
        assert not torch.isnan(Cn).any(), pol


@pytest.mark.parametrize("shape,policy,g", [((1000, 700, 900), "sk", 0), ((1000, 700, 900), "sk", 333),
                                            ((384, 384, 1024), "auto", 0), ((4096, 4096, 64), "dp_1tile_sk", 0),
                                            ((4096, 4096, 64), "2tile_sk_dp", 0)])
@pytest.mark.parametrize("tile", TILES)
def test_f64_trace_matches_enumerator(shape, policy, g, tile):
    M, N, K = shape
    a, b = _inputs(M, N, K, seed=9)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    p = sk().get_plan(M, N, K, 0, 0, 0, sk().F64, sk().F64, policy, g, 2, tile)
    tr = torch.full((max(p.trace_capacity(), 1) * 8,), -7, dtype=torch.int32, device=dev())
    C = sk().matmul(A, B, policy=policy, force_g=g, trace=tr, tile=tile)
    torch.cuda.synchronize()
    info = p.info()
    recs = [tuple(int(v) for v in r) for r in tr.cpu().numpy().reshape(-1, 8) if r[0] != -7]
    got = records_to_schedule(recs, info["grid"])
    ref = oracle_plan_for(info, p.model_constants(), policy, force_g=g)
    assert got == S.enumerate_schedule(ref)
    _check(C, _reference(a, b, K))


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("s", [2, 3, 7])
def test_f64_split_fixup_bitwise_equals_owner(s, tile):
    M, N, K = 640, 448, 1600
    a, b = _inputs(M, N, K, seed=s)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    t = sk().Plan(M, N, K, ta=sk().F64, policy="dp", tile=tile).info()["t"]
    plan = sk().get_plan(M, N, K, 0, 0, 0, sk().F64, sk().F64, "sk", s * t, 2, tile, "auto")
    if plan.info()["coop_s"] != s:
        pytest.skip("this GPU's co-resident capacity gives another plan")
    C1 = sk().matmul(A, B, policy="sk", force_g=s * t, fixup="auto", tile=tile)
    C2 = sk().matmul(A, B, policy="sk", force_g=s * t, fixup="owner", tile=tile)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    _check(C1, _reference(a, b, K))


def test_f64_k_zero_and_empty():
    A = torch.zeros((100, 0), dtype=torch.float64, device=dev())
    B = torch.zeros((0, 70), dtype=torch.float64, device=dev())
    C = torch.full((100, 70), 3.0, dtype=torch.float64, device=dev())
    sk().matmul(A, B, out=C, beta=0.5)
    torch.cuda.synchronize()
    assert torch.all(C == 1.5)
    E = sk().matmul(torch.zeros((0, 5), dtype=torch.float64, device=dev()),
                    torch.zeros((5, 4), dtype=torch.float64, device=dev()))
    assert E.shape == (0, 4)
