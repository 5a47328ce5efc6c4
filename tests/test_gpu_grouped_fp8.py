"""GPU parity of the grouped launch and the FP8 path against the oracle.

Grouped: every problem's C against the FP64 oracle (BF16 inputs, FP32 output:
tolerance 1e-5; BF16 output 1e-2), the kernel's schedule trace against the
oracle's grouped enumerator, and replays of a captured HIP graph against
the eager result.

FP8: the quantiser's codes and scale must equal the oracle's bit for bit (the
decision x / s is taken in FP32 on both sides); the FP8 GEMM must match the
FP64 GEMM of the dequantised inputs within 5e-5 and the FP64 GEMM of the
unquantised inputs within 6e-2 (total error including quantisation).  The
kernel-error bound is set by the hardware: gfx950's FP8 MFMA adds its
products at about 16 significant bits before the FP32 accumulate, which
measures as a relative error of ~1.5e-5 independent of K (FP32 accumulation
alone would give ~1e-7).
"""
import json

import numpy as np
import pytest
import torch

import workloads as W
from helpers import oracle_grouped_plan_for, records_to_schedule, to_f64
from oracle import gemm as og
from oracle import grouped as GR
from oracle import lowp

pytestmark = pytest.mark.gpu


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def dev():
    return torch.device("cuda:0")


def _problems(seed, Ms, N, K, dtype=torch.bfloat16):
    g = W.rng(seed)
    As, Bs = [], []
    for M in Ms:
        As.append(torch.from_numpy(W.normal_f32(g, (M, K))).to(dtype).to(dev()))
        Bs.append(torch.from_numpy(W.normal_f32(g, (K, N))).to(dtype).to(dev()))
    return As, Bs


@pytest.mark.parametrize("policy", ["auto", "sk", "dp", "2tile_sk_dp", "dp_1tile_sk"])
@pytest.mark.parametrize("tile", [None, (256, 256, 64), (128, 128, 64, 4), (128, 128, 64, 8)])
def test_grouped_zipf_parity(policy, tile):
    Ms = W.zipf_ms(24, lo=16, hi=1024, seed=1)
    As, Bs = _problems(2, Ms, 1024, 512)
    Cs, _ = sk().grouped_matmul(As, Bs, out_dtype=torch.float32, policy=policy, tile=tile)
    torch.cuda.synchronize()
    for A, B, C in zip(As, Bs, Cs):
        ref = og.gemm_f64(to_f64(A), to_f64(B))
        assert og.rel_frobenius(to_f64(C), ref) <= 1e-5


def test_grouped_ragged_mixed_shapes_bf16_out():
    shapes = [(300, 500, 700), (1, 1, 1), (0, 64, 64), (257, 255, 65), (1000, 130, 5), (64, 3000, 2048)]
    g = W.rng(3)
    As = [torch.from_numpy(W.normal_f32(g, (M, K))).to(torch.bfloat16).to(dev()) for M, N, K in shapes]
    Bs = [torch.from_numpy(W.normal_f32(g, (K, N))).to(torch.bfloat16).to(dev()) for M, N, K in shapes]
    for pol in ("auto", "sk"):
        Cs, _ = sk().grouped_matmul(As, Bs, policy=pol)
        torch.cuda.synchronize()
        for A, B, C in zip(As, Bs, Cs):
            if C.numel() == 0:
                continue
            ref = og.gemm_f64(to_f64(A), to_f64(B))
            assert og.rel_frobenius(to_f64(C), ref) <= 1e-2


@pytest.mark.parametrize("tile", [(256, 256, 64), (128, 128, 64, 4), (128, 128, 64, 8)])
def test_grouped_integer_exact_forced_grids(tile):
    Ms = [37, 300, 16, 520]
    g = W.rng(4)
    As = [torch.from_numpy(W.integer_f32(g, (M, 777))).to(torch.bfloat16).to(dev()) for M in Ms]
    Bs = [torch.from_numpy(W.integer_f32(g, (777, 600))).to(torch.bfloat16).to(dev()) for _ in Ms]
    refs = [og.gemm_f64(to_f64(A), to_f64(B)) for A, B in zip(As, Bs)]
    for fg in (0, 3, 17, 64, 200):
        Cs, _ = sk().grouped_matmul(As, Bs, out_dtype=torch.float32, policy="sk", force_g=fg, tile=tile)
        torch.cuda.synchronize()
        for C, ref in zip(Cs, refs):
            assert np.array_equal(to_f64(C), ref), fg


@pytest.mark.parametrize("policy", ["auto", "paper", "sk", "2tile_sk_dp"])
@pytest.mark.parametrize("tile", [None, (128, 128, 64, 4), (128, 128, 64, 8)])
def test_grouped_trace_matches_enumerator(policy, tile):
    Ms = W.zipf_ms(64, seed=0)
    shapes = [(m, 4096, 2048) for m in Ms]
    A = [torch.ones((m, 2048), dtype=torch.bfloat16, device=dev()) for m in Ms]
    B = [torch.ones((2048, 4096), dtype=torch.bfloat16, device=dev()) for _ in Ms]
    p = sk().GroupedPlan(Ms, [4096] * 64, [2048] * 64, ta=sk().BF16, tc=sk().F32, policy=policy, tile=tile)
    info = p.info()
    tr = torch.full((p.trace_capacity() * 8,), -7, dtype=torch.int32, device=dev())
    sk().grouped_matmul(A, B, out_dtype=torch.float32, policy=policy, trace=tr, tile=tile)
    torch.cuda.synchronize()
    recs = [tuple(int(v) for v in r) for r in tr.cpu().numpy().reshape(-1, 8) if r[0] != -7]
    got = records_to_schedule(recs, info["grid"])
    ref = oracle_grouped_plan_for(shapes, info, p.model_constants(), policy)
    assert got == GR.enumerate_grouped_schedule(ref)


def test_grouped_graph_replay_matches_eager():
    Ms = W.zipf_ms(64, seed=0)
    As, Bs = _problems(5, Ms, 4096, 2048)
    Cs = [torch.empty((m, 4096), dtype=torch.bfloat16, device=dev()) for m in Ms]
    _, table = sk().grouped_matmul(As, Bs, Cs)          # eager, builds the plan, table, workspace
    torch.cuda.synchronize()
    eager = [c.clone() for c in Cs]
    for c in Cs:
        c.zero_()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        sk().grouped_matmul(As, Bs, Cs, table=table)
    torch.cuda.synchronize()
    for rep in range(4):
        for c in Cs:
            c.fill_(float("nan"))                       # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for c, e in zip(Cs, eager):
            assert torch.equal(c, e), rep
    # the oracle on a few sampled problems (full C, sizes the oracle finishes fast)
    for i in range(0, 64, 16):
        ref = og.gemm_f64(to_f64(As[i]), to_f64(Bs[i]))
        assert og.rel_frobenius(to_f64(Cs[i]), ref) <= 1e-2


# ------------------------------------------------------------------ FP8 front end

# (333, 517): unaligned rows (the element-wise kernel); the others have 16-byte
# aligned rows and take the vectorised kernels (same order, or transposed
# through LDS with partial 64 x 64 tiles for (80, 208))
@pytest.mark.parametrize("shape", [(333, 517), (320, 512), (80, 208), (48, 16)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float16])
@pytest.mark.parametrize("layout_in,layout_out", [("row", "row"), ("row", "col"), ("col", "row"), ("col", "col")])
def test_quantize_bit_exact(dtype, layout_in, layout_out, shape):
    rows, cols = shape
    g = W.rng(7 + rows)
    x32 = (W.normal_f32(g, (rows, cols)) * np.exp(g.uniform(-6, 3, (rows, cols)))).astype(np.float32)
    X = torch.from_numpy(x32).to(dtype).to(dev())
    if layout_in == "col":
        X = X.t().contiguous().t()
    Q, s = sk().quantize_e4m3(X, layout_out)
    torch.cuda.synchronize()
    xv = to_f64(X).astype(np.float32)          # the stored input values, exactly
    qref, sref = lowp.quantize_e4m3(xv)
    assert np.float32(s.item()) == sref
    codes = Q.cpu().contiguous().view(torch.uint8).numpy() if layout_out == "row" else \
        Q.t().contiguous().t().cpu().contiguous().view(torch.uint8).numpy()
    assert np.array_equal(codes, qref)


def test_quantize_edge_cases():
    X = torch.zeros((5, 7), dtype=torch.bfloat16, device=dev())
    Q, s = sk().quantize_e4m3(X)
    torch.cuda.synchronize()
    assert s.item() == 1.0 and torch.all(Q.view(torch.uint8) == 0)
    # exact ties of the E4M3 grid after scaling: absmax 448 gives s = 1
    vals = np.array([448.0, 1.0625, 1.1875, 2.0 ** -10, 3 * 2.0 ** -10, -1.0625, 0.0, -448.0], np.float32)
    X = torch.from_numpy(np.tile(vals, (3, 1))).to(dev())
    Q, s = sk().quantize_e4m3(X)
    torch.cuda.synchronize()
    qref, sref = lowp.quantize_e4m3(np.tile(vals, (3, 1)))
    assert s.item() == float(sref) == 1.0
    assert np.array_equal(Q.cpu().view(torch.uint8).numpy(), qref)


@pytest.mark.parametrize("shape", [(333, 517), (320, 512), (80, 208)])
@pytest.mark.parametrize("layout_out", ["row", "col"])
def test_quantize_non_finite_bit_exact(shape, layout_out):
    """NaN and infinite entries give the NaN code with their sign; the scale
    comes from the finite entries (all three kernel forms)."""
    rows, cols = shape
    g = W.rng(11 + rows)
    x32 = W.normal_f32(g, (rows, cols)).astype(np.float32)
    idx = g.choice(rows * cols, size=8, replace=False)
    x32.ravel()[idx[:2]] = np.nan
    x32.ravel()[idx[2:4]] = -np.nan
    x32.ravel()[idx[4:6]] = np.inf
    x32.ravel()[idx[6:]] = -np.inf
    X = torch.from_numpy(x32).to(dev())
    Q, s = sk().quantize_e4m3(X, layout_out)
    torch.cuda.synchronize()
    qref, sref = lowp.quantize_e4m3(x32)
    assert np.float32(s.item()) == sref and np.isfinite(sref)
    codes = Q.cpu().contiguous().view(torch.uint8).numpy() if layout_out == "row" else \
        Q.t().contiguous().t().cpu().contiguous().view(torch.uint8).numpy()
    assert np.array_equal(codes, qref)


@pytest.mark.parametrize("tile", [None, (256, 256, 128), (128, 128, 128)])
@pytest.mark.parametrize("shape", [(256, 256, 128), (300, 500, 700), (1024, 1024, 1024), (128, 2048, 4096),
                                   (1, 1, 1), (513, 257, 131)])
def test_fp8_gemm_parity(shape, tile):
    M, N, K = shape
    a, b = W.normal_pair(M, N, K, seed=M + K)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    for pol in ("auto", "sk", "dp"):
        C, (qa, sa), (qb, sb) = sk().matmul_fp8(A, B, policy=pol, tile=tile)
        torch.cuda.synchronize()
        dqa = to_f64(qa) * sa.item()
        dqb = to_f64(qb) * sb.item()
        kernel_err = og.rel_frobenius(to_f64(C), og.gemm_f64(dqa, dqb))
        total_err = og.rel_frobenius(to_f64(C), og.gemm_f64(a, b))
        assert kernel_err <= 5e-5, (pol, tile, kernel_err)
        assert total_err <= 6e-2, (pol, tile, total_err)


def test_autotuner_picks_tile_and_split(tmp_path):
    """The grouped autotuner times every policy with the planner's tile and
    with each 16-bit tile pinned, keeps the fastest, and caches the decision."""
    from paper_2212_08964_amd import autotune
    Ms = W.zipf_ms(16, lo=16, hi=1024, seed=3)
    As, Bs = _problems(8, Ms, 512, 384)
    Cs = [torch.empty((m, 512), dtype=torch.bfloat16, device=dev()) for m in Ms]
    cache = str(tmp_path / "tune.json")
    autotune._memo.clear()
    best, times = autotune.tune_grouped(As, Bs, Cs, reps=2, cache_path=cache)
    tiles = {json.loads(k)["tile"] and tuple(json.loads(k)["tile"]) for k in times}
    assert {(256, 256, 64), (128, 128, 64, 4), (128, 128, 64, 8), None} <= tiles
    assert json.dumps(best, sort_keys=True) in times
    assert times[json.dumps(best, sort_keys=True)] == min(times.values())
    Cs2, _ = sk().grouped_matmul(As, Bs, **best)
    torch.cuda.synchronize()
    for A, B, C in zip(As, Bs, Cs2):
        assert og.rel_frobenius(to_f64(C), og.gemm_f64(to_f64(A), to_f64(B))) <= 1e-2
    autotune._memo.clear()
    again, fresh = autotune.tune_grouped(As, Bs, Cs, reps=2, cache_path=cache)
    assert again == best and fresh == {}


@pytest.mark.parametrize("tile", [(256, 256, 128), (128, 128, 128)])
def test_fp8_integer_exact_split_fixup(tile):
    """Integer-valued inputs with scale 1 (absmax 2 is not used: the values are
    stored directly as E4M3), every policy and split grids: bit-exact."""
    M, N, K = 700, 900, 1536
    g = W.rng(21)
    a = W.integer_f32(g, (M, K))
    b = W.integer_f32(g, (K, N))
    qa = torch.from_numpy(a).to(torch.float8_e4m3fn).to(dev())
    qb = torch.from_numpy(np.ascontiguousarray(b.T)).to(torch.float8_e4m3fn).to(dev()).t()
    ref = og.gemm_f64(a.astype(np.float64), b.astype(np.float64))
    t = sk().Plan(M, N, K, 0, 1, 0, sk().F8E4M3, sk().F32, policy="dp", tile=tile).info()["t"]
    p = sk().Plan(M, N, K, 0, 1, 0, sk().F8E4M3, sk().F32, policy="dp", tile=tile).info()["p"]
    for pol, fg in [("auto", 0), ("dp", 0), ("sk", 0), ("sk", 2 * t), ("sk", 3 * t), ("sk", 101)]:
        if fg > p:
            continue
        C = sk().matmul(qa, qb, out_dtype=torch.float32, policy=pol, force_g=fg, tile=tile)
        torch.cuda.synchronize()
        assert np.array_equal(to_f64(C), ref), (pol, fg)


@pytest.mark.parametrize("policy", ["auto", "paper", "sk", "dp", "2tile_sk_dp", "dp_1tile_sk"])
def test_grouped_zero_k_problems(policy):
    """Problems with K = 0 get C = beta * C (epilogue-only tiles after the
    others) in the same launch; the others match the oracle and the trace
    matches the enumerator."""
    probs = [(300, 700, 0), (1000, 900, 3000), (64, 64, 0), (0, 50, 0), (500, 256, 640), (900, 900, 0)]
    g = W.rng(5)
    As, Bs, Cin = [], [], []
    for (M, N, K) in probs:
        As.append(torch.from_numpy(W.normal_f32(g, (M, K))).to(torch.bfloat16).to(dev()))
        Bs.append(torch.from_numpy(W.normal_f32(g, (K, N))).to(torch.bfloat16).to(dev()))
        Cin.append(torch.from_numpy(W.normal_f32(g, (M, N))).to(dev()))
    Cs = [c.clone() for c in Cin]
    Ms, Ns, Ks = zip(*probs)
    p = sk().GroupedPlan(Ms, Ns, Ks, ta=sk().BF16, tc=sk().F32, policy=policy)
    info = p.info()
    tr = torch.full((max(p.trace_capacity(), 1) * 8,), -7, dtype=torch.int32, device=dev())
    sk().grouped_matmul(As, Bs, Cs, alpha=1.5, beta=0.5, policy=policy, trace=tr)
    torch.cuda.synchronize()
    for (M, N, K), A, B, C, C0 in zip(probs, As, Bs, Cs, Cin):
        if M * N == 0:
            continue
        if K == 0:
            assert np.array_equal(to_f64(C), np.float32(0.5) * to_f64(C0).astype(np.float32)), (M, N)
        else:
            ref = og.gemm_f64(to_f64(A), to_f64(B), 1.5, 0.5, to_f64(C0))
            assert og.rel_frobenius(to_f64(C), ref) <= 1e-5, (M, N, K)
    recs = [tuple(int(v) for v in r) for r in tr.cpu().numpy().reshape(-1, 8) if r[0] != -7]
    got = records_to_schedule(recs, info["grid"])
    ref = oracle_grouped_plan_for(probs, info, p.model_constants(), policy)
    assert got == GR.enumerate_grouped_schedule(ref)
