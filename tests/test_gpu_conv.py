"""Implicit-GEMM convolution through the C ABI against the float64 convolution
oracle (the definition, tap by tap).

Tolerances as for the GEMM: relative Frobenius error 1e-5 with FP32 output
(accumulation only), 1e-2 with 16-bit output (includes the output rounding).
Integer-valued inputs are exact in FP32 accumulation and fix-up: bit-identical
under every policy and grid.  The schedule trace of a convolution equals the
oracle enumerator's schedule of its GEMM view.
"""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import oracle_plan_for, records_to_schedule, to_f64
from oracle import conv as oc
from oracle import gemm as og
from oracle import schedule as S

pytestmark = pytest.mark.gpu

TOL_OUT32 = 1e-5
TOL_16 = 1e-2
TILES = [(256, 256, 64), (128, 128, 64, 4), (256, 64, 64)]

CASES = [
    # n, h, w, c, k, r, s, pad, stride, dilation
    (2, 14, 14, 64, 96, 3, 3, (1, 1), (1, 1), (1, 1)),
    (3, 17, 11, 128, 200, 3, 3, (1, 1), (2, 2), (1, 1)),
    (1, 9, 13, 64, 64, 3, 3, (2, 2), (1, 1), (2, 2)),
    (4, 7, 7, 256, 130, 1, 1, (0, 0), (1, 1), (1, 1)),
    (2, 23, 23, 64, 64, 7, 7, (3, 3), (2, 2), (1, 1)),
    (1, 5, 8, 192, 33, 2, 3, (0, 1), (1, 2), (1, 1)),
    (5, 12, 12, 64, 300, 3, 3, (0, 0), (1, 1), (1, 1)),
    (3, 15, 13, 128, 40, 3, 3, (1, 1), (1, 1), (1, 1)),        # fewer than 64 output channels: the tall tile
]


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def dev():
    return torch.device("cuda:0")


def inputs(case, dtype, seed, integer=False):
    n, h, w, c, k, r, s = case[:7]
    g = W.rng(seed)
    make = W.integer_f32 if integer else W.normal_f32
    x = torch.from_numpy(make(g, (n, h, w, c))).to(dtype).to(dev())
    f = torch.from_numpy(make(g, (k, r, s, c))).to(dtype).to(dev())
    return x, f


def conv(x, f, case, **kw):
    pad, std, dil = case[7:]
    y = sk().conv2d(x, f, padding=pad, stride=std, dilation=dil, **kw)
    torch.cuda.synchronize()
    return y


def oracle(x, f, case, alpha=1.0, beta=0.0, y=None):
    pad, std, dil = case[7:]
    return oc.conv2d_f64(to_f64(x), to_f64(f), pad, std, dil, alpha, beta, None if y is None else to_f64(y))


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("case", CASES)
def test_conv_parity(case, dtype):
    x, f = inputs(case, dtype, seed=sum(case[:7]))
    ref = oracle(x, f, case)
    for tile in [None] + TILES:
        for pol in ("auto", "dp", "sk"):
            y32 = conv(x, f, case, out_dtype=torch.float32, policy=pol, tile=tile)
            assert y32.shape == ref.shape
            assert og.rel_frobenius(to_f64(y32), ref) <= TOL_OUT32, (tile, pol, "f32 out")
            y16 = conv(x, f, case, policy=pol, tile=tile)
            assert y16.dtype == dtype
            assert og.rel_frobenius(to_f64(y16), ref) <= TOL_16, (tile, pol, "16-bit out")


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[4], CASES[7]])
def test_conv_integer_exact_every_policy(case, tile):
    """Padding, stride and dilation cases with ragged M and N edges: every
    policy and a range of Stream-K grids give the oracle's exact result."""
    x, f = inputs(case, torch.bfloat16, seed=7, integer=True)
    ref = oracle(x, f, case)
    for pol in ["auto", "paper", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"]:
        for fg in ([0] if pol != "sk" else [0, 3, 17, 100, 256]):
            try:
                y = conv(x, f, case, out_dtype=torch.float32, policy=pol, force_g=fg, tile=tile)
            except sk().SkgemmError as e:
                assert fg > 0 and e.status == sk().ERR_CAPACITY, (pol, fg, e)
                continue
            assert np.array_equal(to_f64(y), ref), (pol, fg)


@pytest.mark.parametrize("policy,g", [("sk", 0), ("sk", 37), ("dp", 0), ("dp_1tile_sk", 0), ("2tile_sk_dp", 0)])
@pytest.mark.parametrize("tile", TILES)
def test_conv_trace_matches_enumerator(policy, g, tile):
    case = CASES[1]
    x, f = inputs(case, torch.bfloat16, seed=11)
    n, h, w, c, k, r, s, pad, std, dil = case
    plan = sk().ConvPlan(n, h, w, c, k, r, s, pad, std, dil, ta=sk().BF16, tc=sk().F32, policy=policy, force_g=g,
                         tile=tile)
    info = plan.info()
    tr = torch.full((plan.trace_capacity() * 8,), -7, dtype=torch.int32, device=dev())
    y = conv(x, f, case, out_dtype=torch.float32, policy=policy, force_g=g, tile=tile, trace=tr)
    recs = [tuple(int(v) for v in rec) for rec in tr.cpu().numpy().reshape(-1, 8) if rec[0] != -7]
    ref_plan = oracle_plan_for(info, plan.model_constants(), policy, force_g=g)
    assert records_to_schedule(recs, info["grid"]) == S.enumerate_schedule(ref_plan)
    assert og.rel_frobenius(to_f64(y), oracle(x, f, case)) <= TOL_OUT32


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_conv_alpha_beta(dtype):
    case = CASES[0]
    x, f = inputs(case, dtype, seed=5)
    pad, std, dil = case[7:]
    P, Q = oc.out_size(*case[1:3], *case[5:7], *pad, *std, *dil)
    g = W.rng(6)
    y0 = torch.from_numpy(W.normal_f32(g, (case[0], P, Q, case[4]))).to(dev())
    for pol in ("dp", "sk"):
        y = y0.clone()
        conv(x, f, case, out=y, alpha=-0.75, beta=1.5, policy=pol)
        assert og.rel_frobenius(to_f64(y), oracle(x, f, case, -0.75, 1.5, y0)) <= TOL_OUT32, pol
    # 16-bit output with beta reads the 16-bit y
    y16 = y0.to(dtype)
    yin = y16.clone()
    conv(x, f, case, out=y16, alpha=2.0, beta=-1.0, policy="sk")
    assert og.rel_frobenius(to_f64(y16), oracle(x, f, case, 2.0, -1.0, yin)) <= TOL_16


def test_conv_empty_batch_and_argument_checks():
    x = torch.zeros((0, 8, 8, 64), dtype=torch.bfloat16, device=dev())
    f = torch.zeros((32, 3, 3, 64), dtype=torch.bfloat16, device=dev())
    y = sk().conv2d(x, f, padding=(1, 1))
    assert y.shape == (0, 8, 8, 32)
    x = torch.zeros((1, 8, 8, 96), dtype=torch.bfloat16, device=dev())
    f = torch.zeros((32, 3, 3, 96), dtype=torch.bfloat16, device=dev())
    with pytest.raises(sk().SkgemmError) as e:
        sk().conv2d(x, f)
    assert e.value.status == sk().ERR_UNSUPPORTED


def test_conv_narrow_layer_takes_the_tall_tile():
    """ResNet-50's first-stage 3x3 convolution (64 output channels, 100352
    output pixels) plans on the tall tile; a small narrow case runs its
    automatic plan against the oracle."""
    assert sk().ConvPlan(32, 56, 56, 64, 64, 3, 3, (1, 1), ta=sk().BF16).info()["tile"] == (256, 64, 64, 4)
    case = CASES[7]
    x, f = inputs(case, torch.bfloat16, seed=12)
    y = conv(x, f, case, out_dtype=torch.float32)
    assert og.rel_frobenius(to_f64(y), oracle(x, f, case)) <= TOL_OUT32


def test_conv_resnet_layer_sampled_images():
    """A ResNet-50 stage-1 3x3 convolution at batch 64 (M = 200704 output
    pixels, N = 64, K = 576), in the launch the planner picks: images are
    independent, so sampled images are checked against the oracle run on those
    images alone."""
    case = (64, 56, 56, 64, 64, 3, 3, (1, 1), (1, 1), (1, 1))
    x, f = inputs(case, torch.bfloat16, seed=3)
    y = conv(x, f, case, out_dtype=torch.float32)
    for i in (0, 37, 63):
        ref = oracle(x[i:i + 1], f, case)
        assert og.rel_frobenius(to_f64(y[i:i + 1]), ref) <= TOL_OUT32, i


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[2], CASES[6]])
def test_conv_three_stage_tile_bitwise_and_exact(case):
    """Convolution plans of the 128x128 tile whose grid fits one workgroup per
    CU run the eight-wave three-stage kernel with the gather: bitwise the
    four-wave kernel's result on the same schedule, and exact on
    integer-valued inputs."""
    from helpers import resolved
    n, h, w, c, k, r, s, pad, std, dil = case
    found = 0
    for pol in ("auto", "dp", "sk"):
        plan = sk().ConvPlan(n, h, w, c, k, r, s, pad, std, dil, ta=sk().BF16, tc=sk().F32, policy=pol,
                             tile=(128, 128, 64))
        info = plan.info()
        if info["stages"] != 3:
            continue
        found += 1
        p4, g4 = resolved(info)
        for integer in (False, True):
            x, f = inputs(case, torch.bfloat16, seed=21, integer=integer)
            y8 = conv(x, f, case, out_dtype=torch.float32, policy=p4, force_g=g4, tile=(128, 128, 64))
            y4 = conv(x, f, case, out_dtype=torch.float32, policy=p4, force_g=g4, tile=(128, 128, 64, 4))
            assert torch.equal(y8, y4), (case, pol, integer)
            if integer:
                assert np.array_equal(to_f64(y8), oracle(x, f, case)), (case, pol)
    assert found >= 1
