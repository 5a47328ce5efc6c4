"""GPU parity of the Stream-K GEMM against the FP64 oracle (through the C ABI).

Tolerances (relative Frobenius error against the float64 oracle of the stored
inputs): FP32 1e-5; BF16/FP16 inputs with FP32 output 1e-5 (accumulation
only); BF16/FP16 output 1e-2 (includes the output rounding).  Integer-valued
inputs are exact in FP32 accumulation and fix-up, so those results must be
bit-identical to the oracle under every policy and grid size.
"""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import oracle_plan_for, records_to_schedule, to_f64
from oracle import gemm as og
from oracle import schedule as S

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_16_OUT32 = 1e-5
TOL_16 = 1e-2

POLICIES = ["auto", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"]
# the two 16-bit tile configurations (the planner picks one per problem; tests pin each)
TILES16 = [(256, 256, 64), (128, 128, 64, 4), (128, 128, 64, 8)]


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def dev():
    return torch.device("cuda:0")


def mm(A, B, **kw):
    out = sk().matmul(A, B, **kw)
    torch.cuda.synchronize()
    return out


def oracle(A, B, alpha=1.0, beta=0.0, C=None):
    Cin = to_f64(C) if C is not None else None
    return og.gemm_f64(to_f64(A), to_f64(B), alpha, beta, Cin)


def rel(x, ref):
    return og.rel_frobenius(to_f64(x), ref)


# ------------------------------------------------------------------ FP32 quantisation case

def test_plain_f32_all_policies():
    a, b = W.plain_f32(seed=0)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    ref = og.gemm_f64(a, b)
    bound = (384 * 2.0 ** -24) * (np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)) * 1.01
    for pol in POLICIES:
        C = mm(A, B, policy=pol)
        assert rel(C, ref) <= TOL_F32, pol
        assert np.all(np.abs(to_f64(C) - ref) <= bound * (1024 / 384)), pol


def _capacity(M, N, K, ta):
    return sk().Plan(M, N, K, ta=ta, tc=ta if ta != sk().BF16 else sk().F32, policy="dp").info()["p"]


@pytest.mark.parametrize("g", [1, 2, 9, 16, 36, 64, 100, 200, 256, 288, 500])
def test_integer_f32_bit_exact_every_grid(g):
    """g up to the co-resident capacity p; a g above the 288 iterations is
    reduced to one workgroup per iteration."""
    if g > _capacity(384, 384, 1024, sk().F32):
        pytest.skip("grid larger than the co-resident capacity of this GPU")
    a, b = W.plain_f32(seed=0, integer=True)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    ref = og.gemm_f64(a, b)
    C = mm(A, B, policy="sk", force_g=g)
    assert np.array_equal(to_f64(C), ref)


def test_capacity_refused_beyond_resident():
    p = _capacity(384, 384, 8192, sk().F32)
    with pytest.raises(sk().SkgemmError) as e:
        sk().Plan(384, 384, 8192, ta=sk().F32, policy="sk", force_g=p + 1)   # 2304 iterations > p + 1
    assert e.value.status == sk().ERR_CAPACITY


def test_integer_f32_bit_exact_every_policy():
    a, b = W.plain_f32(seed=0, integer=True)
    A = torch.from_numpy(a).to(dev())
    B = torch.from_numpy(b).to(dev())
    ref = og.gemm_f64(a, b)
    for pol in POLICIES:
        assert np.array_equal(to_f64(mm(A, B, policy=pol)), ref), pol


# ------------------------------------------------------------------ schedule parity

def _trace(A, B, policy, force_g=0, out_dtype=None, tile=None):
    p = sk().get_plan(A.shape[0], B.shape[1], A.shape[1], 0, 0, 0, sk()._torch_dtypes()[A.dtype],
                      sk()._torch_dtypes()[out_dtype or A.dtype], policy, force_g, 2, tile)
    cap = p.trace_capacity()
    tr = torch.full((max(cap, 1) * 8,), -7, dtype=torch.int32, device=dev())
    mm(A, B, policy=policy, force_g=force_g, trace=tr, out_dtype=out_dtype, tile=tile)
    recs = tr.cpu().numpy().reshape(-1, 8)
    info = p.info()
    recs = [tuple(int(v) for v in r) for r in recs if r[0] != -7]
    return p, info, recs


@pytest.mark.parametrize("shape,policy,g", [
    ((384, 384, 1024), "auto", 0), ((384, 384, 1024), "sk", 4), ((384, 384, 1024), "sk", 36),
    ((384, 384, 1024), "sk", 200), ((896, 384, 128), "sk", 4), ((896, 384, 128), "2tile_sk_dp", 0),
    ((2000, 1500, 333), "dp_1tile_sk", 0), ((2000, 1500, 333), "2tile_sk_dp", 0), ((128, 128, 4096), "sk", 0),
])
def test_trace_matches_enumerator_f32(shape, policy, g):
    M, N, K = shape
    g_ = W.rng(1)
    A = torch.from_numpy(W.integer_f32(g_, (M, K))).to(dev())
    B = torch.from_numpy(W.integer_f32(g_, (K, N))).to(dev())
    p, info, recs = _trace(A, B, policy, g)
    got = records_to_schedule(recs, info["grid"])
    ref = oracle_plan_for(info, p.model_constants(), policy, force_g=g)
    assert got == S.enumerate_schedule(ref)


@pytest.mark.parametrize("shape,policy", [((256 * 5 + 7, 256 * 3, 1000), "auto"), ((4096, 4096, 512), "auto"),
                                          ((300, 3000, 2000), "sk"), ((256 * 17, 256 * 16, 256), "auto"),
                                          ((128 * 9 + 5, 128 * 7, 1000), "2tile_sk_dp")])
@pytest.mark.parametrize("tile", TILES16)
def test_trace_matches_enumerator_bf16(shape, policy, tile):
    M, N, K = shape
    A = torch.ones((M, K), dtype=torch.bfloat16, device=dev())
    B = torch.ones((K, N), dtype=torch.bfloat16, device=dev())
    p, info, recs = _trace(A, B, policy, 0, out_dtype=torch.float32, tile=tile)
    assert info["tile"][:len(tile)] == tuple(tile)
    got = records_to_schedule(recs, info["grid"])
    ref = oracle_plan_for(info, p.model_constants(), policy)
    assert got == S.enumerate_schedule(ref)


# ------------------------------------------------------------------ 16-bit inputs

SHAPES16 = [(1, 1, 1), (3, 5, 7), (256, 256, 32), (256, 256, 64), (257, 255, 65), (300, 500, 700), (513, 1031, 129),
            (1000, 130, 5), (64, 3000, 2048), (640, 768, 4099),
            # rows shorter than a 16-byte chunk, and just longer, over many k-slabs
            (300, 7, 1000), (70, 9, 1030), (7, 300, 1000),
            # K a multiple of the k-slab (no K tail) with M and N edges
            (129, 4100, 64), (200, 260, 640)]


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("shape", SHAPES16)
def test_16bit_parity(dtype, shape):
    M, N, K = shape
    a, b = W.normal_pair(M, N, K, seed=M + N + K)
    A = torch.from_numpy(a).to(dtype).to(dev())
    B = torch.from_numpy(b).to(dtype).to(dev())
    ref = oracle(A, B)
    for tile in [None] + TILES16:
        for pol in ("auto", "dp", "sk"):
            C32 = mm(A, B, policy=pol, out_dtype=torch.float32, tile=tile)
            assert rel(C32, ref) <= TOL_16_OUT32, (tile, pol, "f32 out")
            C16 = mm(A, B, policy=pol, tile=tile)
            assert C16.dtype == dtype
            assert rel(C16, ref) <= TOL_16, (tile, pol, "16-bit out")


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("tile", TILES16)
def test_16bit_integer_exact_all_policies(dtype, tile):
    M, N, K = 700, 900, 1500
    g = W.rng(3)
    A = torch.from_numpy(W.integer_f32(g, (M, K))).to(dtype).to(dev())
    B = torch.from_numpy(W.integer_f32(g, (K, N))).to(dtype).to(dev())
    ref = oracle(A, B)
    for pol in POLICIES:
        for fg in ([0] if pol != "sk" else [0, 5, 17, 200, 400]):
            try:
                C = mm(A, B, policy=pol, force_g=fg, out_dtype=torch.float32, tile=tile)
            except sk().SkgemmError as e:
                # a forced grid beyond the co-resident capacity of this tile is refused, never run
                assert fg > 0 and e.status == sk().ERR_CAPACITY, (pol, fg, e)
                continue
            assert np.array_equal(to_f64(C), ref), (pol, fg)


@pytest.mark.parametrize("layouts", ["nn", "nt", "tn", "tt"])
@pytest.mark.parametrize("c_col", [False, True])
@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, "bf16_small"])
def test_layouts(layouts, c_col, dtype):
    tile = None
    if dtype == "bf16_small":
        dtype, tile = torch.bfloat16, (128, 128, 64)
    M, N, K = 333, 517, 290
    a, b = W.normal_pair(M, N, K, seed=11)
    A = torch.from_numpy(a).to(dtype).to(dev())
    B = torch.from_numpy(b).to(dtype).to(dev())
    if layouts[0] == "t":
        A = A.t().contiguous().t()      # column-major view of the same values
    if layouts[1] == "t":
        B = B.t().contiguous().t()
    ref = oracle(A, B)
    odt = torch.float32
    out = torch.empty((N, M), dtype=odt, device=dev()).t() if c_col else torch.empty((M, N), dtype=odt, device=dev())
    for pol in ("auto", "sk", "dp"):
        C = mm(A, B, out=out, policy=pol, tile=tile)
        tol = TOL_F32 if dtype == torch.float32 else TOL_16_OUT32
        assert rel(C, ref) <= tol, (layouts, c_col, pol)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, "bf16_small"])
def test_alpha_beta_and_nan_c(dtype):
    tile = None
    if dtype == "bf16_small":
        dtype, tile = torch.bfloat16, (128, 128, 64)
    M, N, K = 260, 300, 500
    a, b = W.normal_pair(M, N, K, seed=5)
    A = torch.from_numpy(a).to(dtype).to(dev())
    B = torch.from_numpy(b).to(dtype).to(dev())
    c0 = torch.from_numpy(W.normal_f32(W.rng(6), (M, N))).to(dtype).to(dev())
    ref = oracle(A, B, alpha=0.5, beta=-2.0, C=c0)
    for pol in ("sk", "dp", "auto"):
        C = c0.clone()
        mm(A, B, out=C, alpha=0.5, beta=-2.0, policy=pol, tile=tile)
        tol = TOL_F32 if dtype == torch.float32 else TOL_16
        assert rel(C, ref) <= tol, pol
        Cn = torch.full((M, N), float("nan"), dtype=dtype, device=dev())
        mm(A, B, out=Cn, alpha=1.0, beta=0.0, policy=pol, tile=tile)
        assert not torch.isnan(Cn).any(), pol


def test_k_zero_and_empty():
    A = torch.zeros((100, 0), dtype=torch.bfloat16, device=dev())
    B = torch.zeros((0, 70), dtype=torch.bfloat16, device=dev())
    C = torch.full((100, 70), 3.0, dtype=torch.bfloat16, device=dev())
    mm(A, B, out=C, beta=0.5)
    assert torch.all(C.float() == 1.5)
    mm(A, B, out=C, beta=0.0)
    assert torch.all(C.float() == 0.0)
    E = torch.empty((0, 16), dtype=torch.bfloat16, device=dev())
    F = torch.ones((16, 5), dtype=torch.bfloat16, device=dev())
    assert mm(E, F).shape == (0, 5)


@pytest.mark.parametrize("tile", TILES16)
def test_determinism_repeated_runs(tile):
    M, N, K = 1000, 1000, 3000
    a, b = W.normal_pair(M, N, K, seed=9)
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    first = mm(A, B, policy="sk", out_dtype=torch.float32, tile=tile).clone()
    for _ in range(20):
        assert torch.equal(mm(A, B, policy="sk", out_dtype=torch.float32, tile=tile), first)


def test_full_size_sampled_rows_bf16():
    """The benchmark's largest shape (8192^3, bf16, auto policy) on sampled rows."""
    M = N = K = 8192
    g = torch.Generator(device="cpu").manual_seed(0)
    A = torch.randn((M, K), generator=g, dtype=torch.float32).to(torch.bfloat16).to(dev())
    B = torch.randn((K, N), generator=g, dtype=torch.float32).to(torch.bfloat16).to(dev())
    C = mm(A, B)
    rows = np.array([0, 1, 255, 256, 4095, 8191])
    ref = og.gemm_rows_f64(to_f64(A), to_f64(B), rows)
    assert og.rel_frobenius(to_f64(C[torch.from_numpy(rows).to(dev())]), ref) <= TOL_16


# ------------------------------------------------------------------ split fix-up

# (M, N, K, dtype, tile, policy, s): g = s * (Stream-K tiles) with s at most the
# iterations per tile, so the plan reduces each tile with the split fix-up
# (shares of floor / ceil length where s does not divide them); s >= 3 has
# contributors that only store
SPLIT_CASES = [
    (1024, 1024, 1024, torch.bfloat16, (128, 128, 64), "sk", 2),
    (1024, 1024, 1024, torch.bfloat16, (128, 128, 64), "sk", 3),
    (600, 520, 640, torch.float16, (256, 256, 64), "sk", 3),
    (640, 768, 4096, torch.bfloat16, (128, 128, 64), "sk", 7),
    (1000, 1030, 1024, torch.bfloat16, (128, 128, 64), "sk", 4),
    (300, 500, 768, torch.bfloat16, (128, 128, 64), "sk", 3),
    (300, 500, 768, torch.float16, (128, 128, 64), "sk", 12),
    (512, 512, 1536, torch.bfloat16, (256, 256, 64), "sk", 3),
    (600, 520, 640, torch.bfloat16, (256, 256, 64), "sk", 5),
    (384, 384, 1024, torch.float32, None, "sk", 4),
    (384, 384, 1024, torch.float32, None, "sk", 16),
    (2560, 3328, 1024, torch.bfloat16, (128, 128, 64), "dp_1tile_sk", 4),
]


def _split_plan(M, N, K, dtype, tile, policy, s, fixup, out_dtype):
    dts = sk()._torch_dtypes()
    probe = sk().get_plan(M, N, K, 0, 0, 0, dts[dtype], dts[out_dtype], "dp", 0, 2, tile)
    info = probe.info()
    t, p = info["t"], info["p"]
    sk_tiles = t if policy == "sk" else t % p
    return s * sk_tiles, sk().get_plan(M, N, K, 0, 0, 0, dts[dtype], dts[out_dtype], policy, s * sk_tiles, 2,
                                       tile, fixup)


@pytest.mark.parametrize("case", SPLIT_CASES)
def test_split_fixup_bitwise_equals_owner_fixup(case):
    M, N, K, dtype, tile, policy, s = case
    a, b = W.normal_pair(M, N, K, seed=M + N + s)
    A = torch.from_numpy(a).to(dtype).to(dev())
    B = torch.from_numpy(b).to(dtype).to(dev())
    c0 = torch.from_numpy(W.normal_f32(W.rng(s), (M, N))).to(dev())
    for out_dtype in ([torch.float32] if dtype == torch.float32 else [torch.float32, dtype]):
        g, plan = _split_plan(M, N, K, dtype, tile, policy, s, "auto", out_dtype)
        if g > plan.info()["p"] or plan.info()["coop_s"] != s:
            pytest.skip("this GPU's co-resident capacity gives another plan")
        _, owner = _split_plan(M, N, K, dtype, tile, policy, s, "owner", out_dtype)
        assert owner.info()["coop_s"] == 0
        got = {}
        for fx in ("auto", "owner"):
            C = c0.to(out_dtype).clone()
            mm(A, B, out=C, alpha=0.75, beta=0.5, policy=policy, force_g=g, tile=tile, fixup=fx)
            got[fx] = C
        assert torch.equal(got["auto"], got["owner"]), (case, out_dtype)
        tol = TOL_F32 if out_dtype == torch.float32 else TOL_16
        assert rel(got["auto"], oracle(A, B, alpha=0.75, beta=0.5, C=c0.to(out_dtype))) <= tol, (case, out_dtype)


@pytest.mark.parametrize("s", [2, 3, 5, 6])
def test_split_fixup_integer_exact(s):
    M, N, K = 700, 900, 1536
    g = W.rng(40 + s)
    A = torch.from_numpy(W.integer_f32(g, (M, K))).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(W.integer_f32(g, (K, N))).to(torch.bfloat16).to(dev())
    ref = oracle(A, B)
    gs, plan = _split_plan(M, N, K, torch.bfloat16, (128, 128, 64), "sk", s, "auto", torch.float32)
    if gs > plan.info()["p"] or plan.info()["coop_s"] != s:
        pytest.skip("this GPU's co-resident capacity gives another plan")
    for _ in range(3):        # flags are self-cleaning: repeated runs on one workspace
        C = mm(A, B, policy="sk", force_g=gs, out_dtype=torch.float32, tile=(128, 128, 64))
        assert np.array_equal(to_f64(C), ref)


def test_shared_workspace_across_grids():
    """One workspace serves plans with small and large Stream-K grids in turn:
    the partial tiles of a small-grid plan never land on a large-grid plan's
    flags (the flag area has a fixed place)."""
    cases = [(300, 500, 768, 36), (128, 4096, 8192, 256), (300, 500, 768, 144), (128, 4096, 8192, 128)]
    ws = torch.zeros(64 << 20, dtype=torch.uint8, device=dev())
    tile = (128, 128, 64)
    for rep in range(2):
        for (M, N, K, g) in cases:
            a, b = W.normal_pair(M, N, K, seed=M + g)
            A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
            B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
            plan = sk().Plan(M, N, K, ta=sk().BF16, tc=sk().F32, policy="sk", force_g=g, tile=tile)
            nws = plan.workspace_size()
            assert nws <= ws.numel()
            C = torch.empty((M, N), dtype=torch.float32, device=dev())
            stream = torch.cuda.current_stream().cuda_stream
            plan.run(A.data_ptr(), K, B.data_ptr(), N, C.data_ptr(), N, 1.0, 0.0, None, None, ws.data_ptr(), nws,
                     stream=stream)
            sk().check_device_error(ws.data_ptr(), stream)
            assert rel(C, oracle(A, B)) <= TOL_16_OUT32, (rep, M, N, K, g)


@pytest.mark.parametrize("fixup", ["auto", "owner"])
def test_determinism_under_concurrent_noise(fixup):
    """100 runs of one split plan, each beside elementwise kernels on another
    stream (the fix-up waits and the order partials arrive in change from run to
    run): C is bitwise identical every time.  The grid (2 shares x 64 tiles)
    leaves room on the GPU for the other stream's work."""
    M, N, K = 1024, 1024, 2048
    a, b = W.normal_pair(M, N, K, seed=31)
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    tile = (128, 128, 64)
    first = mm(A, B, policy="sk", force_g=128, out_dtype=torch.float32, tile=tile, fixup=fixup).clone()
    noise_stream = torch.cuda.Stream()
    X = torch.randn((2048, 2048), device=dev())
    noise_stream.wait_stream(torch.cuda.current_stream())
    for it in range(100):
        with torch.cuda.stream(noise_stream):
            for _ in range(1 + it % 3):
                X = X * 0.999 + 0.001
        C = sk().matmul(A, B, policy="sk", force_g=128, out_dtype=torch.float32, tile=tile, fixup=fixup)
        torch.cuda.synchronize()
        assert torch.equal(C, first), it
    assert og.rel_frobenius(to_f64(first), oracle(A, B)) <= TOL_16_OUT32


def test_sweep_sample_as_benchmarked():
    """Every 20th shape of the BF16 sweep the benchmark times (bf16 in and out,
    row-major, automatic policy, the planner's tile), on sampled rows against
    the FP64 oracle; the plans cover data-parallel, split and hybrid cases on
    both the two- and the three-stage kernels."""
    shapes = W.sweep_shapes(1000, seed=0)[::20]
    gen = torch.Generator(device="cpu").manual_seed(0)
    seen = set()
    stages = set()
    for (M, N, K) in shapes:
        A = torch.randn((M, K), generator=gen).to(torch.bfloat16).to(dev())
        B = torch.randn((K, N), generator=gen).to(torch.bfloat16).to(dev())
        C = mm(A, B)
        assert C.dtype == torch.bfloat16
        info = sk().get_plan(M, N, K, 0, 0, 0, sk().BF16, sk().BF16, "auto", 0, 2, None).info()
        seen.add((info["policy_name"], info["coop_s"] > 0))
        stages.add(info["stages"])
        rows = np.unique(np.random.default_rng(M + N + K).integers(0, M, 6))
        ref = og.gemm_rows_f64(to_f64(A), to_f64(B), rows)
        got = to_f64(C[torch.from_numpy(rows).to(dev())])
        assert og.rel_frobenius(got, ref) <= TOL_16, (M, N, K, info["policy_name"])
    assert ("sk", True) in seen and ("dp", False) in seen
    assert stages == {2, 3}


@pytest.mark.parametrize("fixup", ["auto", "owner"])
def test_fixup_wait_timeout_reported_and_recovered(fixup):
    """The error path of the bounded fix-up waits, forced from the host with a
    spin limit of one poll: every kernel still exits, skgemm_check_device_error
    reports the timeout, and once the workspace is zero-filled again a plan
    with the default limit gives the exact result in the same workspace."""
    M, N, K = 1000, 700, 900
    g = W.rng(31)
    a = W.integer_f32(g, (M, K))
    b = W.integer_f32(g, (K, N))
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    ref = og.gemm_f64(a.astype(np.float64), b.astype(np.float64))
    tile = (256, 256, 64)
    t = sk().Plan(M, N, K, ta=sk().BF16, tc=sk().F32, policy="dp", tile=tile).info()["t"]
    kw = dict(ta=sk().BF16, tc=sk().F32, policy="sk", force_g=3 * t, tile=tile, fixup=fixup)
    bad = sk().Plan(M, N, K, spin_limit=1, **kw)
    good = sk().Plan(M, N, K, **kw)
    nb = max(bad.workspace_size(), good.workspace_size())
    ws = torch.zeros(nb, dtype=torch.uint8, device=dev())
    C = torch.empty((M, N), dtype=torch.float32, device=dev())
    args = (A.data_ptr(), K, B.data_ptr(), N, C.data_ptr(), N, 1.0, 0.0, None, None, ws.data_ptr(), nb)
    seen = 0
    for _ in range(3):
        bad.run(*args)
        torch.cuda.synchronize()
        try:
            sk().check_device_error(ws.data_ptr())
        except sk().SkgemmError as e:
            assert e.status == sk().ERR_TIMEOUT
            seen += 1
        ws.zero_()
    assert seen > 0
    good.run(*args)
    torch.cuda.synchronize()
    sk().check_device_error(ws.data_ptr())
    assert np.array_equal(C.cpu().numpy().astype(np.float64), ref)


def test_occupancy_per_dtype_and_tile_is_sane_and_stable():
    """The library's per-device occupancy cache holds one entry per input type
    and tile: every entry is a plausible workgroup count, planning one type
    leaves the others' entries alone, and the plan's capacity is CUs times it."""
    cases = [(sk().F32, None), (sk().BF16, (256, 256, 64)), (sk().BF16, (128, 128, 64, 4)),
             (sk().BF16, (128, 128, 64, 8)), (sk().F16, (256, 256, 64)), (sk().F64, (64, 64, 16)),
             (sk().F64, (128, 128, 16))]
    tc = {sk().F32: sk().F32, sk().BF16: sk().BF16, sk().F16: sk().F16, sk().F64: sk().F64}

    def occ(ta, tile):
        info = sk().Plan(512, 512, 512, ta=ta, tc=tc[ta], policy="dp", tile=tile).info()
        assert info["p"] % info["occupancy"] == 0
        return info["occupancy"]

    first = [occ(ta, tile) for ta, tile in cases]
    assert all(1 <= o <= 8 for o in first), first
    assert [occ(ta, tile) for ta, tile in reversed(cases)][::-1] == first
    # FP8 (both operands K-contiguous)
    for tile in [(256, 256, 128), (128, 128, 128)]:
        info = sk().Plan(512, 512, 512, 0, 1, 0, sk().F8E4M3, sk().F32, policy="dp", tile=tile).info()
        assert 1 <= info["occupancy"] <= 8
    assert [occ(ta, tile) for ta, tile in cases] == first


@pytest.mark.parametrize("fixup", ["auto", "owner"])
def test_matmul_reports_timeout_and_clears_its_workspace(fixup):
    """Through the torch layer: with a one-poll spin limit a fix-up wait
    expires, matmul(check=True) raises ERR_TIMEOUT and leaves its cached
    workspace zero-filled, so the next run (default limit) is exact."""
    M, N, K = 1000, 700, 900
    g = W.rng(37)
    a = W.integer_f32(g, (M, K))
    b = W.integer_f32(g, (K, N))
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    ref = og.gemm_f64(a.astype(np.float64), b.astype(np.float64))
    tile = (256, 256, 64)
    t = sk().Plan(M, N, K, ta=sk().BF16, tc=sk().F32, policy="dp", tile=tile).info()["t"]
    kw = dict(policy="sk", force_g=3 * t, tile=tile, fixup=fixup, out_dtype=torch.float32)
    seen = 0
    for _ in range(3):
        try:
            sk().matmul(A, B, spin_limit=1, check=True, **kw)
        except sk().SkgemmError as e:
            assert e.status == sk().ERR_TIMEOUT
            seen += 1
    assert seen > 0
    stream = torch.cuda.current_stream().cuda_stream
    ws = sk()._ws_cache[(dev().index, stream)]
    assert int(ws.count_nonzero().item()) == 0 or seen < 3
    C = sk().matmul(A, B, check=True, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(to_f64(C), ref)


def test_workspaces_are_per_stream():
    """Runs on two streams use two workspaces (their flags and partials must
    not meet); each stream's results match the oracle."""
    M, N, K = 700, 900, 2048
    a, b = W.normal_pair(M, N, K, seed=41)
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    ref = oracle(A, B)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for s in (s1, s2):
        s.wait_stream(torch.cuda.current_stream())
    for it in range(10):
        for s in (s1, s2):
            with torch.cuda.stream(s):
                outs.append(sk().matmul(A, B, policy="sk", out_dtype=torch.float32, tile=(128, 128, 64, 4)))
    torch.cuda.synchronize()
    k1 = (dev().index, s1.cuda_stream)
    k2 = (dev().index, s2.cuda_stream)
    assert sk()._ws_cache[k1].data_ptr() != sk()._ws_cache[k2].data_ptr()
    for C in outs:
        assert rel(C, ref) <= TOL_16_OUT32


def test_graph_keeps_its_workspace_when_an_eager_run_outgrows_it():
    """A grouped launch captured in a HIP graph holds its stream's workspace;
    an eager run on that stream that needs a larger one replaces it in the
    cache, and the graph's replays (which still use the old one) stay equal
    to the eager result."""
    Ms, N, K = [300, 200, 100], 512, 1024
    As = [torch.randn((m, K), device=dev()).to(torch.bfloat16) for m in Ms]
    Bs = [torch.randn((K, N), device=dev()).to(torch.bfloat16) for _ in Ms]
    S_ = torch.cuda.Stream()
    S_.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(S_):
        Cs = [torch.empty((m, N), dtype=torch.float32, device=dev()) for m in Ms]
        _, table = sk().grouped_matmul(As, Bs, Cs, policy="sk", force_g=6)
        want = [C.clone() for C in Cs]
    torch.cuda.synchronize()
    key = (dev().index, S_.cuda_stream)
    old = sk()._ws_cache[key]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=S_):
        sk().grouped_matmul(As, Bs, Cs, policy="sk", force_g=6, table=table)
    # an eager run on the same stream with a much larger Stream-K grid
    M2, N2, K2 = 2048, 2048, 4096
    A2 = torch.randn((M2, K2), device=dev()).to(torch.bfloat16)
    B2 = torch.randn((K2, N2), device=dev()).to(torch.bfloat16)
    torch.cuda.synchronize()
    with torch.cuda.stream(S_):
        C2 = sk().matmul(A2, B2, policy="sk", force_g=128, tile=(256, 256, 64), out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert sk()._ws_cache[key].data_ptr() != old.data_ptr()
    assert any(r is old for r in sk()._ws_retired)
    for rep in range(4):
        for C in Cs:
            C.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for C, w in zip(Cs, want):
            assert torch.equal(C, w), rep
    rows = np.arange(0, M2, 97)
    ref = og.gemm_rows_f64(to_f64(A2), to_f64(B2), rows)
    assert og.rel_frobenius(to_f64(C2[torch.from_numpy(rows).to(dev())]), ref) <= TOL_16_OUT32


@pytest.mark.parametrize("shape,policy,g,fixup", [((1024, 1024, 1024), "sk", 0, "auto"),
                                                   ((384, 384, 1024), "sk", 36, "owner"),
                                                   ((2000, 1500, 333), "dp_1tile_sk", 0, "owner"),
                                                   ((2000, 1500, 333), "2tile_sk_dp", 0, "owner")])
def test_timed_run_stamps_and_schedule(shape, policy, g, fixup):
    """skgemm_run_timed: the schedule records equal the enumerator's, each
    segment's five stamps are in order, a workgroup's segments follow one
    another, only segments that wait for peers show a wait, and C is bitwise
    the untimed run's."""
    M, N, K = shape
    gen = W.rng(3)
    A = torch.from_numpy(W.integer_f32(gen, (M, K))).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(W.integer_f32(gen, (K, N))).to(torch.bfloat16).to(dev())
    kw = dict(policy=policy, force_g=g, fixup=fixup, out_dtype=torch.float32)
    p = sk().get_plan(M, N, K, 0, 0, 0, sk().BF16, sk().F32, policy, g, 2, None, fixup)
    cap = p.trace_capacity()
    tr = torch.full((cap * 8,), -7, dtype=torch.int32, device=dev())
    ts = torch.zeros((cap * 7,), dtype=torch.int64, device=dev())
    C = mm(A, B, trace=tr, times=ts, **kw)
    C0 = mm(A, B, **kw)
    assert torch.equal(C, C0)
    info = p.info()
    recs = tr.cpu().numpy().reshape(-1, 8)
    stamps = ts.cpu().numpy().reshape(-1, 7)
    used = recs[:, 0] != -7
    got = records_to_schedule([tuple(int(v) for v in r) for r in recs[used]], info["grid"])
    assert got == S.enumerate_schedule(oracle_plan_for(info, p.model_constants(), policy, force_g=g))
    st = stamps[used][:, :5]
    clk = stamps[used][:, 5:]
    assert np.all(st > 0) and np.all(np.diff(st, axis=1) >= 0)
    hz = sk().realtime_hz()
    assert 1e6 <= hz <= 1e10
    # the shader clock over the whole launch: between 0.5 and 3 GHz
    ticks = clk[:, 1].astype(np.float64) - clk[:, 0]
    assert np.all(ticks > 0)
    ghz = ticks.sum() / ((st[:, 4] - st[:, 0]).astype(np.float64).sum() / hz) / 1e9
    assert 0.5 < ghz < 3.0, ghz
    per_wg = {}
    for r, s_ in zip(recs[used], st):
        per_wg.setdefault(int(r[0]), []).append((int(r[1]), s_))
    for segs in per_wg.values():
        segs.sort(key=lambda x: x[0])
        for (_, a_), (_, b_) in zip(segs, segs[1:]):
            assert b_[0] >= a_[4]
    # a full tile with no split waits for nobody
    for r, s_ in zip(recs[used], st):
        if r[5] == 0 and info["coop_s"] == 0:
            assert (s_[3] - s_[2]) / hz < 2e-6
    span = (st[:, 4].max() - st[:, 0].min()) / hz
    assert 0 < span < 1.0


def test_matmul_fast_path_repeated_signatures():
    """Repeated matmul calls with one tensor signature take the cached path
    (no layout inference or plan lookup): results equal the first call's; a
    transposed view, a strided view and a non-contiguous operand (copied by
    the slow path, so never cached) stay correct on every call."""
    M, N, K = 300, 700, 900
    a, b = W.normal_pair(M, N, K, seed=51)
    A = torch.from_numpy(a).to(torch.bfloat16).to(dev())
    B = torch.from_numpy(b).to(torch.bfloat16).to(dev())
    ref = oracle(A, B)
    sk()._fast_cache.clear()
    first = mm(A, B, out_dtype=torch.float32)
    for _ in range(3):
        assert torch.equal(mm(A, B, out_dtype=torch.float32), first)
    assert len(sk()._fast_cache) >= 1
    assert rel(first, ref) <= TOL_16_OUT32
    Bt = B.t().contiguous().t()                        # column-major B: another signature
    for _ in range(3):
        assert rel(mm(A, Bt, out_dtype=torch.float32), ref) <= TOL_16_OUT32
    big = torch.zeros((M, 2 * K), dtype=torch.bfloat16, device=dev())
    big[:, ::2] = A                                    # neither dimension contiguous: copied
    As = big[:, ::2]
    n0 = len(sk()._fast_cache)
    for _ in range(3):
        assert rel(mm(As, B, out_dtype=torch.float32), ref) <= TOL_16_OUT32
    assert len(sk()._fast_cache) == n0
    pad = torch.zeros((M, K + 64), dtype=torch.bfloat16, device=dev())
    pad[:, :K] = A                                     # leading dimension K + 64
    for _ in range(3):
        assert rel(mm(pad[:, :K], B, out_dtype=torch.float32), ref) <= TOL_16_OUT32


@pytest.mark.parametrize("c_col", [False, True])
def test_operand_relayout_bitwise_and_parity(c_col):
    """Plans that copy a misaligned operand into 128-byte lines before the
    GEMM: the result is bitwise the one of the same plan run without the copy
    (a workspace of only the fix-up part) and of operands passed with aligned
    leading dimensions (no copy at run time), and matches the FP64 oracle on
    sampled rows."""
    lc = sk().COL_MAJOR if c_col else sk().ROW_MAJOR
    cands = [(777, 5555, 3333), (2049, 6001, 4001), (3333, 777, 5555), (4427, 2519, 3013), (1482, 2519, 3013)]
    found = 0
    for (M, N, K) in cands:
        # relayout=3: copy both operands whenever misaligned (the mechanism,
        # whatever the model would choose)
        plan = sk().Plan(M, N, K, lc=lc, ta=sk().BF16, relayout=3)
        info = plan.info()
        if not (info["pack_a"] or info["pack_b"]):
            continue
        found += 1
        g = W.rng(M)
        A = torch.from_numpy(W.normal_f32(g, (M, K))).to(torch.bfloat16).to(dev())
        B = torch.from_numpy(W.normal_f32(g, (K, N))).to(torch.bfloat16).to(dev())
        # aligned-line copies of the same values (leading dimensions padded to 64 elements)
        Ap = torch.zeros((M, -(-K // 64) * 64), dtype=torch.bfloat16, device=dev())
        Bp = torch.zeros((K, -(-N // 64) * 64), dtype=torch.bfloat16, device=dev())
        Ap[:, :K] = A
        Bp[:, :N] = B
        stream = torch.cuda.current_stream().cuda_stream

        def run(a, lda, b, ldb, ws_bytes):
            C = torch.full((N, M) if c_col else (M, N), float("nan"), dtype=torch.bfloat16, device=dev())
            ws = torch.zeros(max(ws_bytes, 256), dtype=torch.uint8, device=dev())
            plan.run(a.data_ptr(), lda, b.data_ptr(), ldb, C.data_ptr(), M if c_col else N, 1.0, 0.0, None, None,
                     ws.data_ptr() if ws_bytes else None, ws_bytes, stream)
            torch.cuda.synchronize()
            return C.t() if c_col else C

        full = run(A, K, B, N, plan.workspace_size())
        bare = run(A, K, B, N, info["fixup_ws_bytes"])
        aligned = run(Ap, Ap.shape[1], Bp, Bp.shape[1], plan.workspace_size())
        assert torch.equal(full, bare), (M, N, K)
        assert torch.equal(full, aligned), (M, N, K)
        rows = np.sort(W.rng(7).choice(M, 24, replace=False))
        ref = og.gemm_rows_f64(to_f64(A), to_f64(B), rows)
        assert og.rel_frobenius(to_f64(full[torch.from_numpy(rows).to(dev())]), ref) <= TOL_16, (M, N, K)
    assert found == len(cands)


@pytest.mark.parametrize("b_col", [False, True])
@pytest.mark.parametrize("policy,g", [("dp", 0), ("sk", 0), ("sk", 200), ("auto", 0)])
def test_three_stage_tile_bitwise_and_exact(policy, g, b_col):
    """Where a 16-bit 128x128x64 plan's grid fits one workgroup per CU, the
    eight-wave kernel on three LDS stages runs it: the result is bitwise the
    four-wave two-stage kernel's on the same schedule (same k-order per output
    element), integer-valued inputs give the oracle's exact result, and its
    trace is the enumerator's schedule."""
    from helpers import resolved
    shapes = [(1000, 1500, 777), (2048, 2048, 1024), (384, 4096, 5000), (129, 130, 131), (640, 3456, 896)]
    found = 0
    for (M, N, K) in shapes:
        lb = sk().COL_MAJOR if b_col else sk().ROW_MAJOR
        plan = sk().Plan(M, N, K, lb=lb, ta=sk().BF16, tc=sk().F32, policy=policy, force_g=g, tile=(128, 128, 64, 8))
        info = plan.info()
        if info["stages"] != 3:
            assert info["grid"] > info["p"] // info["occupancy"] or info["grid"] > 256, (M, N, K)
            continue
        found += 1
        pol, fg = resolved(info)
        four = dict(policy=pol, force_g=fg, tile=(128, 128, 64, 4))
        assert sk().Plan(M, N, K, lb=lb, ta=sk().BF16, tc=sk().F32, **four).schedule() == plan.schedule()
        gen = W.rng(M + N + K)
        for integer in (False, True):
            make = W.integer_f32 if integer else W.normal_f32
            A = torch.from_numpy(make(gen, (M, K))).to(torch.bfloat16).to(dev())
            B = torch.from_numpy(make(gen, (K, N))).to(torch.bfloat16).to(dev())
            if b_col:
                B = B.t().contiguous().t()
            c8 = mm(A, B, out_dtype=torch.float32, policy=pol, force_g=fg, tile=(128, 128, 64, 8))
            c4 = mm(A, B, out_dtype=torch.float32, **four)
            assert torch.equal(c8, c4), (M, N, K, integer)
            if integer:
                assert np.array_equal(to_f64(c8), oracle(A, B)), (M, N, K)
        # the traced run of the same plan follows the enumerator's schedule
        tr = torch.full((plan.trace_capacity() * 8,), -7, dtype=torch.int32, device=dev())
        mm(A, B, out_dtype=torch.float32, policy=pol, force_g=fg, tile=(128, 128, 64, 8), trace=tr)
        recs = [tuple(int(v) for v in rec) for rec in tr.cpu().numpy().reshape(-1, 8) if rec[0] != -7]
        ref = oracle_plan_for(info, plan.model_constants(), pol, force_g=fg)
        assert records_to_schedule(recs, info["grid"]) == S.enumerate_schedule(ref), (M, N, K)
    assert found >= 2
