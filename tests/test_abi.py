"""Host-side checks of the C ABI (no GPU compute calls).

* libskgemm.so loads and exports every function include/skgemm.h declares;
* argument errors are reported as status codes before anything launches;
* the planner's host-side schedule equals the oracle enumerator's, record by
  record, over many shapes, policies, grid sizes and processor widths.
"""
import ctypes
import itertools
import os
import re

import pytest

from helpers import POLICY_BY_ID, oracle_grouped_plan_for, oracle_plan_for, records_to_schedule, resolved
from oracle import schedule as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2212_08964_amd import skgemm
    return skgemm


def test_library_exports_every_declared_symbol():
    sk = _lib()
    L = sk.lib()
    header = open(os.path.join(ROOT, "include", "skgemm.h")).read()
    names = set(re.findall(r"^\s*(?:const char\*|void|skgemm_status_t)\s+(skgemm_\w+)\s*\(", header, re.M))
    assert len(names) >= 12
    for n in sorted(names):
        assert hasattr(L, n), f"missing export {n}"
    assert set(sk.EXPORTED) == names


def test_plan_argument_errors():
    sk = _lib()
    L = sk.lib()
    h = ctypes.c_void_p()
    o = sk.default_options()
    o.num_cus, o.occupancy = 256, 1
    bad = [
        (-1, 4, 4, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16, sk.ERR_INVALID_ARG),
        (4, 4, 4, 2, 0, 0, sk.BF16, sk.BF16, sk.BF16, sk.ERR_INVALID_ARG),
        (4, 4, 4, 0, 0, 0, sk.BF16, sk.F16, sk.BF16, sk.ERR_UNSUPPORTED),
        (4, 4, 4, 0, 0, 0, sk.F32, sk.F32, sk.BF16, sk.ERR_UNSUPPORTED),
        (4, 4, 4, 0, 0, 0, sk.F8E4M3, sk.F8E4M3, sk.F32, sk.ERR_UNSUPPORTED),   # FP8 needs B column-major
        (4, 4, 4, 0, 0, 0, sk.BF16, sk.BF16, sk.F8E4M3, sk.ERR_UNSUPPORTED),
        (1 << 31, 4, 4, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16, sk.ERR_INVALID_ARG),
    ]
    for M, N, K, la, lb, lc, ta, tb, tc, want in bad:
        assert L.skgemm_plan(ctypes.byref(h), M, N, K, la, lb, lc, ta, tb, tc, ctypes.byref(o)) == want
    assert L.skgemm_plan(None, 4, 4, 4, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16, None) == sk.ERR_INVALID_ARG
    # a Stream-K grid beyond the co-resident capacity is refused
    o.policy, o.force_g = sk.POLICY["sk"], 300
    assert L.skgemm_plan(ctypes.byref(h), 512, 512, 8192, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                         ctypes.byref(o)) == sk.ERR_CAPACITY
    # ... while one beyond the iterations is reduced to one workgroup per iteration
    o.force_g = 40
    pl = sk.Plan(64, 64, 640, ta=sk.BF16, policy="sk", force_g=100, num_cus=256, occupancy=1)
    info = pl.info()
    assert info["t"] * info["ipt"] < 100 and info["g_sk"] == info["grid"] == info["t"] * info["ipt"]
    o.share = 2
    assert L.skgemm_plan(ctypes.byref(h), 512, 512, 4096, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                         ctypes.byref(o)) == sk.ERR_INVALID_ARG
    o.share = 0
    o.tile_m = 32
    o.force_g = 0
    assert L.skgemm_plan(ctypes.byref(h), 512, 512, 4096, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                         ctypes.byref(o)) == sk.ERR_UNSUPPORTED


def test_run_argument_errors_before_launch():
    sk = _lib()
    p = sk.Plan(300, 200, 100, ta=sk.BF16, policy="sk", num_cus=256, occupancy=1)
    ws = p.workspace_size()
    assert ws > 0
    fake = 1 << 40   # never dereferenced: every call below fails its host checks first
    cases = [
        dict(lda=99, ldb=200, ldc=200, ws=fake, wsb=ws, want=sk.ERR_INVALID_ARG),    # lda < K
        dict(lda=100, ldb=199, ldc=200, ws=fake, wsb=ws, want=sk.ERR_INVALID_ARG),   # ldb < N
        dict(lda=100, ldb=200, ldc=199, ws=fake, wsb=ws, want=sk.ERR_INVALID_ARG),   # ldc < N
        dict(lda=100, ldb=200, ldc=200, ws=None, wsb=ws, want=sk.ERR_WORKSPACE),
        dict(lda=100, ldb=200, ldc=200, ws=fake, wsb=ws - 1, want=sk.ERR_WORKSPACE),
        dict(lda=100, ldb=200, ldc=200, ws=fake + 16, wsb=ws, want=sk.ERR_WORKSPACE),  # misaligned
    ]
    for c in cases:
        st = sk.lib().skgemm_run(p.handle, fake, c["lda"], fake, c["ldb"], fake, c["ldc"], 1.0, 0.0,
                                 None, None, c["ws"], c["wsb"], None)
        assert st == c["want"], c
    st = sk.lib().skgemm_run(p.handle, fake, 100, fake, 200, None, 200, 1.0, 0.0, None, None, fake, ws, None)
    assert st == sk.ERR_INVALID_ARG
    z = sk.Plan(0, 200, 100, ta=sk.BF16, num_cus=256, occupancy=1)
    assert sk.lib().skgemm_run(z.handle, None, 100, None, 200, None, 200, 1.0, 0.0, None, None, None, 0,
                               None) == sk.OK
    assert sk.status_string(sk.ERR_TIMEOUT) != sk.status_string(sk.OK)


SHAPES = [(384, 384, 1024), (896, 384, 128), (1, 1, 1), (300, 500, 700), (4096, 4096, 64), (128, 8192, 8192),
          (2048, 2048, 8192), (8192, 8192, 8192), (1000, 130, 5), (7, 3000, 4000), (513, 257, 0),
          (256 * 17, 256 * 16, 1000), (256 * 33, 256 * 9, 300)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("policy", ["auto", "paper", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"])
@pytest.mark.parametrize("share", ["proportional", "leading"])
def test_planner_schedule_matches_enumerator(dtype, policy, share):
    sk = _lib()
    ta = {"f32": sk.F32, "bf16": sk.BF16}[dtype]
    for (M, N, K), (cus, occ), lc in itertools.product(SHAPES, [(256, 1), (256, 2), (4, 1), (37, 3)],
                                                       [sk.ROW_MAJOR, sk.COL_MAJOR]):
        try:
            p = sk.Plan(M, N, K, ta=ta, lc=lc, policy=policy, num_cus=cus, occupancy=occ, share=share)
        except sk.SkgemmError as e:
            assert e.status == sk.ERR_CAPACITY
            continue
        info = p.info()
        ref = oracle_plan_for(info, p.model_constants(), policy)
        assert (ref.policy, ref.sk_tiles, ref.g_sk, ref.grid, ref.sk_first) == (
            POLICY_BY_ID[info["policy"]], info["sk_tiles"], info["g_sk"], info["grid"], bool(info["sk_first"]))
        got = records_to_schedule(p.schedule(), info["grid"])
        want = S.enumerate_schedule(ref)
        assert got == want, (M, N, K, cus, occ, policy)
        if info["t"]:
            S.check_invariants(ref, got)
        assert p.trace_capacity() == info["grid"] * max([len(s) for s in want] + [0])


@pytest.mark.parametrize("g", [1, 2, 3, 5, 9, 16, 36, 100, 288, 300])
@pytest.mark.parametrize("share", ["proportional", "leading"])
def test_planner_forced_grid_matches_enumerator(g, share):
    sk = _lib()
    p = sk.Plan(384, 384, 1024, ta=sk.F32, policy="sk", force_g=g, num_cus=256, occupancy=2, share=share)
    info = p.info()
    ref = oracle_plan_for(info, p.model_constants(), "sk", force_g=g)
    got = records_to_schedule(p.schedule(), info["grid"])
    assert got == S.enumerate_schedule(ref)
    S.check_invariants(ref, got)


def test_workspace_scales_with_grid_not_problem():
    sk = _lib()
    for tile in [(256, 256, 64), (128, 128, 64)]:
        small = sk.Plan(300, 300, 4096, ta=sk.BF16, policy="sk", force_g=64, num_cus=256, occupancy=1, tile=tile)
        big = sk.Plan(3000, 3000, 40960, ta=sk.BF16, policy="sk", force_g=64, num_cus=256, occupancy=1,
                      tile=tile)
        assert small.info()["tile"][:3] == big.info()["tile"][:3] == tile
        # the fix-up part (the rest, if any, holds a re-laid-out operand)
        assert small.info()["fixup_ws_bytes"] == big.info()["fixup_ws_bytes"]
    # one FP32 partial tile per workgroup: the small tile needs a quarter of the partial storage
    w = {t: sk.Plan(3000, 3000, 40960, ta=sk.BF16, policy="sk", force_g=64, num_cus=256, occupancy=1,
                    tile=t).info()["fixup_ws_bytes"] for t in [(256, 256, 64), (128, 128, 64)]}
    assert w[(256, 256, 64)] - w[(128, 128, 64)] == 64 * (256 * 256 - 128 * 128) * 4
    dp = sk.Plan(3000, 3000, 4096, ta=sk.BF16, policy="dp", num_cus=256, occupancy=1)
    assert dp.workspace_size() == 0


@pytest.mark.parametrize("policy", ["auto", "paper", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"])
def test_grouped_planner_matches_enumerator(policy):
    from oracle import grouped as GR
    import workloads as W
    sk = _lib()
    groups = [
        [(m, 4096, 2048) for m in W.zipf_ms(64, seed=0)],
        [(100, 300, 16), (0, 50, 70), (700, 900, 5000), (1, 1, 1)],
        [(256 * 3, 256 * 5, 640)] * 7,
        # K = 0 problems (epilogue-only tiles) between problems with iterations
        [(300, 700, 0), (1000, 900, 3000), (64, 64, 0), (0, 50, 0), (500, 256, 640), (900, 900, 0)],
        [(256, 256, 0)] * 3,
    ]
    for probs, (cus, occ) in itertools.product(groups, [(256, 1), (16, 1), (37, 2)]):
        Ms, Ns, Ks = zip(*probs)
        try:
            p = sk.GroupedPlan(Ms, Ns, Ks, ta=sk.BF16, policy=policy, num_cus=cus, occupancy=occ)
        except sk.SkgemmError as e:
            assert e.status == sk.ERR_CAPACITY
            continue
        info = p.info()
        ref = oracle_grouped_plan_for(probs, info, p.model_constants(), policy)
        assert (ref.policy, ref.sk_tiles, ref.g_sk, ref.grid) == (
            POLICY_BY_ID[info["policy"]], info["sk_tiles"], info["g_sk"], info["grid"])
        got = records_to_schedule(p.schedule(), info["grid"])
        assert got == GR.enumerate_grouped_schedule(ref)
        GR.check_grouped_invariants(ref, got)


def test_grouped_and_quantize_argument_errors():
    sk = _lib()
    L = sk.lib()
    h = ctypes.c_void_p()
    arr = ctypes.c_int64 * 2
    o = sk.default_options()
    o.num_cus, o.occupancy = 256, 1
    assert L.skgemm_grouped_plan(ctypes.byref(h), 0, arr(1, 1), arr(1, 1), arr(1, 1), 0, 0, 0, sk.BF16, sk.BF16,
                                 sk.BF16, ctypes.byref(o)) == sk.ERR_INVALID_ARG
    # a K = 0 problem is planned (its tiles only apply the epilogue)
    assert L.skgemm_grouped_plan(ctypes.byref(h), 2, arr(4, 4), arr(4, 4), arr(4, 0), 0, 0, 0, sk.BF16, sk.BF16,
                                 sk.BF16, ctypes.byref(o)) == sk.OK
    L.skgemm_plan_destroy(h)
    g = sk.GroupedPlan([64, 64], [64, 64], [64, 64], ta=sk.BF16, num_cus=256, occupancy=1)
    fake = 1 << 40
    bad = [(fake, 63, fake, 64, fake, 64, 1.0, 0.0), (fake, 64, fake, 64, fake, 64, 1.0, 0.0)]   # lda < K
    with pytest.raises(sk.SkgemmError):
        g.table(bad)
    n = ctypes.c_size_t()
    assert L.skgemm_quantize_workspace_size(ctypes.byref(n)) == sk.OK and n.value > 0
    assert L.skgemm_quantize_e4m3(fake, sk.F8E4M3, 4, 4, 0, 4, fake, 0, 4, fake, fake, n.value,
                                  None) == sk.ERR_UNSUPPORTED
    assert L.skgemm_quantize_e4m3(fake, sk.BF16, 4, 4, 0, 3, fake, 0, 4, fake, fake, n.value,
                                  None) == sk.ERR_INVALID_ARG
    assert L.skgemm_quantize_e4m3(fake, sk.BF16, 4, 4, 0, 4, fake, 0, 4, fake, fake, n.value - 4,
                                  None) == sk.ERR_WORKSPACE


def test_raster_and_xcd_options():
    """Raster and XCD permutation options are validated and leave the schedule over tile indices unchanged."""
    sk = _lib()
    L = sk.lib()
    h = ctypes.c_void_p()
    for field, bad in (("raster_rows", -1), ("raster_rows", 1 << 17), ("xcds", -1), ("xcds", 65)):
        o = sk.default_options()
        o.num_cus, o.occupancy = 256, 1
        setattr(o, field, bad)
        assert L.skgemm_plan(ctypes.byref(h), 1000, 1000, 1000, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                             ctypes.byref(o)) == sk.ERR_INVALID_ARG, (field, bad)
    scheds = [sk.Plan(3000, 2000, 1000, ta=sk.BF16, policy="sk", num_cus=256, occupancy=1, raster_rows=r,
                      xcds=x).schedule() for r in (0, 1, 3, 8) for x in (0, 1, 8)]
    assert all(s == scheds[0] for s in scheds)


def _one_segment_shares(sched, sk_tiles, g_sk, ipt):
    """s when the enumerated schedule cuts every Stream-K tile into s >= 2
    shares held by s consecutive workgroups with one Stream-K segment each
    (workgroup x on tile x // s, the shares in order and covering the tile),
    else 0."""
    per_wg = [[sg for sg in segs if sg.tile < sk_tiles] for segs in sched[:g_sk]]
    if not sk_tiles or not g_sk or any(len(v) != 1 for v in per_wg) or g_sk % sk_tiles:
        return 0
    s = g_sk // sk_tiles
    if s < 2:
        return 0
    for x, (sg,) in enumerate(per_wg):
        c = x % s
        if sg.tile != x // s or (c == 0 and sg.k_lo != 0) or (c == s - 1 and sg.k_hi != ipt):
            return 0
        if c and per_wg[x - 1][0].k_hi != sg.k_lo:
            return 0
    return s


@pytest.mark.parametrize("share", ["proportional", "leading"])
@pytest.mark.parametrize("policy", ["auto", "sk", "dp_1tile_sk"])
def test_split_fixup_exactly_for_one_segment_shares(policy, share):
    """The plan uses the split fix-up exactly when the enumerator's schedule
    gives every Stream-K workgroup one segment of a cut of its tile (both
    share rules); SKGEMM_FIXUP_OWNER always turns it off."""
    sk = _lib()
    shapes = [(1024, 1024, 1024), (1000, 1030, 1024), (300, 500, 768), (2560, 3328, 1024), (384, 384, 1000),
              (640, 768, 4096), (128, 8192, 8192), (4096, 4096, 64)]
    grids = [0] if policy == "auto" else [0, 5, 24, 36, 64, 96, 128, 144, 256, 320]
    seen = 0
    for (M, N, K), g in itertools.product(shapes, grids):
        try:
            p = sk.Plan(M, N, K, ta=sk.BF16, policy=policy, force_g=g, num_cus=256, occupancy=2,
                        tile=(128, 128, 64), share=share)
        except sk.SkgemmError as e:
            assert e.status == sk.ERR_CAPACITY
            continue
        info = p.info()
        sched = records_to_schedule(p.schedule(), info["grid"])
        want = _one_segment_shares(sched, info["sk_tiles"], info["g_sk"], info["ipt"])
        assert info["coop_s"] == want, (M, N, K, policy, g)
        seen += want > 0
        o = sk.Plan(M, N, K, ta=sk.BF16, policy=policy, force_g=g, num_cus=256, occupancy=2, tile=(128, 128, 64),
                    share=share, fixup="owner")
        assert o.info()["coop_s"] == 0
        assert records_to_schedule(o.schedule(), info["grid"]) == sched
    assert seen > 0


def test_split_fixup_invalid_option():
    sk = _lib()
    L = sk.lib()
    o = sk.default_options()
    o.fixup = 7
    h = ctypes.c_void_p()
    assert L.skgemm_plan(ctypes.byref(h), 64, 64, 64, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                         ctypes.byref(o)) == sk.ERR_INVALID_ARG


def test_spin_limit_option():
    """A negative spin limit is refused; 0 (the default) and positive limits plan,
    and the options structure the binding passes has the header's size (the
    library clears exactly that many bytes in skgemm_default_options)."""
    sk = _lib()
    L = sk.lib()
    h = ctypes.c_void_p()
    o = sk.default_options()
    o.spin_limit = -1
    assert L.skgemm_plan(ctypes.byref(h), 64, 64, 64, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                         ctypes.byref(o)) == sk.ERR_INVALID_ARG
    for lim in (0, 1, 1000):
        p = sk.Plan(300, 200, 900, ta=sk.BF16, policy="sk", num_cus=256, occupancy=2, spin_limit=lim)
        assert p.info()["grid"] > 0
    # 15 int32 fields, in the header's order; the padding after them is not
    # touched by the library
    assert ctypes.sizeof(sk.Options) == 15 * 4
    guard = (ctypes.c_int32 * 17)(*([0x5A5A5A5A] * 17))
    L.skgemm_default_options(ctypes.cast(guard, ctypes.POINTER(sk.Options)))
    assert list(guard[:15]) == [sk.POLICY["auto"], 0, 0, 0, 0, 2] + [0] * 9
    assert list(guard[15:]) == [0x5A5A5A5A] * 2


def test_f64_plans():
    """FP64 in needs FP64 out; its partial tiles are FP64 (8 bytes per element)."""
    sk = _lib()
    for tile in [(64, 64, 16), (128, 128, 16)]:
        t = sk.Plan(1000, 700, 900, ta=sk.F64, policy="sk", force_g=100, num_cus=256, occupancy=2, tile=tile)
        assert t.info()["tile"][:3] == tile
        u = sk.Plan(1000, 700, 900, ta=sk.F64, policy="sk", force_g=50, num_cus=256, occupancy=2, tile=tile)
        assert t.workspace_size() - u.workspace_size() == 50 * tile[0] * tile[1] * 8
    # unpinned, the planner takes the tile with the smaller modelled time
    p = sk.Plan(1000, 700, 900, ta=sk.F64, policy="sk", force_g=100, num_cus=256, occupancy=4)
    info = p.info()
    assert info["tile"][:3] in [(64, 64, 16), (128, 128, 16)]
    for ta, tc in [(sk.F64, sk.F32), (sk.F32, sk.F64), (sk.BF16, sk.F64)]:
        with pytest.raises(sk.SkgemmError) as e:
            sk.Plan(100, 100, 100, ta=ta, tc=tc, num_cus=256, occupancy=1)
        assert e.value.status == sk.ERR_UNSUPPORTED
    ref = oracle_plan_for(info, p.model_constants(), "sk", force_g=100)
    assert records_to_schedule(p.schedule(), info["grid"]) == S.enumerate_schedule(ref)


@pytest.mark.parametrize("policy", ["auto", "paper", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp"])
def test_batched_planner_matches_enumerator(policy):
    """A strided batch of equal problems is one iteration space, problem after
    problem: the planner's schedule equals the grouped enumerator's for the
    list of equal problems (and so, by the equal-ipt pin, one GEMM with the
    tile count summed)."""
    sk = _lib()
    for (batch, M, N, K), (cus, occ) in itertools.product(
            [(4, 300, 500, 700), (16, 128, 256, 2048), (3, 1000, 130, 5), (7, 64, 64, 64), (2, 513, 257, 0)],
            [(256, 1), (16, 1), (37, 2)]):
        try:
            p = sk.BatchedPlan(batch, M, N, K, ta=sk.BF16, policy=policy, num_cus=cus, occupancy=occ)
        except sk.SkgemmError as e:
            assert e.status == sk.ERR_CAPACITY
            continue
        info = p.info()
        assert info["batch"] == batch and info["t"] == batch * info["tm"] * info["tn"]
        ref = oracle_grouped_plan_for([(M, N, K)] * batch, info, p.model_constants(), policy)
        assert (ref.policy, ref.sk_tiles, ref.g_sk, ref.grid) == (
            POLICY_BY_ID[info["policy"]], info["sk_tiles"], info["g_sk"], info["grid"])
        from oracle import grouped as GR
        got = records_to_schedule(p.schedule(), info["grid"])
        assert got == GR.enumerate_grouped_schedule(ref), (batch, M, N, K, cus, occ)
        if info["t"]:
            GR.check_grouped_invariants(ref, got)


def test_batched_argument_errors():
    sk = _lib()
    L = sk.lib()
    h = ctypes.c_void_p()
    o = sk.default_options()
    o.num_cus, o.occupancy = 256, 1
    assert L.skgemm_batched_plan(ctypes.byref(h), 0, 4, 4, 4, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                                 ctypes.byref(o)) == sk.ERR_INVALID_ARG
    p = sk.BatchedPlan(3, 64, 64, 64, ta=sk.BF16, num_cus=256, occupancy=1, policy="dp")
    fake = 1 << 40
    # overlapping C matrices, negative strides: refused before launch
    assert L.skgemm_batched_run(p.handle, fake, 64, 4096, fake, 64, 4096, fake, 64, 4000, 1.0, 0.0, None, None,
                                None, 0, None) == sk.ERR_INVALID_ARG
    assert L.skgemm_batched_run(p.handle, fake, 64, -1, fake, 64, 4096, fake, 64, 4096, 1.0, 0.0, None, None,
                                None, 0, None) == sk.ERR_INVALID_ARG
    # a batched plan needs the batched run (strides), and a single plan runs through either
    assert L.skgemm_run(p.handle, fake, 64, fake, 64, fake, 64, 1.0, 0.0, None, None, None, 0,
                        None) == sk.ERR_INVALID_ARG


CONV_CASES = [
    # n, h, w, c, k, r, s, pad, stride, dilation
    (2, 14, 14, 64, 96, 3, 3, (1, 1), (1, 1), (1, 1)),
    (3, 17, 11, 128, 200, 3, 3, (1, 1), (2, 2), (1, 1)),
    (1, 9, 13, 64, 64, 3, 3, (2, 2), (1, 1), (2, 2)),
    (4, 7, 7, 256, 130, 1, 1, (0, 0), (1, 1), (1, 1)),
    (2, 23, 23, 64, 64, 7, 7, (3, 3), (2, 2), (1, 1)),
    (1, 5, 8, 192, 33, 2, 3, (0, 1), (1, 2), (1, 1)),
]


@pytest.mark.parametrize("case", CONV_CASES)
@pytest.mark.parametrize("policy", ["auto", "paper", "sk", "dp"])
def test_conv_plan_is_the_gemm_view(case, policy):
    """A convolution plan is the plan of its GEMM view (M = n P Q, N = k,
    K = r s c; A K-contiguous, the filters a column-major B, C row-major) on
    the tile of the same size: same resolution, same schedule, and that
    schedule is the oracle enumerator's."""
    from oracle import conv as oc
    sk = _lib()
    n, h, w, c, k, r, s, pad, std, dil = case
    P, Q = oc.out_size(h, w, r, s, pad[0], pad[1], std[0], std[1], dil[0], dil[1])
    for tile, (cus, occ) in itertools.product([(256, 256, 64), (128, 128, 64, 4), (256, 64, 64)],
                                              [(256, 1), (64, 2)]):
        cp = sk.ConvPlan(n, h, w, c, k, r, s, pad, std, dil, ta=sk.BF16, policy=policy, tile=tile, num_cus=cus,
                         occupancy=occ)
        gp = sk.Plan(n * P * Q, k, r * s * c, sk.ROW_MAJOR, sk.COL_MAJOR, sk.ROW_MAJOR, ta=sk.BF16, policy=policy,
                     tile=tile, num_cus=cus, occupancy=occ)
        ci, gi = cp.info(), gp.info()
        assert (ci["M"], ci["N"], ci["K"]) == (n * P * Q, k, r * s * c)
        assert ci == gi, (case, tile)
        assert cp.model_constants() == gp.model_constants()
        assert cp.schedule() == gp.schedule()
        ref = oracle_plan_for(ci, cp.model_constants(), policy)
        assert records_to_schedule(cp.schedule(), ci["grid"]) == S.enumerate_schedule(ref)


def test_conv_chooses_among_its_tiles():
    """256x256 and 128x128 for any channel count (the 128x128 one on eight
    waves and three stages where the grid fits one workgroup per CU); the
    tall 256x64 tile only for at most 64 output channels."""
    sk = _lib()
    big = sk.ConvPlan(32, 56, 56, 64, 256, 3, 3, (1, 1), num_cus=256, occupancy=1).info()
    small = sk.ConvPlan(1, 7, 7, 64, 128, 3, 3, (1, 1), num_cus=256, occupancy=1).info()
    narrow = sk.ConvPlan(32, 56, 56, 64, 64, 3, 3, (1, 1), num_cus=256, occupancy=1).info()
    assert big["tile"] in {(256, 256, 64, 8), (128, 128, 64, 4), (128, 128, 64, 8)}
    assert small["tile"] == (128, 128, 64, 8) and small["stages"] == 3
    assert narrow["tile"] == (256, 64, 64, 4)
    for k in (65, 96, 200):
        assert sk.ConvPlan(8, 14, 14, 64, k, 3, 3, (1, 1), num_cus=256, occupancy=1).info()["tile"] != (256, 64, 64, 4)


def test_conv_argument_errors():
    sk = _lib()
    L = sk.lib()
    o = sk.default_options()
    o.num_cus, o.occupancy = 256, 1
    h = ctypes.c_void_p()

    def plan(*f, ta=sk.BF16, tc=sk.BF16):
        return L.skgemm_conv_plan(ctypes.byref(h), ctypes.byref(sk.ConvDesc(*f)), ta, tc, ctypes.byref(o))

    ok = (2, 8, 8, 64, 32, 3, 3, 1, 1, 1, 1, 1, 1)
    assert plan(*ok) == sk.OK
    L.skgemm_plan_destroy(h)
    assert plan(2, 8, 8, 96, 32, 3, 3, 1, 1, 1, 1, 1, 1) == sk.ERR_UNSUPPORTED      # c not a multiple of 64
    assert plan(*ok, ta=sk.F32, tc=sk.F32) == sk.ERR_UNSUPPORTED
    assert plan(*ok, ta=sk.F8E4M3, tc=sk.F32) == sk.ERR_UNSUPPORTED
    assert plan(2, 8, 8, 64, 32, 3, 3, 1, 1, 1, 1, 1, 1) == sk.OK
    L.skgemm_plan_destroy(h)
    assert plan(2, 2, 8, 64, 32, 3, 3, 0, 0, 1, 1, 1, 1) == sk.ERR_INVALID_ARG      # window taller than the image
    assert plan(2, 8, 8, 64, 32, 3, 3, 1, 1, 0, 1, 1, 1) == sk.ERR_INVALID_ARG      # stride 0
    assert plan(2, 8, 8, 64, 32, 3, 3, -1, 1, 1, 1, 1, 1) == sk.ERR_INVALID_ARG     # negative padding
    assert plan(2, 8, 8, 64, 32, 3, 3, 1, 1, 1, 1, 0, 1) == sk.ERR_INVALID_ARG      # dilation 0
    assert plan(-1, 8, 8, 64, 32, 3, 3, 1, 1, 1, 1, 1, 1) == sk.ERR_INVALID_ARG
    # the input must be addressable with 32-bit offsets
    assert plan(1 << 15, 128, 128, 64, 32, 3, 3, 1, 1, 1, 1, 1, 1) == sk.ERR_UNSUPPORTED
    assert L.skgemm_conv_plan(ctypes.byref(h), None, sk.BF16, sk.BF16, ctypes.byref(o)) == sk.ERR_INVALID_ARG
    # a convolution plan runs only through the convolution entry points, and back
    cp = sk.ConvPlan(2, 8, 8, 64, 32, 3, 3, (1, 1), num_cus=256, occupancy=1)
    gp = sk.Plan(128, 32, 576, sk.ROW_MAJOR, sk.COL_MAJOR, sk.ROW_MAJOR, ta=sk.BF16, num_cus=256, occupancy=1)
    fake = 1 << 40
    assert L.skgemm_run(cp.handle, fake, 576, fake, 576, fake, 32, 1.0, 0.0, None, None, None, 0,
                        None) == sk.ERR_INVALID_ARG
    assert L.skgemm_conv_run(gp.handle, fake, fake, fake, 1.0, 0.0, None, 0, None) == sk.ERR_INVALID_ARG
    assert L.skgemm_conv_run(cp.handle, None, fake, fake, 1.0, 0.0, None, 0, None) == sk.ERR_INVALID_ARG
    # an empty batch is a no-op
    z = sk.ConvPlan(0, 8, 8, 64, 32, 3, 3, (1, 1), num_cus=256, occupancy=1)
    assert z.info()["M"] == 0
    assert L.skgemm_conv_run(z.handle, None, None, None, 1.0, 0.0, None, 0, None) == sk.OK


def test_tall_tile_only_for_narrow_problems():
    """The tall 256x64x64 tile is a candidate only where every launched
    problem has at most 64 columns (and B is K-contiguous), unless named."""
    sk = _lib()
    for (M, N, K), lb, lc in itertools.product([(8192, 16, 8192), (4096, 64, 2048), (3000, 65, 700), (1000, 1, 3000),
                                                (64, 4096, 512)],
                                               [sk.ROW_MAJOR, sk.COL_MAJOR], [sk.ROW_MAJOR, sk.COL_MAJOR]):
        p = sk.Plan(M, N, K, lb=lb, lc=lc, ta=sk.BF16, num_cus=256, occupancy=2)
        info = p.info()
        cols = M if lc == sk.COL_MAJOR else N
        if info["tile"] == (256, 64, 64, 4):
            assert cols <= 64 and info["b_kcontig"], (M, N, K, lb, lc)
        ref = oracle_plan_for(info, p.model_constants(), "auto")
        assert records_to_schedule(p.schedule(), info["grid"]) == S.enumerate_schedule(ref)
    assert sk.Plan(8192, 16, 8192, lb=sk.COL_MAJOR, ta=sk.BF16, num_cus=256, occupancy=2).info()["tile"] == \
        (256, 64, 64, 4)
    with pytest.raises(sk.SkgemmError) as e:      # no tall kernel reads an MN-contiguous B
        sk.Plan(300, 16, 200, lb=sk.ROW_MAJOR, ta=sk.BF16, num_cus=256, occupancy=2, tile=(256, 64, 64))
    assert e.value.status == sk.ERR_UNSUPPORTED


def test_skinny_tile_only_for_short_problems():
    """The skinny 64x256x64 tile is a candidate only where every launched
    problem has at most 64 rows (and A is K-contiguous), unless the options
    name it; its plans follow the enumerator like every other tile's."""
    sk = _lib()
    for (M, N, K), la, lc in itertools.product([(1, 1000, 3000), (16, 8192, 8192), (64, 4096, 2048), (65, 4096, 2048),
                                                (300, 200, 100), (128, 8192, 8192)],
                                               [sk.ROW_MAJOR, sk.COL_MAJOR], [sk.ROW_MAJOR, sk.COL_MAJOR]):
        p = sk.Plan(M, N, K, la=la, lc=lc, ta=sk.BF16, num_cus=256, occupancy=2)
        info = p.info()
        rows = N if lc == sk.COL_MAJOR else M
        if info["tile"] == (64, 256, 64, 4):
            assert rows <= 64 and info["a_kcontig"], (M, N, K, la, lc)
        ref = oracle_plan_for(info, p.model_constants(), "auto")
        assert records_to_schedule(p.schedule(), info["grid"]) == S.enumerate_schedule(ref)
    named = sk.Plan(300, 200, 100, ta=sk.BF16, num_cus=256, occupancy=2, tile=(64, 256, 64))
    assert named.info()["tile"] == (64, 256, 64, 4)
    with pytest.raises(sk.SkgemmError) as e:      # no skinny kernel reads an MN-contiguous A
        sk.Plan(16, 300, 200, la=sk.COL_MAJOR, ta=sk.BF16, num_cus=256, occupancy=2, tile=(64, 256, 64))
    assert e.value.status == sk.ERR_UNSUPPORTED


def test_plan_log_environment_switch():
    """SKGEMM_LOG=1 prints one line per plan built (launch kind, shape, tile,
    resolved policy and grid); unset, the library prints nothing."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2212_08964_amd import skgemm as sk\n"
            "sk.Plan(300, 200, 900, ta=sk.BF16, policy='sk', force_g=12, num_cus=256, occupancy=1)\n"
            "sk.ConvPlan(2, 8, 8, 64, 32, 3, 3, (1, 1), num_cus=256, occupancy=1)\n"
            "sk.GroupedPlan([64, 128], [64, 64], [64, 64], ta=sk.BF16, num_cus=256, occupancy=1)\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    env = dict(os.environ, SKGEMM_LOG="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = [ln for ln in out.stderr.splitlines() if ln.startswith("skgemm: plan")]
    assert len(lines) == 3, out.stderr
    assert " gemm M=300 N=200 K=900 " in lines[0] and "policy=sk" in lines[0] and "g_sk=12" in lines[0]
    assert lines[1].startswith("skgemm: plan conv M=128 N=32 K=576")
    assert lines[2].startswith("skgemm: plan grouped") and "G=2" in lines[2]
    env["SKGEMM_LOG"] = "0"
    quiet = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert quiet.returncode == 0 and "skgemm: plan" not in quiet.stderr


def test_three_stage_small_tile_substitution():
    """A 16-bit 128x128x64 plan whose grid fits one workgroup per CU runs the
    eight-wave kernel on three LDS stages (occupancy 1), with the schedule,
    workspace and model constants of the plan it replaces (a convolution
    plan: the same kernel with the gather); never for larger grids, four
    requested waves, other tiles or other input types."""
    sk = _lib()
    kw = dict(num_cus=256, occupancy=2)
    for ta in (sk.BF16, sk.F16):
        i = sk.Plan(2048, 2048, 1024, ta=ta, policy="dp", tile=(128, 128, 64), **kw).info()   # 256 tiles
        assert (i["stages"], i["waves"], i["occupancy"], i["p"], i["grid"]) == (3, 8, 1, 256, 256)
        i = sk.Plan(2048, 4096, 1024, ta=ta, policy="dp", tile=(128, 128, 64), **kw).info()   # 512 tiles
        assert (i["stages"], i["occupancy"], i["p"]) == (2, 2, 512)
        i = sk.Plan(2048, 2048, 1024, ta=ta, policy="dp", tile=(128, 128, 64, 4), **kw).info()
        assert (i["stages"], i["waves"]) == (2, 4)
        assert sk.Plan(2048, 2048, 1024, ta=ta, tile=(256, 256, 64), **kw).info()["stages"] == 2
    for g, want in ((200, 3), (256, 3), (300, 2)):
        deep = sk.Plan(1000, 1000, 5000, ta=sk.BF16, policy="sk", force_g=g, tile=(128, 128, 64, 8), **kw)
        i = deep.info()
        assert (i["g_sk"], i["stages"]) == (g, want)
        four = sk.Plan(1000, 1000, 5000, ta=sk.BF16, policy="sk", force_g=g, tile=(128, 128, 64, 4), **kw)
        assert deep.schedule() == four.schedule()
        assert deep.workspace_size() == four.workspace_size()
        eight = sk.Plan(1000, 1000, 5000, ta=sk.BF16, policy="sk", force_g=300, tile=(128, 128, 64, 8), **kw)
        assert deep.model_constants() == eight.model_constants()
    # the automatic plan of a one-wave problem; other types and launch kinds never
    assert sk.Plan(1536, 2048, 2048, ta=sk.BF16, **kw).info()["stages"] in (2, 3)
    assert sk.Plan(1024, 1024, 1024, lb=sk.COL_MAJOR, ta=sk.F8E4M3, tc=sk.BF16, tile=(128, 128, 128), policy="dp", **kw).info()["stages"] == 2
    assert sk.Plan(1024, 1024, 1024, ta=sk.F32, tc=sk.F32, **kw).info()["stages"] == 2
    assert sk.Plan(512, 512, 512, ta=sk.F64, tc=sk.F64, tile=(128, 128, 16), **kw).info()["stages"] == 2
    cv = sk.ConvPlan(2, 16, 16, 64, 128, 3, 3, (1, 1), ta=sk.BF16, tile=(128, 128, 64), **kw).info()
    assert (cv["stages"], cv["waves"], cv["occupancy"]) == (3, 8, 1) and cv["grid"] <= 256
    cv4 = sk.ConvPlan(2, 16, 16, 64, 128, 3, 3, (1, 1), ta=sk.BF16, tile=(128, 128, 64, 4), **kw).info()
    assert (cv4["stages"], cv4["waves"]) == (2, 4)
    big = sk.ConvPlan(32, 56, 56, 64, 128, 3, 3, (1, 1), ta=sk.BF16, tile=(128, 128, 64), policy="dp", **kw).info()
    assert big["stages"] == 2 and big["grid"] > 256
    g = sk.GroupedPlan([300, 500], [600, 400], [700, 700], ta=sk.BF16, tile=(128, 128, 64), **kw).info()
    assert g["stages"] == (3 if g["grid"] <= 256 else 2)


def test_calibrate_estimate_terms_match_planner():
    """calibrate.estimate_terms, dotted with a plan's model constants, is the
    planner's own estimate (printed by SKGEMM_LOG) on every 16-bit GEMM tile
    and policy, so constants fitted to it mean what the planner uses; where
    the estimate is larger, the plan's HBM bound set it."""
    import json
    import subprocess
    import sys
    code = ("import sys, json; sys.path.insert(0, %r)\n"
            "from paper_2212_08964_amd import skgemm as sk, calibrate as cal\n"
            "for (M, N, K) in cal.sweep_shapes(40, 3):\n"
            "    for tile in cal.SWEEP_TILES:\n"
            "        occ = 1 if tile[0] * tile[1] == 65536 else 2\n"
            "        for lb in (sk.ROW_MAJOR, sk.COL_MAJOR):\n"
            "            try:\n"
            "                p = sk.Plan(M, N, K, lb=lb, ta=sk.BF16, num_cus=256, occupancy=occ, tile=tile)\n"
            "            except sk.SkgemmError:\n"
            "                continue\n"
            "            t = cal.estimate_terms(p.info())\n"
            "            print(json.dumps(sum(x * y for x, y in zip(t, p.model_constants()))), flush=True)\n"
            "            break\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, SKGEMM_LOG="1"),
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    mine = [json.loads(x) for x in out.stdout.split()]
    logged = [float(ln.split("est_us=")[1].split()[0]) for ln in out.stderr.splitlines()
              if ln.startswith("skgemm: plan")]
    assert len(mine) == len(logged) == 40 * 5
    equal = 0
    for m, e in zip(mine, logged):
        assert e >= m - 0.006, (m, e)
        equal += abs(e - m) <= 0.006
    assert equal >= 0.9 * len(mine)


def test_operand_relayout_plan():
    """Single-GEMM plans keep workspace for a 128-byte-line copy of an operand
    only where its lines (leading dimension = line length) are misaligned and
    the model says the copy pays; the workspace is the fix-up part plus those
    256-byte-aligned regions. Grouped, batched and convolution plans never do."""
    sk = _lib()
    seen = set()
    for (M, N, K), occ, lc in itertools.product(
            [(777, 5555, 3333), (8001, 8001, 8001), (3333, 777, 5555), (4427, 2519, 3013), (1536, 2560, 3072),
             (228, 173, 292), (4096, 4096, 4096), (8000, 8000, 8000)], [1, 2], [sk.ROW_MAJOR, sk.COL_MAJOR]):
        p = sk.Plan(M, N, K, lc=lc, ta=sk.BF16, num_cus=256, occupancy=occ)
        i = p.info()
        Ml, Nl = i["M"], i["N"]
        lines_cols = [(Ml, K) if i["a_kcontig"] else (K, Ml), (Nl, K) if i["b_kcontig"] else (K, Nl)]
        ws = i["fixup_ws_bytes"]
        # the copies go after the fix-up part, never over the shared flag area
        off = max(ws, 256 + 4096 * 128)
        for x, key in enumerate(("pack_a", "pack_b")):
            lines, cols = lines_cols[x]
            if i[key]:
                assert (cols * 2) % 128 != 0, (M, N, K, key)
                off = ((off + 255) // 256) * 256 + ((lines * (-(-cols // 64) * 64) * 2 + 255) // 256) * 256
                ws = off
                seen.add(key)
        assert p.workspace_size() == ws, (M, N, K, occ, lc)
        if M % 64 == 0 and N % 64 == 0 and K % 64 == 0:
            assert not i["pack_a"] and not i["pack_b"]
    assert seen == {"pack_a", "pack_b"}
    g = sk.GroupedPlan([777, 3001], [5555, 4001], [3333, 3333], ta=sk.BF16, num_cus=256, occupancy=1).info()
    b = sk.BatchedPlan(4, 777, 5555, 3333, ta=sk.BF16, num_cus=256, occupancy=1).info()
    c = sk.ConvPlan(8, 57, 57, 64, 96, 3, 3, (1, 1), num_cus=256, occupancy=1).info()
    for info in (g, b, c):
        assert info["pack_a"] == 0 and info["pack_b"] == 0


def test_relayout_option():
    """relayout: -1 never copies, 1 / 2 / 3 copy the caller's A / B / both
    whenever their lines are misaligned (column-major C swaps the launched
    operands, not the caller's names), 0 leaves it to the model; other values
    are refused."""
    sk = _lib()
    M, N, K = 777, 5555, 3333          # K and N both misaligned in BF16
    for lc in (sk.ROW_MAJOR, sk.COL_MAJOR):
        for rl, want in ((-1, (0, 0)), (1, (1, 0)), (2, (0, 1)), (3, (1, 1))):
            i = sk.Plan(M, N, K, lc=lc, ta=sk.BF16, num_cus=256, occupancy=1, relayout=rl).info()
            got = (i["pack_a"], i["pack_b"])
            assert got == (want[::-1] if lc == sk.COL_MAJOR else want), (lc, rl, got)
    aligned = sk.Plan(1024, 2048, 4096, ta=sk.BF16, num_cus=256, occupancy=1, relayout=3).info()
    assert (aligned["pack_a"], aligned["pack_b"]) == (0, 0)
    L = sk.lib()
    h = ctypes.c_void_p()
    o = sk.default_options()
    o.num_cus, o.occupancy = 256, 1
    for bad in (4, -2):
        o.relayout = bad
        assert L.skgemm_plan(ctypes.byref(h), 64, 64, 64, 0, 0, 0, sk.BF16, sk.BF16, sk.BF16,
                             ctypes.byref(o)) == sk.ERR_INVALID_ARG
