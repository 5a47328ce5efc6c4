"""The library's automatic policy (a design choice for MI355X, not the paper's
selection), checked through the C ABI against the properties it is defined by:

* tiles that fill whole waves, or four full waves and more, stay data-parallel;
* otherwise the remainder tiles (all tiles below one wave) are cut into s equal
  shares with g = s * (their count): basic Stream-K below one wave, DP +
  one-tile SK above, data-parallel when s = 1;
* s minimises the documented cost max(a + b[s > 1] + c_n ceil(ipt / s) +
  d (s - 1), (B + 2 (s - 1) count BM BN 4) / 6 TB/s) over
  1 <= s <= min(p / count, ipt), where c_n is c for grids of at most one
  workgroup per CU and c + (e - c)(n - 1)/(occ - 1) for n = ceil(g / CUs)
  workgroups on a CU (ties to the smaller s); when M, N and K are multiples
  of 64, the search stops at the first s >= 3 whose grid exceeds the CU
  count with fewer than 8 iterations per share; B is the split tiles' share
  (count / t) of the operand bytes (A, B read once, C written once);
* its plans use the split fix-up (every Stream-K tile cut into s one-segment
  shares).
The schedules these plans launch are compared with the oracle's enumerator in
the planner and trace tests (through the explicit policy and grid they resolve
to)."""
import itertools
import math

import pytest


def _sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


HBM_BYTES_PER_US = 6.0e6     # the rate the rule assumes for its memory-bound bound


def _cost(s, count, ipt, p, cus, m, op_bytes=0.0, tile_bytes=0.0):
    a, b, c, d, e = m
    occ = max(1, p // cus)
    n = -(-(s * count) // cus)
    cn = c if n <= 1 or occ <= 1 else c + (e - c) * (n - 1) / (occ - 1)
    compute = a + (b if s > 1 else 0.0) + cn * -(-ipt // s) + d * (s - 1)
    return max(compute, (op_bytes + 2.0 * (s - 1) * count * tile_bytes) / HBM_BYTES_PER_US)


SHAPES = [(384, 384, 1024), (1024, 1024, 1024), (300, 500, 700), (4096, 4096, 64), (128, 8192, 8192),
          (2048, 2048, 8192), (8192, 8192, 8192), (1000, 130, 5), (7, 3000, 4000), (256 * 17, 256 * 16, 1000),
          (256 * 33, 256 * 9, 300), (5632, 384, 768), (3328, 2304, 3968), (650, 201, 5611), (128, 128, 64)]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_auto_policy_properties(dtype):
    sk = _sk()
    ta = {"f32": sk.F32, "bf16": sk.BF16, "f64": sk.F64}[dtype]
    seen = set()
    for (M, N, K), (cus, occ) in itertools.product(SHAPES, [(256, 1), (256, 2), (37, 3), (8, 1)]):
        p_ = sk.Plan(M, N, K, ta=ta, policy="auto", num_cus=cus, occupancy=occ)
        info, m = p_.info(), p_.model_constants()
        p, t, ipt = info["p"], info["t"], info["ipt"]
        w, r = divmod(t, p)
        pol = info["policy_name"]
        if r == 0 or w >= 4:
            assert pol == "dp", (M, N, K, cus, occ)
            seen.add("dp-waves")
            continue
        count = t if w == 0 else r
        smax = max(1, min(p // count, ipt))
        aligned = M % 64 == 0 and N % 64 == 0 and K % 64 == 0
        if aligned:
            for s_ in range(3, smax + 1):
                if s_ * count > cus and -(-ipt // s_) < 8:
                    smax = s_ - 1
                    break
        eb = {sk.F32: 4, sk.BF16: 2, sk.F64: 8}[ta]
        op = float((M * K + K * N) * eb + M * N * eb) * count / t     # the split region's share
        tb = float(info["BM"] * info["BN"] * (8 if ta == sk.F64 else 4))
        costs = [_cost(s, count, ipt, p, cus, m, op, tb) for s in range(1, smax + 1)]
        best = 1 + min(range(len(costs)), key=lambda i: (costs[i], i))
        if best == 1:
            assert pol == "dp" and info["grid"] == t, (M, N, K, cus, occ)
            seen.add("dp-model")
            continue
        assert pol == ("sk" if w == 0 else "dp_1tile_sk"), (M, N, K, cus, occ, pol)
        assert (info["sk_tiles"], info["g_sk"]) == (count, best * count), (M, N, K, cus, occ)
        assert info["coop_s"] == best
        assert info["grid"] == (best * count if w == 0 else p)
        seen.add(pol)
    assert {"dp-waves", "dp-model", "sk", "dp_1tile_sk"} <= seen, seen


def test_auto_policy_hand_worked_cases():
    """Cases whose choice follows from the rule without its constants."""
    sk = _sk()
    # 1024 tiles of 256x256 on 256 CUs: four full waves, no remainder
    assert sk.Plan(8192, 8192, 8192, ta=sk.BF16, num_cus=256, occupancy=1, tile=(256, 256, 64)).info()[
        "policy_name"] == "dp"
    # four full waves and a remainder: data-parallel
    info = sk.Plan(256 * (16 * 4 + 1), 256 * 16, 4096, ta=sk.BF16, num_cus=256, occupancy=1,
                   tile=(256, 256, 64)).info()
    assert (info["t"] // info["p"], info["policy_name"]) == (4, "dp")
    # one iteration per tile cannot be split
    info = sk.Plan(1000, 1000, 64, ta=sk.BF16, num_cus=256, occupancy=1, tile=(256, 256, 64)).info()
    assert (info["ipt"], info["policy_name"]) == (1, "dp")
    # one tile with 128 iterations on 256 CUs: split (a data-parallel tile would
    # run all 128 iterations on one CU)
    info = sk.Plan(128, 128, 8192, ta=sk.BF16, num_cus=256, occupancy=2, tile=(128, 128, 64, 4)).info()
    assert info["policy_name"] == "sk" and info["g_sk"] > 1 and info["coop_s"] == info["g_sk"]


def test_paper_policy_is_the_papers_selection_in_the_library():
    """SKGEMM_POLICY_PAPER resolves like the oracle's "auto"."""
    sk = _sk()
    from helpers import oracle_plan_for
    for (M, N, K), (cus, occ) in itertools.product(SHAPES, [(256, 1), (4, 1), (37, 3)]):
        try:
            p_ = sk.Plan(M, N, K, ta=sk.F32, policy="paper", num_cus=cus, occupancy=occ)
        except sk.SkgemmError as e:
            assert e.status == sk.ERR_CAPACITY
            continue
        info = p_.info()
        ref = oracle_plan_for(info, p_.model_constants(), "paper")
        assert (ref.policy, ref.sk_tiles, ref.g_sk, ref.grid, ref.sk_first) == (
            info["policy_name"], info["sk_tiles"], info["g_sk"], info["grid"], bool(info["sk_first"]))


def test_auto_three_stage_rule():
    """Automatic plans of the small 16-bit tile: a split over more workgroups
    than CUs (two-stage kernel) stands only where the three-stage rule does
    not apply (with at most CUs/2 tiles, fewer than 12 iterations per tile;
    with more tiles, 32 or more); the rule's replacements have the forms it
    defines (floor(CUs/t) shares per tile, or data-parallel tiles, on the
    three-stage kernel); explicit policies are never changed."""
    import workloads as W
    sk = _sk()
    cus = 256
    seen = set()
    for (M, N, K) in W.sweep_shapes(600, seed=5):
        got = sk.Plan(M, N, K, ta=sk.BF16, num_cus=cus, occupancy=2, tile=(128, 128, 64)).info()
        t, ipt = got["t"], got["ipt"]
        if got["stages"] == 2 and got["policy_name"] == "sk" and got["g_sk"] > cus and t <= cus:
            assert not (2 * t <= cus and ipt >= 12) and not (2 * t > cus and ipt < 32), (M, N, K)
            seen.add("kept")
        elif got["stages"] == 3 and got["policy_name"] == "sk" and 2 * t <= cus and ipt >= 12 \
                and got["g_sk"] == cus // t * t:
            assert got["p"] == cus and got["waves"] == 8
            seen.add("split")
        elif got["stages"] == 3 and got["policy_name"] == "dp" and 2 * t > cus and ipt < 32:
            assert got["grid"] == t <= cus
            seen.add("dp")
        # explicit policies and forced grids are never changed by the rule
        exp = sk.Plan(M, N, K, ta=sk.BF16, num_cus=cus, occupancy=2, tile=(128, 128, 64), policy="sk").info()
        assert exp["stages"] == (3 if exp["grid"] <= cus else 2)
    assert seen == {"split", "dp", "kept"}
