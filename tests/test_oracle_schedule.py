"""Pins of the schedule enumerator and the grid-size model.

* the paper's worked examples (golden fixture, each entry cites its passage);
* exhaustive tiny problems: every (tile, k) covered once, one writer per tile
  holding k = 0, at most one partial per workgroup, owner peers contiguous
  and above the owner, even share within one, at most two contributors per
  tile when the Stream-K region has at least as many tiles as workgroups;
* the generalisations stated in the Stream-K subsection: g = t behaves like
  data-parallel, g = s * t like fixed-split s (when s divides the iterations
  per tile);
* the model reproduces the three published best grid sizes.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import grouped as GR
from oracle import schedule as S

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "streamk_worked_examples.json")))


def test_dp_ceilings():
    for e in GOLDEN["dp_ceiling"]:
        tm, tn, t, _, _ = S.iteration_space(e["M"], e["N"], e["K"], e["BM"], e["BN"], 1)
        assert t == e["tiles"]
        assert S.dp_utilization_ceiling(t, e["p"]) == pytest.approx(e["ceiling"])


def test_fixed_split_example():
    e = GOLDEN["fixed_split"][0]
    _, _, t, ipt, _ = S.iteration_space(e["M"], e["N"], e["K"], e["BM"], e["BN"], e["BK"])
    sched = S.fixed_split_schedule(t, ipt, e["s"])
    assert len(sched) == e["grid"]
    assert all((segs[0].k_hi - segs[0].k_lo) * e["BK"] == e["k_per_cta"] for segs in sched)
    assert S.dp_utilization_ceiling(len(sched), e["p"]) == pytest.approx(e["efficiency"])


def test_basic_streamk_example():
    e = GOLDEN["basic_streamk"][0]
    pl = S.make_plan(e["M"], e["N"], e["K"], e["BM"], e["BN"], e["BK"], p=e["g"], policy="sk", force_g=e["g"])
    assert pl.ipt == e["iters_per_tile"]
    sched = S.enumerate_schedule(pl)
    for segs in sched:
        n = sum(s.k_hi - s.k_lo for s in segs)
        assert n == e["iters_per_cta"]
        assert n * e["BK"] == e["k_volume_per_cta"]
    S.check_invariants(pl, sched)


def test_skew_example():
    e = GOLDEN["skew"][0]
    pl = S.make_plan(e["M"], e["N"], e["K"], e["BM"], e["BN"], e["BK"], p=e["g"], policy="sk", force_g=e["g"])
    sched = S.enumerate_schedule(pl)
    assert [segs[0].k_lo * e["BK"] for segs in sched] == e["k_offsets"]


def test_hybrid_examples_peer_counts():
    # 896x384x128 on four SMs, 128x128x4 tiles: two-tile SK + DP gives each owner
    # exactly one peer; DP + one-tile SK puts three peers on one owner.
    two = S.make_plan(896, 384, 128, 128, 128, 4, p=4, policy="2tile_sk_dp")
    one = S.make_plan(896, 384, 128, 128, 128, 4, p=4, policy="dp_1tile_sk")
    # the paper's automatic choice for two or more full waves (kept for grouped
    # launches whose problems differ in iterations per tile)
    paper = GR.make_grouped_plan([(896, 384, 128), (128, 128, 8)], 128, 128, 4, p=4)
    assert paper.policy == "2tile_sk_dp"
    owners2 = [s for segs in S.enumerate_schedule(two) for s in segs if s.role == S.OWNER]
    owners1 = [s for segs in S.enumerate_schedule(one) for s in segs if s.role == S.OWNER]
    assert owners2 and all(len(s.peers) == 1 for s in owners2)
    assert len(owners1) == 1 and owners1[0].peers == (1, 2, 3)
    assert two.sk_tiles == 5 and one.sk_tiles == 1
    for pl in (two, one):
        S.check_invariants(pl, S.enumerate_schedule(pl))


def test_model_reproduces_published_grid_sizes():
    tile = GOLDEN["model_tile"]
    for e in GOLDEN["model"]:
        _, _, t, ipt, T = S.iteration_space(e["M"], e["N"], e["K"], tile["BM"], tile["BN"], tile["BK"])
        assert (t, ipt) == (e["tiles"], e["iters_per_tile"])
        g = S.model_best_g(t, ipt, tile["p"], (0.0, 20.0, 1.0, 8.0))
        assert g == e["g_best"]
        pl = S.make_plan(e["M"], e["N"], e["K"], tile["BM"], tile["BN"], tile["BK"], p=tile["p"],
                         policy="sk", force_g=g)
        counts = sorted({sum(s.k_hi - s.k_lo for s in segs) for segs in S.enumerate_schedule(pl)})
        assert counts == e["iters_per_cta"]


def test_model_sensitivity():
    """A dropped term of the model changes at least one published choice."""
    tile = GOLDEN["model_tile"]
    shapes = [(e["M"], e["N"], e["K"]) for e in GOLDEN["model"]]
    want = [e["g_best"] for e in GOLDEN["model"]]
    for consts in [(0, 0, 1, 8), (0, 20, 1, 0), (0, 20, 0, 8)]:
        got = []
        for M, N, K in shapes:
            _, _, t, ipt, _ = S.iteration_space(M, N, K, tile["BM"], tile["BN"], tile["BK"])
            got.append(S.model_best_g(t, ipt, tile["p"], consts))
        assert got != want


def _tiny_cases():
    for M, N, K in itertools.product(range(1, 6), range(1, 6), range(0, 6)):
        yield M, N, K


@pytest.mark.parametrize("policy", ["sk", "dp", "dp_1tile_sk", "2tile_sk_dp", "auto"])
def test_exhaustive_tiny_invariants(policy):
    BM = BN = 2
    BK = 1
    n_checked = 0
    for M, N, K in _tiny_cases():
        _, _, t, ipt, T = S.iteration_space(M, N, K, BM, BN, BK)
        for p in range(1, max(T, t) + 2):
            gs = range(1, T + 1) if policy == "sk" and T else [0]
            for g in gs:
                pl = S.make_plan(M, N, K, BM, BN, BK, p=p, policy=policy, force_g=g)
                sched = S.enumerate_schedule(pl)
                S.check_invariants(pl, sched)
                if pl.g_sk:
                    shares = [sum(s.k_hi - s.k_lo for s in S.streamk_share(x, pl)) for x in range(pl.g_sk)]
                    q = pl.sk_iters // pl.g_sk
                    assert set(shares) <= {q, q + 1}
                    if pl.sk_tiles >= pl.g_sk:
                        contrib = {}
                        for x in range(pl.g_sk):
                            for s in S.streamk_share(x, pl):
                                contrib.setdefault(s.tile, set()).add(x)
                        assert max(len(v) for v in contrib.values()) <= 2
                n_checked += 1
    assert n_checked > 100


def test_sk_with_g_equal_t_is_data_parallel():
    for M, N, K in [(384, 384, 128), (1000, 300, 77), (128, 128, 1)]:
        pl = S.make_plan(M, N, K, 128, 128, 4, p=1024, policy="sk", force_g=0)
        force = S.make_plan(M, N, K, 128, 128, 4, p=1024, policy="sk", force_g=pl.t)
        dp = S.make_plan(M, N, K, 128, 128, 4, p=1024, policy="dp")
        assert S.enumerate_schedule(force) == S.enumerate_schedule(dp)


@pytest.mark.parametrize("s", [2, 4, 8])
def test_sk_with_g_multiple_of_t_is_fixed_split(s):
    M, N, K = 384, 256, 256
    pl = S.make_plan(M, N, K, 128, 128, 8, p=4096, policy="sk", force_g=0)
    assert pl.ipt % s == 0
    sk = S.make_plan(M, N, K, 128, 128, 8, p=4096, policy="sk", force_g=s * pl.t)
    assert S.enumerate_schedule(sk) == S.fixed_split_schedule(pl.t, pl.ipt, s)


def test_auto_policy_is_the_papers_selection():
    """The oracle's "auto" follows the Data-parallel Hybridization subsection,
    each branch pinned by a hand-worked case."""
    # tiles fill whole waves (1024 tiles of 256x256 on 256 workgroups): data-parallel
    pl = S.make_plan(8192, 8192, 8192, 256, 256, 64, 256)
    assert (pl.policy, pl.grid, pl.g_sk) == ("dp", 1024, 0)
    # fewer tiles than workgroups: basic Stream-K with the model's grid, which
    # reproduces the published grid sizes of the model figure
    tile = GOLDEN["model_tile"]
    for e in GOLDEN["model"]:
        pl = S.make_plan(e["M"], e["N"], e["K"], tile["BM"], tile["BN"], tile["BK"], p=tile["p"],
                         model=(0.0, 20.0, 1.0, 8.0))
        assert (pl.policy, pl.sk_tiles, pl.g_sk, pl.grid) == ("sk", e["tiles"], e["g_best"], e["g_best"])
    # two full waves and one tile over (the 896x384 example on four SMs):
    # two-tile SK + DP over r + p = 5 tiles, then the 16 others data-parallel
    pl = S.make_plan(896, 384, 128, 128, 128, 4, p=4)
    assert (pl.policy, pl.sk_tiles, pl.g_sk, pl.grid, pl.sk_first) == ("2tile_sk_dp", 5, 4, 4, True)
    # one full wave and a remainder: DP + one-tile SK, g = min(p, r * ipt)
    pl = S.make_plan(128 * 5, 128, 64, 128, 128, 32, p=4)      # t = 5, r = 1, ipt = 2
    assert (pl.policy, pl.sk_tiles, pl.g_sk, pl.grid, pl.sk_first) == ("dp_1tile_sk", 1, 2, 4, False)
    pl = S.make_plan(128 * 7, 128, 1024, 128, 128, 32, p=4)    # t = 7, r = 3, ipt = 32
    assert (pl.policy, pl.sk_tiles, pl.g_sk, pl.grid) == ("dp_1tile_sk", 3, 4, 4)
    # the two-tile threshold is hybrid_min_waves full waves
    pl = S.make_plan(896, 384, 128, 128, 128, 4, p=4, hybrid_min_waves=6)    # w = 5
    assert (pl.policy, pl.sk_tiles) == ("dp_1tile_sk", 1)
    pl = S.make_plan(896, 384, 128, 128, 128, 4, p=4, hybrid_min_waves=5)
    assert (pl.policy, pl.sk_tiles) == ("2tile_sk_dp", 5)
    # K = 0: epilogue-only tiles, data-parallel whatever the policy
    for pol in S.POLICIES:
        pl = S.make_plan(300, 300, 0, 128, 128, 32, p=4, policy=pol)
        assert (pl.policy, pl.grid) == ("dp", 9)


@pytest.mark.parametrize("t,ipt,s", [(3, 10, 4), (7, 9, 2), (5, 64, 8), (12, 88, 10), (1, 7, 7)])
def test_proportional_share_cuts_every_tile_alike(t, ipt, s):
    """With g = s * t the proportional share cuts every tile at the same k-offsets (the
    offsets of the within-one split of ipt into s parts), whether or not s divides ipt;
    the leading rule does not when s does not divide ipt."""
    M, N, K = 128 * t, 128, 8 * ipt
    prop = S.make_plan(M, N, K, 128, 128, 8, p=4096, policy="sk", force_g=s * t)
    sched = S.enumerate_schedule(prop)
    S.check_invariants(prop, sched)
    cuts = [sorted(seg.k_lo for segs in sched for seg in segs if seg.tile == x) for x in range(t)]
    assert all(c == cuts[0] for c in cuts) and len(cuts[0]) == s
    sizes = [seg.k_hi - seg.k_lo for segs in sched for seg in segs]
    assert max(sizes) - min(sizes) <= 1
    lead = S.make_plan(M, N, K, 128, 128, 8, p=4096, policy="sk", force_g=s * t, share="leading")
    lcuts = [sorted(seg.k_lo for segs in S.enumerate_schedule(lead) for seg in segs if seg.tile == x)
             for x in range(t)]
    assert (all(c == lcuts[0] for c in lcuts)) == (ipt % s == 0 or t == 1)


def test_share_rules_are_within_one():
    for total in (1, 7, 100, 288, 1000):
        for g in (1, 2, 3, 7, 64, total):
            for share in ("proportional", "leading"):
                starts = [S.share_start(x, total, g, share) for x in range(g + 1)]
                sizes = [b - a for a, b in zip(starts, starts[1:])]
                assert starts[0] == 0 and starts[-1] == total
                assert set(sizes) <= {total // g, -(-total // g)}
                for i in range(total):
                    x = S.owner_of(i, total, g, share)
                    assert starts[x] <= i < starts[x + 1]


def test_planted_mistake_is_caught():
    """The invariant checker fails on a schedule with a dropped iteration and on
    one whose owner lists the wrong peer."""
    pl = S.make_plan(896, 384, 128, 128, 128, 4, p=4, policy="sk", force_g=4)
    sched = S.enumerate_schedule(pl)
    broken = [list(x) for x in sched]
    s0 = broken[0][-1]
    broken[0][-1] = S.Segment(s0.tile, s0.k_lo, s0.k_hi - 1, s0.role, s0.peers)
    with pytest.raises(AssertionError):
        S.check_invariants(pl, broken)
    broken = [list(x) for x in sched]
    broken[0][-1] = S.Segment(s0.tile, s0.k_lo, s0.k_hi, s0.role, (2,))
    with pytest.raises(AssertionError):
        S.check_invariants(pl, broken)


# ------------------------------------------------------------------ grouped launches

def test_grouped_single_problem_equals_single_enumerator():
    from oracle import grouped as GR
    for (M, N, K), p, pol in itertools.product([(384, 384, 128), (896, 384, 128), (1000, 130, 77)], [4, 9, 64],
                                               ["auto", "sk", "dp", "dp_1tile_sk", "2tile_sk_dp"]):
        g = GR.make_grouped_plan([(M, N, K)], 128, 128, 4, p, policy=pol, model=(0, 20, 1, 8))
        s = S.make_plan(M, N, K, 128, 128, 4, p, policy=pol, model=(0, 20, 1, 8))
        assert (g.policy, g.sk_tiles, g.g_sk, g.grid) == (s.policy, s.sk_tiles, s.g_sk, s.grid)
        assert GR.enumerate_grouped_schedule(g) == S.enumerate_schedule(s)


def test_grouped_equal_ipt_is_one_long_tile_row():
    """Problems with equal iterations per tile concatenate into the same
    iteration space as one GEMM whose tile count is their sum."""
    from oracle import grouped as GR
    probs = [(128 * 3, 128 * 2, 256), (128, 128 * 5, 256), (128 * 2, 128, 256)]   # 6 + 5 + 2 tiles, ipt 64
    for p, pol in itertools.product([3, 4, 7, 32], ["sk", "2tile_sk_dp", "dp_1tile_sk", "auto"]):
        g = GR.make_grouped_plan(probs, 128, 128, 4, p, policy=pol, model=(0, 20, 1, 8))
        s = S.make_plan(128 * 13, 128, 256, 128, 128, 4, p, policy=pol, model=(0, 20, 1, 8))
        assert GR.enumerate_grouped_schedule(g) == S.enumerate_schedule(s)


def test_grouped_ragged_invariants():
    from oracle import grouped as GR
    rng = __import__("random").Random(0)
    for _ in range(60):
        G = rng.randint(1, 6)
        probs = [(rng.randint(0, 9), rng.randint(1, 9), rng.randint(1, 9)) for _ in range(G)]
        for p in (1, 2, 5, 16):
            for pol in ("auto", "sk", "dp", "dp_1tile_sk", "2tile_sk_dp"):
                g = GR.make_grouped_plan(probs, 2, 2, 1, p, policy=pol)
                GR.check_grouped_invariants(g, GR.enumerate_grouped_schedule(g))


def test_grouped_zero_k_problems_are_epilogue_tiles_after_the_rest():
    """Problems with K = 0 leave the Stream-K schedule of the others unchanged
    wherever they sit in the list: their tiles come last and each is one
    data-parallel segment with no iterations (C = beta * C)."""
    from oracle import grouped as GR
    work = [(1000, 900, 3000), (500, 256, 640), (128, 700, 130)]
    zero = [(300, 700, 0), (64, 64, 0), (0, 50, 0)]
    for p, pol in itertools.product([4, 9, 64], ["auto", "sk", "dp", "dp_1tile_sk", "2tile_sk_dp"]):
        base = GR.make_grouped_plan(work, 128, 128, 32, p, policy=pol, model=(0, 20, 1, 8))
        mixed_list = [zero[0], work[0], zero[1], work[1], zero[2], work[2]]
        mixed = GR.make_grouped_plan(mixed_list, 128, 128, 32, p, policy=pol, model=(0, 20, 1, 8))
        assert mixed.order == [1, 3, 4, 5, 0, 2]     # (0, 50, 0) has no tiles: it stays in place
        n_zero = sum(-(-M // 128) * -(-N // 128) for M, N, K in zero)
        assert mixed.t == base.t + n_zero and mixed.total_iters == base.total_iters
        assert (mixed.sk_tiles, mixed.g_sk, mixed.sk_iters) == (base.sk_tiles, base.g_sk, base.sk_iters)
        sched = GR.enumerate_grouped_schedule(mixed)
        GR.check_grouped_invariants(mixed, sched)
        sk_part = [[s for s in segs if s.tile < base.t] for segs in sched]
        want = GR.enumerate_grouped_schedule(base)
        if mixed.grid == base.grid:
            assert sk_part == want
        else:   # a data-parallel grid grows by the epilogue tiles
            assert pol == "dp" or base.policy == "dp"
        zero_segs = [s for segs in sched for s in segs if s.tile >= base.t]
        assert sorted(s.tile for s in zero_segs) == list(range(base.t, mixed.t))
        assert all((s.k_lo, s.k_hi, s.role) == (0, 0, S.FULL) for s in zero_segs)
