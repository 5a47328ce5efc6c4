"""Oracle (test infrastructure only): schedule of a grouped Stream-K launch.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

Several GEMMs share one persistent launch by concatenating their iteration
spaces: problem 0's tiles (each with its own count of MAC-loop iterations)
come first, then problem 1's, and so on.  The policies of the Stream-K
algorithm and its hybrids then apply to that single space unchanged, with a
workgroup's even share allowed to run from one problem into the next.  The
paper evaluates one GEMM at a time; this generalisation is the reading used
for the grouped launch (problems whose K is 0 but which have tiles go after
all others and never join the Stream-K region: their tiles only apply the
epilogue C = beta * C and run as data-parallel tiles; each problem's tiles
linearised m-major, k innermost,
as for one GEMM; the model uses the mean iterations per tile; "auto" is the
paper's selection from the tile count and the processor width).

Everything is computed from an explicit list of tiles by linear search, so it
can be checked by eye; it shares nothing with the device path.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

from .schedule import FULL, OWNER, PARTIAL, Segment, cdiv, model_best_g, owner_of, share_start


@dataclass
class GroupedPlan:
    problems: List[Tuple[int, int, int]]
    BM: int
    BN: int
    BK: int
    p: int
    order: List[int] = field(default_factory=list)                   # problem index per iteration-space position
    tiles: List[Tuple[int, int, int]] = field(default_factory=list)   # (problem, local tile, ipt) per global tile
    first_iter: List[int] = field(default_factory=list)             # first global iteration of each tile
    t: int = 0
    total_iters: int = 0
    policy: str = "dp"
    sk_tiles: int = 0
    sk_iters: int = 0
    g_sk: int = 0
    grid: int = 0
    sk_first: bool = True
    share: str = "proportional"


def make_grouped_plan(problems, BM, BN, BK, p, policy="auto", force_g=0, hybrid_min_waves=2,
                      model=(0.0, 0.0, 1.0, 0.0), share="proportional") -> GroupedPlan:
    pl = GroupedPlan(list(problems), BM, BN, BK, p, share=share)
    # iteration-space order: problems with MAC-loop iterations first (given
    # order), then the K = 0 problems that have tiles
    pl.order = [i for i, (M, N, K) in enumerate(problems) if not (K == 0 and M > 0 and N > 0)] + \
               [i for i, (M, N, K) in enumerate(problems) if K == 0 and M > 0 and N > 0]
    it = 0
    for pi in pl.order:
        M, N, K = problems[pi]
        tm, tn, ipt = cdiv(M, BM), cdiv(N, BN), cdiv(K, BK)
        for lt in range(tm * tn):
            pl.tiles.append((pi, lt, ipt))
            pl.first_iter.append(it)
            it += ipt
    pl.t, pl.total_iters = len(pl.tiles), it
    t = pl.t
    if t == 0:
        return pl
    if it == 0:
        policy = "dp"
    # the policies split the tiles that have iterations; K = 0 tiles follow as
    # data-parallel (epilogue-only) tiles
    tw = sum(1 for (_, _, ipt) in pl.tiles if ipt > 0)
    w, r = divmod(tw, p)
    if policy == "auto":          # the paper's selection, as for one GEMM
        if r == 0:
            policy = "dp"
        elif w == 0:
            policy = "sk"
        elif w >= hybrid_min_waves:
            policy = "2tile_sk_dp"
        else:
            policy = "dp_1tile_sk"
    pl.policy = policy
    if policy == "dp":
        pl.grid = t
        return pl
    if policy == "sk":
        pl.sk_tiles = tw
    elif policy == "dp_1tile_sk":
        pl.sk_tiles, pl.sk_first = r, False
    else:
        pl.sk_tiles = tw if w == 0 else r + p
    pl.sk_iters = pl.total_iters if pl.sk_tiles >= t else pl.first_iter[pl.sk_tiles]
    if policy == "sk":
        if force_g:
            pl.g_sk = force_g
        elif tw >= p:
            pl.g_sk = p
        else:
            pl.g_sk = model_best_g(tw, cdiv(pl.total_iters, tw), p, model)
        pl.g_sk = min(pl.g_sk, pl.sk_iters)     # at most one workgroup per iteration
        pl.grid = pl.g_sk
    else:
        if pl.sk_tiles:
            pl.g_sk = force_g if force_g else min(p, pl.sk_iters)
            pl.g_sk = min(pl.g_sk, pl.sk_iters)
        pl.grid = max(p if t - pl.sk_tiles > 0 else pl.g_sk, pl.g_sk)
    return pl


def _tile_of_iter(pl: GroupedPlan, i: int) -> int:
    for gt in range(pl.t):
        if pl.first_iter[gt] <= i < pl.first_iter[gt] + pl.tiles[gt][2]:
            return gt
    raise IndexError(i)


def enumerate_grouped_schedule(pl: GroupedPlan) -> List[List[Segment]]:
    """Per-workgroup ordered segments; Segment.tile is the global tile index."""
    out = []
    for x in range(pl.grid):
        sk = []
        if x < pl.g_sk:
            it, end = share_start(x, pl.sk_iters, pl.g_sk, pl.share), share_start(x + 1, pl.sk_iters, pl.g_sk, pl.share)
            while it < end:
                gt = _tile_of_iter(pl, it)
                first, last = pl.first_iter[gt], pl.first_iter[gt] + pl.tiles[gt][2]
                lo, hi = it - first, min(end, last) - first
                if it != first:
                    sk.append(Segment(gt, lo, hi, PARTIAL))
                elif end < last:
                    peers = tuple(range(x + 1, owner_of(last - 1, pl.sk_iters, pl.g_sk, pl.share) + 1))
                    sk.append(Segment(gt, lo, hi, OWNER, peers))
                else:
                    sk.append(Segment(gt, lo, hi, FULL))
                it = last
        dp = [Segment(gt, 0, pl.tiles[gt][2], FULL) for gt in range(pl.sk_tiles + x, pl.t, pl.grid)]
        out.append(sk + dp if pl.sk_first else dp + sk)
    return out


def check_grouped_invariants(pl: GroupedPlan, sched: List[List[Segment]]) -> None:
    """Every (tile, k) of every problem covered once; one writer per tile that
    holds k = 0; at most one partial per workgroup; owners' peers are exactly
    the partial holders of their tile, contiguous and above the owner."""
    cover = set()
    writers, parts = {}, {}
    for x, segs in enumerate(sched):
        n_part = 0
        for s in segs:
            for k in range(s.k_lo, s.k_hi):
                assert (s.tile, k) not in cover
                cover.add((s.tile, k))
            if s.role == PARTIAL:
                n_part += 1
                parts.setdefault(s.tile, []).append(x)
            else:
                assert s.k_lo == 0 and s.tile not in writers
                writers[s.tile] = (x, s)
        assert n_part <= 1
    assert len(cover) == pl.total_iters
    assert set(writers) == set(range(pl.t))
    for tile, (x, s) in writers.items():
        got = sorted(parts.get(tile, []))
        if s.role == OWNER:
            assert list(s.peers) == got == list(range(x + 1, x + 1 + len(got))) and got
        else:
            assert not got
