"""Oracle (test infrastructure only): enumerator of the Stream-K decomposition.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

It lists, for every workgroup (the paper's CTA) of a launch, the ordered
segments of MAC-loop iterations it performs, following the Work Decomposition
Strategies section (data-parallel, fixed-split and basic Stream-K algorithms),
the Data-parallel Hybridization subsection (the "DP + one-tile SK" and
"two-tile SK + DP" schedules) and the analytical grid-size model of the
Kernel Configuration subsection.

Readings taken where the paper is silent or garbled (each is listed with its
reason in the design notes):

* Tiles are linearised m-major then n (tile index -> row block = idx // tn,
  column block = idx % tn), with k innermost.  The printed MacLoop divides by
  ceil(m / BLK_M) for both coordinates, which is only consistent for square
  tile grids; the prose's m -> n -> k linearisation is followed instead.
* Even share "within one": every workgroup gets floor(total / g) or
  ceil(total / g) contiguous iterations.  The printed ceil(total / g) split
  overruns on the last CTA; a within-one split is the one that reproduces the
  132/133 iterations per CTA of the model figure.  Which workgroups get the
  extra iteration the paper does not say; two rules are provided:
  proportional (workgroup x starts at floor(x * total / g), the default) and
  leading (q, r = divmod(total, g); workgroup x starts at x*q + min(x, r)).
  Under the proportional rule a grid g = s * t cuts every tile into s parts
  at the same k-offsets.
* The accumulating workgroup of a tile (the one that ran its k = 0 iteration)
  receives partials from workgroups x+1 .. owner_of(last iteration of the
  tile), in ascending order; the printed "cta_end" expression is a tile index
  and is replaced by that owner.
* The Stream-K region of a hybrid schedule is tiles [0, sk_tiles); the
  data-parallel tiles follow and workgroup x takes sk_tiles + x + i * grid.
  "Two-tile SK + DP" runs its Stream-K share first, "DP + one-tile SK" its
  data-parallel tiles first.
* The automatic policy is the paper's own selection (Data-parallel
  Hybridization subsection): no remainder tiles (t mod p == 0) ->
  data-parallel; fewer tiles than workgroups -> basic Stream-K with g from
  the grid-size model over [t, p]; ``hybrid_min_waves`` (default two) or
  more full waves -> two-tile SK + DP; otherwise DP + one-tile SK with
  g = min(p, sk_tiles * ipt).  A library may resolve "auto" by its own rule;
  such a plan is compared here through the explicit policy and grid it
  resolved to.
* K = 0 gives zero iterations per tile; every policy then degenerates to
  data-parallel tiles that only apply the epilogue (C = beta * C).
* Model ties are broken toward the smallest g (fewer partial tiles).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

FULL = "full"        # starts and ends its tile: writes C directly
PARTIAL = "partial"  # does not start its tile: publishes a partial tile
OWNER = "owner"      # starts but does not end its tile: adds peers' partials, writes C

POLICIES = ("auto", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp")


def cdiv(a: int, b: int) -> int:
    return -(-a // b)


@dataclass(frozen=True)
class Segment:
    tile: int                 # linear output-tile index
    k_lo: int                 # first MAC-loop iteration of the tile covered
    k_hi: int                 # one past the last
    role: str
    peers: Tuple[int, ...] = ()   # OWNER only: workgroups whose partials it adds


@dataclass
class Plan:
    M: int
    N: int
    K: int
    BM: int
    BN: int
    BK: int
    p: int
    tm: int = 0
    tn: int = 0
    t: int = 0
    ipt: int = 0
    policy: str = "dp"        # resolved policy
    sk_tiles: int = 0         # tiles [0, sk_tiles) form the Stream-K region
    g_sk: int = 0             # workgroups sharing the Stream-K region
    grid: int = 0             # workgroups launched
    sk_first: bool = True     # per-workgroup order: Stream-K share before DP tiles
    model: Tuple[float, float, float, float] = (0.0, 0.0, 1.0, 0.0)
    share: str = "proportional"   # even-share rule: "proportional" or "leading"

    @property
    def total_iters(self) -> int:
        return self.t * self.ipt

    @property
    def sk_iters(self) -> int:
        return self.sk_tiles * self.ipt

    @property
    def dp_tiles(self) -> int:
        return self.t - self.sk_tiles


# ---------------------------------------------------------------- iteration space

def iteration_space(M: int, N: int, K: int, BM: int, BN: int, BK: int):
    """(tm, tn, t, ipt, T): tile-grid extents, tile count, MAC-loop iterations
    per tile and total iterations, all by ceiling division."""
    tm, tn = cdiv(M, BM), cdiv(N, BN)
    ipt = cdiv(K, BK)
    t = tm * tn
    return tm, tn, t, ipt, t * ipt


def tile_origin(tile: int, tn: int, BM: int, BN: int) -> Tuple[int, int]:
    """Top-left element (row, column) of a linear tile index (m-major, then n)."""
    return BM * (tile // tn), BN * (tile % tn)


def share_start(x: int, total: int, g: int, share: str = "proportional") -> int:
    """First iteration of workgroup x under the within-one even share."""
    if share == "proportional":
        return x * total // g
    q, r = divmod(total, g)
    return x * q + min(x, r)


def owner_of(i: int, total: int, g: int, share: str = "proportional") -> int:
    """Workgroup whose within-one share contains iteration i (found by
    walking the share boundaries, not by inverting their formula)."""
    lo, hi = 0, g - 1
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if share_start(mid, total, g, share) <= i:
            lo = mid
        else:
            hi = mid - 1
    return lo


# ---------------------------------------------------------------- analytical model

def model_iters_per_cta(g: int, t: int, ipt: int) -> int:
    return cdiv(t * ipt, g)


def model_fixup_peers(g: int, t: int, ipt: int) -> int:
    return cdiv(ipt, model_iters_per_cta(g, t, ipt))


def model_time(g: int, t: int, ipt: int, a: float, b: float, c: float, d: float) -> float:
    """Runtime of one tile-producing workgroup as a function of grid size g:
    fixed cost a, plus b if any tile needs partials from other workgroups,
    plus c per MAC-loop iteration, plus d per extra collaborator."""
    peers = model_fixup_peers(g, t, ipt)
    return a + b * (1 if peers > 1 else 0) + c * model_iters_per_cta(g, t, ipt) + d * (peers - 1)


def model_best_g(t: int, ipt: int, p: int, consts) -> int:
    """Grid size in [t, p] with the smallest modelled time (smallest g on ties)."""
    a, b, c, d = consts[:4]
    lo, hi = t, max(t, p)
    best_g, best = lo, None
    for g in range(lo, hi + 1):
        v = model_time(g, t, ipt, a, b, c, d)
        if best is None or v < best:
            best, best_g = v, g
    return best_g


# ---------------------------------------------------------------- planning

def make_plan(M: int, N: int, K: int, BM: int, BN: int, BK: int, p: int,
              policy: str = "auto", force_g: int = 0, hybrid_min_waves: int = 2,
              model=(0.0, 0.0, 1.0, 0.0), share: str = "proportional") -> Plan:
    """Resolve a policy into the Stream-K region and the launch grid."""
    if policy not in POLICIES:
        raise ValueError(policy)
    tm, tn, t, ipt, T = iteration_space(M, N, K, BM, BN, BK)
    pl = Plan(M, N, K, BM, BN, BK, p, tm, tn, t, ipt, model=tuple(model), share=share)
    if t == 0:
        pl.policy, pl.grid = "dp", 0
        return pl
    if ipt == 0:
        policy = "dp"
    w, r = divmod(t, p)
    if policy == "auto":
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
        pl.sk_tiles, pl.g_sk, pl.grid = 0, 0, t
        return pl
    if policy == "sk":
        pl.sk_tiles = t
        if force_g:
            pl.g_sk = force_g
        elif t >= p:
            pl.g_sk = p
        else:
            pl.g_sk = model_best_g(t, ipt, p, model)
        pl.g_sk = min(pl.g_sk, pl.sk_iters)     # at most one workgroup per iteration
        pl.grid = pl.g_sk
        return pl
    if policy == "dp_1tile_sk":
        pl.sk_tiles = r
        pl.sk_first = False
    else:  # 2tile_sk_dp
        pl.sk_tiles = t if w == 0 else r + p
        pl.sk_first = True
    if pl.sk_tiles:
        pl.g_sk = force_g if force_g else min(p, pl.sk_tiles * ipt)
        pl.g_sk = min(pl.g_sk, pl.sk_iters)
    pl.grid = p if pl.dp_tiles > 0 else pl.g_sk
    pl.grid = max(pl.grid, pl.g_sk)
    return pl


# ---------------------------------------------------------------- enumeration

def streamk_share(x: int, pl: Plan) -> List[Segment]:
    """Segments of workgroup x in the Stream-K region: walk its contiguous
    share of iterations, cutting at tile seams."""
    if x >= pl.g_sk or pl.sk_tiles == 0:
        return []
    total, g, ipt = pl.sk_iters, pl.g_sk, pl.ipt
    it, it_end = share_start(x, total, g, pl.share), share_start(x + 1, total, g, pl.share)
    segs = []
    while it < it_end:
        tile = it // ipt
        first, last = tile * ipt, tile * ipt + ipt
        lo, hi = it - first, min(it_end, last) - first
        if it != first:
            segs.append(Segment(tile, lo, hi, PARTIAL))
        elif it_end < last:
            end_wg = owner_of(last - 1, total, g, pl.share)
            segs.append(Segment(tile, lo, hi, OWNER, tuple(range(x + 1, end_wg + 1))))
        else:
            segs.append(Segment(tile, lo, hi, FULL))
        it = last
    return segs


def dp_share(x: int, pl: Plan) -> List[Segment]:
    """Whole data-parallel tiles of workgroup x."""
    if pl.policy == "dp":
        return [Segment(x, 0, pl.ipt, FULL)] if x < pl.t else []
    return [Segment(tile, 0, pl.ipt, FULL) for tile in range(pl.sk_tiles + x, pl.t, pl.grid)]


def enumerate_schedule(pl: Plan) -> List[List[Segment]]:
    """Ordered segment list of every launched workgroup."""
    out = []
    for x in range(pl.grid):
        sk, dp = streamk_share(x, pl), dp_share(x, pl)
        out.append(sk + dp if pl.sk_first else dp + sk)
    return out


def fixed_split_schedule(t: int, ipt: int, s: int) -> List[List[Segment]]:
    """Fixed-split decomposition with splitting factor s: workgroup (x, y) is
    listed at index x * s + y and covers split y of tile x; split 0 adds the
    partials of splits 1 .. s-1 (ceil-sized splits)."""
    ips = cdiv(ipt, s)
    out = []
    for x in range(t):
        for y in range(s):
            lo = y * ips
            hi = min(ipt, lo + ips)
            lo = min(lo, hi)
            if y != 0:
                out.append([Segment(x, lo, hi, PARTIAL)])
            elif s > 1:
                out.append([Segment(x, lo, hi, OWNER, tuple(x * s + c for c in range(1, s)))])
            else:
                out.append([Segment(x, lo, hi, FULL)])
    return out


def dp_utilization_ceiling(t: int, p: int) -> float:
    """Fraction of the processor kept busy by t equal work units in waves of p."""
    return t / (p * cdiv(t, p))


def check_invariants(pl: Plan, sched: List[List[Segment]]) -> None:
    """Structural invariants of a schedule; raises AssertionError on violation.

    Every (tile, k) pair is covered exactly once; each tile has one writer,
    which holds its k = 0 iteration; each workgroup publishes at most one
    partial; an owner's peers are exactly the workgroups holding partial
    segments of its tile, contiguous and ascending, all above the owner."""
    cover = {}
    writers = {}
    partials_by_tile = {}
    for x, segs in enumerate(sched):
        n_part = 0
        for s in segs:
            for k in range(s.k_lo, s.k_hi):
                key = (s.tile, k)
                assert key not in cover, f"iteration {key} covered twice"
                cover[key] = x
            if s.role == PARTIAL:
                n_part += 1
                assert s.k_lo > 0
                partials_by_tile.setdefault(s.tile, []).append(x)
            else:
                assert s.k_lo == 0, "writer must hold k = 0"
                assert s.tile not in writers, "two writers"
                writers[s.tile] = (x, s)
        assert n_part <= 1, "more than one partial per workgroup"
    assert len(cover) == pl.t * pl.ipt, "iterations missing"
    assert set(writers) == set(range(pl.t)), "tile without writer"
    for tile, (x, s) in writers.items():
        parts = sorted(partials_by_tile.get(tile, []))
        if s.role == OWNER:
            assert list(s.peers) == parts and parts, "owner peers mismatch"
            assert parts == list(range(x + 1, x + 1 + len(parts))), "peers not contiguous"
        else:
            assert not parts, "full tile has partials"
