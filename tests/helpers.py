"""Shared test helpers: tensor/array conversions and schedule comparison.

Nothing here computes the GEMM: expected values come from ``oracle`` only.
"""
from __future__ import annotations

import numpy as np

from oracle import schedule as S

ROLE = {0: S.FULL, 1: S.PARTIAL, 2: S.OWNER}
POLICY_ID = {"auto": 0, "dp": 1, "sk": 2, "dp_1tile_sk": 3, "2tile_sk_dp": 4, "paper": 5}
POLICY_BY_ID = {v: k for k, v in POLICY_ID.items()}


def records_to_schedule(records, grid):
    """Library/kernel schedule records -> per-workgroup Segment lists (oracle form)."""
    out = [[] for _ in range(grid)]
    for wg, seq, tile, lo, hi, role, p0, p1 in sorted(records, key=lambda r: (r[0], r[1])):
        peers = tuple(range(p0, p1 + 1)) if role == 2 else ()
        assert seq == len(out[wg]), f"workgroup {wg}: record {seq} out of order"
        out[wg].append(S.Segment(int(tile), int(lo), int(hi), ROLE[role], peers))
    return out


SHARE_BY_ID = {0: "proportional", 1: "leading"}


def oracle_plan_for(info, model, policy, force_g=0):
    """The oracle's plan for the problem a library plan launches.

    The library resolves "auto" by its own rule (a design choice for the
    target GPU, not the paper's selection); such a plan is rebuilt here from
    the explicit policy and grid it resolved to, so the comparison checks the
    schedule of that resolved plan, not the rule that picked it."""
    if policy == "auto":
        policy, force_g = resolved(info)
    elif policy == "paper":       # the library's name for the paper's own selection
        policy = "auto"
    return S.make_plan(int(info["M"]), int(info["N"]), int(info["K"]), int(info["BM"]), int(info["BN"]),
                       int(info["BK"]), int(info["p"]), policy=policy, force_g=force_g,
                       hybrid_min_waves=int(info["hybrid_min_waves"]), model=tuple(model)[:4],
                       share=SHARE_BY_ID[int(info.get("share", 0))])


def oracle_grouped_plan_for(problems, info, model, policy, force_g=0):
    """The grouped oracle's plan for the problems a grouped library plan
    launches (problems as given; "auto" rebuilt from its resolved form)."""
    from oracle import grouped as GR
    if policy == "auto":
        policy, force_g = resolved(info)
    elif policy == "paper":
        policy = "auto"
    return GR.make_grouped_plan(problems, int(info["BM"]), int(info["BN"]), int(info["BK"]), int(info["p"]),
                                policy=policy, force_g=force_g, hybrid_min_waves=int(info["hybrid_min_waves"]),
                                model=tuple(model)[:4], share=SHARE_BY_ID[int(info.get("share", 0))])


def resolved(info):
    """(explicit policy, forced grid) a library plan resolved to."""
    pol = POLICY_BY_ID[int(info["policy"])]
    return pol, (int(info["g_sk"]) if pol != "dp" else 0)


def bits_u16(t):
    """uint16 numpy view of a 16-bit torch tensor (any device)."""
    import torch
    return t.detach().cpu().contiguous().view(torch.int16).numpy().view(np.uint16)


def to_f64(t):
    """Exact float64 value of a torch tensor's stored elements."""
    import torch
    from oracle import lowp
    t = t.detach().cpu().contiguous()
    if t.dtype == torch.float32:
        return t.numpy().astype(np.float64)
    if t.dtype == torch.bfloat16:
        return lowp.bf16_bits_to_f64(bits_u16(t))
    if t.dtype == torch.float16:
        return lowp.f16_bits_to_f64(bits_u16(t))
    if t.dtype == torch.float8_e4m3fn:
        return lowp.e4m3_bits_to_f64(t.view(torch.uint8).numpy())
    raise TypeError(t.dtype)
