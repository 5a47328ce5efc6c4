"""Shared test helpers: tensor/array conversions and schedule comparison.

Nothing here computes the GEMM: expected values come from ``oracle`` only.
"""
from __future__ import annotations

import numpy as np

from oracle import schedule as S

ROLE = {0: S.FULL, 1: S.PARTIAL, 2: S.OWNER}
POLICY_ID = {"auto": 0, "dp": 1, "sk": 2, "dp_1tile_sk": 3, "2tile_sk_dp": 4}
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
    """The oracle's plan for the problem a library plan launches."""
    return S.make_plan(int(info["M"]), int(info["N"]), int(info["K"]), int(info["BM"]), int(info["BN"]),
                       int(info["BK"]), int(info["p"]), policy=policy, force_g=force_g,
                       hybrid_min_waves=int(info["hybrid_min_waves"]), model=model_with_cus(info, model),
                       share=SHARE_BY_ID[int(info.get("share", 0))])


def model_with_cus(info, model):
    """The library's (a, b, c, d, e) plus the CU count of the plan, the form the
    oracle's split rule takes."""
    return tuple(model)[:5] + (int(info["p"]) // int(info["occupancy"]),)


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
