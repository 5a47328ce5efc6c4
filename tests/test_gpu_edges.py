"""GPU parity at the operands' inner edges, with padded leading dimensions.

Every operand and the output live in storage whose rows are longer than the
matrix (ld > inner extent), with the gap filled with NaN.  The MAC loop loads
16-byte chunks; a chunk that straddles the inner edge of a ragged K (or of a
ragged M or N of an MN-contiguous operand) brings in bytes from the gap, and
those must be cleared before they reach the matrix cores: NaN times the zero
padding of the other operand would otherwise poison valid outputs.  Inputs
are small integers, so every result is exact and compared bit for bit with
the FP64 oracle; the output's gap must still hold NaN afterwards (nothing is
written outside the matrix).
"""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import to_f64
from oracle import gemm as og

pytestmark = pytest.mark.gpu

SHAPES = [(333, 517, 290), (257, 129, 77), (64, 64, 9), (5, 300, 3), (130, 2, 69), (1, 1, 1), (200, 260, 1030)]
PAD = 13   # elements of NaN gap per row (odd: rows start misaligned)


def sk():
    from paper_2212_08964_amd import skgemm
    return skgemm


def dev():
    return torch.device("cuda:0")


def padded(x, dtype, col_major):
    """x (rows x cols, float32 numpy) stored in NaN-padded storage of `dtype`:
    row-major with ld = cols + PAD, or column-major with ld = rows + PAD."""
    r, c = x.shape
    t = torch.from_numpy(x)
    if col_major:
        st = torch.full((c, r + PAD), float("nan"), dtype=torch.float32)
        st[:, :r] = t.t()
        return st.to(dtype).to(dev())[:, :r].t()
    st = torch.full((r, c + PAD), float("nan"), dtype=torch.float32)
    st[:, :c] = t
    return st.to(dtype).to(dev())[:, :c]


CASES = [(torch.float32, None, "nn"), (torch.float32, None, "tt"),
         (torch.bfloat16, (256, 256, 64), "nn"), (torch.bfloat16, (128, 128, 64, 4), "nt"),
         (torch.bfloat16, (128, 128, 64, 8), "tn"), (torch.float16, (256, 256, 64), "tt"),
         (torch.float16, (128, 128, 64, 8), "nn"), (torch.float64, None, "nn"), (torch.float64, None, "tn"),
         (torch.float8_e4m3fn, (256, 256, 128), "nt"), (torch.float8_e4m3fn, (128, 128, 128), "nt")]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype,tile,layouts", CASES)
def test_padded_nan_gaps_exact(shape, dtype, tile, layouts):
    M, N, K = shape
    g = W.rng(M * 7 + N * 3 + K)
    a = W.integer_f32(g, (M, K))
    b = W.integer_f32(g, (K, N))
    A = padded(a, dtype, layouts[0] == "t")
    B = padded(b, dtype, layouts[1] == "t")
    out_dt = torch.float64 if dtype == torch.float64 else torch.float32
    Cst = torch.full((M, N + PAD), float("nan"), dtype=out_dt, device=dev())
    C = Cst[:, :N]
    ref = og.gemm_f64(a.astype(np.float64), b.astype(np.float64))
    for pol in ("auto", "dp", "sk"):
        C.fill_(float("nan"))
        sk().matmul(A, B, out=C, policy=pol, tile=tile)
        torch.cuda.synchronize()
        assert np.array_equal(to_f64(C) if out_dt == torch.float32 else C.cpu().numpy(), ref), pol
        assert torch.isnan(Cst[:, N:]).all(), pol


@pytest.mark.parametrize("policy", ["auto", "sk", "dp"])
@pytest.mark.parametrize("dtype,tile", [(torch.bfloat16, (256, 256, 64)), (torch.bfloat16, (128, 128, 64, 8)),
                                        (torch.float32, None)])
def test_grouped_padded_nan_gaps_exact(policy, dtype, tile):
    """One grouped launch over ragged problems whose operands and outputs all
    sit in NaN-padded storage (leading dimensions from the per-problem table)."""
    shapes = [(333, 517, 290), (64, 64, 9), (130, 2, 69), (200, 260, 1030), (1, 1, 1)]
    g = W.rng(41)
    As, Bs, Cs, Cst, refs = [], [], [], [], []
    for M, N, K in shapes:
        a = W.integer_f32(g, (M, K))
        b = W.integer_f32(g, (K, N))
        As.append(padded(a, dtype, False))
        Bs.append(padded(b, dtype, False))
        st = torch.full((M, N + PAD), float("nan"), dtype=torch.float32, device=dev())
        Cst.append(st)
        Cs.append(st[:, :N])
        refs.append(og.gemm_f64(a.astype(np.float64), b.astype(np.float64)))
    sk().grouped_matmul(As, Bs, Cs, policy=policy, tile=tile)
    torch.cuda.synchronize()
    for (M, N, K), C, st, ref in zip(shapes, Cs, Cst, refs):
        assert np.array_equal(to_f64(C), ref), (M, N, K)
        assert torch.isnan(st[:, N:]).all(), (M, N, K)
