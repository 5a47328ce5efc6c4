"""Stream-K GEMM for AMD MI355X (gfx950).

The work of C = alpha * A * B + beta * C is split by MAC-loop iteration over
persistent workgroups (basic Stream-K and its data-parallel hybrids), with
hand-written HIP kernels behind the C ABI of include/skgemm.h.  This package
is the thin Python layer over that library.
"""
from . import skgemm  # noqa: F401
from .skgemm import (BatchedPlan, ConvPlan, GroupedPlan, Plan, batched_matmul, conv2d, grouped_matmul,  # noqa: F401
                     matmul, matmul_fp8, quantize_e4m3)
