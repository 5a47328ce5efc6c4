"""Stream-K GEMM for AMD MI355X (gfx950).

The work of C = alpha * A * B + beta * C is split by MAC-loop iteration over
persistent workgroups (basic Stream-K and its data-parallel hybrids), with
hand-written HIP kernels behind the C ABI of include/skgemm.h.  This package
is the thin Python layer over that library.
"""
from . import skgemm  # noqa: F401
from .skgemm import GroupedPlan, Plan, grouped_matmul, matmul, matmul_fp8, quantize_e4m3  # noqa: F401
