"""Oracle: plain, slow, obviously correct CPU implementations of what the
Stream-K GEMM path computes.  This package is test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, call, link or execute anything in it.  The device
path (``paper_2212_08964_amd``) never does, and this package imports nothing
from the device path.

Modules:
* ``gemm``     - FP64 GEMM definition (C triple loop) and its gradient.
* ``lowp``     - BF16 / FP16 / FP8-E4M3 decoding, rounding and per-tensor
                 FP8 quantisation, written from the format definitions.
* ``schedule`` - enumerator of the data-parallel, fixed-split, basic Stream-K
                 and hybrid schedules, the analytical grid-size model and the
                 paper's own policy selection.
* ``grouped``  - the schedule of grouped (and strided batched) launches.
* ``conv``     - 2-D convolution from its definition (the implicit-GEMM
                 extension's result).
"""
