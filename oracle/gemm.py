"""Oracle (test infrastructure only): FP64 GEMM and its gradient, from the definition.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

The result oracle is the problem statement of the Background section,
C = alpha * A * B + beta * C, evaluated in float64 by the plain loop nest in
``gemm_ref.c`` (row i, then k, then column j).  Stream-K reaches this same
result; only the FP32 rounding order differs on the device.  Stored
low-precision inputs are first converted exactly to float64 (``lowp.decode``)
and FP8 per-tensor scales multiply alpha, so the oracle computes
alpha * s_A * s_B * sum_k A[i,k] B[k,j] + beta * C[i,j] with no rounding other
than float64's.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build
from . import lowp

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_gemm_f64.argtypes = [i64, i64, i64, dp, dp, ctypes.c_double,
                                        ctypes.c_double, dp, dp]
        lib.oracle_gemm_f64.restype = None
        lib.oracle_gemm_rows_f64.argtypes = [i64, ctypes.POINTER(i64), i64, i64, dp, dp,
                                             ctypes.c_double, ctypes.c_double, dp, dp]
        lib.oracle_gemm_rows_f64.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    """Threads the oracle's OpenMP loop runs on."""
    return int(_load().oracle_num_threads())


def gemm_f64(A, B, alpha: float = 1.0, beta: float = 0.0, C=None) -> np.ndarray:
    """alpha * A @ B + beta * C in float64 (A: M x K, B: K x N, C: M x N).

    beta == 0 never reads C."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    out = np.empty((M, N), dtype=np.float64)
    cin = None
    if beta != 0.0:
        cin = np.ascontiguousarray(C, dtype=np.float64)
        if cin.shape != (M, N):
            raise ValueError("C shape")
    if M and N:
        _load().oracle_gemm_f64(M, N, K, _dptr(A), _dptr(B), float(alpha), float(beta),
                                _dptr(cin) if cin is not None else None, _dptr(out))
    return out


def gemm_rows_f64(A, B, rows, alpha: float = 1.0, beta: float = 0.0, C_rows=None) -> np.ndarray:
    """Rows ``rows`` of alpha * A @ B + beta * C; ``C_rows`` holds those rows of C."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    M, K = A.shape
    N = B.shape[1]
    if rows.size and (rows.min() < 0 or rows.max() >= M):
        raise ValueError("row index out of range")
    out = np.empty((rows.size, N), dtype=np.float64)
    cin = None
    if beta != 0.0:
        cin = np.ascontiguousarray(C_rows, dtype=np.float64)
    if rows.size and N:
        _load().oracle_gemm_rows_f64(rows.size, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     N, K, _dptr(A), _dptr(B), float(alpha), float(beta),
                                     _dptr(cin) if cin is not None else None, _dptr(out))
    return out


def gemm_stored(A_stored, B_stored, dtype: str, alpha: float = 1.0, beta: float = 0.0,
                C=None, scale_a: float = 1.0, scale_b: float = 1.0, rows=None) -> np.ndarray:
    """Oracle for stored low-precision operands (bit patterns for bf16/f16/f8e4m3,
    values for f32): decode exactly, fold the per-tensor scales into alpha, then
    evaluate the float64 definition (all rows, or only ``rows``)."""
    A = lowp.decode(A_stored, dtype)
    B = lowp.decode(B_stored, dtype)
    a_eff = float(alpha) * float(scale_a) * float(scale_b)
    if rows is None:
        return gemm_f64(A, B, a_eff, beta, C)
    return gemm_rows_f64(A, B, rows, a_eff, beta, C)


def gemm_grad(A, B, dC):
    """Gradient of L = <dC, A @ B> with respect to A and B:
    dA = dC @ B^T and dB = A^T @ dC, each evaluated by the float64 definition."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    dC = np.asarray(dC, dtype=np.float64)
    dA = gemm_f64(dC, B.T)
    dB = gemm_f64(A.T, dC)
    return dA, dB


def rel_frobenius(x, ref) -> float:
    """||x - ref||_F / ||ref||_F (0 when both are zero)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(x - ref)
    if den == 0:
        return 0.0 if num == 0 else float("inf")
    return float(num / den)
