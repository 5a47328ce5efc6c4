"""Pins of the FP64 GEMM oracle against things other than itself.

* numpy's float64 matmul (a library routine) on random, ragged shapes;
* exact integer arithmetic (Python integers) on integer-valued inputs, where
  the float64 result must be exact;
* the identity (A = I gives C = B) and the all-ones closed form (C = K);
* BLAS conventions: beta = 0 never reads C, alpha/beta scaling;
* the row-subset entry point against the full product;
* finite differences of L = <dC, A B> against the gradient oracle.
"""
import numpy as np
import pytest

from oracle import gemm as og
from oracle import lowp


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (64, 48, 33), (129, 70, 257), (3, 200, 1)])
def test_matches_numpy_matmul(M, N, K):
    g = np.random.default_rng(M * 1000 + N * 10 + K)
    A = g.standard_normal((M, K))
    B = g.standard_normal((K, N))
    C = g.standard_normal((M, N))
    got = og.gemm_f64(A, B, alpha=0.75, beta=-1.25, C=C)
    ref = 0.75 * (A @ B) - 1.25 * C
    assert og.rel_frobenius(got, ref) <= 1e-13


@pytest.mark.parametrize("M,N,K", [(5, 4, 3), (17, 9, 31), (40, 33, 1000)])
def test_integer_inputs_exact(M, N, K):
    g = np.random.default_rng(1)
    A = g.integers(-2, 3, size=(M, K))
    B = g.integers(-2, 3, size=(K, N))
    got = og.gemm_f64(A.astype(np.float64), B.astype(np.float64))
    # exact products in Python integers
    exact = [[sum(int(A[i, k]) * int(B[k, j]) for k in range(K)) for j in range(N)] for i in range(M)]
    assert np.array_equal(got, np.array(exact, dtype=np.float64))


def test_identity_and_ones():
    g = np.random.default_rng(2)
    B = g.standard_normal((37, 21))
    assert np.array_equal(og.gemm_f64(np.eye(37), B), B)
    ones = og.gemm_f64(np.ones((6, 300)), np.ones((300, 11)))
    assert np.all(ones == 300.0)


def test_beta_zero_never_reads_c():
    A = np.ones((4, 3))
    B = np.ones((3, 5))
    C = np.full((4, 5), np.nan)
    assert np.all(og.gemm_f64(A, B, alpha=2.0, beta=0.0, C=C) == 6.0)


def test_k_zero_is_beta_c():
    C = np.arange(12.0).reshape(3, 4)
    got = og.gemm_f64(np.zeros((3, 0)), np.zeros((0, 4)), alpha=1.0, beta=0.5, C=C)
    assert np.array_equal(got, 0.5 * C)


def test_rows_subset_equals_full_rows():
    g = np.random.default_rng(3)
    A = g.standard_normal((50, 40))
    B = g.standard_normal((40, 30))
    C = g.standard_normal((50, 30))
    rows = np.array([0, 7, 49, 7, 23])
    full = og.gemm_f64(A, B, 1.5, 0.5, C)
    part = og.gemm_rows_f64(A, B, rows, 1.5, 0.5, C[rows])
    assert np.array_equal(part, full[rows])


def test_stored_bf16_folds_scales():
    g = np.random.default_rng(4)
    a = g.standard_normal((8, 16)).astype(np.float32)
    b = g.standard_normal((16, 4)).astype(np.float32)
    abits = (a.view(np.uint32) >> 16).astype(np.uint16)    # truncation: any bf16 pattern will do
    bbits = (b.view(np.uint32) >> 16).astype(np.uint16)
    got = og.gemm_stored(abits, bbits, "bf16", alpha=2.0, scale_a=0.5, scale_b=3.0)
    ref = 3.0 * (lowp.bf16_bits_to_f64(abits) @ lowp.bf16_bits_to_f64(bbits))
    assert og.rel_frobenius(got, ref) <= 1e-14


def test_gradient_matches_central_differences():
    """L = <dC, A B> is bilinear, so central differences in float64 equal the
    derivative up to rounding: dL/dA[i,k] = (L(A + h e_ik) - L(A - h e_ik)) / 2h."""
    g = np.random.default_rng(5)
    n = 64
    A = g.standard_normal((n, n))
    B = g.standard_normal((n, n))
    dC = g.standard_normal((n, n))
    dA, dB = og.gemm_grad(A, B, dC)

    def L(a, b):
        return float(np.sum(dC * og.gemm_f64(a, b)))

    h = 0.5
    idx = [(0, 0), (3, 17), (63, 63), (31, 2), (10, 50)]
    for i, k in idx:
        Ap, Am = A.copy(), A.copy()
        Ap[i, k] += h
        Am[i, k] -= h
        fd = (L(Ap, B) - L(Am, B)) / (2 * h)
        assert abs(fd - dA[i, k]) <= 1e-10 * max(1.0, abs(dA[i, k])) * n
        Bp, Bm = B.copy(), B.copy()
        Bp[i, k] += h
        Bm[i, k] -= h
        fd = (L(A, Bp) - L(A, Bm)) / (2 * h)
        assert abs(fd - dB[i, k]) <= 1e-10 * max(1.0, abs(dB[i, k])) * n


def test_error_bound_for_fp32_accumulation():
    """Sanity of the tolerance used for FP32 device results: summing in float32
    stays within gamma_K |A||B| of the float64 oracle (standard bound)."""
    g = np.random.default_rng(6)
    M, N, K = 16, 16, 1024
    A = g.uniform(-1, 1, (M, K)).astype(np.float32)
    B = g.uniform(-1, 1, (K, N)).astype(np.float32)
    ref = og.gemm_f64(A, B)
    acc = np.zeros((M, N), dtype=np.float32)
    for k in range(K):
        acc = (acc + np.outer(A[:, k], B[k, :]).astype(np.float32)).astype(np.float32)
    u = 2.0 ** -24
    gamma = K * u / (1 - K * u)
    bound = gamma * (np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64))
    assert np.all(np.abs(acc - ref) <= bound)
