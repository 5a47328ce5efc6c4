/*
 * Oracle (test infrastructure only): the plain FP64 definition of GEMM.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path never links or calls it.
 *
 * Computes the problem statement of the Background section (C = alpha*A*B +
 * beta*C) directly, as the sequential loop nest of the "Sequential
 * cache-blocked" algorithm reduces to when the blocking factors equal the
 * matrix extents: for every output element, a sum over k of A[i][k]*B[k][j],
 * accumulated in double precision in increasing k order.
 *
 * All matrices are dense row-major double arrays: A is M x K, B is K x N,
 * C_in and C_out are M x N.  The caller converts stored low-precision values to
 * double (exactly) before calling; per-tensor dequantisation scales are folded
 * into alpha by the caller.  beta == 0 never reads C_in (it may be NULL).
 */
#include <stdint.h>
#include <stddef.h>

/* Full product.  Loop order i, k, j; rows are independent, so OpenMP splits
 * them across threads without changing any element's summation order. */
void oracle_gemm_f64(int64_t M, int64_t N, int64_t K,
                     const double* A, const double* B,
                     double alpha, double beta,
                     const double* C_in, double* C_out)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < M; ++i) {
        double* crow = C_out + i * N;
        for (int64_t j = 0; j < N; ++j) crow[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double a = A[i * K + k];
            const double* brow = B + k * N;
            for (int64_t j = 0; j < N; ++j) crow[j] += a * brow[j];
        }
        for (int64_t j = 0; j < N; ++j) {
            double v = alpha * crow[j];
            if (beta != 0.0) v += beta * C_in[i * N + j];
            crow[j] = v;
        }
    }
}

/* Same definition for a chosen subset of output rows (used where a full
 * product would take too long on the host).  rows[r] names the row of A whose
 * product is written to row r of C_out (n_rows x N); C_in holds the matching
 * n_rows x N rows of the input C. */
void oracle_gemm_rows_f64(int64_t n_rows, const int64_t* rows,
                          int64_t N, int64_t K,
                          const double* A, const double* B,
                          double alpha, double beta,
                          const double* C_in, double* C_out)
{
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < n_rows; ++r) {
        const int64_t i = rows[r];
        double* crow = C_out + r * N;
        for (int64_t j = 0; j < N; ++j) crow[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double a = A[i * K + k];
            const double* brow = B + k * N;
            for (int64_t j = 0; j < N; ++j) crow[j] += a * brow[j];
        }
        for (int64_t j = 0; j < N; ++j) {
            double v = alpha * crow[j];
            if (beta != 0.0) v += beta * C_in[r * N + j];
            crow[j] = v;
        }
    }
}

/* Number of threads the OpenMP runtime will use (reported with timings). */
int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
