/*
 * tso_oracle.c -- CPU oracle for the tall & skinny products of
 * Ernst, Hager, Thies, Wellein, "Performance Engineering for Real and Complex
 * Tall & Skinny Matrix Multiplication Kernels on GPUs" (arXiv 1905.03136).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  It shares no code,
 * header, helper or constant with the GPU library, and the GPU library never
 * calls it.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load it.
 *
 * What it computes (Section 1.1, the problem statement; Section 2.2, Listing 1):
 *   A is K x M, B is K x N, C is M x N, all row-major (Section 1.2: a row of a
 *   block vector holds one entry of each vector), element (k,m) of A at
 *   A[k*lda + m].
 *   TSMTTSM:  C[m][n] = sum_{k=0}^{K-1} op(A[k][m]) * B[k][n]
 *   TSMM:     B[k][n] = alpha * sum_{m=0}^{M-1} op(A[k][m]) * C[m][n]
 *                       + beta * B_old[k][n]          (beta == 0: B_old not read)
 *   op(x) = x, or conj(x) for the conjugate form of the complex case.
 *
 * Arithmetic: IEEE binary64, round to nearest, no contraction into FMA
 * (compile with -ffp-contract=off).  Each entry of C is summed in increasing
 * k exactly as Listing 1 does; each entry of B in increasing m.  Complex
 * numbers are interleaved (re, im) pairs of doubles and multiplied with the
 * textbook formula (ar*br - ai*bi) + i(ar*bi + ai*br).
 *
 * The "compensated" mode evaluates the same sums with the Dot2 algorithm of
 * Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26(6), 2005): an error-free
 * product (via fma) and Knuth's error-free sum, with the errors collected in a
 * second accumulator.  Its result is as accurate as if computed in twice the
 * working precision and is the reference for long sums.
 *
 * Threads only split the set of independent output entries (rows of C for
 * TSMTTSM, rows of B for TSMM); every entry is still summed by one thread in
 * the order above, so the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* error-free product: a*b == p + e exactly (needs a correctly rounded fma) */
static inline void two_prod(double a, double b, double *p, double *e)
{
    double h = a * b;
    *e = fma(a, b, -h);
    *p = h;
}

/* Knuth's error-free sum: a+b == s + e exactly */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* one Dot2 step: (s, c) += x*y */
static inline void dot2_step(double *s, double *c, double x, double y)
{
    double p, ep, t, et;
    two_prod(x, y, &p, &ep);
    two_sum(*s, p, &t, &et);
    *s = t;
    *c = *c + (et + ep);
}

static int clamp_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    return nthreads < 1 ? 1 : nthreads;
}

/* ------------------------------------------------------------------ */
/* TSMTTSM, real: C[m][n] = sum_k A[k][m] * B[k][n]                      */
/* ------------------------------------------------------------------ */
static void tsmttsm_real(int comp, int64_t K, int M, int N,
                         const double *A, int64_t lda, const double *B, int64_t ldb,
                         double *C, int64_t ldc, int nthreads)
{
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int m = 0; m < M; ++m) {
        double *s = calloc((size_t)N, sizeof(double));
        double *c = calloc((size_t)N, sizeof(double));
        for (int64_t k = 0; k < K; ++k) {
            const double a = A[k * lda + m];
            const double *brow = B + k * ldb;
            for (int n = 0; n < N; ++n) {
                if (comp) dot2_step(&s[n], &c[n], a, brow[n]);
                else      s[n] = s[n] + a * brow[n];
            }
        }
        for (int n = 0; n < N; ++n) C[(int64_t)m * ldc + n] = comp ? s[n] + c[n] : s[n];
        free(s);
        free(c);
    }
}

/* ------------------------------------------------------------------ */
/* TSMTTSM, complex: C[m][n] = sum_k op(A[k][m]) * B[k][n]               */
/* op = conj when conjA != 0 (the Hermitian product A^H B)               */
/* ------------------------------------------------------------------ */
static void tsmttsm_cplx(int comp, int conjA, int64_t K, int M, int N,
                         const double *A, int64_t lda, const double *B, int64_t ldb,
                         double *C, int64_t ldc, int nthreads)
{
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int m = 0; m < M; ++m) {
        double *sr = calloc((size_t)N, sizeof(double)), *cr = calloc((size_t)N, sizeof(double));
        double *si = calloc((size_t)N, sizeof(double)), *ci = calloc((size_t)N, sizeof(double));
        for (int64_t k = 0; k < K; ++k) {
            const double ar = A[2 * (k * lda + m)];
            const double ai = conjA ? -A[2 * (k * lda + m) + 1] : A[2 * (k * lda + m) + 1];
            const double *brow = B + 2 * k * ldb;
            for (int n = 0; n < N; ++n) {
                const double br = brow[2 * n], bi = brow[2 * n + 1];
                if (comp) {
                    /* real part: ar*br + (-ai)*bi ; imaginary part: ar*bi + ai*br */
                    dot2_step(&sr[n], &cr[n], ar, br);
                    dot2_step(&sr[n], &cr[n], -ai, bi);
                    dot2_step(&si[n], &ci[n], ar, bi);
                    dot2_step(&si[n], &ci[n], ai, br);
                } else {
                    const double pr = ar * br - ai * bi;
                    const double pi = ar * bi + ai * br;
                    sr[n] = sr[n] + pr;
                    si[n] = si[n] + pi;
                }
            }
        }
        for (int n = 0; n < N; ++n) {
            C[2 * ((int64_t)m * ldc + n)]     = comp ? sr[n] + cr[n] : sr[n];
            C[2 * ((int64_t)m * ldc + n) + 1] = comp ? si[n] + ci[n] : si[n];
        }
        free(sr); free(cr); free(si); free(ci);
    }
}

/* ------------------------------------------------------------------ */
/* TSMM, real: B[k][n] = alpha * sum_m A[k][m] * C[m][n] + beta * B[k][n] */
/* ------------------------------------------------------------------ */
static void tsmm_real(int comp, int64_t K, int M, int N,
                      const double *A, int64_t lda, const double *C, int64_t ldc,
                      double *B, int64_t ldb, double alpha, double beta, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t k = 0; k < K; ++k) {
        const double *arow = A + k * lda;
        double *brow = B + k * ldb;
        for (int n = 0; n < N; ++n) {
            double s = 0.0, c = 0.0;
            for (int m = 0; m < M; ++m) {
                if (comp) dot2_step(&s, &c, arow[m], C[(int64_t)m * ldc + n]);
                else      s = s + arow[m] * C[(int64_t)m * ldc + n];
            }
            if (comp) s = s + c;
            brow[n] = (beta == 0.0) ? alpha * s : alpha * s + beta * brow[n];
        }
    }
}

/* ------------------------------------------------------------------ */
/* TSMM, complex: B[k][n] = alpha * sum_m op(A[k][m]) * C[m][n] + beta*B */
/* alpha and beta are real scalars.                                      */
/* ------------------------------------------------------------------ */
static void tsmm_cplx(int comp, int conjA, int64_t K, int M, int N,
                      const double *A, int64_t lda, const double *C, int64_t ldc,
                      double *B, int64_t ldb, double alpha, double beta, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t k = 0; k < K; ++k) {
        const double *arow = A + 2 * k * lda;
        double *brow = B + 2 * k * ldb;
        for (int n = 0; n < N; ++n) {
            double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
            for (int m = 0; m < M; ++m) {
                const double ar = arow[2 * m];
                const double ai = conjA ? -arow[2 * m + 1] : arow[2 * m + 1];
                const double xr = C[2 * ((int64_t)m * ldc + n)];
                const double xi = C[2 * ((int64_t)m * ldc + n) + 1];
                if (comp) {
                    dot2_step(&sr, &cr, ar, xr);
                    dot2_step(&sr, &cr, -ai, xi);
                    dot2_step(&si, &ci, ar, xi);
                    dot2_step(&si, &ci, ai, xr);
                } else {
                    sr = sr + (ar * xr - ai * xi);
                    si = si + (ar * xi + ai * xr);
                }
            }
            if (comp) { sr = sr + cr; si = si + ci; }
            if (beta == 0.0) {
                brow[2 * n]     = alpha * sr;
                brow[2 * n + 1] = alpha * si;
            } else {
                brow[2 * n]     = alpha * sr + beta * brow[2 * n];
                brow[2 * n + 1] = alpha * si + beta * brow[2 * n + 1];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* exported entry points                                               */
/* Return 0 on success, 1 on an invalid argument.  cplx selects the     */
/* interleaved complex type; leading dimensions count elements (a       */
/* complex element is two doubles).                                     */
/* ------------------------------------------------------------------ */
int tso_tsmttsm(int cplx, int conjA, int compensated, int64_t K, int M, int N,
                const double *A, int64_t lda, const double *B, int64_t ldb,
                double *C, int64_t ldc, int nthreads)
{
    if (K < 0 || M < 1 || N < 1 || lda < M || ldb < N || ldc < N) return 1;
    if (!C || (K > 0 && (!A || !B))) return 1;
    nthreads = clamp_threads(nthreads);
    if (nthreads > M) nthreads = M;
    if (cplx) tsmttsm_cplx(compensated, conjA, K, M, N, A, lda, B, ldb, C, ldc, nthreads);
    else      tsmttsm_real(compensated, K, M, N, A, lda, B, ldb, C, ldc, nthreads);
    return 0;
}

int tso_tsmm(int cplx, int conjA, int compensated, int64_t K, int M, int N,
             const double *A, int64_t lda, const double *C, int64_t ldc,
             double *B, int64_t ldb, double alpha, double beta, int nthreads)
{
    if (K < 0 || M < 1 || N < 1 || lda < M || ldb < N || ldc < N) return 1;
    if (K > 0 && (!A || !B || !C)) return 1;
    nthreads = clamp_threads(nthreads);
    if (cplx) tsmm_cplx(compensated, conjA, K, M, N, A, lda, C, ldc, B, ldb, alpha, beta, nthreads);
    else      tsmm_real(compensated, K, M, N, A, lda, C, ldc, B, ldb, alpha, beta, nthreads);
    return 0;
}

int tso_max_threads(void)
{
    return clamp_threads(0);
}
