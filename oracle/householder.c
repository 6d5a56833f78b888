/*
 * Plain FP64 CPU reference ("oracle") for Householder QR and least squares.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU path is
 * compared against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header or constant with the
 * GPU library and must never be called from the product path.
 *
 * What it computes (paper: "A 3D Parallel Algorithm for QR Decomposition",
 * Ballard, Demmel, Grigori, Jacquelin, Knight):
 *
 *  - A QR decomposition A = Q R of an m x n matrix with m >= n, Q orthogonal,
 *    R upper trapezoidal (Sec. 2.1, "QR Preliminaries").
 *  - Q in Householder representation (Sec. 2.3, "Compact Representations"):
 *    Q = I - V T V^T with V unit lower trapezoidal (m x n) and T upper
 *    triangular (n x n), V's strict lower trapezoid and R's upper triangle
 *    stored in place over A.
 *  - The method of the paper (Elmroth-Gustavson recursion, Alg. 2, with a TSQR
 *    base case, Sec. 5 and App. C) reaches, in exact arithmetic, the same
 *    (V, T, R) as the plain unblocked right-looking Householder algorithm with
 *    b = 1 (Sec. 8.1, the 1D-house variant on one processor), because every
 *    variant applies the same reflectors and the Householder representation of
 *    a given thin Q-factor is unique.  So this oracle is that plain algorithm:
 *    one reflector per column, applied to the trailing columns at once.
 *
 * Reflector sign rule (the paper leaves local-QR unspecified, App. C.1): the
 * LAPACK dlarfg convention.  For x = A[j:m, j], alpha = x[0], sigma^2 =
 * ||x[1:]||^2:
 *     sigma == 0  ->  tau = 0, beta = alpha (no reflection)
 *     otherwise   ->  beta = -sign(alpha) * sqrt(alpha^2 + sigma^2),
 *                     sign(+-0) = +1, tau = (beta - alpha) / beta,
 *                     v = [1; x[1:] / (alpha - beta)],  R_jj = beta.
 * This is the same sign rule that Householder reconstruction (App. C.2) picks
 * through S_jj = sgn(X_jj), so both give identical (V, T, R).
 *
 * T is accumulated column by column: T[0:j, j] = -tau_j T[0:j, 0:j]
 * (V[:, 0:j]^T v_j), T_jj = tau_j; the result satisfies the closed form of
 * Sec. 2.3, T^{-1} = striu(V^T V) + diag(V^T V) / 2.
 *
 * Storage is column-major; element (i, j) of a matrix with leading dimension
 * ld is at p[i + j*ld].  All arithmetic is IEEE FP64; compile with
 * -ffp-contract=off so that no fused multiply-add changes the rounding.
 * OpenMP, when enabled, only splits independent columns of a trailing update
 * among threads; the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AT(p, i, j, ld) ((p)[(int64_t)(i) + (int64_t)(j) * (int64_t)(ld)])

/* Generate the reflector for column j of A (rows j..m-1), dlarfg rule.
 * On return A[j+1:m, j] holds v[1:], A[j, j] holds beta (= R_jj). */
static double make_reflector(int64_t m, int64_t j, double *A, int64_t lda)
{
    double alpha = AT(A, j, j, lda);
    double sigma2 = 0.0;
    for (int64_t i = j + 1; i < m; ++i) {
        double x = AT(A, i, j, lda);
        sigma2 += x * x;
    }
    if (sigma2 == 0.0)
        return 0.0; /* H_j = I, R_jj = alpha */
    double norm = sqrt(alpha * alpha + sigma2);
    double beta = (alpha >= 0.0) ? -norm : norm; /* -0.0 >= 0.0 holds */
    double tau = (beta - alpha) / beta;
    double scale = 1.0 / (alpha - beta);
    for (int64_t i = j + 1; i < m; ++i)
        AT(A, i, j, lda) *= scale;
    AT(A, j, j, lda) = beta;
    return tau;
}

/* Apply H = I - tau v v^T (v stored below row j of column vcol of V, with an
 * implicit 1 at row j) to columns [c0, c1) of C, rows j..m-1. */
static void apply_reflector(int64_t m, int64_t j, const double *V, int64_t ldv,
                            int64_t vcol, double tau, double *C, int64_t ldc,
                            int64_t c0, int64_t c1)
{
    if (tau == 0.0)
        return;
#pragma omp parallel for schedule(static) if ((c1 - c0) * (m - j) > 65536)
    for (int64_t k = c0; k < c1; ++k) {
        double w = AT(C, j, k, ldc);
        for (int64_t i = j + 1; i < m; ++i)
            w += AT(V, i, vcol, ldv) * AT(C, i, k, ldc);
        w *= tau;
        AT(C, j, k, ldc) -= w;
        for (int64_t i = j + 1; i < m; ++i)
            AT(C, i, k, ldc) -= AT(V, i, vcol, ldv) * w;
    }
}

/* Unblocked Householder QR in place.  tau has n entries.  Returns 0, or -1 on
 * bad arguments. */
int oracle_qr(int64_t m, int64_t n, double *A, int64_t lda, double *tau)
{
    if (m < n || n < 0 || lda < (m > 1 ? m : 1) || (!A && n) || (!tau && n))
        return -1;
    for (int64_t j = 0; j < n; ++j) {
        tau[j] = make_reflector(m, j, A, lda);
        apply_reflector(m, j, A, lda, j, tau[j], A, lda, j + 1, n);
    }
    return 0;
}

/* T factor of the Householder representation from V (strict lower part of A
 * after oracle_qr) and tau.  T is n x n upper triangular, zero below the
 * diagonal. */
int oracle_form_t(int64_t m, int64_t n, const double *A, int64_t lda,
                  const double *tau, double *T, int64_t ldt)
{
    if (m < n || n < 0 || ldt < (n > 1 ? n : 1))
        return -1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            AT(T, i, j, ldt) = 0.0;
    double *g = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!g)
        return -2;
    for (int64_t j = 0; j < n; ++j) {
        /* g[i] = V[:, i]^T v_j for i < j.  v_j is zero above row j and one at
         * row j; v_i is one at row i < j. */
        for (int64_t i = 0; i < j; ++i) {
            double s = AT(A, j, i, lda);
            for (int64_t r = j + 1; r < m; ++r)
                s += AT(A, r, i, lda) * AT(A, r, j, lda);
            g[i] = s;
        }
        /* T[0:j, j] = -tau_j * T[0:j, 0:j] * g */
        for (int64_t i = 0; i < j; ++i) {
            double s = 0.0;
            for (int64_t k = i; k < j; ++k)
                s += AT(T, i, k, ldt) * g[k];
            AT(T, i, j, ldt) = -tau[j] * s;
        }
        AT(T, j, j, ldt) = tau[j];
    }
    free(g);
    return 0;
}

/* C <- Q^T C (trans = 'T') or C <- Q C (trans = 'N'), Q = H_0 H_1 ... H_{n-1}
 * from oracle_qr, C is m x k. */
int oracle_apply_q(char trans, int64_t m, int64_t n, int64_t k,
                   const double *A, int64_t lda, const double *tau,
                   double *C, int64_t ldc)
{
    if (m < n || n < 0 || k < 0 || ldc < (m > 1 ? m : 1) ||
        (trans != 'T' && trans != 'N'))
        return -1;
    if (trans == 'T') {
        for (int64_t j = 0; j < n; ++j)
            apply_reflector(m, j, A, lda, j, tau[j], C, ldc, 0, k);
    } else {
        for (int64_t j = n - 1; j >= 0; --j)
            apply_reflector(m, j, A, lda, j, tau[j], C, ldc, 0, k);
    }
    return 0;
}

/* Explicit thin Q (first n columns of Q): Q1 = Q [I_n; 0], m x n. */
int oracle_form_q(int64_t m, int64_t n, const double *A, int64_t lda,
                  const double *tau, double *Q, int64_t ldq)
{
    if (m < n || n < 0 || ldq < (m > 1 ? m : 1))
        return -1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            AT(Q, i, j, ldq) = (i == j) ? 1.0 : 0.0;
    return oracle_apply_q('N', m, n, n, A, lda, tau, Q, ldq);
}

/* Back substitution R x = c for the n x n upper triangle of R (in A), nrhs
 * right-hand sides held in the first n rows of B.  Returns j+1 if R_jj == 0
 * exactly (no division performed), 0 on success. */
int oracle_trsv_upper(int64_t n, int64_t nrhs, const double *R, int64_t ldr,
                      double *B, int64_t ldb)
{
    for (int64_t j = 0; j < n; ++j)
        if (AT(R, j, j, ldr) == 0.0)
            return (int)(j + 1);
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = AT(B, i, c, ldb);
            for (int64_t k = i + 1; k < n; ++k)
                s -= AT(R, i, k, ldr) * AT(B, k, c, ldb);
            AT(B, i, c, ldb) = s / AT(R, i, i, ldr);
        }
    }
    return 0;
}

/* Least squares min ||B_c - A x_c||_2 by Householder QR.  A is overwritten by
 * its factors (as oracle_qr), B (m x nrhs) by [x; Q^T b residual part]:
 * x in rows 0..n-1.  tau is caller-provided scratch of n doubles.  Returns 0,
 * -1 on bad arguments, or j+1 if R_jj == 0 exactly. */
int oracle_lstsq(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda,
                 double *B, int64_t ldb, double *tau)
{
    int rc = oracle_qr(m, n, A, lda, tau);
    if (rc)
        return rc;
    rc = oracle_apply_q('T', m, n, nrhs, A, lda, tau, B, ldb);
    if (rc)
        return rc;
    return oracle_trsv_upper(n, nrhs, A, lda, B, ldb);
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
