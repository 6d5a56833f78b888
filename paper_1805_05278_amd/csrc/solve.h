// Triangular solves, fills and reductions around the factorisation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miqr {

// Zero the strict lower triangle of each nb x nb diagonal block of a matrix
// with n columns (nb = n: the strict lower triangle of an n x n matrix).
void zero_block_lower(hipStream_t s, int64_t n, int64_t nb, double* T, int64_t ldt);
// Q = [I_n; 0] (m x n).
void set_identity(hipStream_t s, int64_t m, int64_t n, double* Q, int64_t ldq);
// Copy an m x n matrix.
void copy_matrix(hipStream_t s, int64_t m, int64_t n, const double* X, int64_t ldx, double* Y,
                 int64_t ldy);
// Q <- Q diag(d).
void scale_columns(hipStream_t s, int64_t m, int64_t n, double* Q, int64_t ldq, const double* d);
// R <- diag(d) R on the upper triangle of the n x n top of A, d = sign(diag R)
// (+1 for >= 0); d is written to `sign`.
void normalize_r(hipStream_t s, int64_t n, double* A, int64_t lda, double* sign);
// For m == n: switch the last reflector from tau = 2 to tau = 0 (negate
// R_{n-1,n-1}, zero the trows entries of T's last column at Tcol).
void square_last_column(hipStream_t s, int64_t n, double* A, int64_t lda, double* Tcol,
                        int64_t trows);
// *flag = smallest 1-based j with R_jj == 0 (or 0); flag is device memory.
void find_zero_diagonal(hipStream_t s, int64_t n, const double* R, int64_t ldr, int* flag);
// X <- R^{-1} X for the n x n upper triangle of R, blocked back substitution.
hipError_t solve_upper(hipStream_t s, int64_t n, int64_t nrhs, const double* R, int64_t ldr,
                       double* X, int64_t ldx, double* scratch, int64_t scratch_doubles);
// X <- R^{-T} X (forward substitution with R^T).
hipError_t solve_upper_trans(hipStream_t s, int64_t n, int64_t nrhs, const double* R,
                             int64_t ldr, double* X, int64_t ldx, double* scratch,
                             int64_t scratch_doubles);
// Y[:, c] += sgn * a[c] * X[:, c] for c < ncols (a: device, one per column).
void axpy_cols(hipStream_t s, int64_t rows, int64_t ncols, double sgn, const double* a,
               const double* X, int64_t ldx, double* Y, int64_t ldy);
// P[:, c] = S[:, c] + b[c] * P[:, c].
void xpby_cols(hipStream_t s, int64_t rows, int64_t ncols, const double* S, int64_t lds,
               const double* b, double* P, int64_t ldp);
// out[j] = sum_i X[i, j]^2 for each of the n columns (fixed-order reduction).
void column_sumsq(hipStream_t s, int64_t m, int64_t n, const double* X, int64_t ldx, double* out);

}  // namespace miqr
