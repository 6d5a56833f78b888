// Triangular solves with R, fills and column reductions.
#include <algorithm>
#include <climits>

#include "common.h"
#include "gemm.h"
#include "profiler.h"
#include "solve.h"

namespace miqr {

static inline unsigned nblocks_for(int64_t n, int per = 256, int64_t cap = 65536) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, cap));
}

// Elementwise kernels over an m x n column-major matrix: blockIdx.y walks the
// columns and blockIdx.x the rows, so no thread divides a flat index.
struct Grid2 {
  dim3 g;
  Grid2(int64_t m, int64_t n) {
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, 256));
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(n, 4096));
    g = dim3((unsigned)gx, (unsigned)gy);
  }
};
#define MIQR_FOR_ELEMENTS(m, n)                                                    \
  for (int64_t j = blockIdx.y; j < (n); j += gridDim.y)                           \
    for (int64_t i = blockIdx.x * 256 + (int64_t)threadIdx.x; i < (m);            \
         i += (int64_t)gridDim.x * 256)

// Strict lower triangle of the nb x nb diagonal blocks of a matrix with n
// columns (nb = n: of the whole n x n matrix), rows below nb untouched.
__global__ __launch_bounds__(256) void k_zero_block_lower(int64_t n, int64_t nb, double* T,
                                                          int64_t ldt) {
  MIQR_FOR_ELEMENTS(nb, n) {
    if (i > j % nb) T[i + j * ldt] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_set_identity(int64_t m, int64_t n, double* Q,
                                                      int64_t ldq) {
  MIQR_FOR_ELEMENTS(m, n) { Q[i + j * ldq] = (i == j) ? 1.0 : 0.0; }
}

__global__ __launch_bounds__(256) void k_copy_matrix(int64_t m, int64_t n, const double* X,
                                                     int64_t ldx, double* Y, int64_t ldy) {
  MIQR_FOR_ELEMENTS(m, n) { Y[i + j * ldy] = X[i + j * ldx]; }
}

__global__ __launch_bounds__(256) void k_scale_columns(int64_t m, int64_t n, double* Q,
                                                       int64_t ldq, const double* d) {
  MIQR_FOR_ELEMENTS(m, n) { Q[i + j * ldq] *= d[j]; }
}

__global__ void k_normalize_r(int64_t n, double* A, int64_t lda, double* sign) {
  // One thread per row i of R: d_i = sign(R_ii), row i of the upper triangle scaled by d_i.
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (A[i + i * lda] < 0.0) ? -1.0 : 1.0;
    sign[i] = d;
    if (d < 0.0)
      for (int64_t j = i; j < n; ++j) A[i + j * lda] = -A[i + j * lda];
  }
}

// Square matrices: the last column has no entries below the diagonal.  The
// reconstruction always reflects there (tau = 2, H = diag(1, .., 1, -1)); the
// reflector rule of the representation does not (tau = 0, H = I).  Switching
// to tau = 0 negates the last row of R (only its diagonal entry) and zeroes
// the last column of T (its trows entries at Tcol).
__global__ void k_square_last_column(int64_t n, double* A, int64_t lda, double* Tcol,
                                     int64_t trows) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < trows;
       i += (int64_t)gridDim.x * blockDim.x) {
    Tcol[i] = 0.0;
    if (i == trows - 1) A[(n - 1) + (n - 1) * lda] = -A[(n - 1) + (n - 1) * lda];
  }
}

__global__ void k_find_zero_diag(int64_t n, const double* R, int64_t ldr, int* flag) {
  __shared__ int best;
  if (threadIdx.x == 0) best = INT_MAX;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    if (R[i + i * ldr] == 0.0) atomicMin(&best, (int)(i + 1));
  __syncthreads();
  if (threadIdx.x == 0) *flag = (best == INT_MAX) ? 0 : best;
}

// Solve with one diagonal block (nb <= 64 rows) of R for up to 4 right-hand
// sides at a time: backward (R x = c) or forward with R^T (R^T x = c).
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsm_diag(int nb, int64_t nrhs, const double* R,
                                                    int64_t ldr, double* X, int64_t ldx) {
  __shared__ double Rs[kNB][kNB + 1];
  __shared__ double xs[2][4];
  const int t = threadIdx.x, row = t & 63, col = t >> 6;
  for (int e = t; e < kTS; e += 256) {
    const int i = e % kNB, j = e / kNB;
    Rs[i][j] = (i < nb && j < nb) ? R[i + (int64_t)j * ldr] : 0.0;
  }
  __syncthreads();
  for (int64_t c0 = 4 * (int64_t)blockIdx.x; c0 < nrhs; c0 += 4 * (int64_t)gridDim.x) {
    const int64_t cc = c0 + col;
    const bool live = cc < nrhs && row < nb;
    double x = live ? X[row + cc * ldx] : 0.0;
    for (int s = 0; s < nb; ++s) {
      const int i = TRANS ? s : nb - 1 - s;
      if (row == i) {
        x = x / Rs[i][i];
        xs[s & 1][col] = x;
      }
      __syncthreads();
      const double xi = xs[s & 1][col];
      if (TRANS) {
        if (row > i) x -= Rs[i][row] * xi;
      } else {
        if (row < i) x -= Rs[row][i] * xi;
      }
    }
    if (live) X[row + cc * ldx] = x;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_column_sumsq(int64_t m, const double* X, int64_t ldx,
                                                       double* out) {
  __shared__ double part[4];
  const int64_t j = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double v = X[i + j * ldx];
    s += v * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = (part[0] + part[1]) + (part[2] + part[3]);
}

static inline unsigned trsm_groups(int64_t nrhs) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((nrhs + 3) / 4, 4096));
}

__global__ __launch_bounds__(256) void k_axpy_cols(int64_t rows, int64_t ncols, double sgn,
                                                   const double* a, const double* X,
                                                   int64_t ldx, double* Y, int64_t ldy) {
  MIQR_FOR_ELEMENTS(rows, ncols) { Y[i + j * ldy] += sgn * a[j] * X[i + j * ldx]; }
}

__global__ __launch_bounds__(256) void k_xpby_cols(int64_t rows, int64_t ncols, const double* S,
                                                   int64_t lds, const double* b, double* P,
                                                   int64_t ldp) {
  MIQR_FOR_ELEMENTS(rows, ncols) { P[i + j * ldp] = S[i + j * lds] + b[j] * P[i + j * ldp]; }
}

void axpy_cols(hipStream_t s, int64_t rows, int64_t ncols, double sgn, const double* a,
               const double* X, int64_t ldx, double* Y, int64_t ldy) {
  if (rows <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_axpy_cols, Grid2(rows, ncols).g, dim3(256), 0, s, rows, ncols, sgn, a, X,
                     ldx, Y, ldy);
}

void xpby_cols(hipStream_t s, int64_t rows, int64_t ncols, const double* S, int64_t lds,
               const double* b, double* P, int64_t ldp) {
  if (rows <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_xpby_cols, Grid2(rows, ncols).g, dim3(256), 0, s, rows, ncols, S, lds, b,
                     P, ldp);
}

void zero_block_lower(hipStream_t s, int64_t n, int64_t nb, double* T, int64_t ldt) {
  if (n <= 0 || nb <= 0) return;
  TimedLaunch tl(s, "zero_block_lower", 4.0 * (double)nb * n, 0.0);
  hipLaunchKernelGGL(k_zero_block_lower, Grid2(nb, n).g, dim3(256), 0, s, n, nb, T, ldt);
}

void set_identity(hipStream_t s, int64_t m, int64_t n, double* Q, int64_t ldq) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_set_identity, Grid2(m, n).g, dim3(256), 0, s, m, n, Q, ldq);
}

void copy_matrix(hipStream_t s, int64_t m, int64_t n, const double* X, int64_t ldx, double* Y,
                 int64_t ldy) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_copy_matrix, Grid2(m, n).g, dim3(256), 0, s, m, n, X, ldx, Y, ldy);
}

void scale_columns(hipStream_t s, int64_t m, int64_t n, double* Q, int64_t ldq, const double* d) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_scale_columns, Grid2(m, n).g, dim3(256), 0, s, m, n, Q, ldq, d);
}

void normalize_r(hipStream_t s, int64_t n, double* A, int64_t lda, double* sign) {
  hipLaunchKernelGGL(k_normalize_r, dim3(nblocks_for(n)), dim3(256), 0, s, n, A, lda, sign);
}

void square_last_column(hipStream_t s, int64_t n, double* A, int64_t lda, double* Tcol,
                        int64_t trows) {
  hipLaunchKernelGGL(k_square_last_column, dim3(nblocks_for(trows)), dim3(256), 0, s, n, A, lda,
                     Tcol, trows);
}

void find_zero_diagonal(hipStream_t s, int64_t n, const double* R, int64_t ldr, int* flag) {
  hipLaunchKernelGGL(k_find_zero_diag, dim3(1), dim3(256), 0, s, n, R, ldr, flag);
}

hipError_t solve_upper(hipStream_t s, int64_t n, int64_t nrhs, const double* R, int64_t ldr,
                       double* X, int64_t ldx, double* scratch, int64_t scratch_doubles) {
  const int64_t nblk = (n + kNB - 1) / kNB;
  for (int64_t bk = nblk - 1; bk >= 0; --bk) {
    const int64_t i0 = bk * kNB, i1 = std::min<int64_t>(n, i0 + kNB);
    {
      TimedLaunch tl(s, "trsm_diag", 8.0 * (double)(i1 - i0) * (i1 - i0 + 2 * nrhs),
                     (double)(i1 - i0) * (i1 - i0) * nrhs);
      hipLaunchKernelGGL(k_trsm_diag<false>, dim3(trsm_groups(nrhs)), dim3(256), 0, s,
                         (int)(i1 - i0), nrhs, R + i0 + i0 * ldr, ldr, X + i0, ldx);
    }
    if (i0 > 0) {
      GemmDesc d;
      d.ta = 'N';
      d.tb = 'N';
      d.M = i0;
      d.N = nrhs;
      d.K = i1 - i0;
      d.alpha = -1.0;
      d.beta = 1.0;
      d.A = R + i0 * ldr;
      d.lda = ldr;
      d.B = X + i0;
      d.ldb = ldx;
      d.C = X;
      d.ldc = ldx;
      hipError_t e = gemm(d, s, scratch, scratch_doubles);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t solve_upper_trans(hipStream_t s, int64_t n, int64_t nrhs, const double* R,
                             int64_t ldr, double* X, int64_t ldx, double* scratch,
                             int64_t scratch_doubles) {
  const int64_t nblk = (n + kNB - 1) / kNB;
  for (int64_t bk = 0; bk < nblk; ++bk) {
    const int64_t i0 = bk * kNB, i1 = std::min<int64_t>(n, i0 + kNB);
    {
      TimedLaunch tl(s, "trsm_diag", 8.0 * (double)(i1 - i0) * (i1 - i0 + 2 * nrhs),
                     (double)(i1 - i0) * (i1 - i0) * nrhs);
      hipLaunchKernelGGL(k_trsm_diag<true>, dim3(trsm_groups(nrhs)), dim3(256), 0, s,
                         (int)(i1 - i0), nrhs, R + i0 + i0 * ldr, ldr, X + i0, ldx);
    }
    if (i1 < n) {
      GemmDesc d;
      d.ta = 'T';
      d.tb = 'N';
      d.M = n - i1;
      d.N = nrhs;
      d.K = i1 - i0;
      d.alpha = -1.0;
      d.beta = 1.0;
      d.A = R + i0 + i1 * ldr;
      d.lda = ldr;
      d.B = X + i0;
      d.ldb = ldx;
      d.C = X + i1;
      d.ldc = ldx;
      hipError_t e = gemm(d, s, scratch, scratch_doubles);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

void column_sumsq(hipStream_t s, int64_t m, int64_t n, const double* X, int64_t ldx, double* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_column_sumsq, dim3((unsigned)n), dim3(256), 0, s, m, X, ldx, out);
}

}  // namespace miqr
