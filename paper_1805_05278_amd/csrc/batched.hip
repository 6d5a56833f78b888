// Batched least squares: one workgroup per problem, popped from a device queue
// by a persistent grid.
//
// A problem min ||B - A X|| (m x n, nrhs right-hand sides) is solved by
// Householder QR of the augmented matrix [A | B] with a flat TSQR sweep (the
// paper's TSQR with a chain as its tree, Sec. 5 / App. C.1): the running R
// (n x (n + nrhs), zero at the start) is stacked over each 64-row block X of
// [A | B] in turn, and [R; X] is reduced column by column.  The reflector of
// column j is v = [e_j; y] (R is upper triangular, so v has a single entry in
// the R part), with the dlarfg sign rule.  After the last block R holds the R
// factor of A and, in its last nrhs columns, the top n rows of Q^T B; back
// substitution gives X.
//
// Two threads own column c of [A | B]: 32 rows each of the current block in
// registers, and column c of R in global memory, which no other column
// touches.  A step is one reflector: the pivot column posts its entries and
// (tau, scale) in LDS; every column to its right forms its dot product with
// them (32 products per thread plus one lane-pair sum, no workgroup
// reduction) and updates itself.  One barrier per step.
#include <climits>

#include "batched.h"
#include "common.h"
#include "profiler.h"

namespace miqr {
namespace {

constexpr int H = kBatchRows;

__global__ void k_batch_reset(int* counter) {
  if (threadIdx.x < kBatchCounters) counter[threadIdx.x] = 0;
}

// Global-address-space views: loads and stores through them wait on the
// vector memory counter only, so a prefetch stays in flight across LDS traffic.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gdouble* gp(double* p) { return (gdouble*)p; }

// Adjacent-lane pair sum (quad_perm [1,0,3,2]) and even-lane broadcast
// (quad_perm [0,0,2,2]) for the two threads that share a column.
__device__ __forceinline__ double pair_sum(double v) { return v + dpp_mov<0xB1>(v); }
__device__ __forceinline__ double from_even(double v) { return dpp_mov<0xA0>(v); }

constexpr int HR = H / 2;  // rows of a block held by each of a column's two threads

// Flat TSQR sweep of one problem (flags without kTaskApply).  Threads 2c and
// 2c+1 hold rows [0, 32) and [32, 64) of column c of the current block; the
// even thread also owns column c of R in global memory.  The pivot posts its
// unscaled column and (tau, scale); the others fold the scale into their
// update coefficient, so the pivot never rescales its column.
__device__ void batch_factor(const BatchTask& t, double (*xs)[H], double (*coef)[2]) {
  const int tid = threadIdx.x, c = tid >> 1, half = tid & 1;
  const int wave = tid >> 6;
  const int n = t.n, N = n + t.nrhs, m = t.m;
  const bool own = c < N;
  const bool keep = (t.flags & kTaskKeep) != 0;
  gdouble* col = nullptr;
  if (own) col = gp(c < n ? t.A + (int64_t)c * t.lda : t.B + (int64_t)(c - n) * t.ldb);
  gdouble* Rc = gp(c < n ? t.R + (int64_t)c * n : t.C + (int64_t)(c - n) * n);
  const int jmax = c < n ? c : n - 1;  // last row of R in column c
  if (own && half == 0)
    for (int j = 0; j <= jmax; ++j) Rc[j] = 0.0;
  const int nblk = (m + H - 1) / H;
  double x[HR];
  double sc_own = 0.0;  // scale of this column's reflector in the current block
  for (int bk = 0; bk < nblk; ++bk) {
    const int r0 = bk * H + half * HR;
    const int rows = max(0, min(HR, m - r0));
    if (own) {
      if (rows == HR) {
#pragma unroll
        for (int r = 0; r < HR; ++r) x[r] = col[r0 + r];
      } else {
#pragma unroll
        for (int r = 0; r < HR; ++r) x[r] = r < rows ? col[r0 + r] : 0.0;
      }
    } else {
#pragma unroll
      for (int r = 0; r < HR; ++r) x[r] = 0.0;
    }
    // Partial sum of squares of the next pivot's column (column 0 first).
    double s2 = 0.0;
    if (c == 0) {
#pragma unroll
      for (int r = 0; r < HR; ++r) s2 += x[r] * x[r];
    }
    double rnext = (own && half == 0) ? Rc[0] : 0.0;
    for (int j = 0; j < n; ++j) {
      const int slot = j & 1;
      const double rj = from_even(rnext);  // R[j, c] in both threads of the column
      if (own && half == 0 && j + 1 <= jmax) rnext = Rc[j + 1];
      if (c == j) {
        const double sig2 = pair_sum(s2);
        const double alpha = rj;
        double tau = 0.0, beta = alpha, sc = 0.0;
        if (sig2 != 0.0) {
          const double nrm = sqrt(alpha * alpha + sig2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          sc = 1.0 / (alpha - beta);
        }
        sc_own = sc;
#pragma unroll
        for (int r = 0; r < HR; ++r) xs[slot][half * HR + r] = x[r];
        if (half == 0) {
          Rc[j] = beta;
          coef[slot][0] = tau;
          coef[slot][1] = sc;
          if (keep) gp(t.tau)[(int64_t)bk * n + j] = tau;
        }
      }
      __syncthreads();
      if (own && c > j) {
        const double tau = coef[slot][0];
        const bool next_wave = ((2 * (j + 1)) >> 6) == wave;  // holds the next pivot
        if (tau != 0.0) {
          const double sc = coef[slot][1];
          const double* y = xs[slot] + half * HR;
          double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
          for (int r = 0; r < HR; r += 4) {
            d0 += y[r] * x[r];
            d1 += y[r + 1] * x[r + 1];
            d2 += y[r + 2] * x[r + 2];
            d3 += y[r + 3] * x[r + 3];
          }
          const double w = rj + sc * pair_sum((d0 + d1) + (d2 + d3));
          if (half == 0) Rc[j] = rj - tau * w;
          const double f = tau * w * sc;
          // Read y from LDS again for the update instead of holding it live
          // across the pair sum (register pressure).
          asm volatile("" ::: "memory");
          if (next_wave) {
            double q0 = 0.0, q1 = 0.0;
#pragma unroll
            for (int r = 0; r < HR; r += 2) {
              x[r] -= f * y[r];
              x[r + 1] -= f * y[r + 1];
              q0 += x[r] * x[r];
              q1 += x[r + 1] * x[r + 1];
            }
            s2 = q0 + q1;
          } else {
#pragma unroll
            for (int r = 0; r < HR; ++r) x[r] -= f * y[r];
          }
        } else if (next_wave) {
          double q0 = 0.0, q1 = 0.0;
#pragma unroll
          for (int r = 0; r < HR; r += 2) {
            q0 += x[r] * x[r];
            q1 += x[r + 1] * x[r + 1];
          }
          s2 = q0 + q1;
        }
      }
    }
    if (keep && c < n) {
#pragma unroll
      for (int r = 0; r < HR; ++r)
        if (r < rows) col[r0 + r] = sc_own * x[r];
    }
  }
}

// Replay stored reflectors on B only (kTaskApply).  Wave k (< nrhs) carries
// right-hand side k with lane r holding row r of the block; a step is a
// wave-wide dot product (DPP/shuffle sum), no workgroup barrier.
__device__ void batch_apply(const BatchTask& t, double (*cbuf)[kBatchMaxCols]) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int n = t.n, m = t.m;
  const int nblk = (m + H - 1) / H;
  double* cb = cbuf[w];  // running top n rows of Q^T b for this wave's column
  for (int k = w; k < t.nrhs; k += kBatchThreads / 64) {
    gdouble* b = gp(t.B + (int64_t)k * t.ldb);
    for (int j = l; j < n; j += 64) cb[j] = 0.0;
    __builtin_amdgcn_wave_barrier();
    for (int bk = 0; bk < nblk; ++bk) {
      const int r0 = bk * H;
      const bool in = r0 + l < m;
      double br = in ? b[r0 + l] : 0.0;
      const gdouble* Y = gp(t.A + r0 + l);
      const gdouble* tb = gp(t.tau + (int64_t)bk * n);
      double ynext = in ? Y[0] : 0.0;
      for (int j = 0; j < n; ++j) {
        const double y = ynext;
        if (j + 1 < n) ynext = in ? Y[(int64_t)(j + 1) * t.lda] : 0.0;
        const double tau = tb[j];
        if (tau == 0.0) continue;
        double d = y * br;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o);
        const double rj = cb[j];
        const double tw = tau * (rj + d);
        br -= tw * y;
        __builtin_amdgcn_wave_barrier();
        if (l == 0) cb[j] = rj - tw;
        __builtin_amdgcn_wave_barrier();
      }
    }
    gdouble* Rk = gp(t.C + (int64_t)k * n);
    for (int j = l; j < n; j += 64) Rk[j] = cb[j];
    __builtin_amdgcn_wave_barrier();
  }
}

// R x = c for the nrhs right-hand sides held in C; thread l owns row
// l.  Returns the 1-based index of the first zero diagonal entry (0 if none);
// then B's top rows receive c unchanged.
__device__ int batch_solve(const BatchTask& t, double (*xbuf)[kBatchMaxRhs], int* s_sing) {
  const int l = threadIdx.x;
  const int n = t.n, nrhs = t.nrhs;
  const gdouble* R = gp(t.R);
  const gdouble* C = gp(t.C);
  if (l == 0) *s_sing = INT_MAX;
  __syncthreads();
  if (l < n && R[l + (int64_t)l * n] == 0.0) atomicMin(s_sing, l);
  __syncthreads();
  const int sing = *s_sing;
  double cv[kBatchMaxRhs];
#pragma unroll
  for (int k = 0; k < kBatchMaxRhs; ++k)
    cv[k] = (k < nrhs && l < n) ? C[l + (int64_t)k * n] : 0.0;
  if (sing == INT_MAX) {
    double rl = l < n ? R[l + (int64_t)(n - 1) * n] : 0.0;  // R[l, n-1]
    for (int i = n - 1; i >= 0; --i) {
      const int slot = i & 1;
      const double rcur = rl;
      if (i >= 1 && l <= i - 1) rl = R[l + (int64_t)(i - 1) * n];
      if (l == i) {
#pragma unroll
        for (int k = 0; k < kBatchMaxRhs; ++k) {
          cv[k] = cv[k] / rcur;
          xbuf[slot][k] = cv[k];
        }
      }
      __syncthreads();
      if (l < i) {
#pragma unroll
        for (int k = 0; k < kBatchMaxRhs; ++k) cv[k] -= rcur * xbuf[slot][k];
      }
    }
  }
  if (l < n)
    for (int k = 0; k < nrhs; ++k) {
      gp(t.B)[l + (int64_t)k * t.ldb] = cv[k];
      if (t.X) gp(t.X)[l + (int64_t)k * n] = cv[k];
    }
  return sing == INT_MAX ? 0 : sing + 1;
}

__global__ __launch_bounds__(kBatchThreads) void k_batched_ls(const BatchHeader* table,
                                                                 int* counter, int* status) {
  const int count = __builtin_amdgcn_readfirstlane(table->count[0]);
  const BatchTask* tasks =
      (const BatchTask*)(table + 1) + __builtin_amdgcn_readfirstlane(table->begin[0]);
  __shared__ __align__(16) double ybuf[2][H];
  __shared__ double tbuf[2][2];
  __shared__ double xbuf[2][kBatchMaxRhs];
  __shared__ double cbuf[kBatchThreads / 64][kBatchMaxCols];
  __shared__ int s_idx, s_sing;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    // Uniform across the workgroup: keeps the task's fields in scalar registers.
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    __syncthreads();
    if (idx >= count) break;
    const BatchTask t = tasks[idx];
    if (t.flags & kTaskApply) {
      batch_apply(t, cbuf);
    } else {
      batch_factor(t, ybuf, tbuf);
    }
    __syncthreads();
    const int st = batch_solve(t, xbuf, &s_sing);
    if ((t.flags & kTaskWriteR) && st == 0) {
      const int c = threadIdx.x;
      if (c < t.n)
        for (int j = 0; j <= c; ++j) gp(t.A)[j + (int64_t)c * t.lda] = gp(t.R)[j + (int64_t)c * t.n];
    }
    if (threadIdx.x == 0) status[t.slot] = st;
    __syncthreads();
  }
}

}  // namespace

int batched_blk_grid(int device, int prec, int queue);
void batched_blk_launch(hipStream_t s, const BatchHeader* table, int queue, int* counter,
                        int* status, int* iters, int grid, int prec);

BatchGrids batched_grids(int device, int prec) {
  BatchGrids g{};
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    cus = 256;
  int per = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batched_ls, kBatchThreads, 0) !=
          hipSuccess ||
      per < 1)
    per = 1;
  g.g[0] = cus * per;
  for (int k = 1; k <= kBatchQueues; ++k) g.g[k] = batched_blk_grid(device, prec, k);
  return g;
}

void batched_ls(hipStream_t s, const BatchHeader* table, int* counter, int* status, int* iters,
                const BatchGrids& grids, int prec, double bytes, double flops) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, counter);
  TimedLaunch tl(s, "batched_ls", bytes, flops);
  // Largest problems first: the queues of more tiles per wave hold them.
  for (int k = kBatchQueues - 1; k >= 1; --k)
    batched_blk_launch(s, table, k, counter, status, iters, grids.g[k], prec);
  if (prec != kBlkF64)
    batched_blk_launch(s, table, kBatchQueues, counter, status, iters, grids.g[kBatchQueues], prec);
  if (grids.g[0] > 0)
    hipLaunchKernelGGL(k_batched_ls, dim3(grids.g[0]), dim3(kBatchThreads), 0, s, table, counter,
                       status);
}

}  // namespace miqr
