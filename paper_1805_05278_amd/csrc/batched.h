// Batched least squares: many independent small problems in one persistent
// launch.  Each workgroup pops problems from a device queue and solves each one
// alone, so a problem's arithmetic does not depend on what else is in the batch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miqr {

constexpr int kBatchRows = 64;     // row block height of the flat TSQR sweep
constexpr int kBatchThreads = 320; // one thread per column: n + nrhs <= 320
constexpr int kBatchMaxRhs = 8;

// Task flags.
constexpr int kTaskKeep = 1;    // store the reflector blocks in A and tau (for later solves)
constexpr int kTaskApply = 2;   // reuse stored reflectors: transform B only, then solve
constexpr int kTaskWriteR = 4;  // copy R into A's upper triangle at the end

struct BatchTask {
  double* A;        // m x n (lda)
  double* B;        // m x nrhs (ldb); rows 0..n-1 receive x
  double* R;        // n x (n + nrhs), ld n: R and the top n rows of Q^T B
  double* tau;      // ceil(m / 64) x n reflector scalars (kTaskKeep / kTaskApply)
  int64_t lda, ldb;
  int m, n, nrhs, flags;
  int slot;         // index into the status array
  int pad;
};

// Solve tasks[0..count) (in that order of popping) with `grid` persistent
// workgroups; status[slot] = 0, or j + 1 if R_jj == 0 exactly (B then holds
// the top n rows of Q^T B).  counter: one device int, reset by the launch.
// bytes / flops: the batch's algorithmic totals, for the kernel timer.
void batched_ls(hipStream_t s, const BatchTask* tasks, int count, int* counter, int* status,
                int grid, double bytes, double flops);

// Workgroups that fit on the device at once for the batched kernel.
int batched_grid(int device, int count);

}  // namespace miqr
