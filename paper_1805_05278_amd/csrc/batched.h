// Batched least squares: many independent small problems in one persistent
// launch.  Each workgroup pops problems from a device queue and solves each one
// alone, so a problem's arithmetic does not depend on what else is in the batch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miqr {

constexpr int kBatchRows = 64;      // row block height of the flat TSQR sweep
constexpr int kBatchMaxCols = 320;  // n + nrhs limit
constexpr int kBatchThreads = 2 * kBatchMaxCols;  // two threads per column
constexpr int kBatchMaxRhs = 8;

// Task flags.
constexpr int kTaskKeep = 1;    // store the reflector blocks in A and tau (for later solves)
constexpr int kTaskApply = 2;   // reuse stored reflectors: transform B only, then solve
constexpr int kTaskWriteR = 4;  // copy R into A's upper triangle at the end

struct BatchTask {
  double* A;        // m x n (lda)
  double* B;        // m x nrhs (ldb); rows 0..n-1 receive x
  double* R;        // n x n, ld n: the R factor (read-only for kTaskApply)
  double* C;        // n x nrhs, ld n: the top n rows of Q^T B
  double* tau;      // ceil(m / 64) x n reflector scalars (kTaskKeep / kTaskApply)
  double* X;        // optional n x nrhs (ld n) second copy of the solution
  int64_t lda, ldb;
  int m, n, nrhs, flags;
  int slot;         // index into the status array
  int pad;
};

// Device task table: a header holding the task count, then the tasks.  The
// kernel reads the count from the header, so one captured launch serves
// tables of any length up to the grid's capacity.
struct BatchHeader {
  int count;
  int pad[15];
};
inline BatchTask* batch_tasks(BatchHeader* h) { return (BatchTask*)(h + 1); }
inline size_t batch_table_bytes(int64_t count) {
  return sizeof(BatchHeader) + (size_t)count * sizeof(BatchTask);
}

// Solve the table's tasks (in table order of popping) with `grid` persistent
// workgroups; status[slot] = 0, or j + 1 if R_jj == 0 exactly (B then holds
// the top n rows of Q^T B).  counter: one device int, reset by the launch.
// bytes / flops: the batch's algorithmic totals, for the kernel timer.
void batched_ls(hipStream_t s, const BatchHeader* table, int* counter, int* status, int grid,
                double bytes, double flops);

// Workgroups that fit on the device at once for the batched kernel.
int batched_grid(int device, int count);

}  // namespace miqr
