// Batched least squares: many independent small problems in persistent
// launches.  Each workgroup pops problems from a device queue and solves each
// one alone, so a problem's arithmetic does not depend on what else is in the
// batch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miqr {

constexpr int kBatchRows = 64;      // row block height of the flat TSQR sweep
constexpr int kBatchMaxCols = 320;  // n + nrhs limit
constexpr int kBatchThreads = 2 * kBatchMaxCols;  // column sweep: two threads per column
constexpr int kBatchMaxRhs = 8;

// Task flags.
constexpr int kTaskKeep = 1;    // store the reflector blocks in A and tau (for later solves)
constexpr int kTaskApply = 2;   // reuse stored reflectors: transform B only, then solve
constexpr int kTaskWriteR = 4;  // copy R into A's upper triangle at the end

// Status of a problem: 0, j + 1 when R_jj == 0 exactly, or kStatusNoConv
// when a mixed-precision solve did not reach its backward-error target (A and
// B are then left as they were, for an FP64 solve).
constexpr int kStatusNoConv = -1;
// A bounded wait inside the batched kernel ran out (a logic error, never
// expected): the problem's results are not valid.
constexpr int kStatusFault = -2;

// Queues: tasks are grouped by kernel.  Queue 0 is the column sweep (replays
// of kept reflectors); queues 1..3 the blocked kernel for problems of at most
// 8, 12 and 20 sixteen-column tiles of [A | B] (two, three and five tiles per
// wave), each compiled for its own register budget.
constexpr int kBatchQueues = 4;
constexpr int kBlkWaves = 4;

// Working precision of the blocked kernel.
enum BlkPrec : int { kBlkF64 = 0, kBlkF32 = 1, kBlkBF16 = 2 };

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

// Queue of a task (by its flags and its number of column tiles).
int batch_queue(const BatchTask& t);

// Device task table: a header, then the tasks grouped by queue (queue k's
// tasks at [begin[k], begin[k] + count[k])).  The kernels read the counts
// from the header, so one captured launch sequence serves tables of any
// length up to the capacity it was sized for.
struct BatchHeader {
  int total;
  int begin[kBatchQueues];
  int count[kBatchQueues];
  int pad[16 - 1 - 2 * kBatchQueues];
};
static_assert(sizeof(BatchHeader) == 64, "BatchHeader is one 64-byte line");
inline BatchTask* batch_tasks(BatchHeader* h) { return (BatchTask*)(h + 1); }
inline size_t batch_table_bytes(int64_t count) {
  return sizeof(BatchHeader) + (size_t)count * sizeof(BatchTask);
}

// Persistent grids (workgroups) of the queues' kernels for one precision;
// entry kBatchQueues is the refinement kernel of the mixed precisions.
struct BatchGrids {
  int g[kBatchQueues + 1];
};
// Device ints the launches use as queue counters.
constexpr int kBatchCounters = kBatchQueues + 1;
BatchGrids batched_grids(int device, int prec);

// Solve the table's tasks: one persistent launch per queue (largest problems
// first), each popping its queue in table order, then for a mixed precision
// one persistent launch that refines the solutions of queues 1..3 in FP64.
// status[slot] receives the problem's status, iters[slot] (if iters is
// non-null; mixed precisions) the refinement iterations or -1.  counter:
// kBatchCounters device ints, reset by the launch.  prec: working precision
// of the blocked kernel (tasks of queue 0 always run in FP64).  bytes / flops:
// the batch's algorithmic totals, for the kernel timer.
void batched_ls(hipStream_t s, const BatchHeader* table, int* counter, int* status, int* iters,
                const BatchGrids& grids, int prec, double bytes, double flops);

}  // namespace miqr
