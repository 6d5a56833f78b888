// Batched least squares, blocked form: one workgroup of four waves per
// problem, popped from a device queue by a persistent grid.
//
// As in the column sweep, min ||B - A X|| (A m x n, nrhs right-hand sides)
// is solved by Householder QR of [A | B] (N = n + nrhs columns) with a flat
// TSQR sweep over 64-row blocks (the TSQR of Sec. 5 / App. C.1 with a chain
// as its tree): the running R (n x N) is stacked over each block X and
// [R; X] is reduced.  Here the block's reflectors are taken sixteen at a
// time (a panel) in the compact WY form of Sec. 2.3.  The reflector of
// column j is v = [e_j; y] (R is upper triangular), so the panel's
// V^T V = I + Y^T Y, its T follows the Sec. 2.3 recurrence on the Gram
// entries y_i . y_j, and it updates each sixteen-column tile c right of it by
//   W = R[panel rows, c] + Y^T X[:, c],   W' = T^T W,
//   R[panel rows, c] -= W',   X[:, c] -= Y W',
// three products on MFMA.
//
// Register layout: tile c of the block lives in wave c mod 4; lane l
// (q = l / 16, cl = l % 16) holds rows 16 t + rho(q, r) (t, r = 0..3) of
// column 16 c + cl, rho being the row map of the MFMA accumulator.  The tile
// is therefore both the B operand of Y^T X (the contraction over the block's
// rows runs in the order the registers hold them, with Y read in that same
// order) and the accumulator of X -= Y W', with no data movement.  R stays in
// global memory (L2): tile (p, c) is read and written once per block, always
// by the wave that owns column tile c.
//
// A panel is factored by the wave that owns its tile, column by column
// (dlarfg sign rule; norm, beta and tau in FP64): the pivot column reaches
// the other lanes through LDS, dot products are per-lane partial sums and one
// cross-row sum in registers (v_permlane16/32_swap), and the same sums give
// the Gram entries of T.  Look-ahead: the owner of panel p + 1 updates that
// tile first and factors it while the other waves still apply panel p, so a
// panel costs one barrier.
//
// Precisions: FP64 throughout (FP64 MFMA), or a working copy of the block in
// FP32 with Y^T X and Y W' on FP32 MFMA or on BF16 MFMA with FP32
// accumulation; reflector generation, T and R stay in FP64 and T^T W runs on
// FP32 MFMA.  The mixed forms then refine each solution in FP64 against the
// original A and B: conjugate gradients on the normal equations with R as
// preconditioner (CGLS on min ||b - (A R^-1) y||, x = R^-1 y), the residual
// b - A x recomputed from A each iteration, until every right-hand side's
// backward error ||A^T r|| / (||A||_F (||A||_F ||x|| + ||r||)) is at most
// 5e-14 (the 1e-13 gate with a margin).  A and B are only written once that
// holds; otherwise the problem
// reports kStatusNoConv with A and B intact, for an FP64 solve.
#include <climits>

#include "batched.h"
#include "common.h"

namespace miqr {
namespace {

constexpr int H = kBatchRows;
constexpr int NW = kBlkWaves;
constexpr int NT = 64 * NW;
constexpr int KG = 4;  // right-hand sides refined together
// Refinement target: half the 1e-13 gate, a margin for the rounding of the
// estimate itself (another FP64 evaluation of ||A^T r|| differs by about
// u sqrt(m) ||A|| ||r||).
constexpr double kRefineTol = 5e-14;
constexpr int kRefineMaxIt = 40;

static_assert(NW == 4, "tile-to-wave map assumes four waves");
static_assert(kBatchMaxCols <= 2 * NT, "a thread owns at most two rows of R");

typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gdouble* gp(double* p) { return (gdouble*)p; }
__device__ __forceinline__ const gdouble* gp(const double* p) { return (const gdouble*)p; }

typedef short s4 __attribute__((ext_vector_type(4)));

template <int P>
struct Prec {
  typedef float W;
  typedef f4 V;
};
template <>
struct Prec<kBlkF64> {
  typedef double W;
  typedef d4 V;
};

// Row map of the 16x16 MFMA accumulators: register r of lane group q holds
// row rho(q, r); the FP64 output interleaves the lane groups, the FP32
// outputs stack them.  rho_q / rho_r invert it.
template <int P>
__device__ __forceinline__ constexpr int rho(int q, int r) {
  return P == kBlkF64 ? q + 4 * r : 4 * q + r;
}
template <int P>
__device__ __forceinline__ constexpr int rho_q(int v) {
  return P == kBlkF64 ? (v & 3) : (v >> 2);
}
template <int P>
__device__ __forceinline__ constexpr int rho_r(int v) {
  return P == kBlkF64 ? (v >> 2) : (v & 3);
}

// 16x16x4 MFMA of the working type: a = A[l % 16][l / 16], b = B[l / 16][l % 16].
__device__ __forceinline__ d4 mma(double a, double b, d4 c) { return mfma64(a, b, c); }
__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Round to nearest even BF16 (finite inputs).
__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ s4 pack_bf16(f4 v) {
  s4 o;
  o[0] = to_bf16(v[0]);
  o[1] = to_bf16(v[1]);
  o[2] = to_bf16(v[2]);
  o[3] = to_bf16(v[3]);
  return o;
}
// 16x16x16 BF16 MFMA: a = A[l % 16][4 (l / 16) + j], b = B[4 (l / 16) + j][l % 16].
__device__ __forceinline__ f4 mma_bf16(f4 a, f4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pack_bf16(a), pack_bf16(b), c, 0, 0, 0);
}

__device__ __forceinline__ unsigned lo32(double v) {
  return (unsigned)(unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ unsigned hi32(double v) {
  return (unsigned)((unsigned long long)__double_as_longlong(v) >> 32);
}
__device__ __forceinline__ double join(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the four lanes cl, cl + 16, cl + 32, cl + 48: rows paired by
// v_permlane16_swap, then halves by v_permlane32_swap; each swap leaves one
// copy holding the lower partner in both places and the other the upper, so
// every lane forms the same sums in the same order.
__device__ __forceinline__ double rows_sum(double v) {
  {
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(v), lo32(v), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(v), hi32(v), false, false);
    v = join(l[0], h[0]) + join(l[1], h[1]);
  }
  {
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(v), lo32(v), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(v), hi32(v), false, false);
    v = join(l[0], h[0]) + join(l[1], h[1]);
  }
  return v;
}

__device__ __forceinline__ double readlane(double v, int lane) {
  return join((unsigned)__builtin_amdgcn_readlane((int)lo32(v), lane),
              (unsigned)__builtin_amdgcn_readlane((int)hi32(v), lane));
}

// The pivot broadcast fused into the FMAs: v_fmac_{f64,f32}_dpp with
// row_newbcast:J reads its first source from lane J of the lane's row.  One
// s_nop 1 at the head of each block gives the two wait states a DPP read
// needs after a VALU write of its source (the compiler does not look inside
// the asm); within a block no instruction DPP-reads a register written by
// the one before it.  xs[4 t + r] is register r of row tile t.
//   d0 += sum_t (x_J[t][0] x[t][0] + x_J[t][2] x[t][2]), d1 likewise for
//   registers 1 and 3 (two chains for latency).
template <int J>
__device__ __forceinline__ void dots_bcast(const double (&xs)[16], double& d0, double& d1) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %2, %2 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %3, %3 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %0, %4, %4 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %5, %5 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %0, %6, %6 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %7, %7 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %0, %8, %8 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %9, %9 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %0, %10, %10 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %11, %11 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %0, %12, %12 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %13, %13 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %0, %14, %14 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %15, %15 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %0, %16, %16 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %17, %17 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      : "+v"(d0), "+v"(d1)
      : "v"(xs[0]), "v"(xs[1]), "v"(xs[2]), "v"(xs[3]), "v"(xs[4]), "v"(xs[5]), "v"(xs[6]), "v"(xs[7]), "v"(xs[8]), "v"(xs[9]), "v"(xs[10]), "v"(xs[11]), "v"(xs[12]), "v"(xs[13]), "v"(xs[14]), "v"(xs[15]), "n"(J));
}
template <int J>
__device__ __forceinline__ void dots_bcast(const float (&xs)[16], float& d0, float& d1) {
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %2, %2 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %3, %3 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %4, %4 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %5, %5 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %6, %6 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %7, %7 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %8, %8 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %9, %9 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %10, %10 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %11, %11 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %12, %12 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %13, %13 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %14, %14 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %15, %15 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %16, %16 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %17, %17 row_newbcast:%18 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      : "+v"(d0), "+v"(d1)
      : "v"(xs[0]), "v"(xs[1]), "v"(xs[2]), "v"(xs[3]), "v"(xs[4]), "v"(xs[5]), "v"(xs[6]), "v"(xs[7]), "v"(xs[8]), "v"(xs[9]), "v"(xs[10]), "v"(xs[11]), "v"(xs[12]), "v"(xs[13]), "v"(xs[14]), "v"(xs[15]), "n"(J));
}
//   x[t][r] += x_J[t][r] nf (lane J's own entries are unchanged when its nf
//   is zero).
template <int J>
__device__ __forceinline__ void update_bcast(double (&xs)[16], double nf) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %0, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %1, %1, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %2, %2, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %3, %3, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %4, %4, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %5, %5, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %6, %6, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %7, %7, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %8, %8, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %9, %9, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %10, %10, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %11, %11, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %12, %12, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %13, %13, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %14, %14, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f64_dpp %15, %15, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      : "+v"(xs[0]), "+v"(xs[1]), "+v"(xs[2]), "+v"(xs[3]), "+v"(xs[4]), "+v"(xs[5]), "+v"(xs[6]), "+v"(xs[7]), "+v"(xs[8]), "+v"(xs[9]), "+v"(xs[10]), "+v"(xs[11]), "+v"(xs[12]), "+v"(xs[13]), "+v"(xs[14]), "+v"(xs[15])
      : "v"(nf), "n"(J));
}
template <int J>
__device__ __forceinline__ void update_bcast(float (&xs)[16], float nf) {
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %0, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %1, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %2, %2, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %3, %3, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %4, %4, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %5, %5, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %6, %6, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %7, %7, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %8, %8, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %9, %9, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %10, %10, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %11, %11, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %12, %12, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %13, %13, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %14, %14, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %15, %15, %16 row_newbcast:%17 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      : "+v"(xs[0]), "+v"(xs[1]), "+v"(xs[2]), "+v"(xs[3]), "+v"(xs[4]), "+v"(xs[5]), "+v"(xs[6]), "+v"(xs[7]), "+v"(xs[8]), "+v"(xs[9]), "+v"(xs[10]), "+v"(xs[11]), "+v"(xs[12]), "+v"(xs[13]), "+v"(xs[14]), "+v"(xs[15])
      : "v"(nf), "n"(J));
}

// Lane group QJ's value to all four groups (lanes cl, cl + 16, cl + 32,
// cl + 48): v_permlane16_swap leaves rows (0, 0, 2, 2) in one copy and
// (1, 1, 3, 3) in the other, v_permlane32_swap then halves (0, 1, 0, 1) and
// (2, 3, 2, 3).
template <int QJ>
__device__ __forceinline__ double group_bcast(double v) {
  unsigned lo = lo32(v), hi = hi32(v);
  {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    lo = (QJ & 1) ? l[1] : l[0];
    hi = (QJ & 1) ? h[1] : h[0];
  }
  {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    lo = (QJ & 2) ? l[1] : l[0];
    hi = (QJ & 2) ? h[1] : h[0];
  }
  return join(lo, hi);
}

// The lane index through an empty asm: addresses, masks and row numbers made
// from it are then computed where they are used.  Otherwise the compiler
// hoists them out of the sweep's loops as invariants and holds dozens of
// them in registers for the whole problem, spilling the tiles.
// Workgroup barrier that orders LDS only: global loads in flight (a
// prefetch) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int lane_id() {
  int l = threadIdx.x & 63;
  asm volatile("" : "+v"(l));
  return l;
}

// LDS buffers for the panels' Y and T: panel p uses buffer p mod NBUF.  With
// three, panel p + 1 reuses panel p - 2's buffer, whose readers finished
// before panel p was published, so no factorisation waits for the previous
// owner's other tiles; with two it waits for the last of panel p - 1's
// readers.  The FP32 working copies take three; FP64 keeps two, which leaves
// LDS for three workgroups per CU where its registers allow them (measured
// faster overall).
template <typename W>
struct Bufs {
  static constexpr int n = sizeof(W) == 8 ? 2 : 3;
};

template <typename W, int NBUF = Bufs<W>::n>
struct FactorLds {
  W ya[NBUF][4][4][16][4];  // Y by accumulator position: [buf][t][q][cl][r] = Y[16 t + rho(q, r)][cl]
  W yt[NBUF][4][16][4][4];  // Y as the A operand of Y W': [buf][t][i][q][r] = Y[16 t + i][rho(q, r)]
  W ts[NBUF][16][4][4];     // T: [buf][j][q][r] = T[rho(q, r)][j]
};
template <typename W, int NBUF = Bufs<W>::n>
struct BlkLds {
  FactorLds<W> f;
  double gram[16][18];  // [k][i] = y_i . y_k, i < k, of the current panel (rows 16-byte aligned)
  double tau[NBUF][16];
  double z[2][8];
  int idx, sing;
  int ready_y;  // last panel of the block whose Y (the ya copy) is in LDS
  int ready;    // last panel of the block whose Y (both copies) and T are in LDS
  int done[NW];  // per wave: panels of the block whose updates it has finished
  int err;    // a bounded wait ran out (a logic error): the problem fails
};

// Bounded wait until an LDS counter reaches `target`.  Every wave of the
// workgroup progresses without the waiting one, so the wait ends; the bound
// turns a logic error into an error status rather than a hang.
// Once one wait has run out, every later wait of the problem returns at
// once, so a fault costs one bound, not one per wait.
constexpr int kSpinLimit = 1 << 20;
__device__ __forceinline__ void wait_at_least(int* v, int target, int* err) {
  if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return;
  int spins = 0;
  while (__hip_atomic_load(v, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
    if (++spins > kSpinLimit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}
// Bounded wait until every wave's counter v[w] reaches `target` (same bound
// and error rule as wait_at_least).
__device__ __forceinline__ void wait_all_at_least(int* v, int target, int* err) {
  if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return;
  int spins = 0;
  for (;;) {
    int lo = __hip_atomic_load(&v[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int w = 1; w < NW; ++w)
      lo = min(lo, __hip_atomic_load(&v[w], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (lo >= target) return;
    if (++spins > kSpinLimit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}
constexpr int RC = 16;       // rows of A per chunk of a refinement pass
constexpr int RCP = RC + 1;  // padded column stride of the chunk: a thread per column reads
                             // one row of it without bank conflicts
struct RefineLds {
  double v[kBatchMaxCols * KG];      // a vector of length n per right-hand side, [row][rhs]
  double a[kBatchMaxCols * RCP];     // the chunk's entries of A, [column][row]
  double part[NT / RC][RC][KG];      // per-group partial sums of A v, [group][row][rhs]
  double rc[RC][KG];                 // the chunk's residual
  double red[NW][KG];
  double z[2][8];
  int idx, sing;
};

__device__ __forceinline__ const double* src_col(const BatchTask& t, int col) {
  return col < t.n ? t.A + (int64_t)col * t.lda : t.B + (int64_t)(col - t.n) * t.ldb;
}
__device__ __forceinline__ double* r_col(const BatchTask& t, int col) {
  return col < t.n ? t.R + (int64_t)col * t.n : t.C + (int64_t)(col - t.n) * t.n;
}

// Tile (p, c) of the running R (rows 16 p.., columns 16 c.. of [R | C]) in
// accumulator order; zero when `zero` (before the first block) and outside
// n x N.  The loads are issued unconditionally (an entry outside reads R[0][0]
// and is replaced by zero): with no branches around them the compiler can
// count them and need not wait for them before unrelated work.
template <int P>
__device__ __forceinline__ void load_r(const BatchTask& t, int p, int c, bool zero, double (&rv)[4]) {
  const int lane = lane_id(), q = lane >> 4, cl = lane & 15;
  const int col = 16 * c + cl;
  const bool in = !zero && col < t.n + t.nrhs;
  const gdouble* rc = gp(r_col(t, in ? col : 0));
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * p + rho<P>(q, r);
    const bool ok = in && row < t.n;
    const double v = rc[ok ? row : 0];
    rv[r] = ok ? v : 0.0;
  }
}
template <int P>
__device__ __forceinline__ void store_r(const BatchTask& t, int p, int c, const double (&rv)[4]) {
  const int lane = lane_id(), q = lane >> 4, cl = lane & 15;
  const int col = 16 * c + cl;
  if (col >= t.n + t.nrhs) return;
  gdouble* rc = gp(r_col(t, col));
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * p + rho<P>(q, r);
    if (row < t.n) rc[row] = rv[r];
  }
}

// Tile c of the block at row r0 of [A | B], in the working precision.
template <int P>
__device__ __forceinline__ void load_tile(const BatchTask& t, int r0, int c,
                                          typename Prec<P>::V (&x)[4]) {
  using W = typename Prec<P>::W;
  const int lane = lane_id(), q = lane >> 4, cl = lane & 15;
  const int col = 16 * c + cl;
  const bool in = col < t.n + t.nrhs;
  const gdouble* src = gp(src_col(t, in ? col : 0));
#pragma unroll
  for (int tt = 0; tt < 4; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + 16 * tt + rho<P>(q, r);
      const bool ok = in && row < t.m;
      const double v = src[ok ? row : 0];  // unconditional load (see load_r)
      x[tt][r] = (W)(ok ? v : 0.0);
    }
}

// Column JJ of a panel (dlarfg sign rule; norm, beta and tau in FP64) by the
// wave holding the panel's tile x, with the diagonal R tile in rd (row JJ in
// register rho_r(JJ) of lane group rho_q(JJ)).  The columns are unrolled, so
// every register index and lane is a constant: the pivot column enters the
// dot products and the update through DPP broadcasts inside the FMAs, R's
// row JJ reaches all four lane groups by lane permutes.
template <int P, int JJ>
__device__ __forceinline__ void column_step(int q, int cl, typename Prec<P>::V (&x)[4],
                                            double (&rd)[4], double& mysc, double& mytau,
                                            BlkLds<typename Prec<P>::W>& S) {
  using W = typename Prec<P>::W;
  using V = typename Prec<P>::V;
  constexpr int qj = rho_q<P>(JJ), rj = rho_r<P>(JJ);
  const double rdj = rd[rj];
  W xs[16];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) xs[4 * tt + r] = x[tt][r];
  const double alpha = readlane(rdj, 16 * qj + JJ);
  W d0 = 0, d1 = 0;
  dots_bcast<JJ>(xs, d0, d1);
  const double dot = rows_sum((double)d0 + (double)d1);  // x_j . x_cl
  // Lane JJ's dot product is the pivot column's squared norm.
  const double sig2 = readlane(dot, JJ);
  const double rjc = group_bcast<qj>(rdj);  // R[j, cl] in all four lanes
  // Reflector (dlarfg rule) without branches; no reflection when the column
  // below the diagonal is zero.
  double bt, tr, z;
  reflector(alpha, sig2, bt, tr, z);
  const bool refl = sig2 != 0.0;
  const double beta = refl ? bt : alpha;
  const double sc = refl ? z : 0.0;
  const double tau = refl ? tr : 0.0;
  // w = R[j, cl] + y_j . x_cl; for cl < JJ it is the Gram entry y_cl . y_j
  // once scaled (entries cl >= JJ are written too and never read).
  const double w = rjc + sc * dot;
  if (q == 0) S.gram[JJ][cl] = mysc * w;
  // Columns right of the pivot: x -= tau w y_j, R[j, cl] -= tau w; the
  // pivot's lane keeps its reflector and takes beta.
  const bool right = cl > JJ, piv = cl == JJ;
  const double tw = tau * w;
  const W nf = right ? (W)(-(tw * sc)) : (W)0;
  update_bcast<JJ>(xs, nf);
#pragma unroll
  for (int tt = 0; tt < 4; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) x[tt][r] = xs[4 * tt + r];
  const double rnew = piv ? beta : (right ? rdj - tw : rdj);
  mysc = piv ? sc : mysc;
  mytau = piv ? tau : mytau;
  rd[rj] = q == qj ? rnew : rd[rj];
}

// Columns JJ .. pw - 1 of a panel (q, cl: the lane's group and column,
// formed once per panel).
template <int P, int JJ>
__device__ __forceinline__ void column_steps(int pw, int q, int cl, typename Prec<P>::V (&x)[4],
                                             double (&rd)[4], double& mysc, double& mytau,
                                             BlkLds<typename Prec<P>::W>& S) {
  if constexpr (JJ < 16) {
    if (JJ < pw) {
      column_step<P, JJ>(q, cl, x, rd, mysc, mytau, S);
      column_steps<P, JJ + 1>(pw, q, cl, x, rd, mysc, mytau, S);
    }
  }
}

// Householder QR of panel p (columns 16 p .. 16 p + pw - 1) of [R; X] by the
// wave that owns its tile x.  Leaves the reflector tails Y in x's panel
// columns (the tile's other columns, right-hand sides, are updated), Y and T
// in LDS buffer p mod NBUF, the diagonal tile of R in global memory, and tau in
// LDS (and in t.tau for kept factors).
template <int P>
__device__ void panel_factor(const BatchTask& t, int p, int bk, typename Prec<P>::V (&x)[4],
                             double (&rd)[4], BlkLds<typename Prec<P>::W>& S) {
  using W = typename Prec<P>::W;
  using V = typename Prec<P>::V;
  const int lane = lane_id(), q = lane >> 4, cl = lane & 15;
  const int n = t.n;
  const int pw = min(16, n - 16 * p);
  constexpr int NBUF = Bufs<W>::n;
  const int b = p % NBUF;
  const bool keep = (t.flags & kTaskKeep) != 0;
  FactorLds<W>& F = S.f;
  double mysc = 0.0;   // scale of this lane's column reflector (y = sc x)
  double mytau = 0.0;  // and its tau (zero for the missing columns of a narrow panel)
  // A narrow last panel: the Gram rows of the missing columns are zero (T's
  // build below reads all sixteen).
  if (pw < 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = pw + (lane >> 4) + 4 * r;
      if (k < 16) S.gram[k][cl] = 0.0;
    }
  }
  column_steps<P, 0>(pw, q, cl, x, rd, mysc, mytau, S);
  if (lane < 16) {
    S.tau[b][lane] = mytau;
    if (keep && lane < pw) gp(t.tau)[(int64_t)bk * n + 16 * p + lane] = mytau;
  }
  // Y in the panel columns; zero for the tile's other columns in the LDS copies.
  const bool acol = cl < pw;
  const W ys = acol ? (W)mysc : (W)0;
  V yv[4];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    yv[tt] = x[tt] * ys;
    if (acol) x[tt] = yv[tt];
    *(V*)&F.ya[b][tt][q][cl][0] = yv[tt];
  }
  __builtin_amdgcn_wave_barrier();
  // Y is final: the other waves can form Y^T X (which reads the ya copy)
  // while the yt copy is written and T is built; both are published with T.
  if (lane == 0) __hip_atomic_store(&S.ready_y, p, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
  for (int tt = 0; tt < 4; ++tt)
#pragma unroll
    for (int r = 0; r < 4; ++r) F.yt[b][tt][rho<P>(q, r)][rho_q<P>(cl)][rho_r<P>(cl)] = yv[tt][r];
  // T of the panel (Sec. 2.3), by columns.  T is the inverse of the upper
  // triangular S = diag(1 / tau) + striu(V^T V), and V^T V = I + Y^T Y, so
  // column j of T solves S t = e_j by back-substitution: t_j = tau_j and
  // t_i = -tau_i sum_{i < k <= j} G[i][k] t_k (G = Y^T Y), a form that also
  // holds for tau = 0 (zero row and column).  Lane cl computes column cl
  // alone, with no cross-lane sums; G's entries are broadcast reads of LDS.
  // acc[i] collects sum_k G[i][k] t_k until row i's turn, then holds t_i.
  double acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0;
#pragma unroll
  for (int k = 15; k >= 0; --k) {
    // One row of G in registers at a time (the scheduling barrier keeps the
    // compiler from loading them all up front).
    __builtin_amdgcn_sched_barrier(0);
    const double tk = S.tau[b][k];
    acc[k] = fma(-tk, acc[k], cl == k ? tk : 0.0);
#pragma unroll
    for (int i = 0; i < k; ++i) acc[i] = fma(S.gram[k][i], acc[k], acc[i]);
  }
  // ts[j][q][r] = T[rho(q, r)][j]: each lane writes its lane group's four
  // (every lane stores, so the compiler cannot sink the arithmetic into a
  // branch behind the loads).
  V tv;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double v = acc[rho<P>(0, r)];
#pragma unroll
    for (int qq = 1; qq < 4; ++qq) v = q == qq ? acc[rho<P>(qq, r)] : v;
    tv[r] = (W)v;
  }
  *(V*)&F.ts[b][cl][q][0] = tv;
  store_r<P>(t, p, p, rd);
}

// Update of tile x (column tile c) by panel p.  Y of the panel must be
// published; wait_t: T may not be yet, and is waited for after Y^T X.
template <int P>
__device__ __forceinline__ void update_tile(const BatchTask& t, int p, int c, bool first,
                                            typename Prec<P>::V (&x)[4],
                                            BlkLds<typename Prec<P>::W>& S, bool wait_t) {
  using W = typename Prec<P>::W;
  using V = typename Prec<P>::V;
  const FactorLds<W>& F = S.f;
  const int lane = lane_id(), q = lane >> 4, cl = lane & 15;
  constexpr int NBUF = Bufs<W>::n;
  const int b = p % NBUF;
  // Y and T are read from LDS for each tile rather than held across the
  // wave's tiles (register pressure): the empty asm keeps the compiler from
  // merging the reads of consecutive tile updates.
  asm volatile("" ::: "memory");
  double ro[4];
  load_r<P>(t, p, c, first, ro);
  V acc = {};
  if constexpr (P == kBlkBF16) {
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) acc = mma_bf16(*(const V*)&F.ya[b][tt][q][cl][0], x[tt], acc);
  } else {
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      const V ya = *(const V*)&F.ya[b][tt][q][cl][0];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mma(ya[r], x[tt][r], acc);
    }
  }
  V wv;
#pragma unroll
  for (int r = 0; r < 4; ++r) wv[r] = (W)(ro[r] + (double)acc[r]);
  if (wait_t) wait_at_least(&S.ready, p, &S.err);
  const V tv = *(const V*)&F.ts[b][cl][q][0];
  V w2 = {};
#pragma unroll
  for (int r = 0; r < 4; ++r) w2 = mma(tv[r], wv[r], w2);
#pragma unroll
  for (int r = 0; r < 4; ++r) ro[r] -= (double)w2[r];
  store_r<P>(t, p, c, ro);
  const V nw = -w2;
  asm volatile("" ::: "memory");
  if constexpr (P == kBlkBF16) {
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) x[tt] = mma_bf16(*(const V*)&F.yt[b][tt][cl][q][0], nw, x[tt]);
  } else {
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      const V yt = *(const V*)&F.yt[b][tt][cl][q][0];
#pragma unroll
      for (int r = 0; r < 4; ++r) x[tt] = mma(yt[r], nw[r], x[tt]);
    }
  }
}

// Slot i of a wave's tiles holds the wave's tile (i + rot) mod MAXT (tile
// w + NW ((i + rot) mod MAXT)): after factoring a panel the owner rotates its
// slots by one, so the next panel it owns is always in slot 0 and the
// unrolled factorisation exists once rather than once per slot.
template <int MAXT>
__device__ __forceinline__ int slot_tile(int w, int i, int rot) {
  const int k = i + rot;
  return w + NW * (k >= MAXT ? k - MAXT : k);
}

// The owner's step for panel pn = p + 1 (its tile in slot 0): update by
// panel p (if any), factor, publish, rotate the slots.
template <int P, int MAXT>
__device__ __forceinline__ void own_panel(const BatchTask& t, int p, int bk,
                                          typename Prec<P>::V (&x)[MAXT][4],
                                          BlkLds<typename Prec<P>::W>& S) {
  using V = typename Prec<P>::V;
  // The panel's diagonal R tile, loaded before the update so that its
  // latency is off the chain (only this wave touches it).
  double rd[4];
  load_r<P>(t, p + 1, p + 1, bk == 0, rd);
  if (p >= 0) update_tile<P>(t, p, p + 1, bk == 0, x[0], S, true);
  // LDS buffer (p + 1) mod NBUF last held panel p + 1 - NBUF: every wave
  // must be done with it (a per-wave count: a total could be reached while
  // one slow wave still reads the buffer).
  wait_all_at_least(S.done, p + 2 - Bufs<typename Prec<P>::W>::n, &S.err);
  panel_factor<P>(t, p + 1, bk, x[0], rd, S);
  if ((threadIdx.x & 63) == 0)
    __hip_atomic_store(&S.ready, p + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  V keep0[4];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) keep0[tt] = x[0][tt];
#pragma unroll
  for (int i = 0; i + 1 < MAXT; ++i)
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) x[i][tt] = x[i + 1][tt];
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) x[MAXT - 1][tt] = keep0[tt];
}

// The sweep over the row blocks; leaves R and C (the top n rows of Q^T B) in
// t.R / t.C.
template <int P, int MAXT>
__device__ void sweep(const BatchTask& t, BlkLds<typename Prec<P>::W>& S) {
  using V = typename Prec<P>::V;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // in a scalar register
  const int n = t.n, N = n + t.nrhs;
  const int CT = (N + 15) >> 4, PT = (n + 15) >> 4;
  const int nblk = (t.m + H - 1) / H;
  const bool keep = (t.flags & kTaskKeep) != 0;
  V x[MAXT][4];
  for (int bk = 0; bk < nblk; ++bk) {
    const bool first = bk == 0;
    // Every wave has left the previous block's panels (and its waits on the
    // counters) before they are reset.
    __syncthreads();
    if (threadIdx.x == 0) {
      S.ready_y = -1;
      S.ready = -1;
#pragma unroll
      for (int k = 0; k < NW; ++k) S.done[k] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXT; ++i) {
      const int c = w + NW * i;
      if (c < CT) load_tile<P>(t, bk * H, c, x[i]);
    }
    int rot = 0;
    // Panels are ordered by LDS counters instead of a barrier per panel: a
    // wave waits for the panel it applies to be published (Y, then T), and a
    // panel's owner waits only until its LDS buffer is free.  The next
    // panel's owner therefore does not wait for this panel's owner to finish
    // its other tiles.
    for (int p = -1; p < PT; ++p) {
      if (p >= 0) wait_at_least(&S.ready_y, p, &S.err);  // Y of panel p published
      const int pn = p + 1;
      // Look-ahead: the owner of panel pn brings its tile up to date first
      // and factors it.
      if (pn < PT && w == (pn & 3)) {
        own_panel<P, MAXT>(t, p, bk, x, S);
        ++rot;
      }
      if (p >= 0) {
        bool wait_t = true;  // the first tile's update waits for T
#pragma unroll
        for (int i = 0; i < MAXT; ++i) {
          const int c = slot_tile<MAXT>(w, i, rot);
          if (c > p && c < CT && (c != pn || pn >= PT)) {
            update_tile<P>(t, p, c, first, x[i], S, wait_t);
            wait_t = false;
          }
        }
        if ((threadIdx.x & 63) == 0)
          __hip_atomic_store(&S.done[w], p + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    if (keep) {
      // Kept factors: the reflector tails of the block into A's rows.
      const int lane = lane_id(), q = lane >> 4, cl = lane & 15;
#pragma unroll
      for (int i = 0; i < MAXT; ++i) {
        const int col = 16 * slot_tile<MAXT>(w, i, rot) + cl;
        if (col < n) {
          gdouble* dst = gp(t.A + (int64_t)col * t.lda);
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = bk * H + 16 * tt + rho<P>(q, r);
              if (row < t.m) dst[row] = (double)x[i][tt][r];
            }
        }
      }
    }
  }
  __syncthreads();
}

// Sum over the workgroup of KK values per thread; every thread receives the
// same totals (butterfly sums within each wave, then the wave totals in
// order).
template <int KK>
__device__ __forceinline__ void wg_sum(double (&v)[KK], double (*red)[KG]) {
  static_assert(KK <= KG, "reduction width");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < KK; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < KK; ++k) red[w][k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KK; ++k) v[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
  __syncthreads();
}

// One step of a triangular solve by rows: the owner of row i divides by the
// diagonal entry and posts z_i; after the barrier every row `act` subtracts
// its entry times z_i.  a0 / a1: this thread's entries (rows l, l + NT) of
// the column (or row) of R that step i uses.
template <int KK>
__device__ __forceinline__ void solve_step(int i, double a0, double a1, bool act0, bool act1,
                                           double (&v)[2][KK], double (*zb)[8]) {
  const int l = threadIdx.x, s = i & 1;
  if (l == i)
#pragma unroll
    for (int k = 0; k < KK; ++k) {
      v[0][k] = v[0][k] / a0;
      zb[s][k] = v[0][k];
    }
  if (l + NT == i)
#pragma unroll
    for (int k = 0; k < KK; ++k) {
      v[1][k] = v[1][k] / a1;
      zb[s][k] = v[1][k];
    }
  __syncthreads();
  if (act0)
#pragma unroll
    for (int k = 0; k < KK; ++k) v[0][k] -= a0 * zb[s][k];
  if (act1)
#pragma unroll
    for (int k = 0; k < KK; ++k) v[1][k] -= a1 * zb[s][k];
}

constexpr int SB = 16;  // steps of a triangular solve whose entries of R load together

// R z = v in place by back substitution (R upper triangular, n x n in t.R);
// thread l holds rows l and l + NT of KK right-hand sides.  One barrier per
// row; the entries of R for SB columns are loaded in one go, so the steps do
// not wait on memory.
template <int KK>
__device__ void backsub(const BatchTask& t, double (&v)[2][KK], double (*zb)[8]) {
  const int l = threadIdx.x, n = t.n, l1 = l + NT;
  const gdouble* R = gp(t.R);
  for (int top = n - 1; top >= 0; top -= SB) {
    double c0[SB], c1[SB];  // R[l][top - u], R[l1][top - u]
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int col = top - u;
      c0[u] = (col >= 0 && l <= col) ? R[(int64_t)col * n + l] : 0.0;
      c1[u] = (col >= 0 && l1 <= col) ? R[(int64_t)col * n + l1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int i = top - u;
      if (i >= 0) solve_step<KK>(i, c0[u], c1[u], l < i, l1 < i, v, zb);
    }
  }
  __syncthreads();
}

// R^T z = v in place by forward substitution (row i of R enters step i;
// R^T is lower triangular).  Entries of SB rows of R load together.
template <int KK>
__device__ void fwdsub_t(const BatchTask& t, double (&v)[2][KK], double (*zb)[8]) {
  const int l = threadIdx.x, n = t.n, l1 = l + NT;
  const gdouble* R = gp(t.R);
  for (int i0 = 0; i0 < n; i0 += SB) {
    double c0[SB], c1[SB];  // R[i0 + u][l], R[i0 + u][l1]
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int i = i0 + u;
      c0[u] = (i < n && l >= i && l < n) ? R[(int64_t)l * n + i] : 0.0;
      c1[u] = (i < n && l1 >= i && l1 < n) ? R[(int64_t)l1 * n + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int i = i0 + u;
      if (i < n) solve_step<KK>(i, c0[u], c1[u], l > i && l < n, l1 > i && l1 < n, v, zb);
    }
  }
  __syncthreads();
}

// First zero diagonal entry of R, or INT_MAX.
__device__ int zero_diagonal(const BatchTask& t, int* sing) {
  if (threadIdx.x == 0) *sing = INT_MAX;
  __syncthreads();
  for (int row = threadIdx.x; row < t.n; row += NT)
    if (gp(t.R)[(int64_t)row * t.n + row] == 0.0) atomicMin(sing, row);
  __syncthreads();
  const int s = *sing;
  __syncthreads();
  return s;
}

// Rows l, l + NT of right-hand sides k0.. of an n x nrhs matrix (ld) into v.
template <int KK>
__device__ __forceinline__ void load_rows(const double* M, int64_t ld, int n, int k0, int kn,
                                          double (&v)[2][KK]) {
  const int l = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int k = 0; k < KK; ++k) {
      const int row = l + h * NT;
      v[h][k] = (row < n && k0 + k < kn) ? gp(M)[(int64_t)(k0 + k) * ld + row] : 0.0;
    }
}
template <int KK>
__device__ __forceinline__ void store_rows(double* M, int64_t ld, int n, int k0, int kn,
                                           const double (&v)[2][KK]) {
  const int l = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int k = 0; k < KK; ++k) {
      const int row = l + h * NT;
      if (row < n && k0 + k < kn) gp(M)[(int64_t)(k0 + k) * ld + row] = v[h][k];
    }
}

// FP64: back substitution R x = c[0:n]; x into B's top rows (and X).  If some
// R_jj == 0, B's top rows receive c and the status is j + 1.
__device__ int finish_f64(const BatchTask& t, BlkLds<double>& S) {
  const int sing = zero_diagonal(t, &S.sing);
  for (int k0 = 0; k0 < t.nrhs; k0 += KG) {
    double v[2][KG];
    load_rows<KG>(t.C, t.n, t.n, k0, t.nrhs, v);
    if (sing == INT_MAX) backsub<KG>(t, v, S.z);
    store_rows<KG>(t.B, t.ldb, t.n, k0, t.nrhs, v);
    if (t.X) store_rows<KG>(t.X, t.n, t.n, k0, t.nrhs, v);
  }
  return sing == INT_MAX ? 0 : sing + 1;
}

// v (rows l, l + NT) into the LDS vector, [row][rhs].
__device__ __forceinline__ void put_vector(const BatchTask& t, const double (&v)[2][KG], double* dst) {
  const int l = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int row = l + h * NT;
    if (row < t.n)
#pragma unroll
      for (int k = 0; k < KG; ++k) dst[row * KG + k] = v[h][k];
  }
}

// One pass over A in chunks of RC rows, v (n x KG) in S.v.  Thread (ri, g) =
// (l % RC, l / RC) forms row ri's partial sums of A v over the columns
// j = g mod (NT / RC), keeping the entries in LDS; the partials are summed
// over g.  RESID: the chunk's residual r = b - A v, then u += A^T r from the
// LDS copy (thread l: columns l and l + NT, the row layout of the solves),
// rr += ||r||^2 and a2 += ||A||_F^2; otherwise rr += ||A v||^2.
template <bool RESID>
__device__ void a_pass(const BatchTask& t, int k0, int kn, RefineLds& S, double (&rr)[KG],
                       double (&u)[2][KG], double& a2) {
  constexpr int G = NT / RC;                          // column groups
  constexpr int PJ = (kBatchMaxCols + G - 1) / G;     // columns per thread
  const int l = threadIdx.x, ri = l % RC, g = l / RC;
  const int m = t.m, n = t.n;
  const gdouble* A = gp(t.A);
  const gdouble* B = gp(t.B);
  // The next chunk's entries (and its right-hand sides) are loaded while
  // the current chunk is reduced (the barriers below order LDS only, so the
  // loads stay in flight).
  double pre[PJ];
  double bpre = 0.0;
  auto fetch = [&](int r0) {
    // The column group through an empty asm: the 20 column offsets are
    // formed here rather than hoisted out of the loop and held.
    int gg = g;
    asm volatile("" : "+v"(gg));
    const int i = r0 + ri;
    const gdouble* ai = A + (i < m ? i : 0) + (int64_t)gg * t.lda;
    const int64_t step = (int64_t)G * t.lda;
#pragma unroll
    for (int s = 0; s < PJ; ++s) pre[s] = (i < m && gg + G * s < n) ? ai[s * step] : 0.0;
    if (RESID && l < RC * KG) {
      // Row l % RC, right-hand side l / RC of the chunk.
      const int row = r0 + l % RC, k = l / RC;
      bpre = (row < m && k < kn) ? B[(int64_t)(k0 + k) * t.ldb + row] : 0.0;
    }
  };
  fetch(0);
  for (int r0 = 0; r0 < m; r0 += RC) {
    double acc[KG] = {};
#pragma unroll
    for (int s = 0; s < PJ; ++s) {
      const int j = g + G * s;
      if (j < n) {
        const double a = pre[s];
        if (RESID) {
          S.a[j * RCP + ri] = a;
          a2 += a * a;
        }
#pragma unroll
        for (int k = 0; k < KG; ++k) acc[k] += a * S.v[j * KG + k];
      }
    }
#pragma unroll
    for (int k = 0; k < KG; ++k) S.part[g][ri][k] = acc[k];
    const double bv = bpre;
    if (r0 + RC < m) fetch(r0 + RC);
    lds_barrier();
    if (l < RC * KG) {
      // Row l % RC, right-hand side l / RC: the partials in group order.
      const int rr_ = l % RC, k = l / RC;
      double sum = 0.0;
#pragma unroll
      for (int gg = 0; gg < G; ++gg) sum += S.part[gg][rr_][k];
      const int row = r0 + rr_;
      double v = sum;
      if (RESID) v = (row < m && k < kn) ? bv - sum : 0.0;
      S.rc[rr_][k] = v;
    }
    lds_barrier();
    if (l < RC) {
#pragma unroll
      for (int k = 0; k < KG; ++k) rr[k] += S.rc[l][k] * S.rc[l][k];
    }
    if (RESID) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int col = l + h * NT;
        if (col < n) {
#pragma unroll
          for (int q = 0; q < RC; ++q) {
            const double a = S.a[col * RCP + q];
#pragma unroll
            for (int k = 0; k < KG; ++k) u[h][k] += a * S.rc[q][k];
          }
        }
      }
    }
    lds_barrier();
  }
}

// FP64 refinement of right-hand sides k0 .. k0 + KG - 1 (see the file
// comment).  Returns the iterations used, or -1 if the target was not met.
// *anorm: ||A||_F, taken from the first residual pass when zero.
// rich: the first iteration is the plain step x += R^-1 R^-T A^T r (one
// pass over A fewer than a CGLS step; with R from an FP32 factorisation the
// singular values of A R^-1 are within about u_32 kappa(A) of one, so the
// step contracts the error by about that much); CGLS from the next
// iteration on.  Otherwise CGLS throughout.
__device__ int refine_group(const BatchTask& t, RefineLds& S, double* anorm, int k0, bool rich) {
  const int n = t.n;
  const int kn = min(KG, t.nrhs - k0);
  double xv[2][KG], pv[2][KG], sv[2][KG];
  load_rows<KG>(t.C, t.n, n, k0, t.nrhs, xv);
  backsub<KG>(t, xv, S.z);
  double gam[KG] = {};
  double h1 = 0.0, h2 = 0.0, h3 = 0.0, h4 = 0.0;  // worst of the last four iterations
  for (int it = 0;; ++it) {
    // r = b - A x and u = A^T r in one pass over A.
    put_vector(t, xv, S.v);
    __syncthreads();
    double rr[KG] = {};
    double a2[1] = {0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < KG; ++k) sv[h][k] = 0.0;
    a_pass<true>(t, k0, kn, S, rr, sv, a2[0]);
    if (*anorm == 0.0) {
      wg_sum<1>(a2, S.red);
      *anorm = sqrt(a2[0]);
    }
    double un[KG], xn[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      un[k] = sv[0][k] * sv[0][k] + sv[1][k] * sv[1][k];
      xn[k] = xv[0][k] * xv[0][k] + xv[1][k] * xv[1][k];
    }
    wg_sum<KG>(rr, S.red);
    wg_sum<KG>(un, S.red);
    wg_sum<KG>(xn, S.red);
    // beta with the quotients taken before any product (no product of norms
    // overflows); a non-finite norm (an overflowed sum of squares) gives NaN,
    // which never counts as converged and ends the refinement.
    double worst = 0.0;
    const double an = *anorm;
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      if (k < kn) {
        const double un_ = sqrt(un[k]), xn_ = sqrt(xn[k]), rn_ = sqrt(rr[k]);
        double be;
        if (!(isfinite(an) && isfinite(un_) && isfinite(xn_) && isfinite(rn_)))
          be = NAN;
        else if (an == 0.0)
          be = un_ == 0.0 ? 0.0 : NAN;
        else {
          const double den = xn_ + rn_ / an;
          be = den > 0.0 ? (un_ / an / an) / den : 0.0;
        }
        worst = (be > worst || be != be) ? be : worst;
      }
    }
    if (worst <= kRefineTol) {
      store_rows<KG>(t.B, t.ldb, n, k0, t.nrhs, xv);
      if (t.X) store_rows<KG>(t.X, t.n, n, k0, t.nrhs, xv);
      return it;
    }
    // Give up at the cap, or when four iterations have not halved the error.
    if (it >= kRefineMaxIt || !(worst == worst) || (it >= 4 && worst > 0.5 * h4)) return -1;
    h4 = h3;
    h3 = h2;
    h2 = h1;
    h1 = worst;
    // s = R^-T u; CGLS: p = s + (gamma' / gamma) p, t = R^-1 p; the plain
    // step: t = R^-1 s, x += t.
    fwdsub_t<KG>(t, sv, S.z);
    const bool plain = rich && it == 0;
    if (!plain) {
      const bool first = it == (rich ? 1 : 0);
      double g2[KG];
#pragma unroll
      for (int k = 0; k < KG; ++k) g2[k] = sv[0][k] * sv[0][k] + sv[1][k] * sv[1][k];
      wg_sum<KG>(g2, S.red);
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        const double be = (first || gam[k] == 0.0) ? 0.0 : g2[k] / gam[k];
#pragma unroll
        for (int h = 0; h < 2; ++h) pv[h][k] = sv[h][k] + be * (first ? 0.0 : pv[h][k]);
        gam[k] = g2[k];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < KG; ++k) sv[h][k] = pv[h][k];
    }
    backsub<KG>(t, sv, S.z);
    if (plain) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < KG; ++k) xv[h][k] += sv[h][k];
      continue;
    }
    // alpha = gamma / ||A t||^2, x += alpha t
    put_vector(t, sv, S.v);
    __syncthreads();
    double qq[KG] = {};
    double none[2][KG];
    double a2q = 0.0;
    a_pass<false>(t, k0, kn, S, qq, none, a2q);
    wg_sum<KG>(qq, S.red);
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const double al = qq[k] > 0.0 ? gam[k] / qq[k] : 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) xv[h][k] += al * sv[h][k];
    }
  }
}

// Copy R into A's upper triangle (kTaskWriteR).
__device__ void write_r(const BatchTask& t) {
  for (int c = 0; c < t.n; ++c)
    for (int j = threadIdx.x; j <= c; j += NT)
      gp(t.A)[j + (int64_t)c * t.lda] = gp(t.R)[j + (int64_t)c * t.n];
}

// Register budgets (waves per SIMD, hence workgroups per CU): 256 VGPRs for
// the FP64 tiles of three or five slots, 168 for two and for five FP32
// slots, 128 for two or three FP32 slots.
template <int P, int MAXT>
struct Budget {
  static constexpr int waves = P == kBlkF64 ? (MAXT >= 3 ? 2 : 3) : (MAXT >= 5 ? 3 : 4);
};

// The sweep of one queue's problems.  FP64 finishes each problem (status,
// X, R into A); the mixed precisions leave R and C for k_batched_refine.
template <int P, int MAXT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(Budget<P, MAXT>::waves)))
void k_batched_blk(const BatchHeader* table, int queue, int* counter, int* status) {
  using W = typename Prec<P>::W;
  __shared__ __align__(16) BlkLds<W> S;
  const int total = __builtin_amdgcn_readfirstlane(table->count[queue]);
  const int base = __builtin_amdgcn_readfirstlane(table->begin[queue]);
  const BatchTask* tasks = (const BatchTask*)(table + 1) + base;
  for (;;) {
    if (threadIdx.x == 0) S.idx = atomicAdd(counter + queue, 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(S.idx);
    __syncthreads();
    if (idx >= total) break;
    const BatchTask t = tasks[idx];
    if (threadIdx.x == 0) S.err = 0;
    sweep<P, MAXT>(t, S);
    const bool err = S.err != 0;
    if constexpr (P == kBlkF64) {
      const int st = err ? kStatusFault : finish_f64(t, S);
      if (st == 0 && (t.flags & kTaskWriteR)) write_r(t);
      if (threadIdx.x == 0) status[t.slot] = st;
    } else {
      // The refinement treats a zero diagonal as a failed low-precision
      // factorisation and leaves the problem to the FP64 pass.
      if (err && threadIdx.x == 0) gp(t.R)[0] = 0.0;
    }
    __syncthreads();
  }
}

// FP64 refinement of the mixed-precision solves of queues 1 .. 3 (one
// problem per workgroup, popped from queue counter kBatchQueues).
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_batched_refine(const BatchHeader* table, int* counter, int* status, int* iters, int prec) {
  __shared__ __align__(16) RefineLds S;
  int total = 0;
  for (int k = 1; k < kBatchQueues; ++k) total += table->count[k];
  total = __builtin_amdgcn_readfirstlane(total);
  const int base = __builtin_amdgcn_readfirstlane(table->begin[1]);
  const BatchTask* tasks = (const BatchTask*)(table + 1) + base;
  for (;;) {
    if (threadIdx.x == 0) S.idx = atomicAdd(counter + kBatchQueues, 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(S.idx);
    __syncthreads();
    if (idx >= total) break;
    const BatchTask t = tasks[idx];
    double anorm = 0.0;  // ||A||_F, from the first pass over A
    int st = zero_diagonal(t, &S.sing) == INT_MAX ? 0 : kStatusNoConv;
    int most = 0;
    for (int k0 = 0; st == 0 && k0 < t.nrhs; k0 += KG) {
      const int it = refine_group(t, S, &anorm, k0, prec == kBlkF32);
      if (it < 0)
        st = kStatusNoConv;
      else
        most = max(most, it);
    }
    if (st == 0 && (t.flags & kTaskWriteR)) write_r(t);
    if (threadIdx.x == 0) {
      status[t.slot] = st;
      if (iters) iters[t.slot] = st == 0 ? most : -1;
    }
    __syncthreads();
  }
}

constexpr int kTiles[kBatchQueues] = {0, 2, 3, 5};

template <int P>
const void* blk_kernel(int queue) {
  switch (queue) {
    case 1:
      return (const void*)k_batched_blk<P, 2>;
    case 2:
      return (const void*)k_batched_blk<P, 3>;
    default:
      return (const void*)k_batched_blk<P, 5>;
  }
}

const void* blk_kernel(int prec, int queue) {
  if (prec == kBlkF32) return blk_kernel<kBlkF32>(queue);
  if (prec == kBlkBF16) return blk_kernel<kBlkBF16>(queue);
  return blk_kernel<kBlkF64>(queue);
}

int occupancy_grid(int device, const void* k) {
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    cus = 256;
  int per = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, NT, 0) != hipSuccess || per < 1) per = 1;
  return cus * per;
}

}  // namespace

int batch_queue(const BatchTask& t) {
  if (t.flags & kTaskApply) return 0;
  const int tiles = (t.n + t.nrhs + 15) / 16;
  for (int k = 1; k < kBatchQueues; ++k)
    if (tiles <= NW * kTiles[k]) return k;
  return kBatchQueues - 1;
}

int batched_blk_grid(int device, int prec, int queue) {
  return occupancy_grid(device, queue == kBatchQueues ? (const void*)k_batched_refine
                                                      : blk_kernel(prec, queue));
}

void batched_blk_launch(hipStream_t s, const BatchHeader* table, int queue, int* counter,
                        int* status, int* iters, int grid, int prec) {
  if (grid <= 0) return;
  if (queue == kBatchQueues) {
    hipLaunchKernelGGL(k_batched_refine, dim3(grid), dim3(NT), 0, s, table, counter, status, iters,
                       prec);
    return;
  }
  const void* k = blk_kernel(prec, queue);
  void* args[] = {(void*)&table, (void*)&queue, (void*)&counter, (void*)&status};
  (void)hipLaunchKernel(k, dim3(grid), dim3(NT), args, 0, s);
}

}  // namespace miqr
