// Dense GEMMs of the EG recursion (Alg. 2's six products) and of apply_q.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miqr {

// Structure of a stored operand, applied to its stored (row, col) indices:
// UNIT_LOWER reads 0 above and 1 on the diagonal (a Householder basis V),
// UPPER reads 0 below the diagonal (a kernel T or an R factor).
enum Mask : int { MASK_NONE = 0, MASK_UNIT_LOWER = 1, MASK_UPPER = 2 };

// Arithmetic of the MFMA products.  FP64 inputs are rounded to the compute
// type while they are staged (round to nearest even); accumulation is FP64
// for FP64 and FP32 otherwise.
enum Compute : int { COMPUTE_F64 = 0, COMPUTE_F32 = 1, COMPUTE_BF16 = 2 };

struct GemmDesc {
  char ta = 'N', tb = 'N';
  int64_t M = 0, N = 0, K = 0;
  double alpha = 1.0, beta = 0.0;
  const double* A = nullptr;
  int64_t lda = 0;
  int maskA = MASK_NONE;
  const double* B = nullptr;
  int64_t ldb = 0;
  int maskB = MASK_NONE;
  double* C = nullptr;
  int64_t ldc = 0;
  int compute = COMPUTE_F64;
  int add_identity = 0;  // C(i, i) += 1 after the product (with beta == 0: C = alpha AB + I)
};

// C = alpha op(A) op(B) + beta C (beta == 0: C is not read).  `scratch` holds
// split-K partial sums (scratch_doubles of capacity; 0 disables split-K).
// Adds the launched multiply-add count to *flops (if non-null).
hipError_t gemm(const GemmDesc& d, hipStream_t s, double* scratch, int64_t scratch_doubles,
                double* flops = nullptr);

}  // namespace miqr
