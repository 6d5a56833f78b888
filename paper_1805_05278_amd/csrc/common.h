// Shared device helpers and workspace constants for the miqr HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miqr {

// Panel (TSQR) width limit and workspace strides.  Every small square matrix
// of a TSQR tree (T, Y of a tree step, R) is stored column-major with leading
// dimension kNB in a slot of kTS doubles; a downsweep block B (nb x nq with nq
// up to 2 nb) takes kBS doubles.
constexpr int kNB = 64;
constexpr int kTS = kNB * kNB;
constexpr int kBS = kNB * 2 * kNB;
constexpr int kMaxLevels = 40;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP64 MFMA 16x16x4.  Operand layout (wave64, lane l):
//   a = A[l % 16][l / 16]   (A is 16 x 4)
//   b = B[l / 16][l % 16]   (B is 4 x 16)
//   acc[r] = D[l / 16 + 4 r][l % 16]
__device__ __forceinline__ d4 mfma64(double a, double b, d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

__device__ __forceinline__ double quad_sum(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace miqr
