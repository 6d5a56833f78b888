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
// A TSQR tree node stacks the R factors of its children (after the first)
// into at most kYL rows; its basis Y takes kYS doubles (leading dim kYL).
constexpr int kYL = 256;
constexpr int kYS = kYL * kNB;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP64 MFMA 16x16x4.  Operand layout (wave64, lane l):
//   a = A[l % 16][l / 16]   (A is 16 x 4)
//   b = B[l / 16][l % 16]   (B is 4 x 16)
//   acc[r] = D[l / 16 + 4 r][l % 16]
__device__ __forceinline__ d4 mfma64(double a, double b, d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// Cross-lane moves through DPP (no LDS round trip).  A double moves as two
// 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  int lo = (int)(unsigned)(b & 0xffffffffull), hi = (int)(unsigned)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}

// Sum over the 4 lanes of a quad (quad_perm [1,0,3,2] then [2,3,0,1]); every
// lane of the quad receives the total.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  return v;
}

// Sum over 8 consecutive lanes (quad sums, then row_half_mirror pairs the two
// quads of each half-row).
__device__ __forceinline__ double oct_sum(double v) {
  v = quad_sum(v);
  v += dpp_mov<0x141>(v);
  return v;
}

// Householder reflector of a column (alpha; x) with ||x||^2 = ss > 0 (the
// dlarfg sign rule): beta = -sign(alpha) ||(alpha; x)||,
// tau = (beta - alpha) / beta = 1 + |alpha| / ||(alpha; x)|| and
// scale = 1 / (alpha - beta), the factor that turns x into the reflector's
// tail.  1 / ||.|| and 1 / (alpha - beta) come from the hardware reciprocal
// square root and reciprocal with two Newton steps each: within a few ulps of
// the correctly rounded values, on a much shorter dependent chain than a
// correctly rounded sqrt and division.  The hardware reciprocal square root
// is accurate to about 2^-26 over the whole range, subnormal inputs included
// (measured on gfx950), and every intermediate stays in range
// (|alpha - beta| >= ||.|| >= 2^-538), so no scaling is needed.
__device__ __forceinline__ void reflector(double alpha, double ss, double& beta, double& tau,
                                          double& scale) {
  const double s2 = fma(alpha, alpha, ss);
  double y = __builtin_amdgcn_rsq(s2);
  y = fma(0.5 * y, fma(-(s2 * y), y, 1.0), y);
  y = fma(0.5 * y, fma(-(s2 * y), y, 1.0), y);  // 1 / ||(alpha; x)||
  const double nrm = s2 * y;
  beta = alpha >= 0.0 ? -nrm : nrm;
  const double dd = alpha - beta;
  double z = __builtin_amdgcn_rcp(dd);
  z = fma(z, fma(-dd, z, 1.0), z);
  z = fma(z, fma(-dd, z, 1.0), z);
  scale = z;
  tau = fma(fabs(alpha), y, 1.0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace miqr
