// MFMA GEMMs for gfx950: the six products of each EG recursion node (Alg. 2:
// M1 = V_L^T C, M2 = T_L^T M1, C -= V_L M2, M3 = V_L^T [0; V_R], M4 = M3 T_R,
// T12 = -T_L M4) and the compact-WY application of Q.
//
// One workgroup (4 waves, 2 x 2) computes a BM x BN tile of C; each wave a
// (BM/2) x (BN/2) block of 16 x 16 MFMA tiles.  Operands are staged through
// LDS in BK = 16 deep slices, k-major, with the next slice prefetched into
// registers while the current one is multiplied.  The MFMA computes C^T tiles
// (A' = op(B)^T, B' = op(A)^T) so that the lane-fast output index runs down a
// column of the column-major C and stores coalesce.
//
// Structure masks turn the stored unit lower trapezoidal V (R above its
// diagonal) and the upper triangular T into their mathematical values while
// they are loaded, so the factors never have to be copied out of A.
//
// Split-K (the paper's 1DMM with the K dimension distributed, Sec. 4 and
// Sec. 6.2) is used when the output has few tiles: each slice of K writes a
// partial product and a second kernel adds the partials in a fixed order, so
// results are bitwise reproducible.
#include <algorithm>

#include "common.h"
#include "gemm.h"
#include "profiler.h"

namespace miqr {

struct GemmArgs {
  int64_t M, N, K, kchunk;
  double alpha, beta;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double* P;  // split-K partials (M x N each) or null
  int maskA, maskB;
  int add_identity;
};

// Tile of this workgroup.  Workgroups are dealt to the 8 XCDs in turn (id
// mod 8), and each XCD has its own L2; the linear id is remapped so that XCD
// k runs a contiguous range of the tile order.  The order walks groups of
// kGroup row tiles across all column tiles (column by column inside a group),
// split by split: the workgroups an XCD runs together share a few row panels
// of the left operand and column panels of the right one (or one split-K
// slice of V) in its L2, instead of every XCD fetching every panel.  Any
// bijection gives the same results: only the placement of the tiles changes.
struct TileId {
  int64_t x, y, z;
  __device__ TileId() {
    constexpr int64_t kXcd = 8, kGroup = 8;
    const int64_t gx = gridDim.x, gy = gridDim.y;
    const int64_t nb = gx * gy * gridDim.z;
    const int64_t id = blockIdx.x + gx * (blockIdx.y + gy * (int64_t)blockIdx.z);
    const int64_t q = nb / kXcd, r = nb % kXcd, k = id % kXcd, j = id / kXcd;
    const int64_t lid = k * q + min(k, r) + j;
    const int64_t per = gx * gy, t = lid % per;
    z = lid / per;
    const int64_t g = t / (kGroup * gy), x0 = g * kGroup, gs = min(gx - x0, kGroup);
    const int64_t u = t - g * kGroup * gy;
    x = x0 + u % gs;
    y = u / gs;
  }
};

template <int CMP>
struct MfmaTraits;

template <>
struct MfmaTraits<COMPUTE_F64> {
  typedef double T;
  typedef d4 Acc;
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};

template <>
struct MfmaTraits<COMPUTE_F32> {
  typedef float T;
  typedef f4 Acc;
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// Per-thread global->register staging of one BK-deep slice of op(A) (BM x BK)
// or op(B)^T (BN x BK).  Element (i, k) of the slice is stored at
// (i, k) -> p[i + k ld] when the operand runs along i (not transposed A,
// transposed B) and at p[k + i ld] otherwise.  Each thread owns a fixed
// (i, k) pattern and a pointer advanced by a constant per slice, so the hot
// loop does no 64-bit multiplies.
template <int BX, int BK, bool ALONG_I>
struct SliceLoader {
  static constexpr int L = BX * BK / 256;  // elements per thread
  const double* p;                         // this thread's first element
  int64_t step;                            // pointer advance per slice
  int64_t estride;                         // distance between a thread's elements
  int i, k;                                // position of the first element
  int di, dk;                              // position delta between elements
  __device__ void init(const double* base, int64_t ld, int64_t x0, int64_t kbeg, int t) {
    if (ALONG_I) {
      i = t % BX;
      k = t / BX;
      di = 0;
      dk = 256 / BX;
      p = base + (x0 + i) + (kbeg + k) * ld;
      estride = (int64_t)dk * ld;
      step = (int64_t)BK * ld;
    } else {
      k = t % BK;
      i = t / BK;
      di = 256 / BK;
      dk = 0;
      p = base + (kbeg + k) + (x0 + i) * ld;
      estride = (int64_t)di * ld;
      step = BK;
    }
  }
  // Issue the slice's loads.  Elements out of range read `safe` (a valid
  // address) instead; store() zeroes them and applies the structure mask.
  // No branch selects between loaded values here, so the loads stay in
  // flight across the MFMAs of the current slice.
  __device__ void load(double (&r)[L], bool plain, const double* safe, int64_t x0, int64_t X,
                       int64_t k0, int64_t kend) const {
#pragma unroll
    for (int s = 0; s < L; ++s) {
      const int64_t x = x0 + i + s * di, kk = k0 + k + s * dk;
      const bool ok = plain || (x < X && kk < kend);
      r[s] = *(ok ? p + s * estride : safe);
    }
  }
  // Store a loaded slice: out-of-range elements become 0, the structure
  // mask is applied on the stored (row, col) = along_i ? (x, kk) : (kk, x).
  template <typename T, int LD, bool TRANS>
  __device__ void store_masked(T (*S)[LD], const double (&r)[L], bool plain, int64_t x0, int64_t X,
                               int64_t k0, int64_t kend, int mask) const {
#pragma unroll
    for (int s = 0; s < L; ++s) {
      double v = r[s];
      if (!plain) {
        const int64_t x = x0 + i + s * di, kk = k0 + k + s * dk;
        const int64_t row = ALONG_I ? x : kk, col = ALONG_I ? kk : x;
        if (mask == MASK_UNIT_LOWER) v = (row < col) ? 0.0 : ((row == col) ? 1.0 : v);
        else if (mask == MASK_UPPER) v = (row > col) ? 0.0 : v;
        v = (x < X && kk < kend) ? v : 0.0;  // after the mask: no unit diagonal outside
      }
      if (TRANS) S[i + s * di][k + s * dk] = (T)v;
      else S[k + s * dk][i + s * di] = (T)v;
    }
  }
  // Loads and stores of a slice known to be plain (in range, mask-free).
  __device__ void load_plain(double (&r)[L]) const {
#pragma unroll
    for (int s = 0; s < L; ++s) r[s] = p[s * estride];
  }
  template <typename T, int LD, bool TRANS>
  __device__ void store_plain(T (*S)[LD], const double (&r)[L]) const {
#pragma unroll
    for (int s = 0; s < L; ++s) {
      if (TRANS) S[i + s * di][k + s * dk] = (T)r[s];
      else S[k + s * dk][i + s * di] = (T)r[s];
    }
  }
  __device__ void advance() { p += step; }
};

// Whether every element of a slice (rows x0 .. x0+BX-1 of op, k0 .. k0+BK-1)
// is in range and unaffected by the structure mask.
template <int BX, int BK, bool ALONG_I>
__host__ __device__ __forceinline__ bool slice_is_plain(int64_t x0, int64_t X, int64_t k0,
                                                        int64_t kend, int mask) {
  if (x0 + BX > X || k0 + BK > kend) return false;
  // stored row/col ranges
  const int64_t r0 = ALONG_I ? x0 : k0, r1 = ALONG_I ? x0 + BX - 1 : k0 + BK - 1;
  const int64_t c0 = ALONG_I ? k0 : x0, c1 = ALONG_I ? k0 + BK - 1 : x0 + BX - 1;
  if (mask == MASK_UNIT_LOWER) return r0 > c1;  // strictly below the diagonal
  if (mask == MASK_UPPER) return r1 <= c0;      // on or above the diagonal
  (void)r1; (void)c0;
  return true;
}

// The slabs s (k0 = kbeg + s BK) for which slice_is_plain holds form an
// interval: the masks cut a half-plane in (row, col), so the plain slabs of
// one operand are a prefix or a suffix of the full slabs.  Narrows [*lo, *hi)
// to that interval.
template <int BX, int BK, bool ALONG_I>
__host__ __device__ __forceinline__ void plain_slab_range(int64_t x0, int64_t X, int64_t kbeg,
                                                          int64_t kend, int mask, int* lo,
                                                          int* hi) {
  const int64_t nfull = (kend - kbeg) / BK;  // slabs wholly inside [kbeg, kend)
  int64_t l = *lo, h = min((int64_t)*hi, nfull);
  if (x0 + BX > X) h = 0;
  // first slab index with kbeg + s BK >= need, last with kbeg + s BK <= lim
  auto from = [&](int64_t need) {
    need -= kbeg;
    l = max(l, need <= 0 ? (int64_t)0 : (need + BK - 1) / BK);
  };
  auto upto = [&](int64_t lim) {
    lim -= kbeg;
    h = min(h, lim < 0 ? (int64_t)0 : lim / BK + 1);
  };
  if (mask == MASK_UNIT_LOWER) {
    if (ALONG_I) upto(x0 - BK);  // stored (x, kk): plain iff x0 > k0 + BK - 1
    else from(x0 + BX);          // stored (kk, x): plain iff k0 > x0 + BX - 1
  } else if (mask == MASK_UPPER) {
    if (ALONG_I) from(x0 + BX - 1);  // plain iff x0 + BX - 1 <= k0
    else upto(x0 - BK + 1);          // plain iff k0 + BK - 1 <= x0
  }
  if (l > h) l = h;
  *lo = (int)l;
  *hi = (int)h;
}

template <int BM, int BN, bool TA, bool TB, int CMP>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  typedef MfmaTraits<CMP> Tr;
  typedef typename Tr::T T;
  typedef typename Tr::Acc Acc;
  constexpr int BK = 16;
  constexpr int PAD = 1;
  constexpr int WM = BM / 2, WN = BN / 2, SA = WM / 16, SB = WN / 16;
  // op(A) runs along i in memory when A is not transposed; op(B)^T (N x K)
  // runs along j when B is transposed.
  constexpr bool A_ALONG = !TA, B_ALONG = TB;
  typedef SliceLoader<BM, BK, A_ALONG> LA_t;
  typedef SliceLoader<BN, BK, B_ALONG> LB_t;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = l >> 4;
  const int wm = w & 1, wn = w >> 1;
  const TileId tid;
  const int64_t i0 = tid.x * BM, j0 = tid.y * BN;
  const int64_t kbeg = tid.z * g.kchunk;
  const int64_t kend = min(g.K, kbeg + g.kchunk);
  const int nslab = (int)((kend - kbeg + BK - 1) / BK);

  Acc acc[SA][SB];
#pragma unroll
  for (int a = 0; a < SA; ++a)
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;

  LA_t la;
  LB_t lb;
  la.init(g.A, g.lda, i0, kbeg, t);
  lb.init(g.B, g.ldb, j0, kbeg, t);
  double ra[LA_t::L], rb[LB_t::L];
  int64_t kf = kbeg;  // first k of the slice held in ra / rb
  bool pa = true, pb = true;
  auto fetch = [&](int64_t k0) {
    kf = k0;
    pa = slice_is_plain<BM, BK, A_ALONG>(i0, g.M, k0, kend, g.maskA);
    pb = slice_is_plain<BN, BK, B_ALONG>(j0, g.N, k0, kend, g.maskB);
    la.load(ra, pa, g.A, i0, g.M, k0, kend);
    lb.load(rb, pb, g.B, j0, g.N, k0, kend);
    la.advance();
    lb.advance();
  };

  // Slabs [s1, s2) are plain for both operands: they are loaded and staged
  // without per-element range and mask selects.  The others (a prefix and a
  // suffix: the slabs that meet a structure mask, the ragged last slab, and
  // every slab of a tile that crosses the matrix edge) take the checked
  // path.  Each loop below prefetches the slab after the current one with the
  // path that slab needs, so no loaded value is merged across paths.
  int s1 = 0, s2 = nslab;
  plain_slab_range<BM, BK, A_ALONG>(i0, g.M, kbeg, kend, g.maskA, &s1, &s2);
  plain_slab_range<BN, BK, B_ALONG>(j0, g.N, kbeg, kend, g.maskB, &s1, &s2);
  if (nslab > 0) {
    if (s1 == 0 && s2 > 0) {
      la.load_plain(ra);
      lb.load_plain(rb);
      la.advance();
      lb.advance();
      la.template store_plain<T, BM + PAD, false>(As[0], ra);
      lb.template store_plain<T, BN + PAD, false>(Bs[0], rb);
    } else {
      fetch(kbeg);
      la.template store_masked<T, BM + PAD, false>(As[0], ra, pa, i0, g.M, kf, kend, g.maskA);
      lb.template store_masked<T, BN + PAD, false>(Bs[0], rb, pb, j0, g.N, kf, kend, g.maskB);
    }
  }
  __syncthreads();
  auto compute = [&](int cur) {
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      T af[SA], bf[SB];
#pragma unroll
      for (int a = 0; a < SA; ++a) af[a] = As[cur][4 * ks + lk][wm * WM + 16 * a + li];
#pragma unroll
      for (int b = 0; b < SB; ++b) bf[b] = Bs[cur][4 * ks + lk][wn * WN + 16 * b + li];
#pragma unroll
      for (int a = 0; a < SA; ++a)
#pragma unroll
        for (int b = 0; b < SB; ++b) acc[a][b] = Tr::mma(bf[b], af[a], acc[a][b]);
    }
  };
  int it = 0;
  // Next slab before s1: checked.
  for (; it + 1 < s1 && it < nslab; ++it) {
    const int cur = it & 1;
    fetch(kbeg + (int64_t)(it + 1) * BK);
    compute(cur);
    la.template store_masked<T, BM + PAD, false>(As[cur ^ 1], ra, pa, i0, g.M, kf, kend, g.maskA);
    lb.template store_masked<T, BN + PAD, false>(Bs[cur ^ 1], rb, pb, j0, g.N, kf, kend, g.maskB);
    __syncthreads();
  }
  // Next slab in [s1, s2): plain.
  for (; it + 1 < s2; ++it) {
    const int cur = it & 1;
    la.load_plain(ra);
    lb.load_plain(rb);
    la.advance();
    lb.advance();
    compute(cur);
    la.template store_plain<T, BM + PAD, false>(As[cur ^ 1], ra);
    lb.template store_plain<T, BN + PAD, false>(Bs[cur ^ 1], rb);
    __syncthreads();
  }
  // Next slab at or after s2 (or none): checked.
  for (; it < nslab; ++it) {
    const int cur = it & 1;
    const bool more = it + 1 < nslab;
    if (more) fetch(kbeg + (int64_t)(it + 1) * BK);
    compute(cur);
    if (more) {
      la.template store_masked<T, BM + PAD, false>(As[cur ^ 1], ra, pa, i0, g.M, kf, kend, g.maskA);
      lb.template store_masked<T, BN + PAD, false>(Bs[cur ^ 1], rb, pb, j0, g.N, kf, kend, g.maskB);
    }
    __syncthreads();
  }

  // Epilogue, one 16-row slice at a time.  The C values of slice a + 1 are
  // loaded before slice a is stored, so each slice's loads are in flight
  // while the previous slice is written (the read latency of C is otherwise
  // exposed once per slice).
  double cv[SB][4];
  auto load_c = [&](int a) {
    const int64_t i = i0 + wm * WM + 16 * a + li;
    const bool row_ok = i < g.M;
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + wn * WN + 16 * b + Tr::row(lk, r);
        cv[b][r] = (row_ok && j < g.N && !g.P && g.beta != 0.0)
                       ? g.C[i + j * g.ldc] : 0.0;
      }
  };
  load_c(0);
#pragma unroll
  for (int a = 0; a < SA; ++a) {
    const int64_t i = i0 + wm * WM + 16 * a + li;
    const bool row_ok = i < g.M;
    double out[SB][4];
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + wn * WN + 16 * b + Tr::row(lk, r);
        const double v = g.alpha * (double)acc[a][b][r];
        out[b][r] = g.P ? v : v + g.beta * cv[b][r] + ((g.add_identity && i == j) ? 1.0 : 0.0);
      }
    if (a + 1 < SA) load_c(a + 1);
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + wn * WN + 16 * b + Tr::row(lk, r);
        if (!row_ok || j >= g.N) continue;
        if (g.P) g.P[tid.z * g.M * g.N + i + j * g.M] = out[b][r];
        else g.C[i + j * g.ldc] = out[b][r];
      }
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// BF16 inputs (FP64 operands rounded when staged), FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  One MFMA k-step per 32-deep slice; tiles are
// stored i-major so that a lane's fragment (8 consecutive k) is one 16-byte
// LDS read.  Fragment layout: a = A[l % 16][8 (l / 16) + e],
// b = B[8 (l / 16) + e][l % 16], acc[r] = D[4 (l / 16) + r][l % 16].
template <int BM, int BN, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  constexpr int BK = 32, KP = BK + 8;
  constexpr int WM = BM / 2, WN = BN / 2, SA = WM / 16, SB = WN / 16;
  constexpr bool A_ALONG = !TA, B_ALONG = TB;
  typedef SliceLoader<BM, BK, A_ALONG> LA_t;
  typedef SliceLoader<BN, BK, B_ALONG> LB_t;
  __shared__ __align__(16) __bf16 As[2][BM][KP];
  __shared__ __align__(16) __bf16 Bs[2][BN][KP];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = l >> 4;
  const int wm = w & 1, wn = w >> 1;
  const TileId tid;
  const int64_t i0 = tid.x * BM, j0 = tid.y * BN;
  const int64_t kbeg = tid.z * g.kchunk;
  const int64_t kend = min(g.K, kbeg + g.kchunk);
  const int nslab = (int)((kend - kbeg + BK - 1) / BK);
  f4 acc[SA][SB];
#pragma unroll
  for (int a = 0; a < SA; ++a)
#pragma unroll
    for (int b = 0; b < SB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  LA_t la;
  LB_t lb;
  la.init(g.A, g.lda, i0, kbeg, t);
  lb.init(g.B, g.ldb, j0, kbeg, t);
  double ra[LA_t::L], rb[LB_t::L];
  int64_t kf = kbeg;  // first k of the slice held in ra / rb
  bool pa = true, pb = true;
  auto fetch = [&](int64_t k0) {
    kf = k0;
    pa = slice_is_plain<BM, BK, A_ALONG>(i0, g.M, k0, kend, g.maskA);
    pb = slice_is_plain<BN, BK, B_ALONG>(j0, g.N, k0, kend, g.maskB);
    la.load(ra, pa, g.A, i0, g.M, k0, kend);
    lb.load(rb, pb, g.B, j0, g.N, k0, kend);
    la.advance();
    lb.advance();
  };
  // Plain slabs [s1, s2) skip the per-element selects, as in k_gemm.
  int s1 = 0, s2 = nslab;
  plain_slab_range<BM, BK, A_ALONG>(i0, g.M, kbeg, kend, g.maskA, &s1, &s2);
  plain_slab_range<BN, BK, B_ALONG>(j0, g.N, kbeg, kend, g.maskB, &s1, &s2);
  if (nslab > 0) {
    if (s1 == 0 && s2 > 0) {
      la.load_plain(ra);
      lb.load_plain(rb);
      la.advance();
      lb.advance();
      la.template store_plain<__bf16, KP, true>(As[0], ra);
      lb.template store_plain<__bf16, KP, true>(Bs[0], rb);
    } else {
      fetch(kbeg);
      la.template store_masked<__bf16, KP, true>(As[0], ra, pa, i0, g.M, kf, kend, g.maskA);
      lb.template store_masked<__bf16, KP, true>(Bs[0], rb, pb, j0, g.N, kf, kend, g.maskB);
    }
  }
  __syncthreads();
  auto compute = [&](int cur) {
    bf16x8 af[SA], bf[SB];
#pragma unroll
    for (int a = 0; a < SA; ++a) af[a] = *(const bf16x8*)&As[cur][wm * WM + 16 * a + li][8 * lk];
#pragma unroll
    for (int b = 0; b < SB; ++b) bf[b] = *(const bf16x8*)&Bs[cur][wn * WN + 16 * b + li][8 * lk];
#pragma unroll
    for (int a = 0; a < SA; ++a)
#pragma unroll
      for (int b = 0; b < SB; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[b], af[a], acc[a][b], 0, 0, 0);
  };
  int it = 0;
  for (; it + 1 < s1 && it < nslab; ++it) {
    const int cur = it & 1;
    fetch(kbeg + (int64_t)(it + 1) * BK);
    compute(cur);
    la.template store_masked<__bf16, KP, true>(As[cur ^ 1], ra, pa, i0, g.M, kf, kend, g.maskA);
    lb.template store_masked<__bf16, KP, true>(Bs[cur ^ 1], rb, pb, j0, g.N, kf, kend, g.maskB);
    __syncthreads();
  }
  for (; it + 1 < s2; ++it) {
    const int cur = it & 1;
    la.load_plain(ra);
    lb.load_plain(rb);
    la.advance();
    lb.advance();
    compute(cur);
    la.template store_plain<__bf16, KP, true>(As[cur ^ 1], ra);
    lb.template store_plain<__bf16, KP, true>(Bs[cur ^ 1], rb);
    __syncthreads();
  }
  for (; it < nslab; ++it) {
    const int cur = it & 1;
    const bool more = it + 1 < nslab;
    if (more) fetch(kbeg + (int64_t)(it + 1) * BK);
    compute(cur);
    if (more) {
      la.template store_masked<__bf16, KP, true>(As[cur ^ 1], ra, pa, i0, g.M, kf, kend, g.maskA);
      lb.template store_masked<__bf16, KP, true>(Bs[cur ^ 1], rb, pb, j0, g.N, kf, kend, g.maskB);
    }
    __syncthreads();
  }
  // Epilogue as in k_gemm: slice a + 1 of C is loaded before slice a is stored.
  double cv[SB][4];
  auto load_c = [&](int a) {
    const int64_t i = i0 + wm * WM + 16 * a + li;
    const bool row_ok = i < g.M;
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + wn * WN + 16 * b + 4 * lk + r;
        cv[b][r] = (row_ok && j < g.N && !g.P && g.beta != 0.0)
                       ? g.C[i + j * g.ldc] : 0.0;
      }
  };
  load_c(0);
#pragma unroll
  for (int a = 0; a < SA; ++a) {
    const int64_t i = i0 + wm * WM + 16 * a + li;
    const bool row_ok = i < g.M;
    double out[SB][4];
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + wn * WN + 16 * b + 4 * lk + r;
        const double v = g.alpha * (double)acc[a][b][r];
        out[b][r] = g.P ? v : v + g.beta * cv[b][r] + ((g.add_identity && i == j) ? 1.0 : 0.0);
      }
    if (a + 1 < SA) load_c(a + 1);
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + wn * WN + 16 * b + 4 * lk + r;
        if (!row_ok || j >= g.N) continue;
        if (g.P) g.P[tid.z * g.M * g.N + i + j * g.M] = out[b][r];
        else g.C[i + j * g.ldc] = out[b][r];
      }
  }
}

// C = sum_z P[z] (+ beta C).  A block covers 64 consecutive elements with 4
// groups of splits: group g sums partials g, g + 4, g + 8, ... in order, and
// the four group sums are added in a fixed order, so the result does not
// depend on scheduling.
__global__ __launch_bounds__(256) void k_splitk_reduce(const double* P, int nsplit, int64_t M,
                                                       int64_t N, double beta, double* C,
                                                       int64_t ldc, int add_identity) {
  __shared__ double part[4][64];
  const int64_t MN = M * N;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  double s0 = 0.0, s1 = 0.0;
  if (e < MN) {
    int z = g;
    for (; z + 4 < nsplit; z += 8) {
      s0 += P[(int64_t)z * MN + e];
      s1 += P[(int64_t)(z + 4) * MN + e];
    }
    if (z < nsplit) s0 += P[(int64_t)z * MN + e];
  }
  part[g][lane] = s0 + s1;
  __syncthreads();
  if (g == 0 && e < MN) {
    const double s = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    const int64_t i = e % M, j = e / M;
    double* cp = C + i + j * ldc;
    *cp = ((beta == 0.0) ? s : s + beta * *cp) + ((add_identity && i == j) ? 1.0 : 0.0);
  }
}

template <int BM, int BN, int CMP>
static void launch_t(const GemmDesc& d, const GemmArgs& g, dim3 grid, hipStream_t s) {
  if (d.ta == 'N' && d.tb == 'N')
    hipLaunchKernelGGL((k_gemm<BM, BN, false, false, CMP>), grid, dim3(256), 0, s, g);
  else if (d.ta == 'T' && d.tb == 'N')
    hipLaunchKernelGGL((k_gemm<BM, BN, true, false, CMP>), grid, dim3(256), 0, s, g);
  else if (d.ta == 'N' && d.tb == 'T')
    hipLaunchKernelGGL((k_gemm<BM, BN, false, true, CMP>), grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((k_gemm<BM, BN, true, true, CMP>), grid, dim3(256), 0, s, g);
}

template <int BM, int BN>
static void launch_bf16(const GemmDesc& d, const GemmArgs& g, dim3 grid, hipStream_t s) {
  if (d.ta == 'N' && d.tb == 'N')
    hipLaunchKernelGGL((k_gemm_bf16<BM, BN, false, false>), grid, dim3(256), 0, s, g);
  else if (d.ta == 'T' && d.tb == 'N')
    hipLaunchKernelGGL((k_gemm_bf16<BM, BN, true, false>), grid, dim3(256), 0, s, g);
  else if (d.ta == 'N' && d.tb == 'T')
    hipLaunchKernelGGL((k_gemm_bf16<BM, BN, false, true>), grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((k_gemm_bf16<BM, BN, true, true>), grid, dim3(256), 0, s, g);
}

hipError_t gemm(const GemmDesc& d, hipStream_t s, double* scratch, int64_t scratch_doubles,
                double* flops) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.K <= 0) {
    // C = beta C: reuse the reduction kernel with zero partials is wasteful;
    // a K = 0 product only happens for empty panels, which callers avoid.
    return hipSuccess;
  }
  // 128 x 128 tiles when there are enough of them to fill the chip, or when
  // a long K (split below) supplies the parallelism and the larger tile
  // halves the operand re-reads; 64 x 64 tiles otherwise.
  const int64_t t128 = ((d.M + 127) / 128) * ((d.N + 127) / 128);
  const bool big = d.M >= 128 && d.N >= 128 && (t128 >= 128 || d.K >= 4096);
  const int BM = big ? 128 : 64, BN = big ? 128 : 64;
  const int64_t tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
  const int64_t tiles = tm * tn;
  // Split-K when the output has few tiles: slices of at least 512 for long K,
  // of at least 32 for short K (the small products of a recursion node, whose
  // one or few workgroups would otherwise walk K alone).
  int64_t nsplit = 1;
  const int64_t min_chunk = d.K >= 1024 ? 512 : 32;
  if (tiles < 512 && d.K >= 2 * min_chunk && scratch && scratch_doubles >= 2 * d.M * d.N) {
    nsplit = std::min<int64_t>((1024 + tiles - 1) / tiles, d.K / min_chunk);
    nsplit = std::min<int64_t>(nsplit, scratch_doubles / (d.M * d.N));
    nsplit = std::max<int64_t>(nsplit, 1);
  }
  int64_t kchunk = (d.K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 31) / 32 * 32;
  nsplit = (d.K + kchunk - 1) / kchunk;
  GemmArgs g{d.M, d.N, d.K, kchunk, d.alpha, d.beta, d.A, d.lda, d.B, d.ldb,
             d.C, d.ldc, nsplit > 1 ? scratch : nullptr, d.maskA, d.maskB, d.add_identity};
  dim3 grid((unsigned)tm, (unsigned)tn, (unsigned)nsplit);
  const double gbytes = 8.0 * ((double)d.M * d.K + (double)d.K * d.N +
                               (d.beta == 0.0 ? 1.0 : 2.0) * (double)d.M * d.N);
  {
    TimedLaunch tl(s, d.compute == COMPUTE_F32    ? "gemm_f32"
                      : d.compute == COMPUTE_BF16 ? "gemm_bf16"
                                                  : "gemm_f64",
                   gbytes, 2.0 * (double)d.M * d.N * d.K);
    if (d.compute == COMPUTE_BF16) {
      if (big) launch_bf16<128, 128>(d, g, grid, s);
      else launch_bf16<64, 64>(d, g, grid, s);
    } else if (d.compute == COMPUTE_F32) {
      if (big) launch_t<128, 128, COMPUTE_F32>(d, g, grid, s);
      else launch_t<64, 64, COMPUTE_F32>(d, g, grid, s);
    } else {
      if (big) launch_t<128, 128, COMPUTE_F64>(d, g, grid, s);
      else launch_t<64, 64, COMPUTE_F64>(d, g, grid, s);
    }
  }
  if (nsplit > 1) {
    const int64_t MN = d.M * d.N;
    TimedLaunch tr(s, "gemm_splitk_reduce", 8.0 * (double)MN * (nsplit + 2), (double)MN * nsplit);
    const int blocks = (int)((MN + 63) / 64);
    hipLaunchKernelGGL(k_splitk_reduce, dim3(blocks), dim3(256), 0, s, (const double*)scratch,
                       (int)nsplit, d.M, d.N, d.beta, d.C, d.ldc, d.add_identity);
  }
  if (flops) *flops += 2.0 * (double)d.M * (double)d.N * (double)d.K;
  return hipGetLastError();
}

}  // namespace miqr
