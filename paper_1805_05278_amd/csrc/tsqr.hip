// TSQR panel factorisation for gfx950 (App. C of the paper: upsweep,
// downsweep, Householder reconstruction; base case of 1D-CAQR-EG, Sec. 6.1).
//
// Reduction structure.  The panel's rows are split evenly into leaf blocks of
// at most 128 or 256 rows (at least nbr rows each).  A workgroup reduces a
// *chain* of consecutive leaf blocks in sequence: the first block gets a
// local Householder QR of its own rows (App. C.1); every further block X_s is
// stacked under the running R and the stacked matrix is factored,
//     [R; X_s] = Q_s [R_new; 0],   Q_s = I - [I; Y_s] T_s [I; Y_s]^T,
// with the structure of the stacked triangle exploited: the reflector for
// column j touches only row j of R and the rows of X_s.  Above the leaves,
// a tree node takes the R factors of up to `arity` children and performs the
// same step once, with the R factors of children 1.. stacked into one X.  The
// paper's binomial tree is arity 2 with one leaf block per chain; wider nodes
// trade a larger local QR for fewer sequential levels (the paper's
// latency/bandwidth parameter).
//
// Downsweep (App. C.2).  Starting from B at the root, a node hands
// B - T B to its first child and -Y_s (T B) to the others; a leaf chain is
// walked backwards (M = T_s B, block s receives -Y_s M, B <- B - M) and its
// first block receives [B; 0] - V (Z B) with Z = T V_top^T stored by the
// factorisation.  Started from B = I this yields W, the leading columns of
// the Q-factor.
//
// Householder reconstruction (App. C.2).  The root workgroup follows the path
// to leaf block 0 only, forms X (top rows of W), runs the sign-modified LU
// X + S = L U, and returns T = U S L^{-T}, R = -S R_root, and U^{-1}.  The
// downsweep proper starts from [U^{-1}, -S D] so that one pass over the
// leaves yields V = W U^{-1} and, optionally, the thin Q = -W S D (the
// paper's remark that starting from U^{-1} saves the second broadcast).  The
// top rows of V are L, written from the reconstruction, with R above the
// diagonal.
#include <algorithm>

#include "common.h"
#include "profiler.h"
#include "tsqr.h"
#include "plan.h"

namespace miqr {

// A copy of v that the compiler cannot merge with other uses of v: index
// arithmetic built on it is recomputed where it is used instead of being kept
// live (and spilled) across the kernel.
__device__ __forceinline__ int fresh_copy(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

struct ChainQRArgs {
  double* X;       // leaf level: panel (in place); tree level: child R array
  int64_t ldx;
  int64_t xrows;   // leaf level: panel rows
  int nblocks, chain_len, nbr;
  double* Y;       // tree levels: Y per node (kYS doubles, leading dim kYL)
  double* T;       // leaf: per block; tree: per node
  double* R;       // per chain / node
};

// Sum over N consecutive lanes (N = 8, 16 or 32), result in every lane: quad
// sums and half-row / row mirrors through DPP, then (N = 32) an exchange
// between the two 16-lane rows of a 32-lane group through ds_swizzle.
template <int N>
__device__ __forceinline__ double group_sum(double v) {
  v = oct_sum(v);
  if (N == 8) return v;
  v += dpp_mov<0x140>(v);  // row_mirror: lane i <-> 15 - i
  if (N == 32) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)(b & 0xffffffffull), 0x401F);
    int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(b >> 32), 0x401F);
    v += __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
  }
  return v;
}

// Register layout of a block of H rows (H = 64, 128 or 256) in a 512-thread
// workgroup: thread t holds 8 rows of CPT = H / 64 columns cg CPT .. cg CPT +
// CPT - 1 (cg = t / RG, RG = H / 8).  Its rows are four pairs: slot s of lane
// rg is row 2 rg + 2 RG (s / 2) + s % 2, so that for a fixed slot pair the RG
// lanes of a column cover 2 RG consecutive rows: global loads and stores
// coalesce, and the lanes' 16-byte LDS reads of the reflector are
// consecutive.  The RG threads of a column group sit in one wave, so column
// sums are lane reductions.  Each reflector value read from LDS is reused for
// CPT columns.
template <int H>
struct Lay {
  static constexpr int RG = H / 8;
  static constexpr int CPT = RG / 8;
  static __device__ __forceinline__ int row(int rg, int s) {
    return 2 * rg + 2 * RG * (s >> 1) + (s & 1);
  }
};

// One QR step on the rows held in registers (x[u][s]: column cg CPT + u, row
// Lay<H>::row(rg, s)).
//   first:  plain Householder QR of the rows themselves (pivot row j);
//   !first: the rows are stacked under the upper triangular R held in Rs.
// On return x holds the basis (rows below the pivot for `first`, all rows
// otherwise), Rs the new R (for !first), Gs the Gram entries v_i . v_j in its
// strict upper triangle (Gs must be zero below the diagonal and outside nbr on
// entry), and taus the reflector scalars; build_t then turns Gs into T.  The
// two are separate so that a caller can store x first and build T without
// the block's registers live.
template <int H, bool first>
__device__ __forceinline__ void qr_step(double (&x)[Lay<H>::CPT][8], int nbr,
                                        double (*Rs)[kNB + 1], double (*Gs)[kNB + 1],
                                        double (*vbuf)[H], double* taus, double* Wt) {
  constexpr int RG = Lay<H>::RG, CPT = Lay<H>::CPT;
  const int t = threadIdx.x, rg = t % RG, cg = t / RG;
  // The reflector sits in vb in row order: a lane's pair (s, s + 1) is the
  // 16-byte word at row(rg, s) = s RG + 2 rg, and consecutive lanes read
  // consecutive words.
  // Columns are taken CPT at a time so that the owner's register slot U is a
  // compile-time index (a runtime slot would force x out of registers).
  for (int j0 = 0; j0 < nbr; j0 += CPT) {
#pragma unroll
    for (int U = 0; U < CPT; ++U) {
      const int j = j0 + U;
      if (j >= nbr) break;
      double* vb = vbuf[j & 1];
      if (cg == j0 / CPT) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0}, av = 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int r = Lay<H>::row(rg, s);
          if (first) {
            s4[s & 3] += (r > j) ? x[U][s] * x[U][s] : 0.0;
            av = (r == j) ? x[U][s] : av;
          } else {
            s4[s & 3] += x[U][s] * x[U][s];
          }
        }
        const double ss = group_sum<RG>((s4[0] + s4[1]) + (s4[2] + s4[3]));
        const double alpha = first ? group_sum<RG>(av) : Rs[j][j];
        double beta = alpha, tau = 0.0, scale = 1.0;
        if (ss != 0.0) reflector(alpha, ss, beta, tau, scale);
        double nv[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int r = Lay<H>::row(rg, s);
          const double sc = x[U][s] * scale;
          if (first) {
            nv[s] = (r > j) ? sc : ((r == j) ? 1.0 : 0.0);
            x[U][s] = (r > j) ? sc : ((r == j) ? beta : x[U][s]);
          } else {
            nv[s] = sc;
            x[U][s] = sc;
          }
        }
#pragma unroll
        for (int s = 0; s < 8; s += 2)
          *(double2*)&vb[s * RG + 2 * rg] = make_double2(nv[s], nv[s + 1]);
        if (rg == 0) {
          taus[j] = tau;
          if (!first) Rs[j][j] = beta;
        }
      }
      __syncthreads();
      double v[8];
#pragma unroll
      for (int s = 0; s < 8; s += 2) {
        const double2 p = *(const double2*)&vb[s * RG + 2 * rg];
        v[s] = p.x;
        v[s + 1] = p.y;
      }
      double d[CPT];
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          a0 += v[s] * x[u][s];
          a1 += v[s + 1] * x[u][s + 1];
        }
        d[u] = a0 + a1;
      }
#pragma unroll
      for (int u = 0; u < CPT; ++u) d[u] = group_sum<RG>(d[u]);
      const double tau = taus[j];
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int c = cg * CPT + u;
        if (c > j && c < nbr) {
          const double w = tau * (first ? d[u] : d[u] + Rs[j][c]);
#pragma unroll
          for (int s = 0; s < 8; ++s) x[u][s] -= v[s] * w;
          if (rg == 0 && !first) Rs[j][c] -= w;
        } else if (c < j && rg == 0) {
          Gs[c][j] = d[u];  // v_c . v_j
        }
      }
    }
  }
  __syncthreads();
}

// One pairing level of build_t: for each pair of diagonal blocks of size SZ,
// T12 = -T1 (G12 T2).  The sums run over whole block rows / columns: the
// entries outside a triangle are zero in Gs, so no bounds are needed and the
// loads of a sum can all be in flight together.
template <int SZ>
__device__ __forceinline__ void t_pair_level(double (*Gs)[kNB + 1], double* Wt) {
  constexpr int NP = kNB / (2 * SZ);
  const int t = threadIdx.x;
  for (int e = fresh_copy(t); e < NP * SZ * SZ; e += 512) {
    const int pr = e / (SZ * SZ), i = (e / SZ) % SZ, k = e % SZ;
    const int a = 2 * SZ * pr, b = a + SZ;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int m = 0; m < SZ; m += 2) {
      s0 += Gs[a + i][b + m] * Gs[b + m][b + k];
      s1 += Gs[a + i][b + m + 1] * Gs[b + m + 1][b + k];
    }
    Wt[e] = s0 + s1;
  }
  __syncthreads();
  for (int e = fresh_copy(t); e < NP * SZ * SZ; e += 512) {
    const int pr = e / (SZ * SZ), i = (e / SZ) % SZ, k = e % SZ;
    const int a = 2 * SZ * pr, b = a + SZ;
    const double* w = Wt + pr * SZ * SZ + k;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int m = 0; m < SZ; m += 2) {
      s0 += Gs[a + i][a + m] * w[m * SZ];
      s1 += Gs[a + i][a + m + 1] * w[(m + 1) * SZ];
    }
    Gs[a + i][b + k] = -(s0 + s1);
  }
  __syncthreads();
}

// The same pairing level on FP64 MFMA (SZ = 16 or 32): the two products are
// (SZ / 16)^2 output tiles per pair, one wave per tile, SZ / 4 k-steps each.
// Operand layout: a = A[l % 16][l / 16], b = B[l / 16][l % 16],
// acc[r] = D[l / 16 + 4 r][l % 16].
template <int SZ>
__device__ __forceinline__ void t_pair_level_mfma(double (*Gs)[kNB + 1], double* Wt) {
  constexpr int NP = kNB / (2 * SZ), TPS = SZ / 16, NT = NP * TPS * TPS;
  static_assert(NT <= 8, "one tile per wave");
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = l >> 4;
  const int pr = w / (TPS * TPS), ti = (w / TPS) % TPS, tj = w % TPS;
  const int a = 2 * SZ * pr, b = a + SZ;
  double* Wp = Wt + pr * SZ * SZ;  // Wt[pr] as SZ x SZ, row-major
  if (w < NT) {
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < SZ / 4; ++ks)
      acc = mfma64(Gs[a + 16 * ti + li][b + 4 * ks + lk], Gs[b + 4 * ks + lk][b + 16 * tj + li], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[(16 * ti + lk + 4 * r) * SZ + 16 * tj + li] = acc[r];
  }
  __syncthreads();
  if (w < NT) {
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < SZ / 4; ++ks)
      acc = mfma64(Gs[a + 16 * ti + li][a + 4 * ks + lk], Wp[(4 * ks + lk) * SZ + 16 * tj + li], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) Gs[a + 16 * ti + lk + 4 * r][b + 16 * tj + li] = -acc[r];
  }
  __syncthreads();
}

// T from its 16 x 16 diagonal blocks (in place in Gs) and the Gram entries
// above them: blocks of 16 and 32 are paired, T12 = -T1 (G12 T2).
__device__ __forceinline__ void t_from_blocks(double (*Gs)[kNB + 1], double* Wt) {
  t_pair_level_mfma<16>(Gs, Wt);
  t_pair_level_mfma<32>(Gs, Wt);
}

// T in place of the Gram entries left by qr_step (Gs zero below the
// diagonal and outside nbr).
__device__ __forceinline__ void build_t(double (*Gs)[kNB + 1], const double* taus, double* Wt,
                                        int nbr) {
  const int t = threadIdx.x;
  // T from the Gram entries G (strict upper part of Gs) and tau (Sec. 2.3:
  // T^{-1} = striu(V^T V) + diag(tau)^{-1}), built blockwise in place: first
  // the 8 x 8 diagonal blocks by the column recurrence
  // T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j], taken row by row (row i needs
  // only its own earlier entries, so each thread builds one row alone), then
  // blocks of 8, 16, 32 are paired, T12 = -T1 (G12 T2).
  double Tr[8];
  const int bb = t >> 3, i = t & 7, r0 = 8 * bb;
  if (t < kNB) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int col = r0 + j;
      const double tj = (col < nbr) ? taus[col] : 0.0;
      double sacc = 0.0;
#pragma unroll
      for (int k = 0; k < j; ++k) sacc += Tr[k] * Gs[r0 + k][col];
      Tr[j] = (i == j) ? tj : ((i < j) ? -tj * sacc : 0.0);
    }
  }
  __syncthreads();
  if (t < kNB) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j >= i) Gs[r0 + i][r0 + j] = Tr[j];
  }
  __syncthreads();
  // VALU pairing: the two-workgroups-per-CU leaf kernel that uses this has
  // no registers to spare for the MFMA form (t_from_blocks).
  t_pair_level<8>(Gs, Wt);
  t_pair_level<16>(Gs, Wt);
  t_pair_level<32>(Gs, Wt);
}

// LEAF: the chain walks row blocks of the panel (else stacked child R's).
// PART (leaf only): 0 the whole chain; 1 only its first block (local QR);
// 2 the blocks after the first, starting from the R that part 1 left in the
// chain's R slot.  Parts 1 and 2 are separate launches so that part 2, which
// holds no first-block state, fits two workgroups per CU.
template <int H, bool LEAF, int PART>
__device__ __forceinline__ void chain_qr_body(const ChainQRArgs& a) {
  constexpr int RG = Lay<H>::RG, CPT = Lay<H>::CPT;
  const int t = threadIdx.x, rg = t % RG, cg = t / RG;
  const int chain = blockIdx.x;
  const int b0 = chain * a.chain_len;
  const int b1 = min(b0 + a.chain_len, a.nblocks);
  const int nbr = a.nbr;
  __shared__ double Rs[kNB][kNB + 1];
  __shared__ double Gs[kNB][kNB + 1];
  __shared__ __align__(16) double vbuf[2][H];
  __shared__ double taus[kNB];
  __shared__ double Wt[32 * kNB / 2];

  {
    // The starting R (tree: child 0's R; stacked leaf blocks: the chain's R
    // slot), all loads in flight together (slots are always in bounds),
    // masked afterwards.
    const int tt = fresh_copy(t);
    const double* src = !LEAF ? a.X + (int64_t)b0 * kTS
                              : (PART == 2 ? a.R + (int64_t)chain * kTS : nullptr);
    double g[kTS / 512];
#pragma unroll
    for (int e = 0; e < kTS / 512; ++e) g[e] = src ? src[tt + 512 * e] : 0.0;
#pragma unroll
    for (int e = 0; e < kTS / 512; ++e) {
      const int i = tt + 512 * e, r = i % kNB, cc = i / kNB;
      double v = 0.0;
      if (!LEAF && r < nbr && cc < nbr) v = g[e];
      if (LEAF && PART == 2 && r <= cc && cc < nbr) v = g[e];
      Rs[r][cc] = v;
      Gs[r][cc] = 0.0;
    }
  }
  __syncthreads();

  double x[CPT][8];
  if constexpr (LEAF) {
    const int bs = PART == 2 ? b0 + 1 : b0;
    const int be = PART == 1 ? b0 + 1 : b1;
    for (int b = bs; b < be; ++b) {
      const bool first = b == b0;
      const int64_t rstart = ((int64_t)b * a.xrows) / a.nblocks;
      const int rows = (int)((((int64_t)b + 1) * a.xrows) / a.nblocks - rstart);
      double* src = a.X + rstart;
      const int64_t ld = a.ldx;
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int c = cg * CPT + u;
#pragma unroll
        for (int s = 0; s < 8; ++s)
          x[u][s] = (c < nbr && Lay<H>::row(rg, s) < rows)
                        ? src[Lay<H>::row(rg, s) + (int64_t)c * ld] : 0.0;
      }
      if constexpr (PART != 2) {
        if (first) qr_step<H, true>(x, nbr, Rs, Gs, vbuf, taus, Wt);
      }
      if constexpr (PART != 1) {
        if (!first) qr_step<H, false>(x, nbr, Rs, Gs, vbuf, taus, Wt);
      }
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int c = cg * CPT + u;
#pragma unroll
        for (int s = 0; s < 8; ++s)
          if (c < nbr && Lay<H>::row(rg, s) < rows) src[Lay<H>::row(rg, s) + (int64_t)c * ld] = x[u][s];
      }
      build_t(Gs, taus, Wt, nbr);
      double* Tb = a.T + (int64_t)b * kTS;
      if (!first) {
        for (int i = fresh_copy(t); i < kTS; i += 512) {
          const int r = i % kNB, cc = i / kNB;
          Tb[i] = (r <= cc && cc < nbr) ? Gs[r][cc] : 0.0;
        }
      } else if (PART != 2) {
        // Z = T V_top^T (upper triangular) in place of T; Rs holds V_top
        // (unit lower top nbr x nbr part of the block's basis) meanwhile.
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          const int c = cg * CPT + u;
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int r = Lay<H>::row(rg, s);
            if (r < kNB) Rs[r][c] = (r > c) ? x[u][s] : ((r == c) ? 1.0 : 0.0);
          }
        }
        __syncthreads();
        for (int i = fresh_copy(t); i < kTS; i += 512) {
          const int r = i % kNB, cc = i / kNB;
          double z = 0.0;
          if (r <= cc && cc < nbr)
            for (int k = r; k <= cc; ++k) z += Gs[r][k] * Rs[cc][k];
          Tb[i] = z;
        }
        __syncthreads();
        // The block's R (upper triangle of its top rows) seeds the chain.
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          const int c = cg * CPT + u;
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int r = Lay<H>::row(rg, s);
            if (r < kNB) Rs[r][c] = (r <= c && c < nbr) ? x[u][s] : 0.0;
          }
        }
      }
      __syncthreads();
    }
  } else if (b1 - b0 >= 2) {
    // Tree node: children b0+1 .. b1-1 stacked (row stride nbr) under R_{b0}.
    const int rows = (b1 - b0 - 1) * nbr;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int c = cg * CPT + u;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int r = Lay<H>::row(rg, s);
        double v = 0.0;
        if (c < nbr && r < rows) {
          const int sidx = r / nbr, rr = r - sidx * nbr;
          v = a.X[(int64_t)(b0 + 1 + sidx) * kTS + rr + c * kNB];
        }
        x[u][s] = v;
      }
    }
    qr_step<H, false>(x, nbr, Rs, Gs, vbuf, taus, Wt);
    double* Yn = a.Y + (int64_t)chain * kYS;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int c = cg * CPT + u;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int r = Lay<H>::row(rg, s);
        if (c < nbr && r < rows) Yn[r + c * kYL] = x[u][s];
      }
    }
    build_t(Gs, taus, Wt, nbr);
    double* Tn = a.T + (int64_t)chain * kTS;
    for (int i = fresh_copy(t); i < kTS; i += 512) {
      const int r = i % kNB, cc = i / kNB;
      Tn[i] = (r <= cc && cc < nbr) ? Gs[r][cc] : 0.0;
    }
    __syncthreads();
  } else {
    double* Tn = a.T + (int64_t)chain * kTS;
    for (int i = fresh_copy(t); i < kTS; i += 512) Tn[i] = 0.0;
  }

  for (int i = fresh_copy(t); i < kTS; i += 512) {
    const int r = i % kNB, cc = i / kNB;
    a.R[(int64_t)chain * kTS + i] = (r <= cc && cc < nbr) ? Rs[r][cc] : 0.0;
  }
}

// ------------------------------------------------ blocked block QR on MFMA
//
// For blocks of 256 rows the column-by-column step above spends most of its
// issue slots on 32-lane reductions: every reflector is applied to all 64
// columns at once.  The blocked form (the compact-WY recursion of Sec. 2.3
// applied inside the block) factors 16-column sub-panels column by column,
// each column held by half a wave (8 rows per lane, one reduction per
// column), and applies each sub-panel to the columns right of it with two
// FP64 MFMA products:  W = V_b^T X,  W' = T_b^T W,  X -= V_b W'.  The same
// W product, taken over the columns left of the sub-panel too, yields the
// Gram entries V^T V from which the block's T is built.
//
// Register layout ("tile layout"): wave w holds column tile ct = w / 2 and
// row tiles 8 (w % 2) .. 8 (w % 2) + 7 of the 256 x 64 block; lane (g, cl)
// (g = l / 16, cl = l % 16) holds rows g + 4 r (r = 0..3) of each 16 x 16
// tile in column cl, which is the MFMA accumulator layout.  Global rows are
// staged through the sub-panel buffer P, which also carries each sub-panel
// between the tile layout and the column-step layout (thread t: column
// t / 32, rows 8 (t % 32) .. + 7).

constexpr int kPLD = 258;  // column stride of P (doubles)

// Position of row r of a 256-row column in P: rows 8 q + s go to pair q of
// slice s / 2, so that lanes reading 8 consecutive rows as four pairs hit
// consecutive 16-byte words.
__device__ __forceinline__ int ppos(int r) {
  return ((r & 7) >> 1) * 64 + 2 * (r >> 3) + (r & 1);
}

struct MfmaQRShared {
  double P[16][kPLD];        // one 256 x 16 column tile
  double Wred[8][16][17];    // per-wave partial W tiles (also build_t's scratch)
  double W[16][kNB + 1];     // W = V_b^T [R; X] of the sub-panel, trailing columns
  double Wp[16][kNB + 1];    // W' = T_b^T W
  double Tsub[16][17];
  __align__(16) double vbuf[2][256];
};

// Tile-layout coordinates of thread t.
struct TileCoord {
  int w, g, cl, ct, rt0;
  __device__ TileCoord(int t) {
    w = t >> 6;
    const int l = t & 63;
    g = l >> 4;
    cl = l & 15;
    ct = w >> 1;
    rt0 = (w & 1) * 8;
  }
  __device__ int row(int k, int r) const { return 16 * (rt0 + k) + g + 4 * r; }
};

// ppos(16 m + x) = ppos(x) + 4 m for x < 16: a tile's rows sit at a fixed
// pattern plus 4 per tile, so the k loops below address P as one base per r
// plus an immediate offset (instead of 32 live addresses).
__device__ __forceinline__ int tile_base(const TileCoord& tc, int r) {
  return tc.cl * kPLD + ppos(fresh_copy(tc.g) + 4 * r) + 4 * tc.rt0;
}

// Move column tile ct_ between the column-step layout in P and the tile
// registers of its two owner waves.
__device__ __forceinline__ void tiles_to_p(const TileCoord& tc, int ct_, const double (&xt)[8][4],
                                           MfmaQRShared& S) {
  if (tc.ct == ct_)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double* p = &S.P[0][0] + tile_base(tc, r);
#pragma unroll
      for (int k = 0; k < 8; ++k) p[4 * k] = xt[k][r];
    }
}
__device__ __forceinline__ void p_to_tiles(const TileCoord& tc, int ct_, double (&xt)[8][4],
                                           const MfmaQRShared& S) {
  if (tc.ct == ct_)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double* p = &S.P[0][0] + tile_base(tc, r);
#pragma unroll
      for (int k = 0; k < 8; ++k) xt[k][r] = p[4 * k];
    }
}

// Column-step layout: thread t holds rows 8 q .. 8 q + 7 (q = t % 32) of
// column t / 32 of P.
__device__ __forceinline__ void p_read8(const MfmaQRShared& S, int c, int q, double (&v)[8]) {
#pragma unroll
  for (int s = 0; s < 8; s += 2) {
    const double2 p = *(const double2*)&S.P[c][(s >> 1) * 64 + 2 * q];
    v[s] = p.x;
    v[s + 1] = p.y;
  }
}
__device__ __forceinline__ void p_write8(MfmaQRShared& S, int c, int q, const double (&v)[8]) {
#pragma unroll
  for (int s = 0; s < 8; s += 2)
    *(double2*)&S.P[c][(s >> 1) * 64 + 2 * q] = make_double2(v[s], v[s + 1]);
}

// Load a 256 x 64 block into the tile registers; at(row, col) gives the
// global element (rows < nrows and cols < nbr only; the rest reads 0).  All
// global loads are issued before the first exchange through P.
template <typename At>
__device__ __forceinline__ void load_block(const TileCoord& tc, double (&xt)[8][4], int nrows,
                                           int nbr, MfmaQRShared& S, At at) {
  // Thread (c, q) moves rows q + 32 s of column c: a half-wave covers 32
  // consecutive rows, so the global accesses coalesce.
  const int t = threadIdx.x, c = t >> 5, q = t & 31;
  double v[4][8];
#pragma unroll
  for (int ct_ = 0; ct_ < 4; ++ct_) {
    const int col = 16 * ct_ + c;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      // Clamped into the valid corner and masked after the load, so that no
      // load waits on a predicate and all of them are in flight together.
      const int row = q + 32 * s;
      const double g = at(min(row, nrows - 1), min(col, nbr - 1));
      v[ct_][s] = (col < nbr && row < nrows) ? g : 0.0;
    }
  }
#pragma unroll
  for (int ct_ = 0; ct_ < 4; ++ct_) {
#pragma unroll
    for (int s = 0; s < 8; ++s) S.P[c][ppos(q + 32 * s)] = v[ct_][s];
    __syncthreads();
    p_to_tiles(tc, ct_, xt, S);
    __syncthreads();
  }
}

// Store the tile registers; put(row, col, value) for rows < nrows, cols < nbr.
// The global stores are issued after the last exchange through P, so that no
// barrier waits for them.
template <typename Put>
__device__ __forceinline__ void store_block(const TileCoord& tc, const double (&xt)[8][4],
                                            int nrows, int nbr, MfmaQRShared& S, Put put) {
  const int t = threadIdx.x, c = t >> 5, q = t & 31;
  double v[4][8];
#pragma unroll
  for (int ct_ = 0; ct_ < 4; ++ct_) {
    tiles_to_p(tc, ct_, xt, S);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) v[ct_][s] = S.P[c][ppos(q + 32 * s)];
    __syncthreads();
  }
#pragma unroll
  for (int ct_ = 0; ct_ < 4; ++ct_) {
    const int col = 16 * ct_ + c;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int row = q + 32 * s;
      if (col < nbr && row < nrows) put(row, col, v[ct_][s]);
    }
  }
}

// Sum over the 32 lanes of a half-wave, result in every lane: the 16-lane
// sums of group_sum, then the two rows exchanged in registers by
// v_permlane16_swap (one copy ends up holding the even row in both rows, the
// other the odd row) instead of a ds_swizzle round trip through the LDS unit.
__device__ __forceinline__ double half_wave_sum(double v) {
  v = group_sum<16>(v);
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)(u & 0xffffffffull), hi = (unsigned)(u >> 32);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double e =
      __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | (unsigned long long)l[0]));
  const double o =
      __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | (unsigned long long)l[1]));
  return e + o;
}

// Column jp of T_b (Sec. 2.3 recurrence, T[0:jp, jp] = -tau_jp T[0:jp, 0:jp]
// G[0:jp, jp]), entry of row i.  Row i of T_b was cleared at the start of the
// sub-panel, so the sum can run over all 16 terms: T[i][k] is zero for k < i
// and for k >= jp (not built yet), and G is zero below its diagonal, where
// only zero T entries meet it.  No bounds, so the loads overlap.
__device__ __forceinline__ void tsub_column(MfmaQRShared& S, double (*Gs)[kNB + 1],
                                            const double* taus, int b, int jp, int i) {
  if (jp < 0) return;
  const int jv = 16 * b + jp;
  const double tj = taus[jv];
  double p0 = 0.0, p1 = 0.0;
#pragma unroll
  for (int k = 0; k < 16; k += 2) {
    p0 += S.Tsub[i][k] * Gs[16 * b + k][jv];
    p1 += S.Tsub[i][k + 1] * Gs[16 * b + k + 1][jv];
  }
  S.Tsub[i][jp] = (i == jp) ? tj : ((i < jp) ? -tj * (p0 + p1) : 0.0);
}

// Blocked Householder QR of the block in xt (first: the rows themselves;
// else stacked under the upper triangular R in Rs).  On return xt holds the
// basis (first: R on and above the diagonal of the top rows), Rs the new R
// (stacked), Gs the Gram entries v_i . v_j (i < j) in its strict upper part,
// taus the reflector scalars.  Gs must be zero elsewhere, taus zero beyond
// nbr.
template <bool first>
__device__ void mfma_block_qr(const TileCoord& tc, double (&xt)[8][4], int nbr,
                              double (*Rs)[kNB + 1], double (*Gs)[kNB + 1], double* taus,
                              MfmaQRShared& S) {
  const int t = threadIdx.x, c = t >> 5, q = t & 31;
  const int nsub = (nbr + 15) >> 4;
  for (int b = 0; b < nsub; ++b) {
    // Sub-panel b into the column-step layout; T_b cleared (its rows are
    // built during the column steps).
    tiles_to_p(tc, b, xt, S);
    if (t < 16 * 17) (&S.Tsub[0][0])[t] = 0.0;
    __syncthreads();
    const int jc = 16 * b + c;
    double xf[8];
    p_read8(S, c, q, xf);
    for (int j = 0; j < 16; ++j) {
      const int jg = 16 * b + j;
      if (jg >= nbr) break;
      double* vb = S.vbuf[j & 1];
      if (c == j) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0}, av = 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int r = 8 * q + s;
          if (first) {
            s4[s & 3] += (r > jg) ? xf[s] * xf[s] : 0.0;
            av = (r == jg) ? xf[s] : av;
          } else {
            s4[s & 3] += xf[s] * xf[s];
          }
        }
        const double ss = half_wave_sum((s4[0] + s4[1]) + (s4[2] + s4[3]));
        const double alpha = first ? half_wave_sum(av) : Rs[jg][jg];
        double beta = alpha, tau = 0.0, scale = 1.0;
        if (ss != 0.0) reflector(alpha, ss, beta, tau, scale);
        double nv[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int r = 8 * q + s;
          const double sc = xf[s] * scale;
          if (first) {
            nv[s] = (r > jg) ? sc : ((r == jg) ? 1.0 : 0.0);
            xf[s] = (r > jg) ? sc : ((r == jg) ? beta : xf[s]);
          } else {
            nv[s] = sc;
            xf[s] = sc;
          }
        }
#pragma unroll
        for (int s = 0; s < 8; s += 2)
          *(double2*)&vb[(s >> 1) * 64 + 2 * q] = make_double2(nv[s], nv[s + 1]);
        if (q == 0) {
          taus[jg] = tau;
          if (!first) Rs[jg][jg] = beta;
        }
      }
      __syncthreads();
      if (c > j && jc < nbr) {
        double v[8];
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          const double2 p = *(const double2*)&vb[(s >> 1) * 64 + 2 * q];
          v[s] = p.x;
          v[s + 1] = p.y;
        }
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          a0 += v[s] * xf[s];
          a1 += v[s + 1] * xf[s + 1];
        }
        const double d = half_wave_sum(a0 + a1);
        const double wv = taus[jg] * (first ? d : d + Rs[jg][jc]);
#pragma unroll
        for (int s = 0; s < 8; ++s) xf[s] -= v[s] * wv;
        if (!first && q == 0) Rs[jg][jc] -= wv;
      } else if (c < j) {
        // Columns left of the pivot are final: their half-waves form the
        // Gram entries v_c . v_j (v_j is zero above its pivot row, where a
        // first block's column still holds R), and half-wave 0 builds
        // column j - 1 of T_b, whose Gram column is complete.
        double v[8];
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          const double2 p = *(const double2*)&vb[(s >> 1) * 64 + 2 * q];
          v[s] = p.x;
          v[s + 1] = p.y;
        }
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          a0 += v[s] * xf[s];
          a1 += v[s + 1] * xf[s + 1];
        }
        const double d = half_wave_sum(a0 + a1);
        if (q == 0) Gs[jc][jg] = d;
        if (c == 0 && q < 16) tsub_column(S, Gs, taus, b, j - 1, q);
      }
    }
    // The factored sub-panel back into P and into its owners' tiles.
    p_write8(S, c, q, xf);
    __syncthreads();
    p_to_tiles(tc, b, xt, S);
    if (t < 16) tsub_column(S, Gs, taus, b, min(16, nbr - 16 * b) - 1, t);

    // Partial W = V_b^T X over this wave's 128 rows, all column tiles (the
    // tiles left of b and b itself give Gram entries, the rest the update).
    // MFMA operands: A = V_b^T (lane: V_b[row][16 b + cl]), B = X (lane:
    // xt[k][r]); the k index of the product runs over rows g + 4 r.
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    if (16 * tc.ct < nbr) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double* pv = &S.P[0][0] + tile_base(tc, r);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          double av = pv[4 * k];
          double bx = xt[k][r];
          if (first) {
            const int row = tc.row(k, r);
            const int vc = 16 * b + tc.cl, xc = 16 * tc.ct + tc.cl;
            av = (row < vc) ? 0.0 : ((row == vc) ? 1.0 : av);
            if (tc.ct <= b) bx = (row < xc) ? 0.0 : ((row == xc) ? 1.0 : bx);
          }
          acc = mfma64(av, bx, acc);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) S.Wred[tc.w][tc.g + 4 * r][tc.cl] = acc[r];
    __syncthreads();
    for (int e = fresh_copy(t); e < 16 * kNB; e += 512) {
      const int m = e & 15, col = e >> 4, ct_ = col >> 4, n = col & 15;
      const int jv = 16 * b + m;
      const double val = S.Wred[2 * ct_][m][n] + S.Wred[2 * ct_ + 1][m][n];
      if (ct_ < b) {
        if (jv < nbr) Gs[col][jv] = val;
      } else if (ct_ > b) {
        S.W[m][col] = val + ((first || jv >= nbr || col >= nbr) ? 0.0 : Rs[jv][col]);
      }
    }
    // T_b into the diagonal block of Gs (its Gram entries are used up).
    if (t < 256) {
      const int i = t >> 4, jj = t & 15;
      if (i <= jj) Gs[16 * b + i][16 * b + jj] = S.Tsub[i][jj];
    }
    __syncthreads();
    if (16 * (b + 1) >= nbr) continue;  // no columns right of the last sub-panel
    // W' = T_b^T W on the trailing columns; R rows of the sub-panel (stacked).
    for (int e = fresh_copy(t); e < 16 * kNB; e += 512) {
      const int m = e & 15, col = e >> 4;
      if (col < 16 * (b + 1)) continue;
      double sacc = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) sacc += S.Tsub[k][m] * S.W[k][col];  // T_b upper: 0 for k > m
      S.Wp[m][col] = sacc;
      if (!first && 16 * b + m < nbr && col < nbr) Rs[16 * b + m][col] -= sacc;
    }
    __syncthreads();
    // X -= V_b W' on the column tiles right of b.  A = V_b (lane: V_b[row
    // 16 (rt0 + k) + cl][16 b + 4 p + g]), B = W' (lane: W'[4 p + g][16 ct + cl]).
    if (tc.ct > b && 16 * tc.ct < nbr) {
      // Row 16 (rt0 + k) + cl of column 4 p + g of P sits at
      // pa + 4 k + 4 p kPLD; W'[4 p + g][16 ct + cl] at pw + 4 p (kNB + 1).
      const double* pa = &S.P[0][0] + fresh_copy(tc.g) * kPLD + ppos(tc.cl) + 4 * tc.rt0;
      const double* pw = &S.Wp[0][0] + fresh_copy(tc.g) * (kNB + 1) + 16 * tc.ct + tc.cl;
      double wp[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) wp[p] = -pw[4 * p * (kNB + 1)];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        d4 xa = d4{xt[k][0], xt[k][1], xt[k][2], xt[k][3]};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          double av = pa[4 * k + 4 * p * kPLD];
          if (first) {
            const int row = 16 * (tc.rt0 + k) + tc.cl, vc = 16 * b + 4 * p + tc.g;
            av = (row < vc) ? 0.0 : ((row == vc) ? 1.0 : av);
          }
          xa = mfma64(av, wp[p], xa);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) xt[k][r] = xa[r];
      }
    }
    __syncthreads();
  }
}

// Chain / node body for 256-row blocks on the blocked MFMA factorisation
// (same roles of LEAF and PART as chain_qr_body).
template <bool LEAF, int PART>
__device__ __forceinline__ void chain_qr_body_mfma(const ChainQRArgs& a) {
  const int t = threadIdx.x;
  const TileCoord tc(t);
  const int chain = blockIdx.x;
  const int b0 = chain * a.chain_len;
  const int b1 = min(b0 + a.chain_len, a.nblocks);
  const int nbr = a.nbr;
  __shared__ double Rs[kNB][kNB + 1];
  __shared__ double Gs[kNB][kNB + 1];
  __shared__ double taus[kNB];
  __shared__ MfmaQRShared S;
  double* Wt = &S.Wred[0][0][0];

  {
    // The starting R (tree: child 0's R; stacked leaf blocks: the chain's R
    // slot), all loads in flight together (slots are always in bounds),
    // masked afterwards.
    const int tt = fresh_copy(t);
    const double* src = !LEAF ? a.X + (int64_t)b0 * kTS
                              : (PART == 2 ? a.R + (int64_t)chain * kTS : nullptr);
    double g[kTS / 512];
#pragma unroll
    for (int e = 0; e < kTS / 512; ++e) g[e] = src ? src[tt + 512 * e] : 0.0;
#pragma unroll
    for (int e = 0; e < kTS / 512; ++e) {
      const int i = tt + 512 * e, r = i % kNB, cc = i / kNB;
      double v = 0.0;
      if (!LEAF && r < nbr && cc < nbr) v = g[e];
      if (LEAF && PART == 2 && r <= cc && cc < nbr) v = g[e];
      Rs[r][cc] = v;
      Gs[r][cc] = 0.0;
    }
  }
  if (t < kNB) taus[t] = 0.0;
  __syncthreads();

  double xt[8][4];
  if constexpr (LEAF) {
    const int bs = PART == 2 ? b0 + 1 : b0;
    const int be = PART == 1 ? b0 + 1 : b1;
    for (int b = bs; b < be; ++b) {
      const bool first = b == b0;
      const int64_t rstart = ((int64_t)b * a.xrows) / a.nblocks;
      const int rows = (int)((((int64_t)b + 1) * a.xrows) / a.nblocks - rstart);
      double* src = a.X + rstart;
      const int64_t ld = a.ldx;
      load_block(tc, xt, rows, nbr, S,
                 [&](int row, int col) { return src[row + (int64_t)col * ld]; });
      if constexpr (PART != 2) {
        if (first) mfma_block_qr<true>(tc, xt, nbr, Rs, Gs, taus, S);
      }
      if constexpr (PART != 1) {
        if (!first) mfma_block_qr<false>(tc, xt, nbr, Rs, Gs, taus, S);
      }
      store_block(tc, xt, rows, nbr, S,
                  [&](int row, int col, double v) { src[row + (int64_t)col * ld] = v; });
      t_from_blocks(Gs, Wt);
      double* Tb = a.T + (int64_t)b * kTS;
      if (!first) {
        for (int i = fresh_copy(t); i < kTS; i += 512) {
          const int r = i % kNB, cc = i / kNB;
          Tb[i] = (r <= cc && cc < nbr) ? Gs[r][cc] : 0.0;
        }
      } else if (PART != 2) {
        // Z = T V_top^T (upper triangular) in place of T; Rs holds V_top
        // (unit lower top nbr x nbr part of the block's basis) meanwhile.
        if (tc.rt0 == 0) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = tc.row(k, r), col = 16 * tc.ct + tc.cl;
              Rs[row][col] = (row > col) ? xt[k][r] : ((row == col) ? 1.0 : 0.0);
            }
        }
        __syncthreads();
        for (int i = fresh_copy(t); i < kTS; i += 512) {
          const int r = i % kNB, cc = i / kNB;
          double z = 0.0;
          if (r <= cc && cc < nbr)
            for (int k = r; k <= cc; ++k) z += Gs[r][k] * Rs[cc][k];
          Tb[i] = z;
        }
        __syncthreads();
        // The block's R (upper triangle of its top rows) seeds the chain.
        if (tc.rt0 == 0) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = tc.row(k, r), col = 16 * tc.ct + tc.cl;
              Rs[row][col] = (row <= col && col < nbr) ? xt[k][r] : 0.0;
            }
        }
      }
      __syncthreads();
    }
  } else if (b1 - b0 >= 2) {
    // Tree node: children b0+1 .. b1-1 stacked (row stride nbr) under R_{b0}.
    const int rows = (b1 - b0 - 1) * nbr;
    const double* X = a.X;
    // Child index of a stacked row by a float reciprocal: (row + 1/2) / nbr
    // is never within 1/(2 nbr) of an integer, far above float rounding.
    const float inv_nbr = 1.0f / (float)nbr;
    load_block(tc, xt, rows, nbr, S, [&](int row, int col) {
      const int sidx = (int)(((float)row + 0.5f) * inv_nbr), rr = row - sidx * nbr;
      return X[(int64_t)(b0 + 1 + sidx) * kTS + rr + col * kNB];
    });
    mfma_block_qr<false>(tc, xt, nbr, Rs, Gs, taus, S);
    double* Yn = a.Y + (int64_t)chain * kYS;
    store_block(tc, xt, rows, nbr, S,
                [&](int row, int col, double v) { Yn[row + col * kYL] = v; });
    t_from_blocks(Gs, Wt);
    double* Tn = a.T + (int64_t)chain * kTS;
    for (int i = fresh_copy(t); i < kTS; i += 512) {
      const int r = i % kNB, cc = i / kNB;
      Tn[i] = (r <= cc && cc < nbr) ? Gs[r][cc] : 0.0;
    }
    __syncthreads();
  } else {
    double* Tn = a.T + (int64_t)chain * kTS;
    for (int i = fresh_copy(t); i < kTS; i += 512) Tn[i] = 0.0;
  }

  for (int i = fresh_copy(t); i < kTS; i += 512) {
    const int r = i % kNB, cc = i / kNB;
    a.R[(int64_t)chain * kTS + i] = (r <= cc && cc < nbr) ? Rs[r][cc] : 0.0;
  }
}

template <int H, bool LEAF, int PART>
__global__ __launch_bounds__(512) void k_chain_qr(ChainQRArgs a) {
  if constexpr (H == 256) chain_qr_body_mfma<LEAF, PART>(a);
  else chain_qr_body<H, LEAF, PART>(a);
}

// Blocks after the first of each leaf chain, at two workgroups per CU.  This
// launch has enough chains to fill the chip twice over, so it keeps the
// column-by-column body, which fits two workgroups per CU; the blocked body
// needs 140 KB of LDS (one workgroup per CU) and only pays off where a CU has
// one workgroup anyway (tree nodes, first blocks).
template <int H>
__global__ __launch_bounds__(512, 4) void k_chain_qr_rest(ChainQRArgs a) {
  chain_qr_body<H, true, 2>(a);
}

struct HRArgs {
  int L;  // number of tree levels above the leaves
  const double* T[kMaxLevels];
  int nblocks[kMaxLevels];
  int chain_len[kMaxLevels];
  const double* Rtop;    // R of the top node
  const double* A0;      // leaf block 0 (its basis, in place), leading dim lda
  int64_t lda;
  int nbr, nq, normalize;
  double* Tp;            // nbr x nbr kernel, leading dim ldt
  int64_t ldt;
  double* LR;            // kTS: strict lower L, upper R
  double* Broot;         // kBS: downsweep input of the top node
  double* sign;          // optional, nbr doubles
};

// Stage an nbr x nbr column-major matrix (leading dim kNB) from global
// memory into LDS (row-major), zero outside nbr.
__device__ __forceinline__ void hr_stage(double (*S)[kNB + 1], const double* G, int nbr) {
  // All 16 loads of a thread first (the slot is always in bounds), masked
  // afterwards, so that they are in flight together.
  double g[kTS / 256];
#pragma unroll
  for (int e = 0; e < kTS / 256; ++e) g[e] = G[threadIdx.x + 256 * e];
#pragma unroll
  for (int e = 0; e < kTS / 256; ++e) {
    const int i = threadIdx.x + 256 * e, r = i % kNB, cc = i / kNB;
    S[r][cc] = (r < nbr && cc < nbr) ? g[e] : 0.0;
  }
}

// C = A B for 64 x 64 matrices in LDS on FP64 MFMA; wave w computes rows
// [16 w, 16 w + 16).  C must not alias A or B.  TB: read B transposed.
template <bool TB>
__device__ __forceinline__ void hr_mm(double (*C)[kNB + 1], double (*A)[kNB + 1],
                                      double (*B)[kNB + 1]) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = l >> 4;
  d4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const double af = A[16 * w + li][4 * kk + lk];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const double bf = TB ? B[16 * ct + li][4 * kk + lk] : B[4 * kk + lk][16 * ct + li];
      acc[ct] = mfma64(af, bf, acc[ct]);
    }
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) C[16 * w + lk + 4 * r][16 * ct + li] = acc[ct][r];
}

// Every lane of a quad receives lane q's value (quad_perm [q, q, q, q]); q is
// a constant after unrolling.
__device__ __forceinline__ double quad_bcast(double v, int q) {
  switch (q) {
    case 0: return dpp_mov<0x00>(v);
    case 1: return dpp_mov<0x55>(v);
    case 2: return dpp_mov<0xAA>(v);
    default: return dpp_mov<0xFF>(v);
  }
}

// Sign-modified LU without pivoting (App. C.2) of the 64 x 64 X whose rows
// sit in registers: thread (i, p) holds row i's columns p + 4 (s + m) in
// xr[s] during outer step m, and row i of the running L^{-1} (columns p + 4 s)
// in er[s].  Step J = 4 m + q: before eliminating column J, S_JJ = sgn(X^_JJ)
// (+1 for >= 0) and X^_JJ += S_JJ; the pivot row goes to Rb (double-buffered
// by step parity) and every lower row subtracts its multiple.  After the four
// steps of an outer step, column 4 m + p is final in every row: it is stored
// to Xm and the registers shift down one slot, so the pivot column is always
// slot 0 and no register index depends on the step (a loop of 16 outer steps
// instead of 64 unrolled ones).  Row J of L^{-1} is zero right of column J,
// so its update needs no mask.
__device__ __forceinline__ void hr_lu(double (&xr)[16], double (&er)[16], int i, int p, int nbr,
                                      double (*Rb)[2][4][16], double* Sv, double* Ui,
                                      double (*Xm)[kNB + 1]) {
  for (int m = 0; m < 16; ++m) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int J = 4 * m + q;
      if (J < nbr) {
        const int slot = q & 1;
        if (i == J) {
          if (p == q) {
            const double sg = (xr[0] >= 0.0) ? 1.0 : -1.0;
            xr[0] += sg;
            Sv[J] = sg;
            Ui[J] = 1.0 / xr[0];
          }
#pragma unroll
          for (int t = 0; t < 16; t += 2) {
            *(double2*)&Rb[slot][0][p][t] = make_double2(xr[t], xr[t + 1]);
            *(double2*)&Rb[slot][1][p][t] = make_double2(er[t], er[t + 1]);
          }
        }
        __syncthreads();
        if (i > J && i < nbr) {
          // Multiplier l = X[i][J] / U_JJ, formed by the thread holding
          // column J and shared with the other three threads of the row.
          double l = (p == q) ? xr[0] * Ui[J] : 0.0;
          l = quad_bcast(l, q);
          if (p == q) xr[0] = l;
#pragma unroll
          for (int t = 0; t < 16; t += 2) {
            const double2 rx = *(const double2*)&Rb[slot][0][p][t];
            const double2 re = *(const double2*)&Rb[slot][1][p][t];
            // slot 0 holds column 4 m + p: updated only right of the pivot
            xr[t] -= ((t > 0 || p > q) ? l : 0.0) * rx.x;
            xr[t + 1] -= l * rx.y;
            er[t] -= l * re.x;
            er[t + 1] -= l * re.y;
          }
        }
      }
    }
    Xm[i][4 * m + p] = xr[0];
#pragma unroll
    for (int t = 0; t < 15; ++t) xr[t] = xr[t + 1];
    xr[15] = 0.0;
  }
}

// U^{-1} by backward elimination (U in the upper triangle of Xm): for J
// descending, rows above J lose U[i][J] / U_JJ times row J of the running
// inverse mr (thread (i, p): columns p + 4 s).  Row J of the running inverse
// is zero left of column J, so the update needs no mask; the rows are scaled
// by 1 / U_ii afterwards.
__device__ __forceinline__ void hr_uinv(double (&mr)[16], int i, int p, int nbr,
                                        double (*Rb)[2][4][16], const double* Ui,
                                        double (*Xm)[kNB + 1]) {
  for (int J = nbr - 1; J >= 1; --J) {
    const int slot = J & 1;
    if (i == J) {
#pragma unroll
      for (int t = 0; t < 16; t += 2)
        *(double2*)&Rb[slot][0][p][t] = make_double2(mr[t], mr[t + 1]);
    }
    __syncthreads();
    if (i < J) {
      const double f = Xm[i][J] * Ui[J];
#pragma unroll
      for (int t = 0; t < 16; t += 2) {
        const double2 rm = *(const double2*)&Rb[slot][0][p][t];
        mr[t] -= f * rm.x;
        mr[t + 1] -= f * rm.y;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_tsqr_hr(HRArgs a) {
  __shared__ double Bm[kNB][kNB + 1];
  __shared__ double Mm[kNB][kNB + 1];
  __shared__ double Xm[kNB][kNB + 1];
  __shared__ double Sm[kNB][kNB + 1];
  __shared__ double Sv[kNB], Dv[kNB], Ui[kNB];
  __shared__ __align__(16) double Rb[2][2][4][16];  // [slot][x / e][p][m]: the step's pivot row
  const int t = threadIdx.x;
  const int nbr = a.nbr;
  for (int i = t; i < kTS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    Bm[r][cc] = (r == cc && r < nbr) ? 1.0 : 0.0;
  }
  __syncthreads();
  // B <- B - T B for the T of every node on the path to leaf block 0 and for
  // the stacked steps of leaf chain 0, then M = Z B for leaf block 0.  Step
  // k's T (path(k)) is loaded into registers while step k - 1's product runs.
  const int b1c = min(a.chain_len[0], a.nblocks[0]);
  int nlev = 0;  // path nodes above the leaves
  for (int lev = a.L; lev >= 1; --lev) nlev += (min(a.chain_len[lev], a.nblocks[lev]) >= 2);
  const int np = nlev + (b1c - 1) + 1;
  auto path = [&](int k) -> const double* {
    if (k < nlev) {
      int seen = 0;
      for (int lev = a.L; lev >= 1; --lev)
        if (min(a.chain_len[lev], a.nblocks[lev]) >= 2 && seen++ == k) return a.T[lev];
    }
    if (k < np - 1) return a.T[0] + (int64_t)(b1c - 1 - (k - nlev)) * kTS;
    return a.T[0];  // leaf block 0: Z
  };
  double g[kTS / 256];
  auto load_t = [&](const double* G) {
#pragma unroll
    for (int e = 0; e < kTS / 256; ++e) g[e] = G[t + 256 * e];
  };
  auto stage_t = [&]() {
#pragma unroll
    for (int e = 0; e < kTS / 256; ++e) {
      const int i = t + 256 * e, r = i % kNB, cc = i / kNB;
      Sm[r][cc] = (r < nbr && cc < nbr) ? g[e] : 0.0;
    }
  };
  load_t(path(0));
  stage_t();
  __syncthreads();
  for (int k = 0; k < np; ++k) {
    if (k + 1 < np) load_t(path(k + 1));
    hr_mm<false>(Mm, Sm, Bm);
    __syncthreads();
    if (k + 1 == np) break;  // M = Z B of leaf block 0 stays in Mm
    stage_t();
    for (int i = t; i < kTS; i += 256) {
      const int r = i % kNB, cc = i / kNB;
      Bm[r][cc] -= Mm[r][cc];
    }
    __syncthreads();
  }
  // Leaf block 0 (local QR with basis V, stored Z = T V_top^T):
  // X = top rows of [B; 0] - V (Z B).
  {
    // V_top of leaf block 0, all loads in flight together (indices clamped
    // into the nbr x nbr corner, masked afterwards).
    double g[kTS / 256];
#pragma unroll
    for (int e = 0; e < kTS / 256; ++e) {
      const int i = t + 256 * e, r = min(i % kNB, nbr - 1), cc = min(i / kNB, nbr - 1);
      g[e] = a.A0[r + (int64_t)cc * a.lda];
    }
#pragma unroll
    for (int e = 0; e < kTS / 256; ++e) {
      const int i = t + 256 * e, r = i % kNB, cc = i / kNB;
      double v = 0.0;
      if (r < nbr && cc < nbr) v = (r > cc) ? g[e] : ((r == cc) ? 1.0 : 0.0);
      Sm[r][cc] = v;
    }
  }
  __syncthreads();
  hr_mm<false>(Xm, Sm, Mm);
  __syncthreads();
  for (int i = t; i < kTS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    Xm[r][cc] = (r < nbr && cc < nbr) ? Bm[r][cc] - Xm[r][cc] : 0.0;
    Bm[r][cc] = (r == cc) ? 1.0 : 0.0;  // becomes L^{-1}
    Mm[r][cc] = (r == cc) ? 1.0 : 0.0;  // becomes U^{-1}
  }
  __syncthreads();
  // Sign-modified LU without pivoting (App. C.2): before eliminating column j,
  // S_jj = sgn(X^_jj) (+1 for >= 0) and X^_jj += S_jj.  The row operations are
  // applied to the identity alongside, which therefore ends as L^{-1}; then
  // U^{-1} by backward elimination.  Thread (i, p) keeps row i's columns
  // p, p + 4, ... in registers (hr_lu, hr_uinv).
  {
    const int i = t >> 2, p = t & 3;
    double xr[16], er[16], mr[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int k = p + 4 * m;
      xr[m] = Xm[i][k];
      er[m] = (i == k) ? 1.0 : 0.0;
      mr[m] = (i == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    hr_lu(xr, er, i, p, nbr, Rb, Sv, Ui, Xm);  // X (L below, U on and above) to Xm
    __syncthreads();
    hr_uinv(mr, i, p, nbr, Rb, Ui, Xm);
    // L^{-1} in Bm, U^{-1} (rows scaled by 1/U_ii) in Mm.
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int k = p + 4 * m;
      Bm[i][k] = er[m];
      Mm[i][k] = (i < nbr) ? mr[m] * Ui[i] : mr[m];
    }
    __syncthreads();
  }
  // R = -S R_root, optional D = sign(diag R).
  if (t < nbr) {
    const double r = -Sv[t] * a.Rtop[t + t * kNB];
    const double d = (a.normalize && r < 0.0) ? -1.0 : 1.0;
    Dv[t] = d;
    if (a.sign) a.sign[t] = d;
  }
  __syncthreads();
  // T = U S L^{-T}: stage U S (upper) and multiply by L^{-1} transposed.
  for (int e = t; e < kTS; e += 256) {
    const int r = e % kNB, cc = e / kNB;
    Sm[r][cc] = (r <= cc && cc < nbr) ? Xm[r][cc] * Sv[cc] : 0.0;
  }
  __syncthreads();
  {
    const int w = t >> 6, l = t & 63, li = l & 15, lk = l >> 4;
    d4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = d4{0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < 16; ++kk) {
      const double af = Sm[16 * w + li][4 * kk + lk];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma64(af, Bm[16 * ct + li][4 * kk + lk], acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + lk + 4 * r, cc = 16 * ct + li;
        if (row < nbr && cc < nbr) a.Tp[row + cc * a.ldt] = (row <= cc) ? acc[ct][r] : 0.0;
      }
  }
  for (int e = t; e < kTS; e += 256) {
    const int r = e % kNB, cc = e / kNB;
    const double rt = a.Rtop[e];  // the slot is always in bounds
    double lr = 0.0;
    if (r < nbr && cc < nbr) lr = (r > cc) ? Xm[r][cc] : -Dv[r] * Sv[r] * rt;
    a.LR[e] = lr;
  }
  for (int e = t; e < kBS; e += 256) {
    const int r = e % kNB, cc = e / kNB;
    double v = 0.0;
    if (r < nbr && cc < a.nq) {
      if (cc < nbr) v = Mm[r][cc];
      else if (cc - nbr == r) v = -Sv[r] * Dv[r];
    }
    a.Broot[e] = v;
  }
}

struct DownArgs {
  const double* Bin;   // per chain (leaf) / node (tree) of this level
  double* Bout;        // tree levels: per child (= per chain of the level below)
  const double* T;     // leaf: per block; tree: per node
  const double* Y;     // tree levels: per node
  double* A;           // leaf level: panel (basis in, V out), leading dim lda
  int64_t lda, xrows;
  double* Q;           // leaf level, optional
  int64_t ldq;
  const double* LR;
  int nblocks, chain_len, nbr, nq;
};

// M = T B into Ms (T upper triangular from global, B in Bs); wave w computes
// rows [16w, 16w + 16) of M.  MFMA operand roles: A = T tile, B = B tile.
template <int NQM, int NW>
__device__ __forceinline__ void down_tb(const double* Tb, double (*Bs)[NQM + 4],
                                        double (*Ms)[NQM + 4], int nbr, int CT) {
  // NW waves: wave w computes row tile w % 4 of M and the column tiles of
  // part w / 4 (with 8 waves the columns are split in two).
  constexpr int NCP = NW / 4, CTP = NQM / 16 / NCP;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = l >> 4;
  const int rt = w & 3, cp = w >> 2;
  d4 acc[CTP];
#pragma unroll
  for (int c2 = 0; c2 < CTP; ++c2) acc[c2] = d4{0.0, 0.0, 0.0, 0.0};
  const int i = 16 * rt + li;
  // The wave's T values eight at a time (the slot is always in bounds),
  // masked afterwards: a predicated load per step would wait out a global
  // latency before each MFMA.
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double tv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) tv[e] = Tb[i + (4 * (8 * h + e) + lk) * kNB];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 4 * (8 * h + e) + lk;
      const double av = (i < nbr && k < nbr) ? tv[e] : 0.0;
#pragma unroll
      for (int c2 = 0; c2 < CTP; ++c2) {
        const int ct = cp * CTP + c2;
        if (ct < CT) acc[c2] = mfma64(av, Bs[k][16 * ct + li], acc[c2]);
      }
    }
  }
#pragma unroll
  for (int c2 = 0; c2 < CTP; ++c2) {
    const int ct = cp * CTP + c2;
    if (ct < CT)
#pragma unroll
      for (int r = 0; r < 4; ++r) Ms[16 * rt + lk + 4 * r][16 * ct + li] = acc[c2][r];
  }
}

// Rows of one leaf block (or one node's stacked children) receive
// -Y M (+ B on the top rows of a leaf chain's first block).
template <int RT, int NQM, bool LEAF, int NW>
__device__ __forceinline__ void down_emit(const DownArgs& a, double (*Bs)[NQM + 4],
                                          double (*Ms)[NQM + 4], const double* Yb, int64_t ldy,
                                          int rows, bool first, int64_t rstart, bool top_block,
                                          int b0, int CT) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = l >> 4;
  const int nbr = a.nbr, nq = a.nq;
  double yf[RT][16];
#pragma unroll
  for (int s = 0; s < RT; ++s) {
    const int row = 16 * (w + NW * s) + li;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 4 * kk + lk;
      double v = (row < rows && k < nbr) ? Yb[row + (int64_t)k * ldy] : 0.0;
      if (first && row <= k) v = (row == k && k < nbr) ? 1.0 : 0.0;
      yf[s][kk] = v;
    }
  }
  for (int ct0 = 0; ct0 < CT; ct0 += 2) {
    d4 acc[RT][2];
#pragma unroll
    for (int s = 0; s < RT; ++s) acc[s][0] = acc[s][1] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const double af = Ms[4 * kk + lk][16 * (ct0 + g) + li];
#pragma unroll
        for (int s = 0; s < RT; ++s) acc[s][g] = mfma64(af, yf[s][kk], acc[s][g]);
      }
    }
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int row = 16 * (w + NW * s) + li;
      if (row >= rows) continue;
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int cc = 16 * (ct0 + g) + lk + 4 * r;
          if (cc >= nq) continue;
          double v = -acc[s][g][r];
          if (first && row < nbr) v += Bs[row][cc];
          if (LEAF) {
            if (cc < nbr) {
              if (top_block && row < nbr) v = a.LR[row + cc * kNB];
              a.A[rstart + row + (int64_t)cc * a.lda] = v;
            } else if (a.Q) {
              a.Q[rstart + row + (int64_t)(cc - nbr) * a.ldq] = v;
            }
          } else {
            const int sidx = row / nbr, rr = row - sidx * nbr;
            a.Bout[(int64_t)(b0 + 1 + sidx) * kBS + rr + cc * kNB] = v;
          }
        }
    }
  }
}

// RT: 16-row tiles per wave (block height 16 NW RT); NQM: max columns of B;
// LEAF: emit the panel rows (else the children's B blocks); NW: waves per
// workgroup (the leaf launch uses 8, so that each wave holds half as many
// basis rows and the workgroup has twice the waves to hide its loads).
template <int RT, int NQM, bool LEAF, int NW>
__global__ __launch_bounds__(64 * NW) void k_chain_down(DownArgs a) {
  constexpr int BLD = NQM + 4;
  __shared__ __align__(16) double Bs[kNB][BLD];
  __shared__ __align__(16) double Ms[kNB][BLD];
  const int t = threadIdx.x;
  const int chain = blockIdx.x;
  const int b0 = chain * a.chain_len;
  const int b1 = min(b0 + a.chain_len, a.nblocks);
  const int nbr = a.nbr, nq = a.nq;
  const int CT = (nq + 15) >> 4;

  {
    // B of this chain / node, all loads in flight together (the slot holds
    // kNB x 2 kNB, so every index is in bounds), masked afterwards.
    constexpr int NE = kNB * NQM / (64 * NW);
    const double* bin = a.Bin + (int64_t)chain * kBS;
    double g[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) g[e] = bin[t + 64 * NW * e];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = t + 64 * NW * e, r = i % kNB, cc = i / kNB;
      Bs[r][cc] = (r < nbr && cc < nq) ? g[e] : 0.0;
      Ms[r][cc] = 0.0;
    }
  }
  __syncthreads();

  if constexpr (LEAF) {
    for (int b = b1 - 1; b >= b0; --b) {
      const bool first = b == b0;
      down_tb<NQM, NW>(a.T + (int64_t)b * kTS, Bs, Ms, nbr, CT);
      __syncthreads();
      if (!first)
        for (int i = t; i < kNB * NQM; i += 64 * NW) {
          const int r = i / NQM, cc = i % NQM;
          Bs[r][cc] -= Ms[r][cc];
        }
      const int64_t rstart = ((int64_t)b * a.xrows) / a.nblocks;
      const int rows = (int)((((int64_t)b + 1) * a.xrows) / a.nblocks - rstart);
      down_emit<RT, NQM, true, NW>(a, Bs, Ms, a.A + rstart, a.lda, rows, first, rstart, b == 0, b0, CT);
      __syncthreads();
    }
  } else {
    if (b1 - b0 >= 2) {
      down_tb<NQM, NW>(a.T + (int64_t)chain * kTS, Bs, Ms, nbr, CT);
      __syncthreads();
      down_emit<RT, NQM, false, NW>(a, Bs, Ms, a.Y + (int64_t)chain * kYS, kYL, (b1 - b0 - 1) * nbr, false,
                         0, false, b0, CT);
      __syncthreads();
    }
    // First child: B - M (M is zero when the node has a single child).
    for (int i = t; i < kBS; i += 64 * NW) {
      const int r = i % kNB, cc = i / kNB;
      a.Bout[(int64_t)b0 * kBS + i] = (r < nbr && cc < nq) ? Bs[r][cc] - Ms[r][cc] : 0.0;
    }
  }
}

// ---------------------------------------------------------------- host side

TsqrPlan tsqr_plan(int64_t rows, int nbr, int leaf_rows, int chain, int arity, double* ws) {
  TsqrPlan p;
  p.rows = rows;
  p.nbr = nbr;
  const TsqrGeom g = tsqr_geometry(rows, nbr, leaf_rows, chain, arity);
  p.leaf_rows = g.leaf_rows;
  int64_t off = 0;
  auto take = [&](int64_t n) {
    double* ptr = ws ? ws + off : nullptr;
    off += (n + 31) & ~int64_t(31);
    return ptr;
  };
  TsqrLevel l0;
  l0.nblocks = (int)g.blocks;
  l0.chain_len = g.chain;
  l0.nchains = (int)g.chains;
  p.levels.push_back(l0);
  for (int l = 0; l < g.levels; ++l) {
    TsqrLevel lv;
    lv.nblocks = p.levels.back().nchains;
    lv.chain_len = g.arity;
    lv.nchains = (lv.nblocks + g.arity - 1) / g.arity;
    p.levels.push_back(lv);
  }
  for (size_t i = 0; i < p.levels.size(); ++i) {
    TsqrLevel& lv = p.levels[i];
    if (i == 0) {
      lv.T = take((int64_t)lv.nblocks * kTS);
    } else {
      lv.T = take((int64_t)lv.nchains * kTS);
      lv.Y = take((int64_t)lv.nchains * kYS);
    }
    lv.R = take((int64_t)lv.nchains * kTS);
    lv.B = take((int64_t)lv.nchains * kBS);
  }
  p.LR = take(kTS);
  p.workspace_doubles = off;
  return p;
}

hipError_t tsqr_factor(const TsqrPlan& p, hipStream_t s, double* P, int64_t ldp, double* Tp,
                       int64_t ldt, double* Q, int64_t ldq, int normalize, double* sign) {
  const int nbr = p.nbr;
  const int L = (int)p.levels.size() - 1;
  const double tri = 8.0 * nbr * (nbr + 1) / 2.0;  // bytes of one packed triangle
  const double pan = 8.0 * (double)p.rows * nbr;     // bytes of the panel
  // Upsweep.
  {
    const TsqrLevel& l0 = p.levels[0];
    ChainQRArgs a{P, ldp, p.rows, l0.nblocks, l0.chain_len, nbr, nullptr, l0.T, l0.R};
    // Read A, write V; write T per block and R per chain.  Flops: QR 2 m nb^2
    // plus the Gram products for T, m nb^2.  First blocks and the rest of
    // each chain are separate launches; the byte and flop counts are split
    // by the share of rows.
    const double f1 = (double)l0.nchains / l0.nblocks;
    {
      TimedLaunch tl(s, "tsqr_chain_qr_leaf", 2.0 * pan * f1 + tri * 2.0 * l0.nchains,
                     3.0 * (double)p.rows * nbr * nbr * f1);
      if (p.leaf_rows == 256)
        hipLaunchKernelGGL((k_chain_qr<256, true, 1>), dim3(l0.nchains), dim3(512), 0, s, a);
      else
        hipLaunchKernelGGL((k_chain_qr<128, true, 1>), dim3(l0.nchains), dim3(512), 0, s, a);
    }
    if (l0.chain_len > 1) {
      TimedLaunch tl(s, "tsqr_chain_qr_leaf_rest",
                     2.0 * pan * (1.0 - f1) + tri * (l0.nblocks - l0.nchains + 2.0 * l0.nchains),
                     3.0 * (double)p.rows * nbr * nbr * (1.0 - f1));
      if (p.leaf_rows == 256)
        hipLaunchKernelGGL((k_chain_qr_rest<256>), dim3(l0.nchains), dim3(512), 0, s, a);
      else
        hipLaunchKernelGGL((k_chain_qr_rest<128>), dim3(l0.nchains), dim3(512), 0, s, a);
    }
  }
  for (int lev = 1; lev <= L; ++lev) {
    const TsqrLevel& lv = p.levels[lev];
    ChainQRArgs a{p.levels[lev - 1].R, kNB, 0, lv.nblocks, lv.chain_len, nbr, lv.Y, lv.T, lv.R};
    TimedLaunch tl(s, "tsqr_chain_qr_tree", tri * (2.0 * lv.nblocks + 3.0 * lv.nchains),
                   3.0 * (double)lv.nblocks * nbr * nbr * nbr);
    // A node stacks (arity - 1) child R factors; the kernel's register
    // layout is sized to that height.
    const int stacked = (lv.chain_len - 1) * nbr;
    if (stacked <= 64)
      hipLaunchKernelGGL((k_chain_qr<64, false, 0>), dim3(lv.nchains), dim3(512), 0, s, a);
    else if (stacked <= 128)
      hipLaunchKernelGGL((k_chain_qr<128, false, 0>), dim3(lv.nchains), dim3(512), 0, s, a);
    else
      hipLaunchKernelGGL((k_chain_qr<kYL, false, 0>), dim3(lv.nchains), dim3(512), 0, s, a);
  }
  // Householder reconstruction at the root.
  const int nq = Q ? 2 * nbr : nbr;
  {
    HRArgs h{};
    h.L = L;
    for (int lev = 0; lev <= L; ++lev) {
      h.T[lev] = p.levels[lev].T;
      h.nblocks[lev] = p.levels[lev].nblocks;
      h.chain_len[lev] = p.levels[lev].chain_len;
    }
    h.Rtop = p.levels[L].R;
    h.A0 = P;
    h.lda = ldp;
    h.nbr = nbr;
    h.nq = nq;
    h.normalize = normalize;
    h.Tp = Tp;
    h.ldt = ldt;
    h.LR = p.LR;
    h.Broot = p.levels[L].B;
    h.sign = sign;
    TimedLaunch tl(s, "tsqr_hr_root", tri * 8.0, 6.0 * (double)nbr * nbr * nbr * (L + 2));
    hipLaunchKernelGGL(k_tsqr_hr, dim3(1), dim3(256), 0, s, h);
  }
  // Downsweep through the tree levels, then the leaves.
  for (int lev = L; lev >= 1; --lev) {
    const TsqrLevel& lv = p.levels[lev];
    DownArgs d{};
    d.Bin = lv.B;
    d.Bout = p.levels[lev - 1].B;
    d.T = lv.T;
    d.Y = lv.Y;
    d.nblocks = lv.nblocks;
    d.chain_len = lv.chain_len;
    d.nbr = nbr;
    d.nq = nq;
    TimedLaunch tl(s, "tsqr_down_tree", 8.0 * nbr * nq * 2.0 * lv.nblocks + tri * 2.0 * lv.nblocks,
                   3.0 * (double)lv.nblocks * nbr * nbr * nq);
    const int stacked = (lv.chain_len - 1) * nbr;  // rows of -Y M per node
    if (stacked <= 64) {
      if (nq > kNB)
        hipLaunchKernelGGL((k_chain_down<1, 128, false, 4>), dim3(lv.nchains), dim3(256), 0, s, d);
      else
        hipLaunchKernelGGL((k_chain_down<1, 64, false, 4>), dim3(lv.nchains), dim3(256), 0, s, d);
    } else {
      if (nq > kNB)
        hipLaunchKernelGGL((k_chain_down<4, 128, false, 4>), dim3(lv.nchains), dim3(256), 0, s, d);
      else
        hipLaunchKernelGGL((k_chain_down<4, 64, false, 4>), dim3(lv.nchains), dim3(256), 0, s, d);
    }
  }
  {
    const TsqrLevel& l0 = p.levels[0];
    DownArgs d{};
    d.Bin = l0.B;
    d.T = l0.T;
    d.A = P;
    d.lda = ldp;
    d.xrows = p.rows;
    d.Q = Q;
    d.ldq = ldq;
    d.LR = p.LR;
    d.nblocks = l0.nblocks;
    d.chain_len = l0.chain_len;
    d.nbr = nbr;
    d.nq = nq;
    // Read the basis, write V (and Q); T per block.  Flops: 2 m nb nq for
    // -Y M plus nb^2 nq per block for M = T B.
    TimedLaunch tl(s, "tsqr_down_leaf", pan * (Q ? 3.0 : 2.0) + tri * l0.nblocks,
                   2.0 * (double)p.rows * nbr * nq + (double)l0.nblocks * nbr * nbr * nq);
    if (p.leaf_rows == 256) {
      if (nq > kNB)
        hipLaunchKernelGGL((k_chain_down<4, 128, true, 4>), dim3(l0.nchains), dim3(256), 0, s, d);
      else
        hipLaunchKernelGGL((k_chain_down<2, 64, true, 8>), dim3(l0.nchains), dim3(512), 0, s, d);
    } else {
      if (nq > kNB)
        hipLaunchKernelGGL((k_chain_down<2, 128, true, 4>), dim3(l0.nchains), dim3(256), 0, s, d);
      else
        hipLaunchKernelGGL((k_chain_down<1, 64, true, 8>), dim3(l0.nchains), dim3(512), 0, s, d);
    }
  }
  return hipGetLastError();
}

}  // namespace miqr
