// TSQR panel factorisation for gfx950 (App. C of the paper: upsweep,
// downsweep, Householder reconstruction; base case of 1D-CAQR-EG, Sec. 6.1).
//
// Reduction structure.  The panel's rows are split evenly into leaf blocks of
// at most 128 or 256 rows (at least nbr rows each).  A workgroup reduces a
// *chain* of consecutive blocks in sequence.  A leaf chain starts with the
// local Householder QR of its first block (App. C.1); a tree chain starts from
// its first child's R.  Every further step factors the stacked matrix [R; X_s]
// with the next block X_s,
//     [R; X_s] = Q_s [R_new; 0],   Q_s = I - [I; Y_s] T_s [I; Y_s]^T,
// which is the paper's local QR of stacked R factors (App. C.1) with the
// block structure of the stacked triangle exploited: the reflector for column
// j touches only row j of R and the rows of X_s.  The R factors of one level's
// chains are the blocks of the next level, until one chain remains (a tree of
// arity `arity` above chains of `chain` leaves; the paper's binomial tree is
// arity 2 with chain 1).
//
// Downsweep (App. C.2).  Starting from B at the root, each chain is walked
// backwards: M = T_s B, block s receives -Y_s M, and B <- B - M; the first
// child of a tree chain receives the remaining B, the first block of a leaf
// chain receives [B; 0] - V M with M = Z B, Z = T V_top^T stored by the
// factorisation.  Started from B = I this yields W, the leading columns of the
// Q-factor.
//
// Householder reconstruction (App. C.2).  The root workgroup follows the path
// to leaf block 0 only, forms X (top rows of W), runs the sign-modified LU
// X + S = L U, and returns T = U S L^{-T}, R = -S R_root, and U^{-1}.  The
// downsweep proper then starts from [U^{-1}, -S D] so that one pass over the
// leaves yields V = W U^{-1} and, optionally, the thin Q = -W S D (App. C.2's
// remark that starting from U^{-1} saves the second broadcast).  The top rows
// of V are L (written from the reconstruction), R replaces them above the
// diagonal.
#include <algorithm>

#include "common.h"
#include "tsqr.h"

namespace miqr {

struct ChainQRArgs {
  double* X;        // leaf level: panel (in place); tree level: child R array
  int64_t ldx;
  int64_t xrows;    // leaf level: panel rows
  int nblocks, chain_len, nbr, leaf;
  double* Y;        // tree levels: Y per block
  double* T;        // per block
  double* R;        // per chain
};

// Thread layout: t = 4 c + q.  Thread (c, q) holds column c of the current
// block for rows r(e) = 8 (e / 2) + 2 q + (e % 2), e < RPT (4 RPT rows).
template <int RPT>
__global__ __launch_bounds__(256) void k_chain_qr(ChainQRArgs a) {
  constexpr int H = 4 * RPT;
  const int t = threadIdx.x, c = t >> 2, q = t & 3;
  const int chain = blockIdx.x;
  const int b0 = chain * a.chain_len;
  const int b1 = min(b0 + a.chain_len, a.nblocks);
  const int nbr = a.nbr;
  __shared__ double Rs[kNB][kNB + 1];
  __shared__ double Gs[kNB][kNB + 1];  // Gram entries y_c . y_j, then T in place
  __shared__ __align__(16) double vbuf[2][H];
  __shared__ double taus[kNB];

  for (int i = t; i < kTS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    double v = 0.0;
    if (!a.leaf && r < nbr && cc < nbr) v = a.X[(int64_t)b0 * kTS + i];
    Rs[r][cc] = v;
  }
  __syncthreads();

  double x[RPT];
  for (int b = a.leaf ? b0 : b0 + 1; b < b1; ++b) {
    int64_t rstart = 0;
    int rows;
    double* src;
    int64_t ld;
    if (a.leaf) {
      rstart = ((int64_t)b * a.xrows) / a.nblocks;
      rows = (int)((((int64_t)b + 1) * a.xrows) / a.nblocks - rstart);
      src = a.X + rstart;
      ld = a.ldx;
    } else {
      rows = nbr;
      src = a.X + (int64_t)b * kTS;
      ld = kNB;
    }
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
      const int r = 8 * (e >> 1) + 2 * q + (e & 1);
      x[e] = (c < nbr && r < rows) ? src[r + (int64_t)c * ld] : 0.0;
    }

    // The first block of a leaf chain is a plain Householder QR of its own rows
    // (the paper's local QR, App. C.1): reflector j pivots on row j of the
    // block and leaves the rows above it (R) alone.  Later blocks are stacked
    // under the running R.
    const bool first = a.leaf && b == b0;
    for (int j = 0; j < nbr; ++j) {
      double* vb = vbuf[j & 1];
      if (c == j) {
        double ss = 0.0, alpha;
        if (first) {
          double av = 0.0;
#pragma unroll
          for (int e = 0; e < RPT; ++e) {
            const int r = 8 * (e >> 1) + 2 * q + (e & 1);
            if (r > j) ss += x[e] * x[e];
            if (r == j) av = x[e];
          }
          ss = quad_sum(ss);
          alpha = quad_sum(av);
        } else {
#pragma unroll
          for (int e = 0; e < RPT; ++e) ss += x[e] * x[e];
          ss = quad_sum(ss);
          alpha = Rs[j][j];
        }
        double beta = alpha, tau = 0.0, scale = 1.0;
        if (ss != 0.0) {
          const double nrm = sqrt(alpha * alpha + ss);
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        if (first) {
#pragma unroll
          for (int e = 0; e < RPT; e += 2) {
            double v[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int r = 8 * (e >> 1) + 2 * q + u;
              if (r > j) {
                x[e + u] *= scale;
                v[u] = x[e + u];
              } else if (r == j) {
                x[e + u] = beta;
                v[u] = 1.0;
              } else {
                v[u] = 0.0;
              }
            }
            *(double2*)&vb[8 * (e >> 1) + 2 * q] = make_double2(v[0], v[1]);
          }
          if (q == 0) taus[j] = tau;
        } else {
#pragma unroll
          for (int e = 0; e < RPT; e += 2) {
            x[e] *= scale;
            x[e + 1] *= scale;
            *(double2*)&vb[8 * (e >> 1) + 2 * q] = make_double2(x[e], x[e + 1]);
          }
          if (q == 0) {
            Rs[j][j] = beta;
            taus[j] = tau;
          }
        }
      }
      __syncthreads();
      if (c < nbr && c != j) {
        double d = 0.0;
#pragma unroll
        for (int e = 0; e < RPT; e += 2) {
          const double2 v = *(const double2*)&vb[8 * (e >> 1) + 2 * q];
          d += v.x * x[e] + v.y * x[e + 1];
        }
        d = quad_sum(d);
        if (c > j) {
          const double w = taus[j] * (first ? d : d + Rs[j][c]);
#pragma unroll
          for (int e = 0; e < RPT; e += 2) {
            const double2 v = *(const double2*)&vb[8 * (e >> 1) + 2 * q];
            x[e] -= v.x * w;
            x[e + 1] -= v.y * w;
          }
          if (q == 0 && !first) Rs[j][c] -= w;
        } else if (q == 0) {
          Gs[c][j] = d;  // v_c . v_j for c < j
        }
      }
    }
    __syncthreads();

    // T_s from the Gram entries, column by column over G's upper triangle:
    // T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j], T_jj = tau_j.
    for (int j = 0; j < nbr; ++j) {
      const int i = t >> 2, p = t & 3;
      double s = 0.0;
      if (i < j) {
        for (int k = i + p; k < j; k += 4) s += Gs[i][k] * Gs[k][j];
        s = quad_sum(s);
      }
      __syncthreads();
      if (p == 0) {
        if (i < j) Gs[i][j] = -taus[j] * s;
        else if (i == j) Gs[j][j] = taus[j];
      }
      __syncthreads();
    }

    double* ydst;
    int64_t ldy;
    if (a.leaf) {
      ydst = src;
      ldy = ld;
    } else {
      ydst = a.Y + (int64_t)b * kTS;
      ldy = kNB;
    }
    if (c < nbr) {
#pragma unroll
      for (int e = 0; e < RPT; ++e) {
        const int r = 8 * (e >> 1) + 2 * q + (e & 1);
        if (r < rows) ydst[r + (int64_t)c * ldy] = x[e];
      }
    }
    if (!first) {
      for (int i = t; i < kTS; i += 256) {
        const int r = i % kNB, cc = i / kNB;
        a.T[(int64_t)b * kTS + i] = (r <= cc && cc < nbr) ? Gs[r][cc] : 0.0;
      }
    } else {
      // Store Z = T V_top^T (upper triangular) in place of T, V_top the unit
      // lower top nbr x nbr part of the block's V, so that the downsweep and
      // the reconstruction apply this block as M = Z B, out = [B; 0] - V M.
      // Rs (unused by the first block) holds V_top row-major for the product.
#pragma unroll
      for (int e = 0; e < RPT; ++e) {
        const int r = 8 * (e >> 1) + 2 * q + (e & 1);
        if (r < kNB && c < kNB) Rs[r][c] = (r > c) ? x[e] : ((r == c) ? 1.0 : 0.0);
      }
      __syncthreads();
      for (int i = t; i < kTS; i += 256) {
        const int r = i % kNB, cc = i / kNB;
        double z = 0.0;
        if (r <= cc && cc < nbr)
          for (int k = r; k <= cc; ++k) z += Gs[r][k] * Rs[cc][k];
        a.T[(int64_t)b * kTS + i] = z;
      }
      __syncthreads();
      // The block's R (upper triangle of its top rows) seeds the chain.
#pragma unroll
      for (int e = 0; e < RPT; ++e) {
        const int r = 8 * (e >> 1) + 2 * q + (e & 1);
        if (r < kNB && c < kNB) Rs[r][c] = (r <= c && c < nbr) ? x[e] : 0.0;
      }
    }
    __syncthreads();
  }

  for (int i = t; i < kTS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    a.R[(int64_t)chain * kTS + i] = (r <= cc && cc < nbr) ? Rs[r][cc] : 0.0;
  }
}

struct HRArgs {
  int L;  // number of tree levels above the leaves
  const double* T[kMaxLevels];
  int nblocks[kMaxLevels];
  int chain_len[kMaxLevels];
  const double* Rtop;    // R of the single chain of the top level
  const double* A0;      // leaf block 0 (its Y, in place), leading dim lda
  int64_t lda;
  int nbr, nq, normalize;
  double* Tp;            // nbr x nbr kernel, leading dim ldt
  int64_t ldt;
  double* LR;            // kTS: strict lower L, upper R
  double* Broot;         // kBS: downsweep input of the top chain
  double* sign;          // optional, nbr doubles
};

// C = A_glob (upper triangular, column-major, ld kNB) * B  (nbr x nbr), all in LDS except A.
__device__ void hr_tri_mul(double (*C)[kNB + 1], const double* A, double (*B)[kNB + 1], int nbr) {
  const int t = threadIdx.x;
  const int cc = t & 63, i0 = (t >> 6) * 16;
  for (int i = i0; i < i0 + 16; ++i) {
    double s = 0.0;
    if (i < nbr && cc < nbr)
      for (int k = i; k < nbr; ++k) s += A[i + k * kNB] * B[k][cc];
    C[i][cc] = s;
  }
}

__global__ __launch_bounds__(256) void k_tsqr_hr(HRArgs a) {
  __shared__ double Bm[kNB][kNB + 1];
  __shared__ double Mm[kNB][kNB + 1];
  __shared__ double Xm[kNB][kNB + 1];
  __shared__ double Sv[kNB], Dv[kNB];
  const int t = threadIdx.x;
  const int nbr = a.nbr;
  for (int i = t; i < kTS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    Bm[r][cc] = (r == cc && r < nbr) ? 1.0 : 0.0;
  }
  __syncthreads();
  // Walk the path from the root to leaf block 0 (child 0 of every chain 0).
  for (int lev = a.L; lev >= 0; --lev) {
    const int b1 = min(a.chain_len[lev], a.nblocks[lev]);
    const double* T = a.T[lev];
    for (int b = b1 - 1; b >= 1; --b) {
      hr_tri_mul(Mm, T + (int64_t)b * kTS, Bm, nbr);
      __syncthreads();
      for (int i = t; i < kTS; i += 256) {
        const int r = i % kNB, cc = i / kNB;
        Bm[r][cc] -= Mm[r][cc];
      }
      __syncthreads();
    }
  }
  // Leaf block 0 (a local QR with basis V and stored Z = T V_top^T):
  // X = top rows of [B; 0] - V (Z B).
  hr_tri_mul(Mm, a.T[0], Bm, nbr);
  __syncthreads();
  {
    const int cc = t & 63, i0 = (t >> 6) * 16;
    for (int i = i0; i < i0 + 16; ++i) {
      double s = 0.0;
      if (i < nbr && cc < nbr) {
        for (int k = 0; k < i; ++k) s += a.A0[i + (int64_t)k * a.lda] * Mm[k][cc];
        s += Mm[i][cc];
      }
      Xm[i][cc] = (i < nbr && cc < nbr) ? Bm[i][cc] - s : 0.0;
    }
  }
  __syncthreads();
  // Sign-modified LU without pivoting: S_jj = sgn(X^_jj) (+1 for >= 0), X^_jj += S_jj.
  for (int j = 0; j < nbr; ++j) {
    if (t == 0) {
      const double s = (Xm[j][j] >= 0.0) ? 1.0 : -1.0;
      Sv[j] = s;
      Xm[j][j] += s;
    }
    __syncthreads();
    const int i = t >> 2, p = t & 3;
    if (i > j && i < nbr) {
      const double l = Xm[i][j] / Xm[j][j];
      for (int k = j + 1 + p; k < nbr; k += 4) Xm[i][k] -= l * Xm[j][k];
      if (p == 0) Xm[i][j] = l;
    }
    __syncthreads();
  }
  // Bm <- L^{-1} (unit lower), Mm <- U^{-1} (upper).
  for (int i = t; i < kTS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    Bm[r][cc] = (r == cc) ? 1.0 : 0.0;
    Mm[r][cc] = (r == cc && r < nbr) ? 1.0 / Xm[r][r] : 0.0;
  }
  __syncthreads();
  for (int s = 1; s < nbr; ++s) {
    const int cc = t >> 2, p = t & 3;
    const int il = s;             // L^{-1} row il, columns cc < il
    if (cc < il) {
      double acc = 0.0;
      for (int k = cc + p; k < il; k += 4) acc += Xm[il][k] * Bm[k][cc];
      acc = quad_sum(acc);
      if (p == 0) Bm[il][cc] = -acc;
    }
    const int iu = nbr - 1 - s;   // U^{-1} row iu, columns iu < cc < nbr
    if (cc > iu && cc < nbr) {
      double acc = 0.0;
      for (int k = iu + 1 + p; k <= cc; k += 4) acc += Xm[iu][k] * Mm[k][cc];
      acc = quad_sum(acc);
      if (p == 0) Mm[iu][cc] = -acc / Xm[iu][iu];
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
  for (int i = t; i < kTS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    double lr = 0.0, tv = 0.0;
    if (r < nbr && cc < nbr) {
      if (r > cc) {
        lr = Xm[r][cc];
      } else {
        lr = -Dv[r] * Sv[r] * a.Rtop[r + cc * kNB];
        // T = U S L^{-T}: T[r][cc] = sum_{k=r..cc} U[r][k] S_k Linv[cc][k]
        for (int k = r; k <= cc; ++k) tv += Xm[r][k] * Sv[k] * Bm[cc][k];
      }
      a.Tp[r + cc * a.ldt] = tv;
    }
    a.LR[i] = lr;
  }
  for (int i = t; i < kBS; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    double v = 0.0;
    if (r < nbr && cc < a.nq) {
      if (cc < nbr) v = Mm[r][cc];
      else if (cc - nbr == r) v = -Sv[r] * Dv[r];
    }
    a.Broot[i] = v;
  }
}

struct DownArgs {
  const double* Bin;   // per chain of this level
  double* Bout;        // tree levels: per block (= per chain of the level below)
  const double* T;     // per block
  const double* Y;     // tree levels: per block
  double* A;           // leaf level: panel (Y in, V out), leading dim lda
  int64_t lda, xrows;
  double* Q;           // leaf level, optional
  int64_t ldq;
  const double* LR;
  int nblocks, chain_len, nbr, nq, leaf;
};

// RT: 16-row tiles per wave (block height 64 RT); NQM: max columns of B.
template <int RT, int NQM>
__global__ __launch_bounds__(256) void k_chain_down(DownArgs a) {
  constexpr int BLD = NQM + 4;
  constexpr int CTM = NQM / 16;
  __shared__ __align__(16) double Bs[kNB][BLD];
  __shared__ __align__(16) double Ms[kNB][BLD];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int li = l & 15, lk = l >> 4;
  const int chain = blockIdx.x;
  const int b0 = chain * a.chain_len;
  const int b1 = min(b0 + a.chain_len, a.nblocks);
  const int nbr = a.nbr, nq = a.nq;
  const int CT = (nq + 15) >> 4;

  for (int i = t; i < kNB * NQM; i += 256) {
    const int r = i % kNB, cc = i / kNB;
    Bs[r][cc] = (r < nbr && cc < nq) ? a.Bin[(int64_t)chain * kBS + r + cc * kNB] : 0.0;
    Ms[r][cc] = 0.0;
  }
  __syncthreads();

  const int bfirst = a.leaf ? b0 : b0 + 1;
  for (int b = b1 - 1; b >= bfirst; --b) {
    const bool first = a.leaf && b == b0;
    // M = T_b B (Z_b B for a leaf chain's first block): wave w computes rows
    // [16w, 16w + 16).
    {
      const double* Tb = a.T + (int64_t)b * kTS;
      d4 acc[CTM];
#pragma unroll
      for (int ct = 0; ct < CTM; ++ct) acc[ct] = d4{0.0, 0.0, 0.0, 0.0};
      const int i = 16 * w + li;
      for (int kk = 4 * w; kk < 16; ++kk) {
        const int k = 4 * kk + lk;
        const double av = (i < nbr && k < nbr) ? Tb[i + k * kNB] : 0.0;
#pragma unroll
        for (int ct = 0; ct < CTM; ++ct)
          if (ct < CT) acc[ct] = mfma64(av, Bs[k][16 * ct + li], acc[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < CTM; ++ct)
        if (ct < CT)
#pragma unroll
          for (int r = 0; r < 4; ++r) Ms[16 * w + lk + 4 * r][16 * ct + li] = acc[ct][r];
    }
    __syncthreads();
    if (!first)
      for (int i = t; i < kNB * NQM; i += 256) {
        const int r = i / NQM, cc = i % NQM;
        Bs[r][cc] -= Ms[r][cc];
      }
    // Block b receives -Y_b M.
    {
      int64_t rstart = 0;
      int rows;
      const double* Yb;
      int64_t ldy;
      if (a.leaf) {
        rstart = ((int64_t)b * a.xrows) / a.nblocks;
        rows = (int)((((int64_t)b + 1) * a.xrows) / a.nblocks - rstart);
        Yb = a.A + rstart;
        ldy = a.lda;
      } else {
        rows = nbr;
        Yb = a.Y + (int64_t)b * kTS;
        ldy = kNB;
      }
      double yf[RT][16];
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int row = 16 * (w + 4 * s) + li;
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
          const int row = 16 * (w + 4 * s) + li;
          if (row >= rows) continue;
#pragma unroll
          for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int cc = 16 * (ct0 + g) + lk + 4 * r;
              if (cc >= nq) continue;
              double v = -acc[s][g][r];
              if (first && row < nbr) v += Bs[row][cc];
              if (a.leaf) {
                if (cc < nbr) {
                  if (b == 0 && row < nbr) v = a.LR[row + cc * kNB];
                  a.A[rstart + row + (int64_t)cc * a.lda] = v;
                } else if (a.Q) {
                  a.Q[rstart + row + (int64_t)(cc - nbr) * a.ldq] = v;
                }
              } else {
                a.Bout[(int64_t)b * kBS + row + cc * kNB] = v;
              }
            }
        }
      }
    }
    __syncthreads();
  }
  if (!a.leaf) {
    for (int i = t; i < kBS; i += 256) {
      const int r = i % kNB, cc = i / kNB;
      a.Bout[(int64_t)b0 * kBS + i] = (r < nbr && cc < nq) ? Bs[r][cc] : 0.0;
    }
  }
}

// ---------------------------------------------------------------- host side

TsqrPlan tsqr_plan(int64_t rows, int nbr, int leaf_rows, int chain, int arity, double* ws) {
  TsqrPlan p;
  p.rows = rows;
  p.nbr = nbr;
  if (leaf_rows != 128 && leaf_rows != 256) leaf_rows = (rows >= 256 * 1024) ? 256 : 128;
  p.leaf_rows = leaf_rows;
  const int64_t P0 = std::max<int64_t>(1, (rows + leaf_rows - 1) / leaf_rows);
  if (chain <= 0) chain = (int)std::max<int64_t>(1, std::min<int64_t>(8, P0 / 1024));
  if (arity < 2) arity = 2;
  int64_t off = 0;
  auto take = [&](int64_t n) {
    double* ptr = ws ? ws + off : nullptr;
    off += (n + 31) & ~int64_t(31);
    return ptr;
  };
  TsqrLevel l0;
  l0.nblocks = (int)P0;
  l0.chain_len = chain;
  l0.nchains = (int)((P0 + chain - 1) / chain);
  p.levels.push_back(l0);
  while (p.levels.back().nchains > 1 && (int)p.levels.size() < kMaxLevels) {
    TsqrLevel lv;
    lv.nblocks = p.levels.back().nchains;
    lv.chain_len = arity;
    lv.nchains = (lv.nblocks + arity - 1) / arity;
    p.levels.push_back(lv);
  }
  for (size_t i = 0; i < p.levels.size(); ++i) {
    TsqrLevel& lv = p.levels[i];
    lv.T = take((int64_t)lv.nblocks * kTS);
    if (i > 0) lv.Y = take((int64_t)lv.nblocks * kTS);
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
  // Upsweep.
  {
    const TsqrLevel& l0 = p.levels[0];
    ChainQRArgs a{P, ldp, p.rows, l0.nblocks, l0.chain_len, nbr, 1, nullptr, l0.T, l0.R};
    if (p.leaf_rows == 256)
      hipLaunchKernelGGL(k_chain_qr<64>, dim3(l0.nchains), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(k_chain_qr<32>, dim3(l0.nchains), dim3(256), 0, s, a);
  }
  for (int lev = 1; lev <= L; ++lev) {
    const TsqrLevel& lv = p.levels[lev];
    ChainQRArgs a{p.levels[lev - 1].R, kNB, 0, lv.nblocks, lv.chain_len, nbr, 0, lv.Y, lv.T, lv.R};
    hipLaunchKernelGGL(k_chain_qr<16>, dim3(lv.nchains), dim3(256), 0, s, a);
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
    d.leaf = 0;
    if (nq > kNB)
      hipLaunchKernelGGL((k_chain_down<1, 128>), dim3(lv.nchains), dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL((k_chain_down<1, 64>), dim3(lv.nchains), dim3(256), 0, s, d);
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
    d.leaf = 1;
    if (p.leaf_rows == 256) {
      if (nq > kNB)
        hipLaunchKernelGGL((k_chain_down<4, 128>), dim3(l0.nchains), dim3(256), 0, s, d);
      else
        hipLaunchKernelGGL((k_chain_down<4, 64>), dim3(l0.nchains), dim3(256), 0, s, d);
    } else {
      if (nq > kNB)
        hipLaunchKernelGGL((k_chain_down<2, 128>), dim3(l0.nchains), dim3(256), 0, s, d);
      else
        hipLaunchKernelGGL((k_chain_down<2, 64>), dim3(l0.nchains), dim3(256), 0, s, d);
    }
  }
  return hipGetLastError();
}

}  // namespace miqr
