// Accuracy-preserving local POD: the singular values come from a QR factor
// of the snapshot matrix instead of its Gram matrix, so the squared condition
// number of the method of snapshots (Rem. 2.3) never enters.
//
//   S = Q R                 Cholesky-QR passes, shifted (Fukaya, Kannan,
//                           Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci.
//                           Comput. 2020) while Q^T Q is far from I: the Gram,
//                           Cholesky and lift kernels of this library
//   R V = U_R diag(sigma)   one-sided Jacobi (Hestenes 1958) on R's columns,
//                           this file
//   modes = Q U_R           (scaled: Q U_R diag(sigma) = Q (R V))
//
// Kernels: the diagonal shift, the distance of a Gram matrix from I, the
// upper-triangle copy and the Jacobi SVD.

#include <algorithm>

#include "internal.hpp"

namespace hapod {
namespace {

constexpr int kOsjThreads = 1024;
constexpr int kOsjWaves = kOsjThreads / 64;
constexpr int kOsjMaxSweeps = 60;
constexpr int kOsjGroup = 16;                       // lanes per column pair
constexpr int kOsjGroups = kOsjThreads / kOsjGroup;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// G[k][k] += coef * trace(G)   (one workgroup)
__global__ __launch_bounds__(256) void shift_diag_kernel(double* G, int64_t ldg, int64_t m, double coef) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < m; k += 256) s += G[k * ldg + k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double shift = coef * (red[0] + red[1] + red[2] + red[3]);
  for (int64_t k = threadIdx.x; k < m; k += 256) G[k * ldg + k] += shift;
}

// out[0] = max_{i <= j} |G_ij - delta_ij|   (one workgroup)
__global__ __launch_bounds__(256) void identity_dev_kernel(const double* __restrict__ G, int64_t ldg, int64_t m,
                                                           double* out) {
  __shared__ double red[4];
  double d = 0.0;
  for (int64_t j = 0; j < m; ++j)
    for (int64_t i = threadIdx.x; i <= j; i += 256) d = fmax(d, fabs(G[j * ldg + i] - (i == j ? 1.0 : 0.0)));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Column equilibration and zero columns of a Gram matrix G = Q^T Q (upper
// triangle used).  zero[j] |= (G_jj == 0); with D: D_j = sqrt(G_jj) (1 for a
// zero column) and G <- D^-1 G D^-1; then every zero column's diagonal is
// set to 1, so that it factors as a unit column (its Q column stays zero).
__global__ __launch_bounds__(256) void gram_zero_scale_kernel(double* G, int64_t ldg, int64_t m, int32_t* zero,
                                                              double* D) {
  for (int64_t j = threadIdx.x; j < m; j += 256) {
    const double d = G[j * ldg + j];
    if (d == 0.0) zero[j] = 1;
    if (D) D[j] = d > 0.0 ? sqrt(d) : 1.0;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < m * m; e += 256) {
    const int64_t j = e / m, i = e - j * m;
    if (i > j) continue;
    double g = G[j * ldg + i];
    if (D) g = g / (D[i] * D[j]);
    if (i == j && zero[j]) g = 1.0;
    G[j * ldg + i] = g;
  }
}

// R (column-major, may be null) column j *= D_j; Rinv (row-major) row i *= 1 / D_i
__global__ void unscale_factors_kernel(double* R, int64_t ldr, double* Rinv, int64_t ldi, int64_t m,
                                       const double* D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int64_t j = e / m, i = e - j * m;
  if (R) R[j * ldr + i] *= D[j];
  Rinv[i * ldi + j] /= D[i];
}

// row j of R (column-major m x m) = 0 for every zero column j
__global__ void zero_rows_kernel(double* R, int64_t ldr, int64_t m, const int32_t* zero) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int64_t c = e / m, j = e - c * m;
  if (zero[j]) R[c * ldr + j] = 0.0;
}

// R = upper triangle of W (column-major), zeros below
__global__ void triu_kernel(const double* __restrict__ W, int64_t ldw, int64_t N, double* __restrict__ R, int64_t ldr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i < N) R[j * ldr + i] = (i <= j) ? W[j * ldw + i] : 0.0;
}

// The plane rotation [c s; -s c] that makes columns x, y (squared norms a,
// b, inner product g) orthogonal, the smaller angle (Golub & Van Loan): x <-
// c x - s y, y <- s x + c y, a <- a - t g, b <- b + t g.
__device__ __forceinline__ void jacobi_angle(double a, double b, double g, double& c, double& s, double& t) {
  const double zeta = (b - a) / (2.0 * g);
  t = fabs(zeta) > 1e150 ? 0.5 / zeta : (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  c = 1.0 / sqrt(1.0 + t * t);
  s = c * t;
}

// sigma_c = ||x_c||, sorted descending (equal values by index), and B
// (row-major, ld m) column p = x_c (scaled) or x_c / sigma_c, for the
// converged columns of X (m x m, ld m); one workgroup.
__device__ void osj_finish(const double* X, int64_t m, double* sigma, double* B, int scaled, double* sg, int32_t* pos) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int64_t c = wv; c < m; c += kOsjWaves) {
    double s = 0.0;
    for (int64_t k = lane; k < m; k += 64) s += X[c * m + k] * X[c * m + k];
    s = wave_sum(s);
    if (lane == 0) sg[c] = sqrt(s);
  }
  __syncthreads();
  for (int64_t c = t; c < m; c += kOsjThreads) {
    int32_t rk = 0;
    for (int64_t d = 0; d < m; ++d) rk += (sg[d] > sg[c] || (sg[d] == sg[c] && d < c)) ? 1 : 0;
    pos[c] = rk;
    sigma[rk] = sg[c];
  }
  __syncthreads();
  for (int64_t e = t; e < m * m; e += kOsjThreads) {
    const int64_t c = e / m, k = e - c * m;
    const double sc = scaled ? 1.0 : (sg[c] > 0.0 ? 1.0 / sg[c] : 0.0);
    B[k * m + pos[c]] = X[c * m + k] * sc;
  }
}

// One-sided Jacobi on the columns of X (m x m, column-major, ld m, m <= 128)
// in one workgroup with X in LDS: plane rotations on column pairs until every
// pair is orthogonal to m u of its norms; the pairs of a round are disjoint
// (round-robin order), a group of 16 lanes per pair (four pairs per
// wavefront at once), the squared norms carried across the rotations of a
// sweep.  Then osj_finish.  info: sweeps taken, or -1 without convergence.
__global__ __launch_bounds__(kOsjThreads) void osj_kernel(double* A, int64_t m, double* sigma, double* B, int scaled,
                                                          int32_t* info) {
  extern __shared__ double osj_lds[];
  __shared__ double sg[kQrMaxM];
  __shared__ int32_t pos[kQrMaxM];
  __shared__ double nrm[kQrMaxM];  // squared column norms, carried across rotations
  __shared__ int nrot;
  double* X = osj_lds;
  const int t = threadIdx.x;
  const int gl = t & (kOsjGroup - 1), grp = t / kOsjGroup;
  for (int64_t e = t; e < m * m; e += kOsjThreads) X[e] = A[e];
  const int mi = (int)m;
  const int mm = mi + (mi & 1);
  const double tol = (double)m * 1.1102230246251565e-16;
  int sweep = 0;
  bool done = false;
  for (; sweep < kOsjMaxSweeps && !done; ++sweep) {
    if (t == 0) nrot = 0;
    __syncthreads();
    // exact squared norms at the start of every sweep; within it a rotation
    // updates them (||x'||^2 = a - t g, ||y'||^2 = b + t g), so a pair needs
    // one dot product instead of three
    for (int64_t c = grp; c < m; c += kOsjGroups) {
      double q = 0.0;
      for (int64_t k = gl; k < m; k += kOsjGroup) q += X[c * m + k] * X[c * m + k];
#pragma unroll
      for (int off = kOsjGroup / 2; off > 0; off >>= 1) q += __shfl_xor(q, off, kOsjGroup);
      if (gl == 0) nrm[c] = q;
    }
    __syncthreads();
    for (int r = 0; r < mm - 1; ++r) {
      for (int p = grp; p < mm / 2; p += kOsjGroups) {
        int i, j;
        if (p == 0) {
          i = mm - 1;
          j = r;
        } else {
          i = r + p;
          if (i >= mm - 1) i -= mm - 1;
          j = r - p;
          if (j < 0) j += mm - 1;
        }
        if (i >= mi || j >= mi) continue;  // the padding index of an odd m
        double* ci = X + i * mi;
        double* cj = X + j * mi;
        const double a = nrm[i], b = nrm[j];
        double g = 0.0;
        for (int k = gl; k < mi; k += kOsjGroup) g += ci[k] * cj[k];
#pragma unroll
        for (int off = kOsjGroup / 2; off > 0; off >>= 1) g += __shfl_xor(g, off, kOsjGroup);
        if (!(a > 0.0) || !(b > 0.0) || fabs(g) <= tol * sqrt(a) * sqrt(b)) continue;
        double c, s, tt;
        jacobi_angle(a, b, g, c, s, tt);
        for (int k = gl; k < mi; k += kOsjGroup) {
          const double x = ci[k], y = cj[k];
          ci[k] = c * x - s * y;
          cj[k] = s * x + c * y;
        }
        if (gl == 0) {
          atomicAdd(&nrot, 1);
          nrm[i] = fmax(a - tt * g, 0.0);
          nrm[j] = b + tt * g;
        }
      }
      __syncthreads();
    }
    done = (nrot == 0);
    __syncthreads();
  }
  osj_finish(X, m, sigma, B, scaled, sg, pos);
  if (t == 0) info[0] = done ? sweep : -1;
}

// Block one-sided Jacobi (columns in blocks of kOsjBlk; a sweep visits every
// pair of blocks once in round-robin order): one launch per round, one
// workgroup per block pair of the round.  The workgroup loads its
// 2 kOsjBlk columns (m rows each) into LDS, computes their squared norms
// exactly, runs one cyclic sweep over them (2 kOsjBlk - 1 rounds of kOsjBlk
// disjoint pairs, one wavefront per pair, the norms carried across the
// rotations) and writes them back; the rotations it applied are added to
// *count.  Blocks past the last (odd block count) are skipped.
constexpr int kOsjBlk = 16;
__global__ __launch_bounds__(kOsjThreads) void osj_block_round_kernel(double* X, int m, int nbe, int r,
                                                                      int32_t* count) {
  extern __shared__ double osj_lds[];
  __shared__ double nrm[2 * kOsjBlk];
  __shared__ int nrot;
  const int nb1 = nbe - 1, p = blockIdx.x;
  int I, J;
  if (p == 0) {
    I = nb1;
    J = r;
  } else {
    I = r + p;
    if (I >= nb1) I -= nb1;
    J = r - p;
    if (J < 0) J += nb1;
  }
  const int nb = (m + kOsjBlk - 1) / kOsjBlk;
  if (I >= nb || J >= nb) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  constexpr int LC = 2 * kOsjBlk;
  double* L = osj_lds;
  // local column lc: block I's columns, then block J's; columns past m are zero
  for (int e = t; e < LC * m; e += kOsjThreads) {
    const int lc = e / m, k = e - lc * m;
    const int gc = lc < kOsjBlk ? I * kOsjBlk + lc : J * kOsjBlk + (lc - kOsjBlk);
    L[e] = gc < m ? X[(int64_t)gc * m + k] : 0.0;
  }
  if (t == 0) nrot = 0;
  __syncthreads();
  for (int lc = wv; lc < LC; lc += kOsjWaves) {
    double q = 0.0;
    for (int k = lane; k < m; k += 64) q += L[lc * m + k] * L[lc * m + k];
    q = wave_sum(q);
    if (lane == 0) nrm[lc] = q;
  }
  __syncthreads();
  const double tol = (double)m * 1.1102230246251565e-16;
  static_assert(kOsjWaves == kOsjBlk, "one wavefront per pair of a round");
  for (int rr = 0; rr < LC - 1; ++rr) {
    int i, j;
    if (wv == 0) {
      i = LC - 1;
      j = rr;
    } else {
      i = rr + wv;
      if (i >= LC - 1) i -= LC - 1;
      j = rr - wv;
      if (j < 0) j += LC - 1;
    }
    double* ci = L + i * m;
    double* cj = L + j * m;
    const double a = nrm[i], b = nrm[j];
    double g = 0.0;
    for (int k = lane; k < m; k += 64) g += ci[k] * cj[k];
    g = wave_sum(g);
    if (a > 0.0 && b > 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
      double c, s, tt;
      jacobi_angle(a, b, g, c, s, tt);
      for (int k = lane; k < m; k += 64) {
        const double x = ci[k], y = cj[k];
        ci[k] = c * x - s * y;
        cj[k] = s * x + c * y;
      }
      if (lane == 0) {
        nrm[i] = fmax(a - tt * g, 0.0);
        nrm[j] = b + tt * g;
        atomicAdd(&nrot, 1);
      }
    }
    __syncthreads();
  }
  for (int e = t; e < LC * m; e += kOsjThreads) {
    const int lc = e / m, k = e - lc * m;
    const int gc = lc < kOsjBlk ? I * kOsjBlk + lc : J * kOsjBlk + (lc - kOsjBlk);
    if (gc < m) X[(int64_t)gc * m + k] = L[e];
  }
  if (t == 0 && nrot > 0) atomicAdd(count, nrot);
}

__global__ __launch_bounds__(kOsjThreads) void osj_finish_kernel(const double* X, int64_t m, double* sigma, double* B,
                                                                 int scaled, int32_t* info, int sweeps) {
  __shared__ double sg[kQrMaxM];
  __shared__ int32_t pos[kQrMaxM];
  osj_finish(X, m, sigma, B, scaled, sg, pos);
  if (threadIdx.x == 0) info[0] = sweeps;
}

// W = R^T R in place (upper R, column-major), Rinv = R^-1 (row-major, upper,
// zeros below); a pivot <= rel_floor of its original diagonal, or not
// positive, marks the column as dependent (its row of R becomes e_k).
// Right-looking elimination over all (i, j) of the trailing triangle at
// once, then R^-1 row by row from the bottom with each dot product split
// over 8 lanes; in place in W and Rinv (workgroup-scope barriers order the
// global reads and writes).  For N above kCholLdsMaxN; the blocked kernel
// below takes the smaller ones.
__global__ __launch_bounds__(1024) void chol_inv_wg_kernel(double* W, int64_t ldw, int N, double* Rinv, int64_t ldr,
                                                           int32_t* bad, double rel_floor) {
  __shared__ double d0s[kCholWgMaxN];
  __shared__ double piv;
  __shared__ int nbad;
  const int t = threadIdx.x;
  auto P = [&](int i, int j) -> double& { return W[(int64_t)j * ldw + i]; };
  auto Iv = [&](int i, int j) -> double& { return Rinv[(int64_t)i * ldr + j]; };
  auto unpack = [](int e, int& i, int& j) {
    j = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (j * (j + 1) / 2 > e) --j;
    while ((j + 1) * (j + 2) / 2 <= e) ++j;
    i = e - j * (j + 1) / 2;
  };
  for (int k = t; k < N; k += 1024) d0s[k] = W[(int64_t)k * ldw + k];
  if (t == 0) nbad = 0;
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    if (t == 0) {
      const double d = P(k, k);
      if (!(d > rel_floor * d0s[k]) || !(d > 0.0) || !isfinite(d)) {
        piv = 0.0;
        ++nbad;
      } else {
        piv = sqrt(d);
      }
    }
    __syncthreads();
    const double p = piv;
    for (int j = k + 1 + t; j < N; j += 1024) P(k, j) = (p > 0.0) ? P(k, j) / p : 0.0;
    __syncthreads();
    if (t == 0) P(k, k) = (p > 0.0) ? p : 1.0;
    // trailing update of the upper triangle: (i, j), k < i <= j
    const int rem = N - k - 1;
    const int tot = rem * (rem + 1) / 2;
    for (int e = t; e < tot; e += 1024) {
      int i, j;
      unpack(e, i, j);
      i += k + 1;
      j += k + 1;
      P(i, j) -= P(k, i) * P(k, j);
    }
    __syncthreads();
  }
  // R^-1 row by row from the bottom: Rinv[i][j] = -(sum_{i<l<=j} R[i][l] Rinv[l][j]) / R[i][i]
  const int sub = t & 7;
  for (int i = N - 1; i >= 0; --i) {
    for (int j = i + (t >> 3); j < N; j += 128) {
      double s = 0.0;
      for (int l = i + 1 + sub; l <= j; l += 8) s += P(i, l) * Iv(l, j);
#pragma unroll
      for (int off = 4; off > 0; off >>= 1) s += __shfl_xor(s, off, 8);
      if (sub == 0) Iv(i, j) = (j == i) ? 1.0 / P(i, i) : -s / P(i, i);
    }
    __syncthreads();
  }
  for (int e = t; e < N * N; e += 1024) {
    const int j = e / N, i = e - j * N;
    if (i > j) Rinv[(int64_t)i * ldr + j] = 0.0;
  }
  if (t == 0 && bad) *bad = nbad;
}

// The same factorisation and inverse for N <= kCholLdsMaxN, blocked in
// panels of 16 rows so that the workgroup meets at a few barriers per panel
// instead of several per column (one workgroup of 1024 threads).
//   Panel p (rows p0 .. p0 + 15): wavefront 0 factors the panel's rows over
//   all columns p0 .. N - 1 in registers (lane l holds columns p0 + l and
//   p0 + l + 64; the pivot and the panel's own entries travel by lane
//   shuffles), with the same pivot rule as above; then every thread updates
//   the trailing triangle by the panel's 16 rows.
//   R^-1: the 16 x 16 diagonal blocks by back substitution (one wavefront
//   per block, one lane per column), then the blocks at distance d = 1, 2,
//   ... from the diagonal: X_IJ = -X_II sum_{I < L <= J} R_IL X_LJ.
// Both triangles packed in LDS (column-packed upper: (i, j) at
// j (j + 1) / 2 + i).
constexpr int kCholPanel = 16;
__global__ __launch_bounds__(1024) void chol_inv_blk_kernel(double* W, int64_t ldw, int N, double* Rinv, int64_t ldr,
                                                            int32_t* bad, double rel_floor) {
  extern __shared__ double cb_lds[];
  constexpr int PB = kCholPanel;
  constexpr int kMaxBlk = kCholLdsMaxN / PB;
  __shared__ double d0[kCholLdsMaxN];
  __shared__ double T[kMaxBlk - 1][PB][PB];
  const int np = N * (N + 1) / 2;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  auto P = [&](int i, int j) -> double& { return cb_lds[j * (j + 1) / 2 + i]; };
  auto X = [&](int i, int j) -> double& { return cb_lds[np + j * (j + 1) / 2 + i]; };
  for (int j = wave; j < N; j += 16)
    for (int i = lane; i <= j; i += 64) P(i, j) = W[(int64_t)j * ldw + i];
  for (int k = t; k < N; k += 1024) d0[k] = W[(int64_t)k * ldw + k];
  __syncthreads();
  int nbad = 0;  // counted by lane 0 of wavefront 0
  for (int p0 = 0; p0 < N; p0 += PB) {
    const int pw = min(PB, N - p0), pe = p0 + pw;
    if (wave == 0) {
      double v[PB][2];
      int jc[2] = {p0 + lane, p0 + lane + 64};
#pragma unroll
      for (int r = 0; r < PB; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          v[r][c] = (r < pw && jc[c] < N && p0 + r <= jc[c]) ? P(p0 + r, jc[c]) : 0.0;
#pragma unroll
      for (int r = 0; r < PB; ++r) {
        if (r >= pw) continue;  // (uniform; keeps the loop unrolled, v in registers)
        const int k = p0 + r;
        const double d = __shfl(v[r][0], r);  // column k: lane r, first slot
        const bool b = !(d > rel_floor * d0[k]) || !(d > 0.0) || !isfinite(d);
        const double piv = b ? 0.0 : sqrt(d);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (jc[c] > k && jc[c] < N) v[r][c] = b ? 0.0 : v[r][c] / piv;
          else if (jc[c] == k) v[r][c] = b ? 1.0 : piv;
        }
        nbad += b ? 1 : 0;
#pragma unroll
        for (int r2 = r + 1; r2 < PB; ++r2) {
          if (r2 >= pw) continue;
          const double sk = __shfl(v[r][0], r2);  // R(k, p0 + r2)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            if (jc[c] >= p0 + r2 && jc[c] < N) v[r2][c] -= sk * v[r][c];
        }
      }
#pragma unroll
      for (int r = 0; r < PB; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          if (r < pw && jc[c] >= p0 + r && jc[c] < N) P(p0 + r, jc[c]) = v[r][c];
    }
    __syncthreads();
    // trailing triangle pe <= i <= j < N
    for (int j = pe + (t >> 5); j < N; j += 32)
      for (int i = pe + (t & 31); i <= j; i += 32) {
        double s = 0.0;
        for (int r = 0; r < pw; ++r) s += P(p0 + r, i) * P(p0 + r, j);
        P(i, j) -= s;
      }
    __syncthreads();
  }
  // R^-1: diagonal blocks
  const int nb = (N + PB - 1) / PB;
  if (wave < nb && lane < PB) {
    const int J0 = wave * PB, bw = min(PB, N - J0), jl = lane;
    if (jl < bw) {
      double x[PB];
#pragma unroll
      for (int i = 0; i < PB; ++i) x[i] = 0.0;
#pragma unroll
      for (int i = PB - 1; i >= 0; --i) {
        if (i > jl) continue;
        if (i == jl) {
          x[i] = 1.0 / P(J0 + i, J0 + i);
        } else {
          double s = 0.0;
#pragma unroll
          for (int l = i + 1; l < PB; ++l)
            if (l <= jl) s += P(J0 + i, J0 + l) * x[l];
          x[i] = -s / P(J0 + i, J0 + i);
        }
      }
#pragma unroll
      for (int i = 0; i < PB; ++i)
        if (i <= jl) X(J0 + i, J0 + jl) = x[i];
    }
  }
  __syncthreads();
  // blocks at distance d from the diagonal
  for (int d = 1; d < nb; ++d) {
    const int cnt = (nb - d) * PB * PB;
    for (int e = t; e < cnt; e += 1024) {
      const int I = e / (PB * PB), i = (e / PB) % PB, j = e % PB;
      const int gi = I * PB + i, gj = (I + d) * PB + j;
      double s = 0.0;
      if (gi < N && gj < N)
        for (int l = (I + 1) * PB; l <= gj; ++l) s += P(gi, l) * X(l, gj);
      T[I][i][j] = s;
    }
    __syncthreads();
    for (int e = t; e < cnt; e += 1024) {
      const int I = e / (PB * PB), i = (e / PB) % PB, j = e % PB;
      const int gi = I * PB + i, gj = (I + d) * PB + j;
      if (gi < N && gj < N) {
        double s = 0.0;
        for (int l = i; l < PB && I * PB + l < N; ++l) s += X(gi, I * PB + l) * T[I][l][j];
        X(gi, gj) = -s;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < N * N; e += 1024) {
    const int j = e / N, i = e - j * N;
    if (i <= j) W[(int64_t)j * ldw + i] = P(i, j);
    Rinv[(int64_t)i * ldr + j] = (i <= j) ? X(i, j) : 0.0;
  }
  if (t == 0 && bad) *bad = nbad;
}

// dst (n x m) = the columns of a column table, rows past a column's own row
// count zero; dst plain column-major (ld n) for dst_rbs == 0, else
// row-block-tiled with row-block stride dst_rbs
__global__ void gather_cols_kernel(const void* const* __restrict__ cols, const int64_t* __restrict__ rbs,
                                   const int64_t* __restrict__ crows, int64_t n, double* __restrict__ dst,
                                   int64_t dst_rbs) {
  const int64_t c = blockIdx.y;
  const double* src = (const double*)cols[c];
  const int64_t rows = crows[c], rb = rbs[c];
  double* out = dst_rbs > 0 ? dst + c * kRowBlock : dst + c * n;
  const int64_t orb = dst_rbs > 0 ? dst_rbs : kRowBlock;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    out[blk_off(r, orb)] = r < rows ? src[blk_off(r, rb)] : 0.0;
}

}  // namespace

hapod_status launch_gather_cols(const void* const* d_cols, const int64_t* d_rbs, const int64_t* d_rows, int64_t n,
                                int64_t m, double* dst, int64_t dst_rbs, hipStream_t stream) {
  if (n <= 0 || m <= 0) return HAPOD_OK;
  if (m > 65535) {
    set_error("gather: too many columns");
    return HAPOD_E_UNSUPPORTED;
  }
  const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(gather_cols_kernel, dim3(gx, (unsigned)m), dim3(256), 0, stream, d_cols, d_rbs, d_rows, n, dst,
                     dst_rbs);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_chol_inv_wg(double* W, int64_t ldw, int64_t N, double* Rinv, int64_t ldr, int32_t* d_bad,
                                hipStream_t stream, double rel_floor) {
  if (N <= 0) return HAPOD_OK;
  if (N > kCholWgMaxN) {
    set_error("Cholesky: N above 1024");
    return HAPOD_E_UNSUPPORTED;
  }
  if (N <= kCholLdsMaxN) {
    static bool attr = false;
    if (!attr) {
      HAPOD_HIP(hipFuncSetAttribute((const void*)chol_inv_blk_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(sizeof(double) * kCholLdsMaxN * (kCholLdsMaxN + 1))));
      attr = true;
    }
    hipLaunchKernelGGL(chol_inv_blk_kernel, dim3(1), dim3(1024), sizeof(double) * N * (N + 1), stream, W, ldw,
                       (int)N, Rinv, ldr, d_bad, rel_floor);
  } else {
    hipLaunchKernelGGL(chol_inv_wg_kernel, dim3(1), dim3(1024), 0, stream, W, ldw, (int)N, Rinv, ldr, d_bad,
                       rel_floor);
  }
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_shift_diag(double* G, int64_t ldg, int64_t m, double coef, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(shift_diag_kernel, dim3(1), dim3(256), 0, stream, G, ldg, m, coef);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_identity_dev(const double* G, int64_t ldg, int64_t m, double* out, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(identity_dev_kernel, dim3(1), dim3(256), 0, stream, G, ldg, m, out);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_gram_zero_scale(double* G, int64_t ldg, int64_t m, int32_t* zero, double* D, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(gram_zero_scale_kernel, dim3(1), dim3(256), 0, stream, G, ldg, m, zero, D);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_unscale_factors(double* R, int64_t ldr, double* Rinv, int64_t ldi, int64_t m, const double* D,
                                    hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(unscale_factors_kernel, dim3((unsigned)((m * m + 255) / 256)), dim3(256), 0, stream, R, ldr, Rinv,
                     ldi, m, D);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_zero_rows(double* R, int64_t ldr, int64_t m, const int32_t* zero, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)((m * m + 255) / 256)), dim3(256), 0, stream, R, ldr, m, zero);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_triu(const double* W, int64_t ldw, int64_t N, double* R, int64_t ldr, hipStream_t stream) {
  if (N <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(triu_kernel, dim3((unsigned)((N + 255) / 256), (unsigned)N), dim3(256), 0, stream, W, ldw, N, R,
                     ldr);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_osj(double* A, int64_t m, double* sigma, double* B, int scaled, int32_t* info,
                        hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  if (m > kQrMaxM) {
    set_error("one-sided Jacobi: m above 512");
    return HAPOD_E_UNSUPPORTED;
  }
  if (m <= kOsjLdsMaxM / 2) {
    const size_t lds = sizeof(double) * (size_t)m * m;
    static bool attr = false;
    if (!attr) {
      HAPOD_HIP(hipFuncSetAttribute((const void*)osj_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(sizeof(double) * kOsjLdsMaxM * kOsjLdsMaxM)));
      attr = true;
    }
    hipLaunchKernelGGL(osj_kernel, dim3(1), dim3(kOsjThreads), lds, stream, A, m, sigma, B, scaled, info);
    HAPOD_HIP(hipGetLastError());
    return HAPOD_OK;
  }
  // block one-sided Jacobi: a sweep is nbe - 1 rounds of nbe / 2 block pairs;
  // the rotation count of a sweep is read back to decide convergence
  const int nb = (int)((m + kOsjBlk - 1) / kOsjBlk), nbe = nb + (nb & 1);
  const size_t lds = sizeof(double) * 2 * kOsjBlk * (size_t)m;
  static bool attr_b = false;
  if (!attr_b) {
    HAPOD_HIP(hipFuncSetAttribute((const void*)osj_block_round_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(sizeof(double) * 2 * kOsjBlk * kQrMaxM)));
    attr_b = true;
  }
  int32_t* count = info + 1;
  int sweep = 0;
  bool done = false;
  for (; sweep < kOsjMaxSweeps && !done; ++sweep) {
    HAPOD_TRY(launch_zero_bytes(count, sizeof(int32_t), stream));
    for (int r = 0; r < nbe - 1; ++r) {
      hipLaunchKernelGGL(osj_block_round_kernel, dim3(nbe / 2), dim3(kOsjThreads), lds, stream, A, (int)m, nbe, r,
                         count);
      HAPOD_HIP(hipGetLastError());
    }
    int32_t nrot = 0;
    HAPOD_HIP(hipMemcpyAsync(&nrot, count, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HAPOD_HIP(hipStreamSynchronize(stream));
    done = (nrot == 0);
  }
  hipLaunchKernelGGL(osj_finish_kernel, dim3(1), dim3(kOsjThreads), 0, stream, A, m, sigma, B, scaled, info,
                     done ? sweep : -1);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
