// Eigensolver for Gram matrices too large for one workgroup's Jacobi
// (the wide root of a star tree): the leading eigenpairs of G by Lanczos with
// full reorthogonalisation, in FP64.  Runs that need every eigenpair of a
// matrix of at most kHhMaxM columns replace the Krylov steps by a Householder
// reduction to the same tridiagonal form (see tridiag_kernel); everything
// from T on is shared.
//
//   q_0: deterministic pseudo-random unit vector.
//   step j: w = G q_j; two passes of classical Gram-Schmidt against
//           q_0..q_j (h = Q^T w, w -= Q h); alpha_j = sum of the two
//           coefficients of q_j; beta_j = ||w||; q_{j+1} = w / beta_j.
//           If beta_j <= 1e-10 ||G q_j|| the space is numerically invariant:
//           beta_j = 0 and q_{j+1} is a fresh random vector orthogonalised
//           (two passes) against q_0..q_j.
//   T = tridiag(beta, alpha, beta) (k x k).  Its eigenvalues theta_i come from
//   Sturm-sequence multisection (one wavefront per eigenvalue), its
//   eigenvectors z_i from inverse iteration with a pivoted tridiagonal LU
//   (one thread per eigenvector; one thread per cluster of equal
//   eigenvalues, orthogonalising within the cluster).  Ritz pairs: (theta_i, Q z_i), residual beta_{k-1} |z_i[k-1]|.
//
// The pairs returned are the leading Ritz pairs whose residual is below the
// Gram's rounding level or 1e-8 of their value, extended (when the iteration
// stopped at the rounding level) by the further Ritz values above the final
// residual norm; eigenvalues past them are reported as 0, and the rounding
// level floor_abs = max(-theta_min, u_p trace(G) / 10) is handed to the
// truncation, which counts eigenvalues at or below it as zero energy.  The
// caller learns whether the Krylov space reached the rounding level (else the
// spectrum past the block is unknown) and how much of trace(G) the returned
// pairs leave unexplained.
//
// Several matrices are solved together: every kernel of a step takes the list
// of matrices still iterating (grid z), so a level with many wide nodes costs
// one launch per kernel per step instead of one per node; a matrix leaves the
// list when its own stopping test is met.  Small matrices (see kFusedMaxM)
// instead run a whole period of steps in one workgroup of their own
// (lanczos_fused_kernel): the same steps, with sums taken in another order,
// so a matrix's result depends on the path to rounding level only.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mfma.hpp"
#include "wide.hpp"

namespace hapod {
namespace {

constexpr int kMaxSteps = kWideMaxSteps;
constexpr int kMinSteps = 128;      // no stop before this many steps
constexpr int kCheckEvery = 32;     // stopping test period
constexpr double kPlateau = 0.7;    // beta_j >= 0.7 beta_{j-32}: plateau
constexpr double kBreakdownTol = 1e-10;  // beta_j <= 1e-10 ||G q_j||: restart

__device__ __forceinline__ double hash_unit(uint64_t x) {
  // splitmix64 finaliser -> uniform in [-0.5, 0.5)
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  x ^= x >> 31;
  return (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

__device__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-matrix state of the batched Lanczos iteration (device array).
struct LzNode {
  const double* G;
  int64_t ldg;
  int64_t m;
  double* Q;       // m x (k + 1) Lanczos vectors, column-major
  double* w;       // m
  double* h;       // (k + 1) x nrc projection partials
  double* alpha;   // k
  double* beta;    // k + 1
  double* theta;   // k Ritz values (descending)
  double* e2;      // unused
  double* Z;       // k x k eigenvectors of T, Z[r * kk + i]
  double* last;    // k: last components of the z_i
  double* isc;     // unused
  int* ipiv;       // unused
  double* tr;      // trace(G)
  double* wn;      // nrc partial sums of ||G q_j||^2
  double* V;       // outputs
  double* lambda;
  int64_t ldv;
  int32_t nrc;
  int32_t kk;      // steps taken (tridiagonal phase)
  int32_t b;       // eigenpairs returned
  int32_t coop_p;  // workgroups of the cooperative step kernel (0: not used)
  double* xbuf;    // cooperative kernel: three exchange buffers of xlen doubles
  unsigned* bar;   // cooperative kernel: barrier counter (zeroed per launch)
  int64_t xlen;
  double* Z2;      // k x k: the eigenvectors between the two orthogonalisation sweeps
  // device-only full runs (hh_launch): the rounding level and the trace
  // check go to these, and the back-transformation's column table lives here
  double* floor_out;
  double* diag_out;
  double u_p;
  const void** qcols;
  int64_t* qrbs;
  int64_t* qrows;
  int64_t* qrank;
};

// q = random, unnormalised (normalised by the finish kernel)
__global__ void lanczos_init_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.z];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n.m; i += (int64_t)gridDim.x * blockDim.x)
    n.w[i] = hash_unit((uint64_t)i * 7919u + 17u);
}

// w[c] = G[:, c] . q_j  (G symmetric), one wavefront per column
__global__ __launch_bounds__(256) void matvec_kernel(const LzNode* __restrict__ nodes, const int* __restrict__ act,
                                                     int j) {
  const LzNode n = nodes[act[blockIdx.z]];
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n.m) return;
  const double* col = n.G + c * n.ldg;
  const double* q = n.Q + (int64_t)j * n.m;
  double s = 0.0;
  for (int64_t r = lane; r < n.m; r += 64) s += col[r] * q[r];
  s = wave_sum(s);
  if (lane == 0) n.w[c] = s;
}

constexpr int kProjCols = 16;    // Lanczos vectors per projection workgroup
constexpr int kProjRows = 1024;  // rows per projection workgroup

// h[c * nrc + rc] = Q[rows of chunk rc, c] . w[rows of chunk rc], c <= j
__global__ __launch_bounds__(256) void proj_partial_kernel(const LzNode* __restrict__ nodes,
                                                           const int* __restrict__ act, int j, int wn_pass) {
  const LzNode n = nodes[act[blockIdx.z]];
  __shared__ double red[kProjCols][4];
  __shared__ double rn[4];
  const int c0 = blockIdx.x * kProjCols, rc = blockIdx.y;
  if (rc >= n.nrc) return;
  const int ncols = min(kProjCols, j + 1 - c0);
  const int64_t r0 = (int64_t)rc * kProjRows, r1 = min(n.m, r0 + kProjRows);
  // the first pass of a step also records ||w||^2 = ||G q_j||^2 per row chunk
  const bool norm = (blockIdx.x == 0) && (wn_pass != 0);
  double acc[kProjCols];
  double ww = 0.0;
#pragma unroll
  for (int c = 0; c < kProjCols; ++c) acc[c] = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const double wr = n.w[r];
    ww += wr * wr;
#pragma unroll
    for (int c = 0; c < kProjCols; ++c)
      if (c < ncols) acc[c] += n.Q[(int64_t)(c0 + c) * n.m + r] * wr;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kProjCols; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) red[c][wave] = v;
  }
  if (norm) {
    const double v = wave_sum(ww);
    if (lane == 0) rn[wave] = v;
  }
  __syncthreads();
  if (norm && threadIdx.x == 0) n.wn[rc] = rn[0] + rn[1] + rn[2] + rn[3];
  if (threadIdx.x < ncols)
    n.h[(int64_t)(c0 + threadIdx.x) * n.nrc + rc] =
        red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

// hc = sum over row chunks of h[c] (fixed order); w -= Q[:, 0..j] hc;
// alpha_j += hc[j].  64 rows per workgroup, columns split over 4 wavefronts.
__global__ __launch_bounds__(256) void update_kernel(const LzNode* __restrict__ nodes, const int* __restrict__ act,
                                                     int j) {
  const LzNode n = nodes[act[blockIdx.z]];
  if ((int64_t)blockIdx.x * 64 >= n.m) return;  // whole workgroup
  __shared__ double hs[kMaxSteps + 1];
  __shared__ double part[4][64];
  for (int c = threadIdx.x; c <= j; c += blockDim.x) {
    double t = 0.0;
    for (int rc = 0; rc < n.nrc; ++rc) t += n.h[(int64_t)c * n.nrc + rc];
    hs[c] = t;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) n.alpha[j] += hs[j];
  const int rl = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + rl;
  double t = 0.0;
  if (i < n.m)
    for (int c = cg; c <= j; c += 4) t += n.Q[(int64_t)c * n.m + i] * hs[c];
  part[cg][rl] = t;
  __syncthreads();
  if (cg == 0 && i < n.m) n.w[i] -= part[0][rl] + part[1][rl] + part[2][rl] + part[3][rl];
}

// beta_j = ||w||, q_{j+1} = w / beta_j (one workgroup per matrix); j = -1
// normalises the start vector into q_0
__global__ __launch_bounds__(1024) void finish_kernel(const LzNode* __restrict__ nodes, const int* __restrict__ act,
                                                      int j) {
  const LzNode n = act ? nodes[act[blockIdx.z]] : nodes[blockIdx.z];
  __shared__ double part[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n.m; i += blockDim.x) s += n.w[i] * n.w[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += part[i];
  const double beta = sqrt(tot);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  double* q_next = n.Q + (int64_t)(j + 1) * n.m;
  for (int64_t i = threadIdx.x; i < n.m; i += blockDim.x) q_next[i] = n.w[i] * inv;
  if (threadIdx.x == 0 && j >= 0) n.beta[j] = beta;
}

// Breakdown: beta_j this small against ||G q_j|| means the Krylov space is
// (numerically) invariant, and w / beta_j would be rounding noise that the
// two Gram-Schmidt passes could not make orthogonal to Q.  Restart: a fresh
// pseudo-random vector, orthogonalised against q_0..q_j by two classical
// Gram-Schmidt passes, becomes q_{j+1}, and beta_j = 0 (T splits into
// independent blocks).  One workgroup per matrix; the others return at once.
__global__ __launch_bounds__(1024) void breakdown_kernel(const LzNode* __restrict__ nodes,
                                                         const int* __restrict__ act, int j, double rel_tol) {
  const LzNode n = nodes[act[blockIdx.z]];
  double w2 = 0.0;
  for (int rc = 0; rc < n.nrc; ++rc) w2 += n.wn[rc];
  if (!(n.beta[j] <= rel_tol * sqrt(w2))) return;
  __shared__ double hs[kMaxSteps + 1];
  __shared__ double part[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* w = n.w;
  for (int64_t i = threadIdx.x; i < n.m; i += blockDim.x)
    w[i] = hash_unit((uint64_t)i * 7919u + 104729u * (uint64_t)(j + 1) + 17u);
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = wave; c <= j; c += nw) {  // h = Q^T w, one wavefront per column
      const double* q = n.Q + (int64_t)c * n.m;
      double t = 0.0;
      for (int64_t i = lane; i < n.m; i += 64) t += q[i] * w[i];
      t = wave_sum(t);
      if (lane == 0) hs[c] = t;
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n.m; i += blockDim.x) {  // w -= Q h
      double t = 0.0;
      for (int c = 0; c <= j; ++c) t += n.Q[(int64_t)c * n.m + i] * hs[c];
      w[i] -= t;
    }
    __syncthreads();
  }
  double s2 = 0.0;
  for (int64_t i = threadIdx.x; i < n.m; i += blockDim.x) s2 += w[i] * w[i];
  s2 = wave_sum(s2);
  if (lane == 0) part[wave] = s2;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < nw; ++i) tot += part[i];
  const double nrm = sqrt(tot);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  double* q_next = n.Q + (int64_t)(j + 1) * n.m;
  for (int64_t i = threadIdx.x; i < n.m; i += blockDim.x) q_next[i] = w[i] * inv;
  if (threadIdx.x == 0) n.beta[j] = 0.0;
}

// One workgroup runs steps j0 .. j1-1 of one small matrix (m <= kFusedMaxM)
// with the arithmetic of the step kernels above: w = G q_j, two classical
// Gram-Schmidt passes (alpha_j collects both coefficients of q_j), beta_j =
// ||w||, and the breakdown restart.  q_j, w, the projection coefficients and
// the first Lanczos vectors (as many as kFusedQCache doubles hold) live in
// LDS; G and the later vectors are read from global memory (L2 at these
// sizes).  For small matrices one launch per period of steps replaces seven
// launches per step, whose fixed cost dominated.  One workgroup streams L2
// data at a few tens of GB/s, so above kFusedAloneMaxM columns the step
// kernels, spread over many workgroups, are faster for a matrix alone (about
// 35 us against 33 us per step at 243 columns, 37 against 129 at 512); with
// kFusedBatchMin or more such matrices in the batch, the fused workgroups run
// side by side on their own compute units and win again.
constexpr int kFusedMaxM = 512;
constexpr int kFusedAloneMaxM = 224;
constexpr int kFusedBatchMin = 8;
constexpr int kFusedThreads = 512;
constexpr int kFusedQCache = 16384;  // doubles of LDS for leading Lanczos vectors
// Loads go through global-address-space pointers in explicit batches:
// generic (flat) loads mixed with LDS reads would make the compiler wait for
// every load before the next.
constexpr int kFusedBatch = 8;

// Column c of Q: the LDS copy for c < nq, else global memory.
struct FusedQ {
  const double* g;   // global, column-major, ld m
  const double* l;   // LDS copy of columns 0 .. nq-1
  int64_t m;
  int nq;
};

// sum over c = c0, c0 + stride, ... < cend of X[c * ldx + r] * v[c] (v in LDS)
__device__ __forceinline__ double fused_rowdot(const double* __restrict__ X, int64_t ldx, int64_t r, int c0,
                                               int cend, int stride, const double* v) {
  const gptr<double> Xg = as_global(X);
  double acc = 0.0;
  for (int c = c0; c < cend; c += kFusedBatch * stride) {
    double x[kFusedBatch];
#pragma unroll
    for (int u = 0; u < kFusedBatch; ++u) {
      const int cc = c + u * stride;
      x[u] = (cc < cend) ? Xg[(int64_t)cc * ldx + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kFusedBatch; ++u) {
      const int cc = c + u * stride;
      if (cc < cend) acc += x[u] * v[cc];
    }
  }
  return acc;
}

// the same sum over columns of Q (LDS part first, then global memory)
__device__ __forceinline__ double fused_qrowdot(const FusedQ& Q, int64_t r, int c0, int cend, int stride,
                                                const double* v) {
  double acc = 0.0;
  const int lend = min(cend, Q.nq);
  int c = c0;
  for (; c < lend; c += stride) acc += Q.l[(int64_t)c * Q.m + r] * v[c];
  return acc + fused_rowdot(Q.g, Q.m, r, c, cend, stride, v);
}

// 64-lane sums of four values: lane 16 u holds the sum of t[u] (u = 0..3);
// halving exchanges take 7 shuffles instead of 24.
__device__ __forceinline__ double wave_sum4(const double (&t)[4], int lane) {
  const bool a = (lane & 32) != 0, b = (lane & 16) != 0;
  double k0 = a ? t[2] : t[0], k1 = a ? t[3] : t[1];
  const double s0 = a ? t[0] : t[2], s1 = a ? t[1] : t[3];
  k0 += __shfl_xor(s0, 32, 64);
  k1 += __shfl_xor(s1, 32, 64);
  double k = b ? k1 : k0;
  k += __shfl_xor(b ? k0 : k1, 16, 64);
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) k += __shfl_xor(k, off, 64);
  return k;
}

// h = Q[:, 0..j]^T w, then w -= Q h.  Projection: each wavefront takes
// every nw-th column, four at a time, its lanes striding the rows.  Update:
// the rows split over groups of threads, each group summing every groups-th
// column, the groups' partial sums added in a fixed order.  Returns h[j].
__device__ double fused_cgs_pass(const FusedQ& Q, int j, double* w_s, double* hs, double* part, int rows_pad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nw = kFusedThreads / 64;
  const int64_t m = Q.m;
  const gptr<double> Qg = as_global(Q.g);
  for (int c0 = wave; c0 <= j; c0 += 4 * nw) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    if (c0 + 3 * nw < Q.nq) {  // all four columns in LDS
      for (int64_t r = lane; r < m; r += 64) {
        const double wr = w_s[r];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u * nw;
          if (c <= j) t[u] += Q.l[(int64_t)c * m + r] * wr;
        }
      }
    } else {
      for (int64_t r0 = 0; r0 < m; r0 += 128) {
        double x[2][4], wr[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t r = r0 + lane + 64 * h;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * nw;
            x[h][u] = (c <= j && r < m) ? (c < Q.nq ? Q.l[(int64_t)c * m + r] : Qg[(int64_t)c * m + r]) : 0.0;
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t r = r0 + lane + 64 * h;
          wr[h] = (r < m) ? w_s[r] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int u = 0; u < 4; ++u) t[u] += x[h][u] * wr[h];
      }
    }
    const double sum = wave_sum4(t, lane);
    const int u = lane >> 4;
    if ((lane & 15) == 0 && c0 + u * nw <= j) hs[c0 + u * nw] = sum;
  }
  __syncthreads();
  const int groups = kFusedThreads / rows_pad;
  const int r = tid % rows_pad, grp = tid / rows_pad;
  part[tid] = (r < m) ? fused_qrowdot(Q, r, grp, j + 1, groups, hs) : 0.0;
  __syncthreads();
  if (tid < m) {
    double u = 0.0;
    for (int g = 0; g < groups; ++g) u += part[g * rows_pad + tid];
    w_s[tid] -= u;
  }
  const double hj = hs[j];
  __syncthreads();
  return hj;
}

__device__ double fused_block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < kFusedThreads / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kFusedThreads) void lanczos_fused_kernel(const LzNode* __restrict__ nodes,
                                                                       const int* __restrict__ act, int j0, int j1,
                                                                       double rel_tol) {
  const LzNode n = nodes[act[blockIdx.z]];
  const int64_t m = n.m;
  const int k = (int)min(m, (int64_t)kMaxSteps);
  const int jend = min(j1, k);
  extern __shared__ double qcache[];
  __shared__ double q_s[kFusedMaxM], w_s[kFusedMaxM];
  __shared__ double hs[kMaxSteps + 1];
  __shared__ double part[kFusedThreads];
  __shared__ double red[kFusedThreads / 64];
  const int tid = threadIdx.x;
  const int rows_pad = m <= 64 ? 64 : m <= 128 ? 128 : m <= 256 ? 256 : 512;
  if (j0 >= jend) return;
  FusedQ Q{n.Q, qcache, m, (int)min((int64_t)(k + 1), (int64_t)kFusedQCache / m)};
  // the cached columns written by earlier launches
  const int64_t have = (int64_t)min(j0 + 1, Q.nq) * m;
  for (int64_t e = tid; e < have; e += kFusedThreads) qcache[e] = n.Q[e];
  for (int64_t r = tid; r < m; r += kFusedThreads) q_s[r] = n.Q[(int64_t)j0 * m + r];
  __syncthreads();
  for (int j = j0; j < jend; ++j) {
    // w = G q_j = sum_c G[:, c] q_j[c] (G symmetric): the rows split over
    // groups of threads, each group summing every groups-th column
    {
      const int groups = kFusedThreads / rows_pad;
      const int r = tid % rows_pad, grp = tid / rows_pad;
      part[tid] = (r < m) ? fused_rowdot(n.G, n.ldg, r, grp, (int)m, groups, q_s) : 0.0;
      __syncthreads();
      if (tid < m) {
        double u = 0.0;
        for (int g = 0; g < groups; ++g) u += part[g * rows_pad + tid];
        w_s[tid] = u;
      }
      __syncthreads();
    }
    double wv = (tid < m) ? w_s[tid] : 0.0;
    const double gq2 = fused_block_sum(wv * wv, red);  // ||G q_j||^2
    double alpha = 0.0;
    alpha += fused_cgs_pass(Q, j, w_s, hs, part, rows_pad);
    alpha += fused_cgs_pass(Q, j, w_s, hs, part, rows_pad);
    wv = (tid < m) ? w_s[tid] : 0.0;
    const double beta = sqrt(fused_block_sum(wv * wv, red));
    double* q_next = n.Q + (int64_t)(j + 1) * m;
    double* l_next = (j + 1 < Q.nq) ? qcache + (int64_t)(j + 1) * m : nullptr;
    double beta_out = beta;
    double inv;
    if (beta <= rel_tol * sqrt(gq2)) {
      // breakdown: a fresh pseudo-random vector orthogonalised twice
      for (int64_t r = tid; r < m; r += kFusedThreads)
        w_s[r] = hash_unit((uint64_t)r * 7919u + 104729u * (uint64_t)(j + 1) + 17u);
      __syncthreads();
      fused_cgs_pass(Q, j, w_s, hs, part, rows_pad);
      fused_cgs_pass(Q, j, w_s, hs, part, rows_pad);
      wv = (tid < m) ? w_s[tid] : 0.0;
      const double nrm = sqrt(fused_block_sum(wv * wv, red));
      inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      beta_out = 0.0;
    } else {
      inv = beta > 0.0 ? 1.0 / beta : 0.0;
    }
    for (int64_t r = tid; r < m; r += kFusedThreads) {
      const double x = w_s[r] * inv;
      q_next[r] = x;
      q_s[r] = x;
      if (l_next) l_next[r] = x;
    }
    if (tid == 0) {
      n.alpha[j] = alpha;
      n.beta[j] = beta_out;
    }
    __syncthreads();
  }
}

// Mid-size matrices alone (or a few of them): the steps of the fused kernel
// spread over coop_p workgroups, each holding in LDS its slice of rows of G
// (as columns: G is symmetric) and of the Lanczos vectors.  Per step three
// exchanges through global memory, each closed by a barrier among the
// matrix's workgroups: the projection partials of the two Gram-Schmidt
// passes (with ||G q_j||^2 in the first) and the new w with the partial
// norms.  Every workgroup adds the partials in the same fixed order, so all
// take the same branches.  A barrier waits a bounded time; if it runs out
// (it cannot when the launch is cooperative, i.e. every workgroup resident)
// the error flag is set and every workgroup leaves.
constexpr int kCoopMaxM = 512;
constexpr int kCoopThreads = 256;
constexpr long kCoopSpinLimit = 1L << 22;

__host__ __device__ __forceinline__ int coop_pick(int64_t m) { return m <= 320 ? 16 : 32; }
__device__ __host__ __forceinline__ size_t coop_lds_doubles(int64_t m, int P) {
  const int64_t k = m < kMaxSteps ? m : kMaxSteps;
  const int64_t R = (m + P - 1) / P;
  return (size_t)(R * m + R * (k + 1) + m + (k + 1) + R);
}

// all workgroups of one matrix meet; false when the wait ran out (or another
// workgroup's did)
__device__ bool coop_barrier(unsigned* bar, unsigned target, int* err, int* flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    int bad = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > kCoopSpinLimit) {
        bad = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (bad) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *flag = bad;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *flag == 0;
}

__global__ __launch_bounds__(kCoopThreads) void lanczos_coop_kernel(const LzNode* __restrict__ nodes,
                                                                     const int* __restrict__ act, int j0, int j1,
                                                                     double rel_tol, int* err) {
  const LzNode n = nodes[act[blockIdx.z]];
  const int P = n.coop_p;
  const int p = blockIdx.x;
  if (p >= P) return;  // not one of this matrix's workgroups (no barrier met)
  const int64_t m = n.m;
  const int k = (int)min(m, (int64_t)kMaxSteps);
  const int jend = min(j1, k);
  if (j0 >= jend) return;  // the same for all of the matrix's workgroups
  const int R = (int)((m + P - 1) / P);
  const int r0 = p * R;
  const int nr = (int)max((int64_t)0, min(m, (int64_t)r0 + R) - r0);
  const int kq = k + 1;
  const int K2 = k + 2;  // stride of one workgroup's partials
  extern __shared__ double lds[];
  double* Gs = lds;                       // R x m: row rr = column r0 + rr of G
  double* Qs = Gs + (size_t)R * m;        // R x kq: rows r0.. of the Lanczos vectors
  double* qf = Qs + (size_t)R * kq;       // m: q_j
  double* hh = qf + m;                    // kq: summed projection coefficients
  double* wl = hh + kq;                   // R: this slice of w
  __shared__ double sc[2];
  __shared__ int flag;
  __shared__ double part[kCoopThreads];
  __shared__ double rsum[kCoopThreads / 8];
  const int t = threadIdx.x;
  // rsum[rr] = sum over c < len of A[rr * lda + c] v[c], rr < nr: thread
  // rr + nr g takes every ng-th c from g, the ng partial sums are added in a
  // fixed order (no cross-lane shuffles)
  const int ng = kCoopThreads / max(nr, 1);
  auto rowdot = [&](const double* A, int lda, int len, const double* v) {
    const int rr = t % max(nr, 1), g = t / max(nr, 1);
    double u = 0.0;
    if (g < ng && rr < nr)
      for (int c = g; c < len; c += ng) u += A[(size_t)rr * lda + c] * v[c];
    part[t] = u;
    __syncthreads();
    if (t < nr) {
      double w = 0.0;
      for (int q = 0; q < ng; ++q) w += part[q * nr + t];
      rsum[t] = w;
    }
    __syncthreads();
  };
  unsigned nbar = 0;
  int ex = 0;
  auto xb = [&](int e) { return n.xbuf + (size_t)(e % 3) * n.xlen; };

  for (int rr = 0; rr < nr; ++rr)
    for (int64_t c = t; c < m; c += kCoopThreads) Gs[(size_t)rr * m + c] = n.G[(int64_t)(r0 + rr) * n.ldg + c];
  for (int e = t; e < nr * (j0 + 1); e += kCoopThreads) {
    const int rr = e % nr, c = e / nr;
    Qs[(size_t)rr * kq + c] = n.Q[(int64_t)c * m + r0 + rr];
  }
  for (int64_t c = t; c < m; c += kCoopThreads) qf[c] = n.Q[(int64_t)j0 * m + c];
  __syncthreads();

  // one classical Gram-Schmidt pass of wl against q_0..q_j; returns h_j.
  // extra (>= 0) travels with the partials; its sum lands in sc[0]
  auto cgs = [&](int j, double extra, bool with_extra, bool& ok) -> double {
    double* X = xb(ex++);
    for (int c = t; c <= j; c += kCoopThreads) {
      double hp = 0.0;
      for (int rr = 0; rr < nr; ++rr) hp += Qs[(size_t)rr * kq + c] * wl[rr];
      X[(size_t)p * K2 + c] = hp;
    }
    if (with_extra && t == 0) X[(size_t)p * K2 + k + 1] = extra;
    ok = coop_barrier(n.bar, (unsigned)P * ++nbar, err, &flag);
    if (!ok) return 0.0;
    const gptr<double> Xg = as_global(X);
    for (int c = t; c <= j; c += kCoopThreads) {
      double hs = 0.0;
#pragma unroll 8
      for (int q = 0; q < P; ++q) hs += Xg[(size_t)q * K2 + c];
      hh[c] = hs;
    }
    if (with_extra && t == 0) {
      double e2 = 0.0;
#pragma unroll 8
      for (int q = 0; q < P; ++q) e2 += Xg[(size_t)q * K2 + k + 1];
      sc[0] = e2;
    }
    __syncthreads();
    rowdot(Qs, kq, j + 1, hh);
    if (t < nr) wl[t] -= rsum[t];
    const double hj = hh[j];
    __syncthreads();
    return hj;
  };
  // w goes out whole with the slices' squared norms; returns ||w||, the
  // buffer holding w in *Xw
  auto share_w = [&](double** Xw, bool& ok) -> double {
    double* X = xb(ex++);
    for (int rr = t; rr < nr; rr += kCoopThreads) X[r0 + rr] = wl[rr];
    if (t == 0) {
      double s2 = 0.0;
      for (int rr = 0; rr < nr; ++rr) s2 += wl[rr] * wl[rr];
      X[m + p] = s2;
    }
    ok = coop_barrier(n.bar, (unsigned)P * ++nbar, err, &flag);
    if (!ok) return 0.0;
    const gptr<double> Xg = as_global(X);
    double tot = 0.0;
#pragma unroll 8
    for (int q = 0; q < P; ++q) tot += Xg[m + q];
    *Xw = X;
    return sqrt(tot);
  };

  for (int j = j0; j < jend; ++j) {
    // w = G q_j on this slice of rows
    rowdot(Gs, (int)m, (int)m, qf);
    if (t < nr) wl[t] = rsum[t];
    __syncthreads();
    double gq = 0.0;
    if (t == 0)
      for (int rr = 0; rr < nr; ++rr) gq += wl[rr] * wl[rr];
    bool ok = true;
    double alpha = cgs(j, gq, true, ok);
    if (!ok) return;
    const double gq2 = sc[0];
    alpha += cgs(j, 0.0, false, ok);
    if (!ok) return;
    double* Xw = nullptr;
    const double beta = share_w(&Xw, ok);
    if (!ok) return;
    double beta_out = beta, inv;
    if (beta <= rel_tol * sqrt(gq2)) {
      // breakdown: a fresh pseudo-random vector orthogonalised twice
      for (int rr = t; rr < nr; rr += kCoopThreads)
        wl[rr] = hash_unit((uint64_t)(r0 + rr) * 7919u + 104729u * (uint64_t)(j + 1) + 17u);
      __syncthreads();
      cgs(j, 0.0, false, ok);
      if (!ok) return;
      cgs(j, 0.0, false, ok);
      if (!ok) return;
      const double nrm = share_w(&Xw, ok);
      if (!ok) return;
      inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      beta_out = 0.0;
    } else {
      inv = beta > 0.0 ? 1.0 / beta : 0.0;
    }
    {
      const gptr<double> Xg = as_global(Xw);
      for (int64_t c = t; c < m; c += kCoopThreads) qf[c] = Xg[c] * inv;
    }
    __syncthreads();
    for (int rr = t; rr < nr; rr += kCoopThreads) {
      const double v = qf[r0 + rr];
      Qs[(size_t)rr * kq + j + 1] = v;
      n.Q[(int64_t)(j + 1) * m + r0 + rr] = v;
    }
    if (p == 0 && t == 0) {
      n.alpha[j] = alpha;
      n.beta[j] = beta_out;
    }
    __syncthreads();
  }
}

// out[2 a] = beta_j, out[2 a + 1] = beta_0 of active matrix a
__global__ void gather_beta_kernel(const LzNode* __restrict__ nodes, const int* __restrict__ act, int na, int j,
                                   double* __restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  const LzNode n = nodes[act[a]];
  out[2 * a] = n.beta[j];
  out[2 * a + 1] = n.beta[0];
}

__global__ void setup_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.z];
  const int k = (int)min(n.m, (int64_t)kMaxSteps);
  for (int i = threadIdx.x; i < k; i += blockDim.x) n.alpha[i] = 0.0;
  __shared__ double part[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n.m; i += blockDim.x) s += n.G[i * n.ldg + i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += part[i];
    *n.tr = t;
  }
}

// number of eigenvalues of tridiag(e, d, e) below mu (Sturm sequence)
__device__ int sturm_count(const double* d, const double* e2, int k, double mu, double pivmin) {
  int cnt = 0;
  double q = d[0] - mu;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int j = 1; j < k; ++j) {
    q = (d[j] - mu) - e2[j - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

// theta[i] = i-th largest eigenvalue of T, by multisection: one wavefront
// per eigenvalue, 64 Sturm counts per step shrink the bracket 65-fold.
__global__ __launch_bounds__(256) void bisect_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.z];
  const int k = n.kk;
  if (blockIdx.x * 4 >= k) return;  // whole workgroup
  // T (diagonal, off-diagonal and its squares) staged in LDS: every Sturm
  // count reads all of it
  extern __shared__ double bs[];
  double* d = bs;
  double* e = bs + k;
  double* e2buf = bs + 2 * k;
  double* theta = n.theta;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    d[j] = n.alpha[j];
    const double ej = (j < k - 1) ? n.beta[j] : 0.0;
    e[j] = ej;
    e2buf[j] = ej * ej;
  }
  __syncthreads();
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= k) return;
  double lo = 1e300, hi = -1e300, emax2 = 0.0;
  for (int j = 0; j < k; ++j) {
    const double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + (j < k - 1 ? fabs(e[j]) : 0.0);
    lo = fmin(lo, d[j] - r);
    hi = fmax(hi, d[j] + r);
    if (j < k - 1) emax2 = fmax(emax2, e2buf[j]);
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = fmax(2.2250738585072014e-308, 2.2250738585072014e-308 * emax2);
  const double slack = 4.0 * 2.220446049250313e-16 * tnorm + 2.0 * pivmin;
  lo -= slack;
  hi += slack;
  const int target = k - 1 - i;  // ascending index
  for (int it = 0; it < 20; ++it) {
    if (hi - lo <= 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    // lane l tests x_l = lo + (l + 1) (hi - lo) / 65
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    const bool above = sturm_count(d, e2buf, k, x, pivmin) > target;
    const uint64_t mask = __ballot(above);
    // first lane whose point lies above the eigenvalue bounds it from above
    const int first = mask ? __ffsll((unsigned long long)mask) - 1 : 64;
    const double nlo = (first == 0) ? lo : lo + (hi - lo) * (double)first / 65.0;
    const double nhi = (first == 64) ? hi : lo + (hi - lo) * (double)(first + 1) / 65.0;
    if (!(nlo >= lo && nhi <= hi) || (nlo == lo && nhi == hi)) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) theta[i] = 0.5 * (lo + hi);
}

// inverse iteration: z_i solves (T - theta_i) z = z_prev (pivoted LU), three
// times from a pseudo-random start; written as column i of Z (row-major,
// Z[r * ldz + i]).  Scratch: 5 k doubles + k ints per thread.
// One workgroup (one wavefront, its first lane working) per eigenvector:
// the LU factors and the iterate live in LDS (5 k doubles and k ints),
// so the serial recurrences wait on LDS rather than on global memory.
__global__ __launch_bounds__(64) void inviter_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.z];
  const int k = n.kk, nvec = n.kk;
  const int64_t ldz = n.kk;
  const double* d = n.alpha;
  const double* e = n.beta;
  const double* theta = n.theta;
  double* Z = n.Z;
  double* last = n.last;
  const int i = blockIdx.x;
  if (i >= nvec || threadIdx.x != 0) return;
  extern __shared__ double ivs[];
  const int64_t st = 1;
  double* dl = ivs;
  double* dd = dl + k;
  double* du = dd + k;
  double* du2 = du + k;
  double* b = du2 + k;
  int* piv = reinterpret_cast<int*>(b + k);
#define DL(x) dl[(int64_t)(x) * st]
#define DD(x) dd[(int64_t)(x) * st]
#define DU(x) du[(int64_t)(x) * st]
#define DU2(x) du2[(int64_t)(x) * st]
#define BB(x) b[(int64_t)(x) * st]
#define PIV(x) piv[(int64_t)(x) * st]
  double tnorm = 0.0;
  for (int j = 0; j < k; ++j) tnorm = fmax(tnorm, fabs(d[j]) + (j < k - 1 ? fabs(e[j]) : 0.0) + (j > 0 ? fabs(e[j - 1]) : 0.0));
  const double tiny = fmax(2.220446049250313e-16 * tnorm, 1e-300);
  // Ritz values equal to 9 digits (and above the rounding level of T) form
  // a cluster -- an eigenvalue the restarts found several times; inverse
  // iteration alone would return nearly parallel vectors for them, so one
  // thread (the cluster's first) computes them in turn, orthogonalising each
  // iterate against the cluster's earlier vectors (modified Gram-Schmidt).
  const double level = 1e3 * 2.220446049250313e-16 * tnorm;
  auto same = [&](int a, int b2) {
    return fabs(theta[b2]) > level && theta[a] - theta[b2] <= 1e-9 * fabs(theta[b2]);
  };
  if (i > 0 && same(i - 1, i)) return;
  int cend = i + 1;
  while (cend < nvec && same(cend - 1, cend)) ++cend;
  for (int v = i; v < cend; ++v) {
    const double mu = theta[v];
    // LU with partial pivoting of T - mu I (LAPACK gttrf layout)
    for (int j = 0; j < k; ++j) {
      DD(j) = d[j] - mu;
      if (j < k - 1) { DL(j) = e[j]; DU(j) = e[j]; }
      DU2(j) = 0.0;
    }
    for (int j = 0; j < k - 1; ++j) {
      if (fabs(DD(j)) >= fabs(DL(j))) {
        PIV(j) = j;
        if (DD(j) == 0.0) DD(j) = tiny;
        const double f = DL(j) / DD(j);
        DL(j) = f;
        DD(j + 1) -= f * DU(j);
      } else {
        PIV(j) = j + 1;
        const double f = DD(j) / DL(j);
        DD(j) = DL(j);
        DL(j) = f;
        const double tmp = DU(j);
        DU(j) = DD(j + 1);
        DD(j + 1) = tmp - f * DD(j + 1);
        if (j < k - 2) {
          DU2(j) = DU(j + 1);
          DU(j + 1) = -f * DU(j + 1);
        }
      }
    }
    if (DD(k - 1) == 0.0) DD(k - 1) = tiny;
    for (int j = 0; j < k; ++j)
      if (fabs(DD(j)) < tiny) DD(j) = (DD(j) < 0.0 ? -tiny : tiny);
    for (int j = 0; j < k; ++j) BB(j) = hash_unit((uint64_t)v * 1000003u + j) + 1.0;
    for (int it = 0; it < 3; ++it) {
      // forward with L
      for (int j = 0; j < k - 1; ++j) {
        if (PIV(j) == j) {
          BB(j + 1) -= DL(j) * BB(j);
        } else {
          const double t = BB(j);
          BB(j) = BB(j + 1);
          BB(j + 1) = t - DL(j) * BB(j);
        }
      }
      // back substitution with U (diag DD, super DU, super-super DU2)
      BB(k - 1) /= DD(k - 1);
      if (k > 1) BB(k - 2) = (BB(k - 2) - DU(k - 2) * BB(k - 1)) / DD(k - 2);
      for (int j = k - 3; j >= 0; --j) BB(j) = (BB(j) - DU(j) * BB(j + 1) - DU2(j) * BB(j + 2)) / DD(j);
      // against the cluster's earlier vectors
      for (int c = i; c < v; ++c) {
        double dot = 0.0;
        for (int j = 0; j < k; ++j) dot += Z[(int64_t)j * ldz + c] * BB(j);
        for (int j = 0; j < k; ++j) BB(j) -= dot * Z[(int64_t)j * ldz + c];
      }
      double nrm = 0.0;
      for (int j = 0; j < k; ++j) nrm += BB(j) * BB(j);
      nrm = sqrt(nrm);
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int j = 0; j < k; ++j) BB(j) *= inv;
    }
    for (int j = 0; j < k; ++j) Z[(int64_t)j * ldz + v] = BB(j);
    last[v] = BB(k - 1);
  }
#undef DL
#undef DD
#undef DU
#undef DU2
#undef BB
#undef PIV
}

// Inverse iteration leaves each z_v off by about u |T| / gap along the
// eigenvectors of nearby eigenvalues, so vectors of close but unequal
// eigenvalues overlap far above the rounding level (a sine/cosine pair of a
// wave-like snapshot set: ~1e-8).  One sweep replaces every z_v at once by
// z_v - sum_{c < v} (z_c . z_v) z_c, normalised, with the z_c of the sweep's
// input (eigenvalues descending, so the larger eigenvalue's vector leads);
// an overlap e drops to O(e^2), and two sweeps reach the rounding level.
// Each vector's correction is a combination of vectors of nearby
// eigenvalues (the overlaps with the rest are already at rounding level),
// so the residuals stay as they are.  One workgroup per vector; pass 0 reads
// Z and writes Z2, pass 1 reads Z2, writes Z and refreshes last[].
__global__ __launch_bounds__(256) void ortho_sweep_kernel(const LzNode* __restrict__ nodes, int pass) {
  const LzNode n = nodes[blockIdx.z];
  const int k = n.kk;
  const int v = blockIdx.x;
  if (v >= k) return;
  const double* __restrict__ src = pass == 0 ? n.Z : n.Z2;
  double* __restrict__ dst = pass == 0 ? n.Z2 : n.Z;
  const int64_t ldz = k;
  extern __shared__ double osh[];
  double* zv = osh;      // k
  double* d = osh + k;   // v overlaps
  __shared__ double red[4];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int r = t; r < k; r += 256) zv[r] = src[(int64_t)r * ldz + v];
  __syncthreads();
  for (int c = t; c < v; c += 256) {
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += src[(int64_t)r * ldz + c] * zv[r];
    d[c] = s;
  }
  __syncthreads();
  // row r of the correction: sum_c Z[r, c] d[c], one wave per row
  for (int r = wv; r < k; r += 4) {
    double s = 0.0;
    for (int c = lane; c < v; c += 64) s += src[(int64_t)r * ldz + c] * d[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) zv[r] -= s;
  }
  __syncthreads();
  double nrm = 0.0;
  for (int r = t; r < k; r += 256) nrm += zv[r] * zv[r];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
  if (lane == 0) red[wv] = nrm;
  __syncthreads();
  nrm = red[0] + red[1] + red[2] + red[3];
  const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
  for (int r = t; r < k; r += 256) dst[(int64_t)r * ldz + v] = zv[r] * inv;
  if (pass == 1 && t == 0) n.last[v] = zv[k - 1] * inv;
}

// ---- Full spectra of mid-size matrices (m <= kHhMaxM): Householder ------------
// A full run needs every eigenpair, so the Krylov iteration has no early stop
// to gain from; the orthogonal reduction Q^T G Q = T (Householder, Golub & Van
// Loan, Matrix Computations, Sec. 8.3.1) gives the same (alpha, beta, Q) a
// complete Lanczos run would, backward stable and in a fixed number of steps
// with no host decisions.  One workgroup per matrix; the work copy A of G
// (Z2, leading dimension m rounded up to even) stays in the L2 cache.
//
// Step k: the pending rank-2 update of step k-1 is applied to column k, whose
// tail x = A[k+1:, k] gives the reflector H_k = I - tau v v^T (v[k+1] = 1,
// H_k x = beta_k e_{k+1}); then one pass over the trailing block both applies
// the pending update and forms p = A v, and w = tau p - (tau^2 / 2)(p^T v) v
// becomes the next pending update A -= v w^T + w v^T.  Each trailing element
// is read and written once per step.  The reflectors are kept below the
// subdiagonal of A (tau_k in w[k]) for formq_kernel.
constexpr int kHhMaxM = 256;
typedef __attribute__((address_space(1))) dv2 gdv2;
constexpr int kHhThreads = 1024;
constexpr int kHhRowPairs = kHhMaxM / 2;            // threads along the rows, two rows each
constexpr int kHhGroups = kHhThreads / kHhRowPairs;  // column groups

__global__ __launch_bounds__(kHhThreads) void tridiag_kernel(const LzNode* __restrict__ nodes,
                                                             const int* __restrict__ list) {
  const LzNode n = nodes[list ? list[blockIdx.x] : blockIdx.x];
  const int m = (int)n.m;
  const int lda = m + (m & 1);
  double* A = n.Z2;
  double* tau = n.w;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __shared__ double sv[kHhMaxM], sw[kHhMaxM], nv[kHhMaxM];
  __shared__ double pp[kHhGroups][kHhMaxM];
  __shared__ double red[kHhThreads / 64];
  __shared__ double scal[2];
  for (int64_t e = t; e < (int64_t)lda * m; e += kHhThreads) {
    const int j = (int)(e / lda), i = (int)(e - (int64_t)j * lda);
    A[e] = (i < m) ? n.G[(int64_t)j * n.ldg + i] : 0.0;
  }
  for (int i = t; i < kHhMaxM; i += kHhThreads) {
    sv[i] = 0.0;
    sw[i] = 0.0;
  }
  __syncthreads();
  auto block_sum = [&](double x) {
    x = wave_sum(x);
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kHhThreads / 64; ++q) s += red[q];
    return s;
  };
  const int rp = t % kHhRowPairs, cg = t / kHhRowPairs;
  const int r = 2 * rp;
  for (int k = 0; k + 2 < m; ++k) {
    // column k with the pending update; its tail is x
    double xi = 0.0;
    if (t >= k && t < m) xi = A[t + (int64_t)k * lda] - (sv[t] * sw[k] + sw[t] * sv[k]);
    if (t == k) scal[0] = xi;
    if (t == k + 1) scal[1] = xi;
    const double tail = block_sum((t >= k + 2 && t < m) ? xi * xi : 0.0);
    const double d = scal[0], x0 = scal[1];
    double beta = x0, tk = 0.0, scale = 0.0;
    if (tail > 0.0) {
      const double nrm = sqrt(x0 * x0 + tail);
      beta = (x0 >= 0.0) ? -nrm : nrm;
      tk = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    if (t < kHhMaxM) nv[t] = (t == k + 1) ? 1.0 : ((t >= k + 2 && t < m) ? xi * scale : 0.0);
    if (t >= k + 2 && t < m) A[t + (int64_t)k * lda] = xi * scale;
    if (t == 0) {
      n.alpha[k] = d;
      n.beta[k] = beta;
      tau[k] = tk;
    }
    __syncthreads();
    // trailing block (rows and columns k+1 ..): pending update, then p = A v
    double acc0 = 0.0, acc1 = 0.0;
    if (r + 1 >= k + 1 && r < m) {
      const double v0 = sv[r], v1 = sv[r + 1], w0 = sw[r], w1 = sw[r + 1];
      double* col = A + r;
      int j = k + 1 + cg;
      // eight columns' loads issued before any of their stores (a store
      // to A keeps later loads of A from moving above it)
      constexpr int U = 8;
      for (; j + (U - 1) * kHhGroups < m; j += U * kHhGroups) {
        dv2 a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = *(gptr<dv2>)as_global(col + (int64_t)(j + u * kHhGroups) * lda);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int jj = j + u * kHhGroups;
          const double vj = sv[jj], wj = sw[jj], nj = nv[jj];
          const double a0 = a[u][0] - (v0 * wj + w0 * vj), a1 = a[u][1] - (v1 * wj + w1 * vj);
          *(gdv2*)(col + (int64_t)jj * lda) = dv2{a0, a1};
          acc0 += a0 * nj;
          acc1 += a1 * nj;
        }
      }
      for (; j < m; j += kHhGroups) {
        const dv2 a = *(gptr<dv2>)as_global(col + (int64_t)j * lda);
        const double vj = sv[j], wj = sw[j], nj = nv[j];
        const double a0 = a[0] - (v0 * wj + w0 * vj), a1 = a[1] - (v1 * wj + w1 * vj);
        *(gdv2*)(col + (int64_t)j * lda) = dv2{a0, a1};
        acc0 += a0 * nj;
        acc1 += a1 * nj;
      }
    }
    pp[cg][r] = acc0;
    pp[cg][r + 1] = acc1;
    __syncthreads();
    // w = tau p - (tau / 2)(tau p . v) v
    double pi = 0.0, vi = 0.0;
    if (t >= k + 1 && t < m) {
#pragma unroll
      for (int q = 0; q < kHhGroups; ++q) pi += pp[q][t];
      pi *= tk;
      vi = nv[t];
    }
    const double K = 0.5 * tk * block_sum(pi * vi);
    if (t < kHhMaxM) {
      sv[t] = nv[t];
      sw[t] = (t >= k + 1 && t < m) ? pi - K * vi : 0.0;
    }
    __syncthreads();
  }
  // the last 2 x 2 block (or the single entry)
  if (t == 0) {
    if (m >= 2) {
      auto at = [&](int i, int j) { return A[i + (int64_t)j * lda] - (sv[i] * sw[j] + sw[i] * sv[j]); };
      n.alpha[m - 2] = at(m - 2, m - 2);
      n.beta[m - 2] = at(m - 1, m - 2);
      n.alpha[m - 1] = at(m - 1, m - 1);
      tau[m - 2] = 0.0;
    } else if (m == 1) {
      n.alpha[0] = A[0];
    }
    if (m >= 1) {
      n.beta[m - 1] = 0.0;
      tau[m - 1] = 0.0;
    }
  }
}

// Q = H_0 H_1 ... H_{m-3}: column j is H_0 ... H_{j-1} e_j (reflectors with
// index >= j leave e_j alone).  Sixteen columns per workgroup (one wavefront
// each, four rows per lane); the reflectors pass through LDS in chunks of 64,
// highest index first.
constexpr int kFqChunk = 64;
__global__ __launch_bounds__(1024) void formq_kernel(const LzNode* __restrict__ nodes, const int* __restrict__ list) {
  const LzNode n = nodes[list ? list[blockIdx.z] : blockIdx.z];
  const int m = (int)n.m;
  const int lda = m + (m & 1);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int j = blockIdx.x * 16 + wave;
  if (blockIdx.x * 16 >= m) return;  // whole workgroup
  extern __shared__ double rf[];      // kFqChunk x m reflectors, then their tau
  double* rt = rf + (size_t)kFqChunk * m;
  double q[kHhMaxM / 64];
#pragma unroll
  for (int s = 0; s < kHhMaxM / 64; ++s) q[s] = (lane + 64 * s == j) ? 1.0 : 0.0;
  const int jmax = min(m, (int)blockIdx.x * 16 + 16);  // highest column + 1 in this workgroup
  for (int c1 = jmax - 1; c1 > 0; c1 -= kFqChunk) {
    const int c0 = max(0, c1 - kFqChunk);  // reflectors c0 .. c1-1
    const int nc = c1 - c0;
    __syncthreads();
    for (int e = t; e < nc * m; e += 1024) {
      const int c = e / m, row = e - c * m, kk = c0 + c;
      rf[e] = (row == kk + 1) ? 1.0 : (row >= kk + 2 ? n.Z2[row + (int64_t)kk * lda] : 0.0);
    }
    for (int c = t; c < nc; c += 1024) rt[c] = n.w[c0 + c];
    __syncthreads();
    if (j < m)
      for (int kk = min(c1, j) - 1; kk >= c0; --kk) {
        const double tk = rt[kk - c0];
        if (tk == 0.0) continue;
        const double* v = rf + (size_t)(kk - c0) * m;
        double dot = 0.0;
#pragma unroll
        for (int s = 0; s < kHhMaxM / 64; ++s) {
          const int row = lane + 64 * s;
          if (row < m) dot += v[row] * q[s];
        }
        dot = tk * wave_sum(dot);
#pragma unroll
        for (int s = 0; s < kHhMaxM / 64; ++s) {
          const int row = lane + 64 * s;
          if (row < m) q[s] -= dot * v[row];
        }
      }
  }
  if (j < m)
#pragma unroll
    for (int s = 0; s < kHhMaxM / 64; ++s) {
      const int row = lane + 64 * s;
      if (row < m) n.Q[(int64_t)j * m + row] = q[s];
    }
}

// make the largest-magnitude entry of every column positive (one wave per column)
__global__ __launch_bounds__(256) void sign_fix_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.z];
  double* V = n.V;
  const int64_t ldv = n.ldv, m = n.m, ncols = n.b;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= ncols) return;
  double* col = V + c * ldv;
  double best = -1.0;
  int64_t arg = m;
  for (int64_t r = lane; r < m; r += 64) {
    const double a = fabs(col[r]);
    if (a > best) { best = a; arg = r; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int64_t oa = __shfl_xor(arg, off, 64);
    if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; }
  }
  const double sgn = (arg < m && col[arg] < 0.0) ? -1.0 : 1.0;
  if (sgn < 0.0)
    for (int64_t r = lane; r < m; r += 64) col[r] = -col[r];
}

__global__ void write_lambda_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.z];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n.m; i += (int64_t)gridDim.x * blockDim.x)
    n.lambda[i] = (i < n.b) ? n.theta[i] : 0.0;
}



size_t al(size_t x) { return (x + 255) / 256 * 256; }

// the rounding level and the trace check of a device-only full run; the
// column table of Q and the lift's rank for the back-transformation
__global__ __launch_bounds__(256) void hh_finish_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.x];
  const int k = n.kk;
  __shared__ double part[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) s += n.theta[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tr = *n.tr;
    const double theta_min = k > 0 ? n.theta[k - 1] : 0.0;
    *n.floor_out = fmax(fmax(-theta_min, 0.0), 0.1 * n.u_p * fabs(tr));
    n.diag_out[0] = tr;
    n.diag_out[1] = part[0] + part[1] + part[2] + part[3];
  }
}

__global__ __launch_bounds__(256) void hh_qtable_kernel(const LzNode* __restrict__ nodes) {
  const LzNode n = nodes[blockIdx.z];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) *n.qrank = n.b;
  if (j >= n.kk) return;
  n.qcols[j] = n.Q + j * n.m;
  n.qrbs[j] = kRowBlock;
  n.qrows[j] = n.m;
}

}  // namespace

size_t hh_node_bytes() { return sizeof(LzNode); }

bool hh_available() {
  static const bool force_lanczos = [] {
    const char* e = std::getenv("HAPOD_FULL_LANCZOS");
    return e && e[0] == '1';
  }();
  return !force_lanczos;
}

// Q (m x (m + 1)), w, alpha, beta (m + 1), theta, Z, last, Z2 (m x (m + 1)),
// trace, the back-transformation's column table and rank
size_t hh_scratch_bytes(int64_t m) {
  const size_t k = (size_t)m;
  return al(sizeof(double) * k * (k + 1)) + al(sizeof(double) * k) * 5 + al(sizeof(double) * (k + 1)) +
         al(sizeof(double) * k * k) + al(sizeof(double) * k * (k + 1)) + al(sizeof(double)) + al(sizeof(void*) * k) +
         al(sizeof(int64_t) * k) * 2 + al(sizeof(int64_t));
}

void hh_describe(int64_t m, const double* G, int64_t ldg, double* lambda, double* V, int64_t ldv, char* scratch,
                 double u_p, double* floor_out, double* diag_out, void* node, LiftNode* lift) {
  const size_t k = (size_t)m;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = scratch + o;
    o += al(bytes);
    return p;
  };
  LzNode n{};
  n.G = G;
  n.ldg = ldg;
  n.m = m;
  n.Q = (double*)take(sizeof(double) * k * (k + 1));
  n.w = (double*)take(sizeof(double) * k);
  n.alpha = (double*)take(sizeof(double) * k);
  n.beta = (double*)take(sizeof(double) * (k + 1));
  n.theta = (double*)take(sizeof(double) * k);
  n.last = (double*)take(sizeof(double) * k);
  n.wn = (double*)take(sizeof(double) * k);
  n.Z = (double*)take(sizeof(double) * k * k);
  n.Z2 = (double*)take(sizeof(double) * k * (k + 1));
  n.tr = (double*)take(sizeof(double));
  n.h = n.wn;  // unused by the full-run kernels
  n.qcols = (const void**)take(sizeof(void*) * k);
  n.qrbs = (int64_t*)take(sizeof(int64_t) * k);
  n.qrows = (int64_t*)take(sizeof(int64_t) * k);
  n.qrank = (int64_t*)take(sizeof(int64_t));
  n.V = V;
  n.lambda = lambda;
  n.ldv = ldv;
  n.nrc = 1;
  n.kk = (int32_t)m;
  n.b = (int32_t)m;
  n.floor_out = floor_out;
  n.diag_out = diag_out;
  n.u_p = u_p;
  std::memcpy(node, &n, sizeof(n));
  LiftNode l{};
  l.cols = (const void* const*)n.qcols;
  l.rbs = n.qrbs;
  l.crows = n.qrows;
  l.B = n.Z;
  l.rank = n.qrank;
  l.out = V;
  l.n = m;
  l.ldb = m;
  l.ocs = ldv;
  l.obs = kRowBlock;
  l.m = (int32_t)m;
  l.row_tiles = (int32_t)((m + kLiftTileM - 1) / kLiftTileM);
  l.col_tiles = (int32_t)((m + kLiftTileN - 1) / kLiftTileN);
  l.rt_per = 1;
  *lift = l;
}

hapod_status hh_launch(const void* d_nodes_v, int nn, int64_t m_max, const LiftNode* d_lifts, int lift_items,
                       hipStream_t stream) {
  if (nn <= 0 || m_max <= 0) return HAPOD_OK;
  const LzNode* dn = (const LzNode*)d_nodes_v;
  const int kk = (int)m_max;
  hipLaunchKernelGGL(setup_kernel, dim3(1, 1, nn), dim3(1024), 0, stream, dn);
  hipLaunchKernelGGL(tridiag_kernel, dim3(nn), dim3(kHhThreads), 0, stream, dn, (const int*)nullptr);
  static bool fq_attr = false;
  if (!fq_attr) {
    HAPOD_HIP(hipFuncSetAttribute((const void*)formq_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(sizeof(double) * ((size_t)kFqChunk * kHhMaxM + kFqChunk))));
    fq_attr = true;
  }
  hipLaunchKernelGGL(formq_kernel, dim3((unsigned)((m_max + 15) / 16), 1, nn), dim3(1024),
                     sizeof(double) * ((size_t)kFqChunk * m_max + kFqChunk), stream, dn, (const int*)nullptr);
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)((kk + 3) / 4), 1, nn), dim3(256), sizeof(double) * 3 * (size_t)kk,
                     stream, dn);
  hipLaunchKernelGGL(inviter_kernel, dim3((unsigned)kk, 1, nn), dim3(64), (sizeof(double) * 5 + sizeof(int)) * (size_t)kk,
                     stream, dn);
  for (int pass = 0; pass < 2; ++pass)
    hipLaunchKernelGGL(ortho_sweep_kernel, dim3((unsigned)kk, 1, nn), dim3(256), sizeof(double) * 2 * (size_t)kk,
                       stream, dn, pass);
  hipLaunchKernelGGL(hh_qtable_kernel, dim3((unsigned)((kk + 255) / 256), 1, nn), dim3(256), 0, stream, dn);
  HAPOD_HIP(hipGetLastError());
  HAPOD_TRY(launch_lift(0, d_lifts, nn, lift_items, stream));
  hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)((kk + 3) / 4), 1, nn), dim3(256), 0, stream, dn);
  hipLaunchKernelGGL(write_lambda_kernel, dim3(64, 1, nn), dim3(256), 0, stream, dn);
  hipLaunchKernelGGL(hh_finish_kernel, dim3(nn), dim3(256), 0, stream, dn);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status wide_eigh_batch(std::vector<WideJob>& jobs, double u_p, wide_alloc_fn alloc, wide_free_fn release,
                             void* ctx, hipStream_t stream) {
  const int nn = (int)jobs.size();
  if (nn == 0) return HAPOD_OK;
  for (auto& jb : jobs)
    if (jb.full && jb.m > kMaxSteps) {
      set_error("wide_eigh: a full run needs m <= 768");
      return HAPOD_E_UNSUPPORTED;
    }
  // ---- which matrices take which step kernels ---------------------------------------
  // small matrices: the fused one-workgroup kernel; mid-size ones alone or
  // few: the cooperative kernel (as many as the compute units hold, one
  // workgroup each); the rest: the step kernels
  int n_small = 0;
  for (auto& jb : jobs) n_small += (jb.m > 0 && jb.m <= kFusedMaxM);
  auto fused_node = [&](int i) {
    return jobs[i].m <= kFusedMaxM && (jobs[i].m <= kFusedAloneMaxM || n_small >= kFusedBatchMin);
  };
  static int n_cu = 0;
  if (n_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      n_cu = 0;
    (void)hipGetLastError();
    if (n_cu <= 0) n_cu = 1;
  }
  // (the cooperative grid is the widest matrix's workgroup count times the
  // number of matrices, one workgroup per CU by its LDS: all must be resident)
  // full runs of at most kHhMaxM columns: Householder reduction instead of
  // the Krylov iteration (HAPOD_FULL_LANCZOS=1 keeps them on Lanczos)
  const bool force_lanczos = !hh_available();
  std::vector<char> hh(nn, 0);
  std::vector<int> hh_list;
  for (int i = 0; i < nn; ++i)
    if (!force_lanczos && jobs[i].full && jobs[i].m > 0 && jobs[i].m <= kHhMaxM) {
      hh[i] = 1;
      hh_list.push_back(i);
    }
  std::vector<char> coop(nn, 0);
  {
    int count = 0;
    for (int i = 0; i < nn; ++i) {
      const int64_t m = jobs[i].m;
      if (m <= 0 || hh[i] || fused_node(i) || m > kCoopMaxM) continue;
      if ((count + 1) * coop_pick(kCoopMaxM) > n_cu) break;
      coop[i] = 1;
      ++count;
    }
  }
  // ---- scratch: one block for every matrix -----------------------------------------
  std::vector<size_t> off(nn);
  std::vector<int> kmax(nn), nrc(nn);
  size_t total = 0;
  auto sizes = [&](int i, bool assign, char* base, LzNode* nd) {
    const int64_t m = jobs[i].m;
    const int k = (int)std::min<int64_t>(m, kMaxSteps);
    size_t o = assign ? off[i] : total;
    auto take = [&](size_t bytes) {
      char* p = base ? base + o : nullptr;
      o += al(bytes);
      return p;
    };
    double* Q = (double*)take(sizeof(double) * m * (k + 1));
    double* w = (double*)take(sizeof(double) * m);
    const int nr = (int)((m + kProjRows - 1) / kProjRows);
    double* h = (double*)take(sizeof(double) * (size_t)(k + 1) * nr);
    double* alpha = (double*)take(sizeof(double) * k);
    double* beta = (double*)take(sizeof(double) * (k + 1));
    double* theta = (double*)take(sizeof(double) * k);
    double* e2 = nullptr;  // bisection works in LDS
    double* Z = (double*)take(sizeof(double) * (size_t)k * k);
    double* last = (double*)take(sizeof(double) * k);
    // (k + 1 columns: the Householder work copy's leading dimension is m rounded up to even)
    double* Z2 = (double*)take(sizeof(double) * (size_t)k * (k + 1));
    double* isc = nullptr;  // inverse iteration works in LDS
    int* ipiv = nullptr;
    double* tr = (double*)take(sizeof(double));
    take(sizeof(void*) * k);     // Ritz-lift column table
    take(sizeof(int64_t) * k);   // its row-block strides
    take(sizeof(int64_t) * k);   // its row counts
    take(sizeof(int64_t));       // its rank
    double* wn = (double*)take(sizeof(double) * nr);
    const int cp = coop_pick(m);
    const int64_t xlen = std::max<int64_t>((int64_t)cp * (k + 2), m + cp);
    double* xbuf = (coop[i] ? (double*)take(sizeof(double) * 3 * xlen) : nullptr);
    if (nd) {
      *nd = LzNode{};
      nd->G = jobs[i].G;
      nd->ldg = jobs[i].ldg;
      nd->m = m;
      nd->Q = Q; nd->w = w; nd->h = h; nd->alpha = alpha; nd->beta = beta; nd->theta = theta; nd->e2 = e2;
      nd->Z = Z; nd->last = last; nd->isc = isc; nd->ipiv = ipiv; nd->tr = tr; nd->wn = wn;
      nd->V = jobs[i].V;
      nd->lambda = jobs[i].lambda;
      nd->ldv = jobs[i].ldv;
      nd->nrc = nr;
      nd->coop_p = coop[i] ? cp : 0;
      nd->xbuf = xbuf;
      nd->xlen = xlen;
      nd->Z2 = Z2;
    }
    kmax[i] = k;
    nrc[i] = nr;
    if (!assign) {
      off[i] = total;
      total = o;
    }
    return o;
  };
  for (int i = 0; i < nn; ++i) sizes(i, false, nullptr, nullptr);
  const size_t o_nodes = total;
  total = al(total + sizeof(LzNode) * nn);
  const size_t o_act = total;
  total = al(total + sizeof(int) * nn);
  const size_t o_gb = total;
  total = al(total + sizeof(double) * 2 * nn);
  const size_t o_lift = total;
  total = al(total + sizeof(LiftNode) * nn);
  const size_t o_hh = total;
  total = al(total + sizeof(int) * nn);
  const size_t o_bar = total;  // barrier counters, then the error flag
  total = al(total + sizeof(unsigned) * (nn + 1));
  char* blk = (char*)alloc(ctx, total);
  if (!blk) {
    set_error("wide_eigh: scratch allocation failed");
    return HAPOD_E_NOMEM;
  }
  struct Rel {
    wide_free_fn f;
    void* c;
    void* p;
    ~Rel() { f(c, p); }
  } rel{release, ctx, blk};
  std::vector<LzNode> hn(nn);
  unsigned* dbar = (unsigned*)(blk + o_bar);
  int* derr = (int*)(dbar + nn);
  for (int i = 0; i < nn; ++i) {
    sizes(i, true, blk, &hn[i]);
    hn[i].bar = dbar + i;
  }
  HAPOD_TRY(launch_zero_bytes(dbar, sizeof(unsigned) * (nn + 1), stream));
  LzNode* dn = (LzNode*)(blk + o_nodes);
  int* dact = (int*)(blk + o_act);
  double* dgb = (double*)(blk + o_gb);
  int64_t m_max = 0;
  int kmax_all = 0, nrc_max = 1;
  for (int i = 0; i < nn; ++i) {
    m_max = std::max(m_max, jobs[i].m);
    kmax_all = std::max(kmax_all, kmax[i]);
    nrc_max = std::max(nrc_max, nrc[i]);
  }
  HAPOD_HIP(hipMemcpyAsync(dn, hn.data(), sizeof(LzNode) * nn, hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(setup_kernel, dim3(1, 1, nn), dim3(1024), 0, stream, dn);
  hipLaunchKernelGGL(lanczos_init_kernel, dim3(64, 1, nn), dim3(256), 0, stream, dn);
  hipLaunchKernelGGL(finish_kernel, dim3(1, 1, nn), dim3(1024), 0, stream, dn, (const int*)nullptr, -1);
  HAPOD_HIP(hipGetLastError());
  // the rounding level of each G's spectrum, for the stopping test
  std::vector<double> trace(nn, 0.0), floor_trace(nn);
  for (int i = 0; i < nn; ++i)
    HAPOD_HIP(hipMemcpyAsync(&trace[i], hn[i].tr, sizeof(double), hipMemcpyDeviceToHost, stream));
  HAPOD_HIP(hipStreamSynchronize(stream));
  for (int i = 0; i < nn; ++i) floor_trace[i] = 0.1 * u_p * std::fabs(trace[i]);
  std::vector<int> steps(kmax), act;
  std::vector<char> stopped(nn, 0);
  std::vector<double> prev_check(nn, 0.0);
  // Householder nodes: the reduction, then Q from its reflectors
  if (!hh_list.empty()) {
    int* dhh = (int*)(blk + o_hh);
    const unsigned nh = (unsigned)hh_list.size();
    HAPOD_HIP(hipMemcpyAsync(dhh, hh_list.data(), sizeof(int) * nh, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(tridiag_kernel, dim3(nh), dim3(kHhThreads), 0, stream, dn, dhh);
    HAPOD_HIP(hipGetLastError());
    int64_t hm = 0;
    for (int i : hh_list) hm = std::max(hm, jobs[i].m);
    const size_t shm = sizeof(double) * ((size_t)kFqChunk * hm + kFqChunk);
    static bool fq_attr = false;
    if (!fq_attr) {
      HAPOD_HIP(hipFuncSetAttribute((const void*)formq_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(sizeof(double) * ((size_t)kFqChunk * kHhMaxM + kFqChunk))));
      fq_attr = true;
    }
    hipLaunchKernelGGL(formq_kernel, dim3((unsigned)((hm + 15) / 16), 1, nh), dim3(1024), shm, stream, dn, dhh);
    HAPOD_HIP(hipGetLastError());
  }
  // the active list: fused matrices, then cooperative ones, then the rest
  for (int i = 0; i < nn; ++i) stopped[i] = (kmax[i] == jobs[i].m);
  for (int i = 0; i < nn; ++i)
    if (jobs[i].m > 0 && !hh[i] && fused_node(i)) act.push_back(i);
  for (int i = 0; i < nn; ++i)
    if (jobs[i].m > 0 && !hh[i] && coop[i]) act.push_back(i);
  for (int i = 0; i < nn; ++i)
    if (jobs[i].m > 0 && !hh[i] && !fused_node(i) && !coop[i]) act.push_back(i);
  const char* venv = std::getenv("HAPOD_VERBOSE");
  const bool verbose = venv && venv[0] == '1';
  bool act_dirty = true;
  for (int j = 0; j < kmax_all && !act.empty(); ++j) {
    // matrices whose Krylov space is complete (j = k) leave the list
    {
      std::vector<int> keep;
      for (int i : act)
        if (j < kmax[i]) keep.push_back(i);
      if (keep.size() != act.size()) {
        act.swap(keep);
        act_dirty = true;
        if (act.empty()) break;
      }
    }
    if (act_dirty) {
      HAPOD_HIP(hipMemcpyAsync(dact, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice, stream));
      act_dirty = false;
    }
    const unsigned na = (unsigned)act.size();
    unsigned nf = 0;
    while (nf < na && fused_node(act[nf])) ++nf;
    // small matrices: one fused launch per period of kCheckEvery steps (each
    // stops at its own k)
    if (nf > 0 && j % kCheckEvery == 0) {
      static bool attr_set = false;
      if (!attr_set) {
        HAPOD_HIP(hipFuncSetAttribute((const void*)lanczos_fused_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(kFusedQCache * sizeof(double))));
        attr_set = true;
      }
      hipLaunchKernelGGL(lanczos_fused_kernel, dim3(1, 1, nf), dim3(kFusedThreads), kFusedQCache * sizeof(double),
                         stream, dn, dact, j, j + kCheckEvery, kBreakdownTol);
    }
    unsigned nc = 0;
    while (nf + nc < na && coop[act[nf + nc]]) ++nc;
    if (nc > 0 && j % kCheckEvery == 0) {
      static bool coop_attr = false;
      if (!coop_attr) {
        HAPOD_HIP(hipFuncSetAttribute((const void*)lanczos_coop_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(coop_lds_doubles(kCoopMaxM, coop_pick(kCoopMaxM)) * sizeof(double))));
        coop_attr = true;
      }
      size_t shm = 0;
      int pmax = 0;
      for (unsigned a = nf; a < nf + nc; ++a) {
        const int64_t m = jobs[act[a]].m;
        shm = std::max(shm, coop_lds_doubles(m, coop_pick(m)) * sizeof(double));
        pmax = std::max(pmax, coop_pick(m));
      }
      HAPOD_TRY(launch_zero_bytes(dbar, sizeof(unsigned) * nn, stream));
      const int* dact_c = dact + nf;
      int j0 = j, j1 = j + kCheckEvery;
      double tol = kBreakdownTol;
      void* args[] = {(void*)&dn, (void*)&dact_c, (void*)&j0, (void*)&j1, (void*)&tol, (void*)&derr};
      HAPOD_HIP(hipLaunchCooperativeKernel((const void*)lanczos_coop_kernel, dim3((unsigned)pmax, 1, nc),
                                           dim3(kCoopThreads), args, (unsigned)shm, stream));
    }
    const unsigned nr = na - nf - nc;
    const int* dact_r = dact + nf + nc;
    int64_t am = 0;
    int anrc = 1;
    for (unsigned a = nf + nc; a < na; ++a) {
      am = std::max(am, jobs[act[a]].m);
      anrc = std::max(anrc, nrc[act[a]]);
    }
    if (nr > 0) {
      hipLaunchKernelGGL(matvec_kernel, dim3((unsigned)((am + 3) / 4), 1, nr), dim3(256), 0, stream, dn, dact_r, j);
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(proj_partial_kernel, dim3((unsigned)((j + kProjCols) / kProjCols), (unsigned)anrc, nr),
                           dim3(256), 0, stream, dn, dact_r, j, pass == 0 ? 1 : 0);
        hipLaunchKernelGGL(update_kernel, dim3((unsigned)((am + 63) / 64), 1, nr), dim3(256), 0, stream, dn, dact_r,
                           j);
      }
      hipLaunchKernelGGL(finish_kernel, dim3(1, 1, nr), dim3(1024), 0, stream, dn, dact_r, j);
      // restart the matrices whose step broke down
      hipLaunchKernelGGL(breakdown_kernel, dim3(1, 1, nr), dim3(1024), 0, stream, dn, dact_r, j, kBreakdownTol);
    }
    // Stop once the Krylov space has taken in everything above the rounding
    // level of G: the residual norms beta_j then stop falling (they sit at
    // that level).  Test every kCheckEvery steps: beta_j at or below
    // u_p trace(G) / 10, or beta_j fell less than kPlateau-fold over the last
    // period after having fallen 1000-fold from beta_0.  Full runs never stop.
    if ((j + 1) % kCheckEvery == 0) {
      bool any = false;
      for (int i : act) any |= !jobs[i].full && j + 1 < kmax[i];
      if (!any) continue;
      hipLaunchKernelGGL(gather_beta_kernel, dim3((na + 255) / 256), dim3(256), 0, stream, dn, dact, (int)na, j, dgb);
      std::vector<double> gb(2 * na);
      HAPOD_HIP(hipMemcpyAsync(gb.data(), dgb, sizeof(double) * 2 * na, hipMemcpyDeviceToHost, stream));
      HAPOD_HIP(hipStreamSynchronize(stream));
      std::vector<int> keep;
      for (unsigned a = 0; a < na; ++a) {
        const int i = act[a];
        const double bj = gb[2 * a], b0 = gb[2 * a + 1];
        bool stop = false;
        if (!jobs[i].full && j + 1 < kmax[i]) {
          if (verbose)
            std::fprintf(stderr, "[hapod wide] m=%lld step %d beta %.3e floor_trace %.3e\n", (long long)jobs[i].m,
                         j + 1, bj, floor_trace[i]);
          const bool plateau = prev_check[i] > 0.0 && bj >= kPlateau * prev_check[i] && bj <= 1e-3 * b0;
          prev_check[i] = bj;
          stop = j + 1 >= kMinSteps && (bj <= floor_trace[i] || plateau);
        }
        if (stop) {
          steps[i] = j + 1;
          stopped[i] = 1;
        } else {
          keep.push_back(i);
        }
      }
      if (keep.size() != act.size()) {
        act.swap(keep);
        act_dirty = true;
      }
    }
  }
  HAPOD_HIP(hipGetLastError());
  {
    int e = 0;
    HAPOD_HIP(hipMemcpyAsync(&e, derr, sizeof(int), hipMemcpyDeviceToHost, stream));
    HAPOD_HIP(hipStreamSynchronize(stream));
    if (e) {
      set_error("wide_eigh: a barrier of the cooperative Lanczos kernel timed out");
      return HAPOD_E_DEVICE;
    }
  }
  // ---- tridiagonal eigenproblems of the steps taken ----------------------------------
  int kk_max = 0;
  for (int i = 0; i < nn; ++i) {
    hn[i].kk = jobs[i].m > 0 ? steps[i] : 0;
    kk_max = std::max(kk_max, hn[i].kk);
  }
  HAPOD_HIP(hipMemcpyAsync(dn, hn.data(), sizeof(LzNode) * nn, hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)((kk_max + 3) / 4), 1, nn), dim3(256),
                     sizeof(double) * 3 * (size_t)kk_max, stream, dn);
  HAPOD_HIP(hipGetLastError());
  hipLaunchKernelGGL(inviter_kernel, dim3((unsigned)kk_max, 1, nn), dim3(64),
                     (sizeof(double) * 5 + sizeof(int)) * (size_t)kk_max, stream, dn);
  HAPOD_HIP(hipGetLastError());
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(ortho_sweep_kernel, dim3((unsigned)kk_max, 1, nn), dim3(256),
                       sizeof(double) * 2 * (size_t)kk_max, stream, dn, pass);
    HAPOD_HIP(hipGetLastError());
  }
  // ---- choose each converged leading block (host) ----------------------------------
  std::vector<std::vector<double>> th(nn), lz(nn), bet(nn);
  for (int i = 0; i < nn; ++i) {
    const int kk = hn[i].kk;
    th[i].resize(kk);
    lz[i].resize(kk);
    bet[i].resize(kk);
    if (kk == 0) continue;
    HAPOD_HIP(hipMemcpyAsync(th[i].data(), hn[i].theta, sizeof(double) * kk, hipMemcpyDeviceToHost, stream));
    HAPOD_HIP(hipMemcpyAsync(lz[i].data(), hn[i].last, sizeof(double) * kk, hipMemcpyDeviceToHost, stream));
    HAPOD_HIP(hipMemcpyAsync(bet[i].data(), hn[i].beta, sizeof(double) * kk, hipMemcpyDeviceToHost, stream));
  }
  HAPOD_HIP(hipStreamSynchronize(stream));
  std::vector<LiftNode> lifts;
  int items = 0, b_max = 0;
  for (int i = 0; i < nn; ++i) {
    const int kk = hn[i].kk;
    const int64_t m = jobs[i].m;
    if (kk == 0) continue;
    const double bk = bet[i][kk - 1];
    const double theta_min = *std::min_element(th[i].begin(), th[i].end());
    const double floor_abs = std::max(std::max(-theta_min, 0.0), floor_trace[i]);
    // a Ritz pair counts as converged when its residual is below 1e-8 of its
    // own value or below the Gram's rounding level
    int b = 0;
    while (b < kk && std::fabs(bk * lz[i][b]) <= std::max(1e-8 * std::fabs(th[i][b]), floor_abs)) ++b;
    if (kk == m) b = kk;  // complete tridiagonalisation: every pair is exact
    // Ritz vectors of one Krylov space are orthonormal and diagonalise G on it
    // (V^T G V = diag(theta)), so the energy of S on the modes S v_i / sqrt(theta_i)
    // is at least sum theta_i whether or not the pairs have converged: the block
    // is extended by every Ritz value above the noise level max(floor_abs,
    // beta_{k-1}) (below it a Ritz value cannot be told from zero), and only
    // what lies beyond the Krylov space is left unresolved.
    const double noise = std::max(floor_abs, std::fabs(bk));
    if (stopped[i]) {
      int e = b;
      while (e < kk && th[i][e] > noise) ++e;
      b = e;
    }
    double missing = 0.0, captured = 0.0;
    for (int t = b; t < kk; ++t)
      if (th[i][t] > noise) missing += th[i][t];
    for (int t = 0; t < b; ++t) captured += th[i][t];
    if (verbose)
      std::fprintf(stderr, "[hapod wide] m=%lld steps %d block %d theta_1 %.6e theta_min %.3e floor %.3e\n",
                   (long long)m, kk, b, th[i][0], theta_min, floor_abs);
    hn[i].b = b;
    b_max = std::max(b_max, b);
    if (jobs[i].res) {
      WideResult& r = *jobs[i].res;
      r.iterations = kk;
      r.block = b;
      r.floor_abs = floor_abs;
      r.exhausted = stopped[i] != 0;
      r.missing = missing;
      r.unresolved = std::max(0.0, trace[i] - captured);
      r.trace = trace[i];
      r.noise = (b < m) ? noise : 0.0;
    }
    if (b == 0) continue;
    // Ritz vectors V[:, :b] = Q_k Z[:, :b] (FP64 lift GEMM, all matrices in one launch)
    char* tbl = (char*)(hn[i].tr) + al(sizeof(double));
    const void** qcols = (const void**)tbl;
    int64_t* qrbs = (int64_t*)(tbl + al(sizeof(void*) * kmax[i]));
    int64_t* qrows = (int64_t*)((char*)qrbs + al(sizeof(int64_t) * kmax[i]));
    int64_t* drank = (int64_t*)((char*)qrows + al(sizeof(int64_t) * kmax[i]));
    HAPOD_TRY(launch_fill_colptrs(hn[i].Q, m, kk, 8, qcols, stream));
    HAPOD_TRY(launch_fill_i64(qrbs, kRowBlock, kk, stream));
    HAPOD_TRY(launch_fill_i64(qrows, m, kk, stream));
    HAPOD_TRY(launch_set_scalar_i64(drank, b, stream));
    LiftNode l{};
    l.cols = (const void* const*)qcols;
    l.rbs = qrbs;
    l.crows = qrows;
    l.B = hn[i].Z;
    l.rank = drank;
    l.out = jobs[i].V;
    l.n = m;
    l.ldb = kk;
    l.ocs = jobs[i].ldv;
    l.obs = kRowBlock;
    l.m = kk;
    l.row_tiles = (int32_t)((m + kLiftTileM - 1) / kLiftTileM);
    l.col_tiles = (int32_t)((b + kLiftTileN - 1) / kLiftTileN);
    l.item_base = items;
    items += l.row_tiles * l.col_tiles;
    lifts.push_back(l);
  }
  HAPOD_HIP(hipMemcpyAsync(dn, hn.data(), sizeof(LzNode) * nn, hipMemcpyHostToDevice, stream));
  if (!lifts.empty()) {
    LiftNode* dl = (LiftNode*)(blk + o_lift);
    HAPOD_HIP(hipMemcpyAsync(dl, lifts.data(), sizeof(LiftNode) * lifts.size(), hipMemcpyHostToDevice, stream));
    HAPOD_TRY(launch_lift(0, dl, (int)lifts.size(), items, stream));
    hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)((b_max + 3) / 4), 1, nn), dim3(256), 0, stream, dn);
  }
  hipLaunchKernelGGL(write_lambda_kernel, dim3(64, 1, nn), dim3(256), 0, stream, dn);
  HAPOD_HIP(hipGetLastError());
  HAPOD_HIP(hipStreamSynchronize(stream));
  return HAPOD_OK;
}

hapod_status wide_eigh(const double* G, int64_t ldg, int64_t m, double* lambda, double* V, int64_t ldv, double u_p,
                       wide_alloc_fn alloc, wide_free_fn release, void* ctx, hipStream_t stream, WideResult* res,
                       bool full) {
  if (m <= 0) return HAPOD_OK;
  std::vector<WideJob> jobs(1);
  jobs[0] = WideJob{G, ldg, m, lambda, V, ldv, full, res};
  return wide_eigh_batch(jobs, u_p, alloc, release, ctx, stream);
}

}  // namespace hapod
