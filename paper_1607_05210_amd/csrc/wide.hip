// Eigensolver for Gram matrices too large for one workgroup's Jacobi
// (the wide root of a star tree): the leading eigenpairs of G by Lanczos with
// full reorthogonalisation, in FP64.
//
//   q_0: deterministic pseudo-random unit vector.
//   step j: w = G q_j; two passes of classical Gram-Schmidt against
//           q_0..q_j (h = Q^T w, w -= Q h); alpha_j = sum of the two
//           coefficients of q_j; beta_j = ||w||; q_{j+1} = w / beta_j.
//   T = tridiag(beta, alpha, beta) (k x k).  Its eigenvalues theta_i come from
//   Sturm-sequence bisection (one thread per eigenvalue), its eigenvectors
//   z_i from inverse iteration with a pivoted tridiagonal LU (one thread per
//   eigenvector).  Ritz pairs: (theta_i, Q z_i), residual beta_{k-1} |z_i[k-1]|.
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
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mfma.hpp"
#include "wide.hpp"

namespace hapod {
namespace {

constexpr int kMaxSteps = kWideMaxSteps;
constexpr int kMinSteps = 128;      // no stop before this many steps
constexpr int kCheckEvery = 32;     // stopping test period
constexpr double kPlateau = 0.7;    // beta_j >= 0.7 beta_{j-32}: plateau

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

// q = random, unnormalised (normalised by the finish kernel)
__global__ void lanczos_init_kernel(double* w, int64_t m) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = hash_unit((uint64_t)i * 7919u + 17u);
}

// w[c] = G[:, c] . q  (G symmetric), one wavefront per column
__global__ __launch_bounds__(256) void matvec_kernel(const double* __restrict__ G, int64_t ldg, int64_t m,
                                                     const double* __restrict__ q, double* __restrict__ w) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= m) return;
  const double* col = G + c * ldg;
  double s = 0.0;
  for (int64_t r = lane; r < m; r += 64) s += col[r] * q[r];
  s = wave_sum(s);
  if (lane == 0) w[c] = s;
}

constexpr int kProjCols = 16;    // Lanczos vectors per projection workgroup
constexpr int kProjRows = 1024;  // rows per projection workgroup

// partial[c * nrc + rc] = Q[rows of chunk rc, c] . w[rows of chunk rc], c <= j
__global__ __launch_bounds__(256) void proj_partial_kernel(const double* __restrict__ Q, int64_t m, int j,
                                                           const double* __restrict__ w,
                                                           double* __restrict__ partial, int nrc) {
  __shared__ double red[kProjCols][4];
  const int c0 = blockIdx.x * kProjCols, rc = blockIdx.y;
  const int ncols = min(kProjCols, j + 1 - c0);
  const int64_t r0 = (int64_t)rc * kProjRows, r1 = min(m, r0 + kProjRows);
  double acc[kProjCols];
#pragma unroll
  for (int c = 0; c < kProjCols; ++c) acc[c] = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const double wr = w[r];
#pragma unroll
    for (int c = 0; c < kProjCols; ++c)
      if (c < ncols) acc[c] += Q[(int64_t)(c0 + c) * m + r] * wr;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kProjCols; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < ncols)
    partial[(int64_t)(c0 + threadIdx.x) * nrc + rc] =
        red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

// h[c] = sum over row chunks of partial[c] (fixed order); w -= Q[:, 0..j] h;
// alpha_j += h[j].  64 rows per workgroup, columns split over 4 wavefronts.
__global__ __launch_bounds__(256) void update_kernel(const double* __restrict__ Q, int64_t m, int j,
                                                     double* __restrict__ w, const double* __restrict__ partial,
                                                     int nrc, double* __restrict__ alpha) {
  __shared__ double hs[kMaxSteps + 1];
  __shared__ double part[4][64];
  for (int c = threadIdx.x; c <= j; c += blockDim.x) {
    double t = 0.0;
    for (int rc = 0; rc < nrc; ++rc) t += partial[(int64_t)c * nrc + rc];
    hs[c] = t;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) alpha[j] += hs[j];
  const int rl = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + rl;
  double t = 0.0;
  if (i < m)
    for (int c = cg; c <= j; c += 4) t += Q[(int64_t)c * m + i] * hs[c];
  part[cg][rl] = t;
  __syncthreads();
  if (cg == 0 && i < m) w[i] -= part[0][rl] + part[1][rl] + part[2][rl] + part[3][rl];
}

// beta = ||w||, q_next = w / beta (single workgroup)
__global__ __launch_bounds__(1024) void finish_kernel(const double* __restrict__ w, int64_t m,
                                                      double* __restrict__ q_next, double* __restrict__ beta_out) {
  __shared__ double part[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) s += w[i] * w[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += part[i];
  const double beta = sqrt(tot);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) q_next[i] = w[i] * inv;
  if (threadIdx.x == 0 && beta_out) *beta_out = beta;
}

__global__ void zero_kernel(double* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void trace_kernel(const double* G, int64_t ldg, int64_t m, double* out) {
  __shared__ double part[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) s += G[i * ldg + i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += part[i];
    *out = t;
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
__global__ __launch_bounds__(256) void bisect_kernel(const double* __restrict__ d, const double* __restrict__ e,
                                                     int k, double* __restrict__ e2all,
                                                     double* __restrict__ theta) {
  double* e2buf = e2all + (int64_t)blockIdx.x * k;
  for (int j = threadIdx.x; j < k - 1; j += blockDim.x) e2buf[j] = e[j] * e[j];
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
__global__ void inviter_kernel(const double* __restrict__ d, const double* __restrict__ e, int k,
                               const double* __restrict__ theta, int nvec, double* __restrict__ scratch,
                               int* __restrict__ iscratch, double* __restrict__ Z, int64_t ldz,
                               double* __restrict__ last) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvec) return;
  // interleaved scratch: entry j of this thread's array X at X[j * nvec]
  const int64_t st = nvec;
  double* dl = scratch + i;
  double* dd = dl + st * k;
  double* du = dd + st * k;
  double* du2 = du + st * k;
  double* b = du2 + st * k;
  int* piv = iscratch + i;
#define DL(x) dl[(int64_t)(x) * st]
#define DD(x) dd[(int64_t)(x) * st]
#define DU(x) du[(int64_t)(x) * st]
#define DU2(x) du2[(int64_t)(x) * st]
#define BB(x) b[(int64_t)(x) * st]
#define PIV(x) piv[(int64_t)(x) * st]
  double tnorm = 0.0;
  for (int j = 0; j < k; ++j) tnorm = fmax(tnorm, fabs(d[j]) + (j < k - 1 ? fabs(e[j]) : 0.0) + (j > 0 ? fabs(e[j - 1]) : 0.0));
  const double tiny = fmax(2.220446049250313e-16 * tnorm, 1e-300);
  const double mu = theta[i];
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
  for (int j = 0; j < k; ++j) BB(j) = hash_unit((uint64_t)i * 1000003u + j) + 1.0;
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
    double nrm = 0.0;
    for (int j = 0; j < k; ++j) nrm += BB(j) * BB(j);
    nrm = sqrt(nrm);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int j = 0; j < k; ++j) BB(j) *= inv;
  }
  for (int j = 0; j < k; ++j) Z[(int64_t)j * ldz + i] = BB(j);
  last[i] = BB(k - 1);
#undef DL
#undef DD
#undef DU
#undef DU2
#undef BB
#undef PIV
}

// make the largest-magnitude entry of every column positive (one wave per column)
__global__ __launch_bounds__(256) void sign_fix_kernel(double* V, int64_t ldv, int64_t m, int64_t ncols) {
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

__global__ void write_lambda_kernel(const double* theta, int b, double* lambda, int64_t m) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    lambda[i] = (i < b) ? theta[i] : 0.0;
}

}  // namespace

hapod_status wide_eigh(const double* G, int64_t ldg, int64_t m, double* lambda, double* V, int64_t ldv, double u_p,
                       wide_alloc_fn alloc, wide_free_fn release, void* ctx, hipStream_t stream, WideResult* res,
                       bool full) {
  if (m <= 0) return HAPOD_OK;
  if (full && m > kMaxSteps) {
    set_error("wide_eigh: a full run needs m <= 768");
    return HAPOD_E_UNSUPPORTED;
  }
  const int k = (int)std::min<int64_t>(m, kMaxSteps);
  // ---- scratch ------------------------------------------------------------------
  std::vector<void*> owned;
  auto get = [&](size_t bytes) -> void* {
    void* p = alloc(ctx, bytes);
    if (p) owned.push_back(p);
    return p;
  };
  struct Rel {
    std::vector<void*>& o;
    wide_free_fn f;
    void* c;
    ~Rel() {
      for (void* p : o) f(c, p);
    }
  } rel{owned, release, ctx};
  double* Q = (double*)get(sizeof(double) * m * (k + 1));
  double* w = (double*)get(sizeof(double) * m);
  const int nrc = (int)((m + kProjRows - 1) / kProjRows);
  double* h = (double*)get(sizeof(double) * (size_t)(k + 1) * nrc);
  double* alpha = (double*)get(sizeof(double) * k);
  double* beta = (double*)get(sizeof(double) * (k + 1));
  double* theta = (double*)get(sizeof(double) * k);
  double* e2 = (double*)get(sizeof(double) * (size_t)k * ((k + 3) / 4));
  double* Z = (double*)get(sizeof(double) * (size_t)k * k);
  double* last = (double*)get(sizeof(double) * k);
  double* isc = (double*)get(sizeof(double) * (size_t)5 * k * k);
  int* ipiv = (int*)get(sizeof(int) * (size_t)k * k);
  double* tr = (double*)get(sizeof(double));
  const void** qcols = (const void**)get(sizeof(void*) * k);
  int64_t* qrbs = (int64_t*)get(sizeof(int64_t) * k);
  int64_t* qrows = (int64_t*)get(sizeof(int64_t) * k);
  int64_t* drank = (int64_t*)get(sizeof(int64_t));
  void* dnode = get(sizeof(LiftNode));
  if (!Q || !w || !h || !alpha || !beta || !theta || !e2 || !Z || !last || !isc || !ipiv || !tr || !qcols || !qrbs || !qrows || !drank ||
      !dnode) {
    set_error("wide_eigh: scratch allocation failed");
    return HAPOD_E_NOMEM;
  }
  hipLaunchKernelGGL(zero_kernel, dim3(4), dim3(256), 0, stream, alpha, (int64_t)k);
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(1024), 0, stream, G, ldg, m, tr);
  // q_0
  hipLaunchKernelGGL(lanczos_init_kernel, dim3(64), dim3(256), 0, stream, w, m);
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(1024), 0, stream, w, m, Q, (double*)nullptr);
  const unsigned mv_blocks = (unsigned)((m + 3) / 4);
  const unsigned up_blocks = (unsigned)((m + 63) / 64);
  // the rounding level of G's spectrum, for the stopping test
  double trace = 0.0;
  HAPOD_HIP(hipMemcpyAsync(&trace, tr, sizeof(double), hipMemcpyDeviceToHost, stream));
  HAPOD_HIP(hipStreamSynchronize(stream));
  const double floor_trace = 0.1 * u_p * std::fabs(trace);
  int steps = k;
  bool stopped = (k == m);
  double prev_check = 0.0;
  const char* venv = std::getenv("HAPOD_VERBOSE");
  const bool verbose = venv && venv[0] == '1';
  for (int j = 0; j < k; ++j) {
    const double* qj = Q + (int64_t)j * m;
    hipLaunchKernelGGL(matvec_kernel, dim3(mv_blocks), dim3(256), 0, stream, G, ldg, m, qj, w);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(proj_partial_kernel, dim3((unsigned)((j + kProjCols) / kProjCols), (unsigned)nrc),
                         dim3(256), 0, stream, Q, m, j, w, h, nrc);
      hipLaunchKernelGGL(update_kernel, dim3(up_blocks), dim3(256), 0, stream, Q, m, j, w, h, nrc, alpha);
    }
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(1024), 0, stream, w, m, Q + (int64_t)(j + 1) * m, beta + j);
    // Stop once the Krylov space has taken in everything above the rounding
    // level of G: the residual norms beta_j then stop falling (they sit at
    // that level).  Test every kCheckEvery steps: beta_j at or below
    // u_p trace(G) / 10, or beta_j fell less than kPlateau-fold over the last
    // period after having fallen 1000-fold from beta_0.
    if (!full && (j + 1) % kCheckEvery == 0 && j + 1 < k) {
      double bj = 0.0, b0 = 0.0;
      HAPOD_HIP(hipMemcpyAsync(&bj, beta + j, sizeof(double), hipMemcpyDeviceToHost, stream));
      HAPOD_HIP(hipMemcpyAsync(&b0, beta, sizeof(double), hipMemcpyDeviceToHost, stream));
      HAPOD_HIP(hipStreamSynchronize(stream));
      if (verbose)
        std::fprintf(stderr, "[hapod wide] m=%lld step %d beta %.3e floor_trace %.3e\n", (long long)m, j + 1, bj,
                     floor_trace);
      const bool plateau = prev_check > 0.0 && bj >= kPlateau * prev_check && bj <= 1e-3 * b0;
      prev_check = bj;
      if (j + 1 >= kMinSteps && (bj <= floor_trace || plateau)) {
        steps = j + 1;
        stopped = true;
        break;
      }
    }
  }
  HAPOD_HIP(hipGetLastError());
  // ---- tridiagonal eigenproblem of the steps taken ---------------------------------
  const int kk = steps;
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)((kk + 3) / 4)), dim3(256), 0, stream, alpha, beta, kk, e2, theta);
  HAPOD_HIP(hipGetLastError());
  const unsigned bblocks = (unsigned)((kk + 255) / 256);
  hipLaunchKernelGGL(inviter_kernel, dim3(bblocks), dim3(256), 0, stream, alpha, beta, kk, theta, kk, isc, ipiv, Z,
                     (int64_t)kk, last);
  HAPOD_HIP(hipGetLastError());
  // ---- choose the converged leading block (host) ----------------------------------
  std::vector<double> th(kk), lz(kk), bet(kk);
  HAPOD_HIP(hipMemcpyAsync(th.data(), theta, sizeof(double) * kk, hipMemcpyDeviceToHost, stream));
  HAPOD_HIP(hipMemcpyAsync(lz.data(), last, sizeof(double) * kk, hipMemcpyDeviceToHost, stream));
  HAPOD_HIP(hipMemcpyAsync(bet.data(), beta, sizeof(double) * kk, hipMemcpyDeviceToHost, stream));
  HAPOD_HIP(hipStreamSynchronize(stream));
  const double bk = bet[kk - 1];
  const double theta_min = *std::min_element(th.begin(), th.end());
  const double floor_abs = std::max(std::max(-theta_min, 0.0), floor_trace);
  // a Ritz pair counts as converged when its residual is below 1e-8 of its
  // own value or below the Gram's rounding level
  int b = 0;
  while (b < kk && std::fabs(bk * lz[b]) <= std::max(1e-8 * std::fabs(th[b]), floor_abs)) ++b;
  if (kk == m) b = kk;  // complete tridiagonalisation: every pair is exact
  // Ritz vectors of one Krylov space are orthonormal and diagonalise G on it
  // (V^T G V = diag(theta)), so the energy of S on the modes S v_i / sqrt(theta_i)
  // is at least sum theta_i whether or not the pairs have converged: the block
  // is extended by every Ritz value above the noise level max(floor_abs,
  // beta_{k-1}) (below it a Ritz value cannot be told from zero), and only
  // what lies beyond the Krylov space is left unresolved.
  const double noise = std::max(floor_abs, std::fabs(bk));
  if (stopped) {
    int e = b;
    while (e < kk && th[e] > noise) ++e;
    b = e;
  }
  double missing = 0.0, captured = 0.0;
  for (int i = b; i < kk; ++i)
    if (th[i] > noise) missing += th[i];
  for (int i = 0; i < b; ++i) captured += th[i];
  if (verbose)
    std::fprintf(stderr, "[hapod wide] m=%lld steps %d block %d theta_1 %.6e theta_min %.3e floor %.3e\n",
                 (long long)m, kk, b, th[0], theta_min, floor_abs);
  // ---- Ritz vectors V[:, :b] = Q_k Z[:, :b] (FP64 lift GEMM) ------------------------
  if (b > 0) {
    HAPOD_TRY(launch_fill_colptrs(Q, m, kk, 8, qcols, stream));
    HAPOD_TRY(launch_fill_i64(qrbs, kRowBlock, kk, stream));
    HAPOD_TRY(launch_fill_i64(qrows, m, kk, stream));
    HAPOD_TRY(launch_set_scalar_i64(drank, b, stream));
    LiftNode l{};
    l.cols = (const void* const*)qcols;
    l.rbs = qrbs;
    l.crows = qrows;
    l.B = Z;
    l.rank = drank;
    l.out = V;
    l.n = m;
    l.ldb = kk;
    l.ocs = ldv;
    l.obs = kRowBlock;
    l.m = kk;
    l.row_tiles = (int32_t)((m + kLiftTileM - 1) / kLiftTileM);
    l.col_tiles = (int32_t)((b + kLiftTileN - 1) / kLiftTileN);
    l.item_base = 0;
    HAPOD_HIP(hipMemcpyAsync(dnode, &l, sizeof(l), hipMemcpyHostToDevice, stream));
    HAPOD_TRY(launch_lift(0, (const LiftNode*)dnode, 1, l.row_tiles * l.col_tiles, stream));
    hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)((b + 3) / 4)), dim3(256), 0, stream, V, ldv, m, (int64_t)b);
  }
  hipLaunchKernelGGL(write_lambda_kernel, dim3(64), dim3(256), 0, stream, theta, b, lambda, m);
  HAPOD_HIP(hipGetLastError());
  HAPOD_HIP(hipStreamSynchronize(stream));
  if (res) {
    res->iterations = kk;
    res->block = b;
    res->floor_abs = floor_abs;
    res->exhausted = stopped;
    res->missing = missing;
    res->unresolved = std::max(0.0, trace - captured);
    res->trace = trace;
    res->noise = (b < m) ? noise : 0.0;
  }
  return HAPOD_OK;
}

}  // namespace hapod
