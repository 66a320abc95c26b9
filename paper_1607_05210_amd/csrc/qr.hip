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

#include "internal.hpp"

namespace hapod {
namespace {

constexpr int kOsjThreads = 1024;
constexpr int kOsjWaves = kOsjThreads / 64;
constexpr int kOsjMaxSweeps = 60;

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

// R = upper triangle of W (column-major), zeros below
__global__ void triu_kernel(const double* __restrict__ W, int64_t ldw, int64_t N, double* __restrict__ R, int64_t ldr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i < N) R[j * ldr + i] = (i <= j) ? W[j * ldw + i] : 0.0;
}

// One-sided Jacobi on the columns of X (m x m, column-major, ld m): plane
// rotations on column pairs until every pair is orthogonal to m u of its
// norms; the pairs of a round are disjoint (round-robin order), one
// wavefront per pair.  Then sigma_c = ||x_c||, sorted descending, and
// B (row-major, ld m) column p = x_c (scaled) or x_c / sigma_c.
// info: sweeps taken, or -1 without convergence.
template <bool kLds>
__global__ __launch_bounds__(kOsjThreads) void osj_kernel(double* A, int64_t m, double* sigma, double* B, int scaled,
                                                          int32_t* info) {
  extern __shared__ double osj_lds[];
  __shared__ double sg[kQrMaxM];
  __shared__ int32_t pos[kQrMaxM];
  __shared__ int nrot;
  double* X = kLds ? osj_lds : A;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (kLds) {
    for (int64_t e = t; e < m * m; e += kOsjThreads) X[e] = A[e];
  }
  const int64_t mm = m + (m & 1);
  const double tol = (double)m * 1.1102230246251565e-16;
  int sweep = 0;
  bool done = false;
  for (; sweep < kOsjMaxSweeps && !done; ++sweep) {
    if (t == 0) nrot = 0;
    __syncthreads();
    for (int64_t r = 0; r < mm - 1; ++r) {
      for (int64_t p = wv; p < mm / 2; p += kOsjWaves) {
        int64_t i, j;
        if (p == 0) {
          i = mm - 1;
          j = r;
        } else {
          i = (r + p) % (mm - 1);
          j = (r - p + mm - 1) % (mm - 1);
        }
        if (i >= m || j >= m) continue;  // the padding index of an odd m
        double* ci = X + i * m;
        double* cj = X + j * m;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int64_t k = lane; k < m; k += 64) {
          const double x = ci[k], y = cj[k];
          a += x * x;
          b += y * y;
          g += x * y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        g = wave_sum(g);
        if (!(a > 0.0) || !(b > 0.0) || fabs(g) <= tol * sqrt(a) * sqrt(b)) continue;
        // rotation [c s; -s c] that makes the pair orthogonal, the smaller angle
        const double zeta = (b - a) / (2.0 * g);
        const double tt = fabs(zeta) > 1e150 ? 0.5 / zeta
                                             : (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
        for (int64_t k = lane; k < m; k += 64) {
          const double x = ci[k], y = cj[k];
          ci[k] = c * x - s * y;
          cj[k] = s * x + c * y;
        }
        if (lane == 0) atomicAdd(&nrot, 1);
      }
      __syncthreads();
    }
    done = (nrot == 0);
    __syncthreads();
  }
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
  if (t == 0) info[0] = done ? sweep : -1;
}

}  // namespace

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
  if (m <= kOsjLdsMaxM) {
    const size_t lds = sizeof(double) * (size_t)m * m;
    static bool attr = false;
    if (!attr) {
      HAPOD_HIP(hipFuncSetAttribute((const void*)osj_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(sizeof(double) * kOsjLdsMaxM * kOsjLdsMaxM)));
      attr = true;
    }
    hipLaunchKernelGGL(osj_kernel<true>, dim3(1), dim3(kOsjThreads), lds, stream, A, m, sigma, B, scaled, info);
  } else {
    hipLaunchKernelGGL(osj_kernel<false>, dim3(1), dim3(kOsjThreads), 0, stream, A, m, sigma, B, scaled, info);
  }
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
