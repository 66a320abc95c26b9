// Batched truncation (Def. 2.5 with Thm. 2.4) and preparation of the lift
// operand, one 256-thread workgroup per node.
//
// For eigenvalues lambda_1 >= ... >= lambda_m of a Gram matrix the rank is
//   N = min{N' in 0..m : sum_{n > N'} e_n <= eps^2},
// where e_n is the energy counted for eigenvalue n:
//   policy 0 (clamp): e_n = max(lambda_n, 0) -- negative values are rounding
//                     artefacts of a positive semi-definite product;
//   policy 1 (floor): e_n = lambda_n if lambda_n > theta else 0, with
//                     theta = max(-lambda_min, floor_abs): eigenvalues inside
//                     the rounding band of the Gram product count as zero.
// Tails are summed in FP64: every thread sums its contiguous segment from the
// end, segment totals are combined across lanes with wavefront shuffles and
// across the four wavefronts through LDS.
//
// The lift operand is written row-major: B[k][n] = V[k][n] (inner node:
// S B = U Sigma, the scaled modes) or V[k][n] / sqrt(lambda_n) (root:
// orthonormal modes), for n < N.
#include "internal.hpp"

namespace hapod {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// inclusive suffix sum over the 64 lanes of a wavefront: lane i gets the sum
// of the values of lanes i..63
__device__ __forceinline__ double wave_suffix_sum(double x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    double y = __shfl_down(x, off, 64);
    if (lane + off < 64) x += y;
  }
  return x;
}

__device__ int block_min_int(int v, int* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  if (lane == 0) sh[w] = v;
  __syncthreads();
  int r = sh[0];
  for (int i = 1; i < kWaves; ++i) r = min(r, sh[i]);
  __syncthreads();
  return r;
}

__device__ double block_sum_double(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < kWaves; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// rank for one energy policy; returns N and (for thread 0) tail(N) in *tailN
__device__ int rank_for(const double* lam, int m, int policy, double theta, double eps2,
                        double* shd, int* shi, double* tailN) {
  const int tid = threadIdx.x;
  const int seg = (m + kThreads - 1) / kThreads;
  const int b = tid * seg, e = min(m, b + seg);
  auto energy = [&](int i) -> double {
    const double x = lam[i];
    return policy == 0 ? fmax(x, 0.0) : (x > theta ? x : 0.0);
  };
  // local total of my segment
  double local = 0.0;
  for (int i = e - 1; i >= b; --i) local += energy(i);
  // sum of the segments after mine: suffix over lanes, then over waves
  const int lane = tid & 63, w = tid >> 6;
  const double inc = wave_suffix_sum(local);          // my segment .. end of my wave
  if (lane == 0) shd[w] = inc;                        // wave totals
  __syncthreads();
  double later_waves = 0.0;
  for (int i = kWaves - 1; i > w; --i) later_waves += shd[i];
  const double later = (inc - local) + later_waves;   // strictly after my segment
  __syncthreads();
  // tail[i] = e_i + ... + e_{m-1} for i in my segment; tail[m] = 0
  int first = m;
  double acc = later, my_tail = 0.0;
  for (int i = e - 1; i >= b; --i) {
    // tail after i modes = sum_{n >= i} (0-based), evaluated from the end
    acc += energy(i);
    if (acc <= eps2) { first = i; my_tail = acc; }
  }
  const int N = block_min_int(first, shi);
  // thread owning index N reports tail(N)
  if (N < m && b <= N && N < e) shd[kWaves] = my_tail;
  if (N == m && tid == 0) shd[kWaves] = 0.0;
  __syncthreads();
  if (tid == 0) *tailN = shd[kWaves];
  __syncthreads();
  return N;
}

__global__ __launch_bounds__(kThreads) void truncate_kernel(const TruncNode* __restrict__ nodes) {
  __shared__ double shd[kWaves + 1];
  __shared__ int shi[kWaves];
  const TruncNode nd = nodes[blockIdx.x];
  const int m = nd.m, tid = threadIdx.x;
  if (m <= 0) {
    if (tid == 0) {
      *nd.rank = 0;
      if (nd.info) for (int i = 0; i < 6; ++i) nd.info[i] = 0.0;
    }
    return;
  }
  const double lam1 = nd.lambda[0], lmin = nd.lambda[m - 1];
  double nneg = 0.0;
  for (int i = tid; i < m; i += kThreads) nneg += (nd.lambda[i] < 0.0) ? 1.0 : 0.0;
  nneg = block_sum_double(nneg, shd);
  const double theta = fmax(fmax(-lmin, nd.floor_ptr ? *nd.floor_ptr : nd.floor_abs), 0.0);

  double tail_clamp = 0.0, tail_pol = 0.0;
  const int N_clamp = rank_for(nd.lambda, m, 0, 0.0, nd.eps2, shd, shi, &tail_clamp);
  int N = N_clamp;
  tail_pol = tail_clamp;
  if (nd.policy == 1) N = rank_for(nd.lambda, m, 1, theta, nd.eps2, shd, shi, &tail_pol);

  if (tid == 0) {
    *nd.rank = N;
    if (nd.info) {
      nd.info[0] = tail_pol;
      nd.info[1] = lam1;
      nd.info[2] = lmin;
      nd.info[3] = nneg;
      nd.info[4] = (nd.policy == 1) ? theta : 0.0;
      nd.info[5] = (double)N_clamp;
    }
  }
  for (int n = tid; n < N; n += kThreads) nd.sigma[n] = sqrt(nd.lambda[n]);
  // lift operand, row-major B[k * ldb + n], transposed from V through LDS in
  // 32 x 32 tiles so that reads of V and writes of B are both coalesced
  if (nd.V == nullptr) return;
  __shared__ double tile[32][33];
  const int tx = tid & 31, ty = tid >> 5;  // 32 x 8 threads
  for (int n0 = 0; n0 < N; n0 += 32)
    for (int k0 = 0; k0 < m; k0 += 32) {
      const int n = n0 + tx;
      const double sc = (nd.root && n < N) ? 1.0 / sqrt(nd.lambda[n]) : 1.0;
      for (int r = ty; r < 32; r += 8) {   // column n0 + r of V, rows k0 .. k0 + 31
        const int nn = n0 + r, k = k0 + tx;
        tile[r][tx] = (nn < N && k < m) ? nd.V[(int64_t)nn * nd.ldv + k] : 0.0;
      }
      __syncthreads();
      for (int r = ty; r < 32; r += 8) {   // row k0 + r of B, columns n0 .. n0 + 31
        const int k = k0 + r;
        if (k < m && n < N) {
          const double v = tile[tx][r] * sc;
          nd.B[(int64_t)k * nd.ldb + n] = v;
          if (nd.B32) nd.B32[(int64_t)k * nd.ldb + n] = (float)v;
        }
      }
      __syncthreads();
    }
}

__global__ void lift_operand_kernel(const double* V, int64_t ldv, const double* lambda, int64_t m,
                                    int64_t N, double* B, float* B32, int64_t ldb) {
  const int64_t total = m * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = idx % m, n = idx / m;
    double v = V[n * ldv + k];
    if (lambda) v /= sqrt(lambda[n]);
    B[k * ldb + n] = v;
    if (B32) B32[k * ldb + n] = (float)v;
  }
}

__global__ void to_f32_kernel(const double* src, float* dst, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

}  // namespace

hapod_status launch_lift_operand(const double* V, int64_t ldv, const double* lambda, int64_t m, int64_t N,
                                 double* B, float* B32, int64_t ldb, hipStream_t stream) {
  if (m <= 0 || N <= 0) return HAPOD_OK;
  const unsigned g = (unsigned)std::min<int64_t>((m * N + 255) / 256, 4096);
  hipLaunchKernelGGL(lift_operand_kernel, dim3(g), dim3(256), 0, stream, V, ldv, lambda, m, N, B, B32, ldb);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_to_f32(const double* src, float* dst, int64_t count, hipStream_t stream) {
  if (count <= 0) return HAPOD_OK;
  const unsigned g = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(to_f32_kernel, dim3(g), dim3(256), 0, stream, src, dst, count);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_truncate(const TruncNode* d_nodes, int num_nodes, hipStream_t stream) {
  if (num_nodes <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(truncate_kernel, dim3(num_nodes), dim3(kThreads), 0, stream, d_nodes);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
