// Small helper kernels: column-pointer tables, column copies, the Gram
// diagonal check, and the Cholesky factor / triangular inverse used by the
// Cholesky-QR re-orthonormalisation.
#include "internal.hpp"
#include "mfma.hpp"

namespace hapod {
namespace {

// The pre-split twin: for row block b and column c, 128 hi then 128 lo
// bfloat16 values at dst + (b m + c) 128.  A thread splits a run of 4 rows
// (one 16-byte load, two 8-byte stores); a 256-thread block covers 8 columns
// of one row block.
__global__ __launch_bounds__(256) void split_cols_kernel(int64_t n, int64_t m, const void* const* cols,
                                                         const int64_t* rbs, const int64_t* crows, float* dst) {
  const int64_t b = blockIdx.x;
  const int64_t c = (int64_t)blockIdx.y * 8 + (threadIdx.x >> 5);
  if (c >= m) return;
  const int q = threadIdx.x & 31;
  const int64_t r = b * kRowBlock + 4 * q;
  const float* src = reinterpret_cast<const float*>(cols[c]) + blk_off(r, rbs[c]);
  const int64_t avail = min(n, crows[c]) - r;
  float x[4];
  if (avail >= 4 && (((uintptr_t)src & 15u) == 0)) {
    const float4 v = *reinterpret_cast<const float4*>(src);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = (e < avail) ? src[e] : 0.f;
  }
  uint32_t h01, l01, h23, l23;
  split_bf16x2(x[0], x[1], h01, l01);
  split_bf16x2(x[2], x[3], h23, l23);
  uint16_t* blk = reinterpret_cast<uint16_t*>(dst + (b * m + c) * kRowBlock);
  typedef __attribute__((ext_vector_type(2))) uint32_t u2;
  *reinterpret_cast<u2*>(blk + 4 * q) = u2{h01, h23};
  *reinterpret_cast<u2*>(blk + kRowBlock + 4 * q) = u2{l01, l23};
}

__global__ void fill_colptrs_kernel(const char* base, int64_t ld_bytes, int64_t m, const void** out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) out[j] = base + j * ld_bytes;
}

template <typename E>
__global__ void copy_cols_kernel(int64_t n, int64_t m, const void* const* cols, const int64_t* rbs,
                                 const int64_t* crows, E* out, int64_t ldo) {
  const int64_t j = blockIdx.y;
  const E* src = reinterpret_cast<const E*>(cols[j]);
  const int64_t s = rbs[j], rows = crows[j];
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    out[j * ldo + r] = (r < rows) ? src[blk_off(r, s)] : E(0);
}

__global__ void zero_u32_kernel(uint32_t* p, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void check_diag_kernel(const double* G, int64_t ldg, int64_t m, int32_t* flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = G[i * ldg + i];
    if (!isfinite(d)) *flag = 1;
  }
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) { *p = v; }

__global__ void fill_i64_kernel(int64_t* p, int64_t v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// C = A B, column-major FP64 (M x K times K x N), 16 x 16 tiles through LDS;
// for the small products that compose right singular vectors.
__global__ __launch_bounds__(256) void dgemm_nn_kernel(int64_t M, int64_t N, int64_t K, const double* __restrict__ A,
                                                       int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                       double* __restrict__ C, int64_t ldc) {
  __shared__ double As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t row = (int64_t)blockIdx.x * 16 + tx, col = (int64_t)blockIdx.y * 16 + ty;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    const int64_t ka = k0 + ty, kb = k0 + tx;
    As[ty][tx] = (row < M && ka < K) ? A[ka * lda + row] : 0.0;
    Bs[ty][tx] = (kb < K && col < N) ? B[col * ldb + kb] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += As[k][tx] * Bs[ty][k];
    __syncthreads();
  }
  if (row < M && col < N) C[col * ldc + row] = acc;
}

__global__ void set_identity_kernel(double* T, int64_t n, int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  T[j * ld + i] = (i == j) ? 1.0 : 0.0;
}

}  // namespace

hapod_status launch_fill_colptrs(const void* base, int64_t ld, int64_t m, int elem_bytes,
                                 const void** d_out, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(fill_colptrs_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream,
                     (const char*)base, ld * elem_bytes, m, d_out);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_zero_bytes(void* p, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return HAPOD_OK;
  const size_t words = bytes / 4;  // callers pass multiples of 4
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)std::min<size_t>((words + 255) / 256, 4096)), dim3(256), 0,
                     stream, (uint32_t*)p, words);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_copy_cols(int elem_bytes, int64_t n, int64_t m, const void* const* cols, const int64_t* rbs,
                              const int64_t* crows, void* out, int64_t ldo, hipStream_t stream) {
  if (m <= 0 || n <= 0) return HAPOD_OK;
  if (m > 65535) {
    set_error("launch_copy_cols: too many columns");
    return HAPOD_E_UNSUPPORTED;
  }
  const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  if (elem_bytes == 8)
    hipLaunchKernelGGL(copy_cols_kernel<double>, dim3(gx, (unsigned)m), dim3(256), 0, stream, n, m, cols, rbs,
                       crows, (double*)out, ldo);
  else
    hipLaunchKernelGGL(copy_cols_kernel<float>, dim3(gx, (unsigned)m), dim3(256), 0, stream, n, m, cols, rbs, crows,
                       (float*)out, ldo);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_check_diag(const double* G, int64_t ldg, int64_t m, int32_t* d_flag, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(check_diag_kernel, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 64)), dim3(256), 0,
                     stream, G, ldg, m, d_flag);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_set_scalar_i64(int64_t* p, int64_t v, hipStream_t stream) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(1), 0, stream, p, v);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_fill_i64(int64_t* p, int64_t v, int64_t count, hipStream_t stream) {
  if (count <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(fill_i64_kernel, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 1024)), dim3(256), 0,
                     stream, p, v, count);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_split_cols(int64_t n, int64_t m, const void* const* cols, const int64_t* rbs,
                               const int64_t* crows, float* dst, hipStream_t stream) {
  if (n <= 0 || m <= 0) return HAPOD_OK;
  if (m > 65535) {
    set_error("launch_split_cols: too many columns");
    return HAPOD_E_UNSUPPORTED;
  }
  const unsigned nb = (unsigned)((n + kRowBlock - 1) / kRowBlock);
  hipLaunchKernelGGL(split_cols_kernel, dim3(nb, (unsigned)((m + 7) / 8)), dim3(256), 0, stream, n, m, cols, rbs,
                     crows, dst);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_chol_inv(double* W, int64_t ldw, int64_t N, double* Rinv, int64_t ldr, int32_t* d_bad,
                             hipStream_t stream, double rel_floor) {
  return launch_chol_inv_wg(W, ldw, N, Rinv, ldr, d_bad, stream, rel_floor);
}

hapod_status launch_dgemm_nn(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                             int64_t ldb, double* C, int64_t ldc, hipStream_t stream) {
  if (M <= 0 || N <= 0) return HAPOD_OK;
  const dim3 g((unsigned)((M + 15) / 16), (unsigned)((N + 15) / 16));
  hipLaunchKernelGGL(dgemm_nn_kernel, g, dim3(256), 0, stream, M, N, K, A, lda, B, ldb, C, ldc);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_set_identity(double* T, int64_t n, int64_t ld, hipStream_t stream) {
  if (n <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(set_identity_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, stream, T, n, ld);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
