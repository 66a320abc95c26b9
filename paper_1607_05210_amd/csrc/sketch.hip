// Helpers of the sketched local POD (randomized range finder, Halko,
// Martinsson & Tropp, SIAM Review 2011): the Gaussian test matrix and a
// square transpose.  The products of that route run on the Gram and lift
// kernels (cross-product and residual modes).
#include "internal.hpp"

namespace hapod {
namespace {

// splitmix64 finaliser (Steele, Lea & Flood, OOPSLA 2014) of a counter:
// 53 uniform bits in (0, 1], never 0
__device__ __forceinline__ double unit_open(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  x ^= x >> 31;
  return ((double)(x >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

// out[2 i], out[2 i + 1]: one Box-Muller pair from the uniforms of counters
// (seed, 2 i) and (seed, 2 i + 1).  Deterministic for a given seed, whatever
// the launch shape.
__global__ __launch_bounds__(256) void normal_fill_kernel(double* __restrict__ out, int64_t count, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * i >= count) return;
  const uint64_t base = seed * 0xd1342543de82ef95ull;
  const double u1 = unit_open(base ^ (uint64_t)(2 * i)), u2 = unit_open(base ^ (uint64_t)(2 * i + 1));
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  out[2 * i] = r * c;
  if (2 * i + 1 < count) out[2 * i + 1] = r * s;
}

__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ A, int64_t lda, int64_t m,
                                                        double* __restrict__ T, int64_t ldt) {
  __shared__ double tile[32][33];
  const int64_t bi = (int64_t)blockIdx.x * 32, bj = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi + tx, j = bj + r;
    tile[r][tx] = (i < m && j < m) ? A[j * lda + i] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bj + tx, j = bi + r;  // T(i, j) = A(j, i)
    if (i < m && j < m) T[j * ldt + i] = tile[tx][r];
  }
}

// C (row-major, ld ld): rows [0, rows_c) negated, rows [rows_c, rows_c +
// cols) set to the identity, so that [L, Y] C = Y - L C_old
__global__ __launch_bounds__(256) void neg_ident_kernel(double* __restrict__ C, int64_t rows_c, int64_t cols,
                                                        int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (rows_c + cols) * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  double* p = C + i * ld + j;
  *p = (i < rows_c) ? -*p : (i - rows_c == j ? 1.0 : 0.0);
}

// R[(c0 + j) * ldr + i] += C[i * ldc + j], i < rows, j < cols (C row-major)
__global__ __launch_bounds__(256) void acc_transposed_kernel(double* __restrict__ R, int64_t ldr, int64_t c0,
                                                             const double* __restrict__ C, int64_t ldc, int64_t rows,
                                                             int64_t cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t j = e / rows, i = e - j * rows;
  R[(c0 + j) * ldr + i] += C[i * ldc + j];
}

}  // namespace

hapod_status launch_acc_transposed(double* R, int64_t ldr, int64_t c0, const double* C, int64_t ldc, int64_t rows,
                                   int64_t cols, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(acc_transposed_kernel, dim3((unsigned)((rows * cols + 255) / 256)), dim3(256), 0, stream, R, ldr,
                     c0, C, ldc, rows, cols);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_neg_ident(double* C, int64_t rows_c, int64_t cols, int64_t ld, hipStream_t stream) {
  const int64_t total = (rows_c + cols) * cols;
  if (total <= 0) return HAPOD_OK;
  hipLaunchKernelGGL(neg_ident_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, C, rows_c, cols,
                     ld);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_normal_fill(double* out, int64_t count, uint64_t seed, hipStream_t stream) {
  if (count <= 0) return HAPOD_OK;
  const int64_t pairs = (count + 1) / 2;
  hipLaunchKernelGGL(normal_fill_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, stream, out, count,
                     seed);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_transpose(const double* A, int64_t lda, int64_t m, double* T, int64_t ldt, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  const unsigned nb = (unsigned)((m + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, dim3(nb, nb), dim3(256), 0, stream, A, lda, m, T, ldt);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
