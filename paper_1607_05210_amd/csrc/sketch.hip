// Helpers of the sketched local POD (randomized range finder, Halko,
// Martinsson & Tropp, SIAM Review 2011): the sparse sign sketch Y = S Omega,
// the Gaussian test matrix and a square transpose.  The other products of
// that route run on the Gram and lift kernels (cross-product and residual
// modes).
#include "internal.hpp"
#include "mfma.hpp"

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

// The sparse sign map (a sparse dimension reduction map with kSignNnz
// nonzeros per row, Martinsson & Tropp, Acta Numerica 2020, Sec. 9.2): row k
// of Omega (m x ell) holds +-1/sqrt(kSignNnz) in each of the kSignNnz
// column blocks of width ell / kSignNnz, at the position and with the sign
// drawn from the splitmix64 finaliser of the counter (seed, kSignNnz k + t).
// sign_table_kernel writes, per (k, t), position + ell * (sign < 0) at
// tab[t * sign_table_ld(m) + k].
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
__global__ __launch_bounds__(256) void sign_table_kernel(int32_t* __restrict__ tab, int64_t m, int32_t ell,
                                                         uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // counter kSignNnz k + t
  if (e >= m * kSignNnz) return;
  const int t = (int)(e % kSignNnz);
  const int64_t k = e / kSignNnz;
  const uint32_t bw = (uint32_t)(ell / kSignNnz);
  const uint64_t z = mix64((seed * 0xd1342543de82ef95ull) ^ (uint64_t)e);
  const uint32_t pos = (uint32_t)(((z >> 32) * (uint64_t)bw) >> 32);  // uniform in [0, bw)
  tab[t * sign_table_ld(m) + k] = (int32_t)(t * bw + pos) + ((z & 1u) ? ell : 0);
}

// Y = S Omega for the sparse sign map: one workgroup per 32-row slice of S,
// whose 32 x ell slice of Y accumulates in LDS (rows padded to ell + 1
// doubles against bank conflicts).  Thread (t, i) = (threadIdx.x / 32,
// threadIdx.x % 32) owns row i's entries in column block t, so each entry is
// summed by one thread, in input-column order (deterministic); the sums go
// to LDS as atomic adds whose results are not returned, so consecutive
// updates do not wait for each other (one lane per entry: the order is the
// lane's program order).  A slice that every column holds in full reads
// 32 contiguous rows per column with no guards, kSketchBatch columns and
// their table entries loaded ahead of their use; other slices, and the
// columns past the last whole batch pair, read one column at a time with
// rows past a column's own count as zero.  Rows of Y past n are not
// written.  Y element (r, c) at Y[c * ocs + blk_off(r, obs)].
__global__ __launch_bounds__(256, 1) void sign_sketch_kernel(const void* const* __restrict__ cols,
                                                          const int64_t* __restrict__ rbs,
                                                          const int64_t* __restrict__ crows, int64_t n, int64_t m,
                                                          int64_t full_rows, const int32_t* __restrict__ tab,
                                                          int32_t ell, double* __restrict__ Y, int64_t ocs,
                                                          int64_t obs) {
  extern __shared__ double ys[];
  constexpr int U = kSketchBatch;
  const int i = threadIdx.x & 31, t = threadIdx.x >> 5;
  const int ld = ell + 1;
  const int bw = ell / kSignNnz;
  const int64_t row = (int64_t)blockIdx.x * 32 + i;
  double* yr = ys + i * ld;
  for (int q = 0; q < bw; ++q) yr[t * bw + q] = 0.0;
  // (each thread touches only its own entries: no barrier needed before use)
  auto add = [&](int32_t e, double x) {
    const bool neg = e >= ell;
    atomicAdd(&yr[neg ? e - ell : e], neg ? -x : x);
  };
  const int64_t tld = sign_table_ld(m);
  const int32_t* tr = tab + t * tld;  // this thread's block: entries of consecutive columns
  int64_t k0 = 0;
  if ((int64_t)blockIdx.x * 32 + 32 <= full_rows) {
    // The slice's 32 rows lie in one 128-row block: per column one base
    // pointer (column start + block times row-block stride), computed by the
    // lane of the column's place in a group of 64 columns (one vector load
    // of the column table per lane, a group ahead) and handed to the whole
    // wavefront by readlane, so the loop carries no scalar loads.
    typedef __attribute__((ext_vector_type(4))) int i4;
    constexpr int UQ = U / 4, G = 64, NBG = G / U;
    static_assert(G % U == 0 && U % 4 == 0, "whole batches per column group");
    const int lane = threadIdx.x & 63;
    const int64_t blk = ((int64_t)blockIdx.x * 32) >> 7;
    const int64_t roff = row & (kRowBlock - 1);
    const int64_t mg = m / G * G;  // columns in whole groups
    // a group's column-table entries (loaded a group before they are needed)
    // and the lane's base pointer from them
    struct Raw {
      const void* c;
      int64_t rb;
    };
    auto group_raw = [&](int64_t g0) -> Raw {
      const int64_t k = min(g0 + lane, m - 1);
      return Raw{*as_global(cols + k), *as_global(rbs + k)};
    };
    auto base = [&](const Raw& r) -> uint64_t {
      return (uint64_t)(reinterpret_cast<const double*>(r.c) + blk * r.rb);
    };
    auto col_ptr = [&](uint64_t gb, int u) -> const double* {
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)gb, u);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(gb >> 32), u);
      return reinterpret_cast<const double*>(((uint64_t)hi << 32) | lo);
    };
    double xa[U], xb[U];
    i4 ea[UQ], eb[UQ];
    // batch j (U columns) of the group whose bases are in gb, first column k
    auto load = [&](uint64_t gb, int j, int64_t k, double (&x)[U], i4 (&e)[UQ]) {
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = *as_global(col_ptr(gb, j * U + u) + roff);
#pragma unroll
      for (int q = 0; q < UQ; ++q) e[q] = *as_global(reinterpret_cast<const i4*>(tr + k + 4 * q));
    };
    auto apply = [&](const double (&x)[U], const i4 (&e)[UQ]) {
#pragma unroll
      for (int u = 0; u < U; ++u) add(e[u / 4][u % 4], x[u]);
    };
    if (mg > 0) {
      uint64_t gcur = base(group_raw(0));
      Raw rnext = group_raw(min<int64_t>(G, mg - G));
      load(gcur, 0, 0, xa, ea);
      for (; k0 < mg; k0 += G) {
        const uint64_t gnext = base(rnext);
        // batches 1 .. NBG - 1 of this group, then batch 0 of the next one
        // (past the last group: this group's last batch again, unused); the
        // refills are unconditional, so each wait is for a fixed count
#pragma unroll
        for (int j = 1; j <= NBG; ++j) {
          const bool odd = (j & 1) != 0;
          const bool next = (j == NBG);
          const uint64_t gb = next ? (k0 + G < mg ? gnext : gcur) : gcur;
          const int jj = next ? (k0 + G < mg ? 0 : NBG - 1) : j;
          const int64_t kk = next ? (k0 + G < mg ? k0 + G : k0 + (NBG - 1) * U) : k0 + j * U;
          if (odd) load(gb, jj, kk, xb, eb);
          else load(gb, jj, kk, xa, ea);
          __builtin_amdgcn_sched_barrier(0);
          if (odd) apply(xa, ea);
          else apply(xb, eb);
        }
        gcur = gnext;
        rnext = group_raw(min<int64_t>(k0 + 2 * G, mg - G));
      }
    }
  }
  for (int64_t k = k0; k < m; ++k) {
    const double* c = reinterpret_cast<const double*>(cols[k]);
    const double x = (row < crows[k]) ? c[blk_off(row, rbs[k])] : 0.0;
    add(tr[k], x);
  }
  __syncthreads();
  // write the slice: column c, 32 consecutive rows per pass
  const double scale = 1.0 / sqrt((double)kSignNnz);
  for (int c = t; c < ell; c += 8)
    if (row < n) Y[(int64_t)c * ocs + blk_off(row, obs)] = ys[i * ld + c] * scale;
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

hapod_status launch_sign_table(int32_t* tab, int64_t m, int64_t ell, uint64_t seed, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  if (ell % kSignNnz != 0 || ell <= 0 || ell > kSketchMaxCols) {
    set_error("sparse sign sketch: ell must be a positive multiple of 8 up to 512");
    return HAPOD_E_UNSUPPORTED;
  }
  const int64_t total = m * kSignNnz;
  hipLaunchKernelGGL(sign_table_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, tab, m, (int32_t)ell,
                     seed);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

hapod_status launch_sign_sketch(const void* const* d_cols, const int64_t* d_rbs, const int64_t* d_rows, int64_t n,
                                int64_t m, int64_t full_rows, const int32_t* tab, int64_t ell, double* Y, int64_t ocs,
                                int64_t obs, hipStream_t stream) {
  if (n <= 0 || m <= 0) return HAPOD_OK;
  if (ell % kSignNnz != 0 || ell <= 0 || ell > kSketchMaxCols) {
    set_error("sparse sign sketch: ell must be a positive multiple of 8 up to 512");
    return HAPOD_E_UNSUPPORTED;
  }
  const size_t lds = sizeof(double) * 32 * (size_t)(ell + 1);
  static bool attr = false;
  if (!attr) {
    HAPOD_HIP(hipFuncSetAttribute((const void*)sign_sketch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(sizeof(double) * 32 * (kSketchMaxCols + 1))));
    attr = true;
  }
  const int64_t slices = (n + 31) / 32;
  if (slices > INT32_MAX) {
    set_error("sparse sign sketch: too many rows");
    return HAPOD_E_UNSUPPORTED;
  }
  hipLaunchKernelGGL(sign_sketch_kernel, dim3((unsigned)slices), dim3(256), lds, stream, d_cols, d_rbs, d_rows, n, m,
                     full_rows, tab, (int32_t)ell, Y, ocs, obs);
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
