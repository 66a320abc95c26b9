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
// nonzeros per row, Martinsson & Tropp, Acta Numerica 2020, Sec. 9.2), in a
// block-shifted form: Omega (m x ell) has kSignNnz column blocks of width
// bw = ell / kSignNnz, and row k of Omega holds +-1/sqrt(kSignNnz) once in
// each block.  The input columns go in chunks of bw; in block t, chunk g's
// column g bw + j sits at position (j + shift) mod bw, with the shift
// uniform in [0, bw) and the sign of every position an independent fair
// bit, both drawn from the splitmix64 finaliser of the counter (seed,
// kSignNnz g + t).  Each row of Omega thus has one nonzero per block, as in
// the i.i.d. form; two columns of one chunk never share a position, and
// columns of different chunks share one in a block with probability 1 / bw.
// The positions of a chunk being a cyclic shift, a thread can keep its
// block's bw sums of one row in registers.  Record kSignNnz g + t holds the
// sign bits (bit p: position p negative) and the shift; the sketch kernel
// draws each where it needs it.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
// record e = kSignNnz g + t of the map: its sign bits and shift
struct SignRecord {
  uint64_t signs;
  uint32_t shift;
};
__device__ __forceinline__ SignRecord sign_record(uint64_t seed, uint64_t e, uint32_t bw) {
  const uint64_t z = mix64((seed * 0xd1342543de82ef95ull) ^ e);
  return SignRecord{mix64(z), (uint32_t)(((z >> 32) * (uint64_t)bw) >> 32)};  // shift uniform in [0, bw)
}
// Y = S Omega for that map: one workgroup of kSignNnz wavefronts per slice of
// kSketchRows rows (one row per lane), wavefront t holding, per lane, the
// row's bw sums of column block t in registers.  Per chunk of bw columns the
// wavefronts t < bw / 8 load eight columns each (one column's 64 rows, 512
// contiguous bytes, per load; kSketchDepth chunks ahead) into LDS, every
// column stored twice in a row ([x_0 .. x_{bw-1}, x_0 .. x_{bw-1}]), so
// that each wavefront reads its shifted order as one contiguous window and
// adds it, signed, to its sums: each sum in chunk order, deterministic.  The
// column bases come from one vector load of the column table per chunk,
// handed out by readlane.  SAFE (slices some column does not hold in full)
// reads rows past a column's own count as zero; columns past m (the last
// chunk's rest) read as zero.  Rows of Y past n are not written.  Y element
// (r, c) at Y[c * ocs + blk_off(r, obs)].
template <int BW, bool SAFE>
__global__ __launch_bounds__(kSignNnz * 64, 1) void sign_sketch_kernel(
    const void* const* __restrict__ cols, const int64_t* __restrict__ rbs, const int64_t* __restrict__ crows,
    int64_t n, int64_t m, int64_t chunks, int64_t slice0, uint64_t seed, double* __restrict__ Y, int64_t ocs,
    int64_t obs) {
  constexpr int R = kSketchRows, D = kSketchDepth, CPW = 8, G = 8;
  static_assert(R == 64 && BW % CPW == 0 && BW <= 64 && BW % G == 0 && D % 2 == 0, "sketch shape");
  extern __shared__ double stg[];  // two buffers of 2 BW staged columns x R rows
  const int lane = threadIdx.x & 63;
  const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // this wavefront's column block
  const bool loader = (BW == 64) || t * CPW < BW;
  const int64_t s0 = (slice0 + blockIdx.x) * R;
  const int64_t row = s0 + lane;
  const int64_t blk = s0 >> 7, soff = s0 & (kRowBlock - 1);
  const int64_t steps = (chunks + D - 1) / D * D;  // whole steps of D chunks; chunks past the last are all zero
  double acc[BW];
#pragma unroll
  for (int p = 0; p < BW; ++p) acc[p] = 0.0;
  struct Raw {
    const void* c;
    int64_t rb;
    int64_t rows;
  };
  // the column table of chunk g, one column per lane (lanes past bw repeat
  // the last; columns past m read as column m - 1, their values dropped)
  auto load_ct = [&](int64_t g) -> Raw {
    const int64_t k = min(g * BW + min(lane, BW - 1), m - 1);
    Raw r{*as_global(cols + k), *as_global(rbs + k), 0};
    if constexpr (SAFE) r.rows = *as_global(crows + k);
    return r;
  };
  auto readlane64 = [&](uint64_t v, int idx) -> uint64_t {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, idx);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), idx);
    return ((uint64_t)hi << 32) | lo;
  };
  double sv[D][CPW];
  Raw rr[D];
  // Slot s (static) takes chunk jj (past the last: chunk jj's clamped
  // columns, dropped).  Loads are unconditional in the full-slice form, so
  // every wait is for a fixed count.
  auto refill = [&](int s, int64_t jj) {
    // chunk jj's column table (loaded D chunks ago), used up before the slot
    // is refilled, so that the new load can take the same registers
    const uint64_t cb = (uint64_t)(reinterpret_cast<const double*>(rr[s].c) + blk * rr[s].rb + soff);
    const uint64_t crows_s = (uint64_t)rr[s].rows;
    rr[s] = load_ct(jj + D);
    if (loader) {
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        const int c = t * CPW + q;
        const double* p = reinterpret_cast<const double*>(readlane64(cb, c)) + lane;
        if constexpr (SAFE) {
          const int64_t rk = (int64_t)readlane64(crows_s, c);
          sv[s][q] = (row < rk) ? *as_global(p) : 0.0;
        } else {
          sv[s][q] = *as_global(p);
        }
      }
    }
    // (indexed by the lane's own wavefront number, a vector register, so that
    // the load stays a vector load counted with the others)
  };
#pragma unroll
  for (int s = 0; s < D; ++s) rr[s] = load_ct(s);
#pragma unroll
  for (int s = 0; s < D; ++s) {
    refill(s, s);
    // the column table loaded for the slot's next chunk, marked as used here
    // (an empty asm), so that it is not sunk past the drain below
    asm volatile("" : "+v"(rr[s].c), "+v"(rr[s].rb), "+v"(rr[s].rows));
    __builtin_amdgcn_sched_barrier(0);
  }
  // Nothing in flight on entry: the loop's waits are then those of its own
  // issue order (the compiler merges the entry state into every iteration's).
  __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
  for (int64_t j0 = 0; j0 < steps; j0 += D) {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int64_t j = j0 + s;
      // buffer s & 1 (D even: the chunk's parity) was last read two chunks
      // ago, before the last barrier
      double* st = stg + (s & 1) * (2 * BW * R);
      if (loader) {
#pragma unroll
        for (int q = 0; q < CPW; ++q) {
          const int c = t * CPW + q;
          const double v = (j * BW + c < m) ? sv[s][q] : 0.0;
          st[c * R + lane] = v;
          st[(c + BW) * R + lane] = v;
        }
      }
      const SignRecord rec = sign_record(seed, (uint64_t)(j * kSignNnz + t), (uint32_t)BW);  // scalar arithmetic
      const uint32_t mlo = (uint32_t)rec.signs, mhi = (uint32_t)(rec.signs >> 32);
      const int shift = (int)rec.shift;
      __syncthreads();
      // position p takes column (p - shift) mod bw: entry BW - shift + p of the doubled row
      const double* xr = st + (BW - shift) * R + lane;
      double xa[G], xb[G];
      auto read = [&](int g0, double (&x)[G]) {
#pragma unroll
        for (int u = 0; u < G; ++u) x[u] = xr[(g0 + u) * R];
      };
      auto add = [&](int g0, const double (&x)[G]) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int p = g0 + u;
          const uint32_t word = (p < 32) ? mlo : mhi;
          const uint32_t sb = (word << (31 - (p & 31))) & 0x80000000u;
          const uint64_t bits = __builtin_bit_cast(uint64_t, x[u]) ^ ((uint64_t)sb << 32);
          acc[p] += __builtin_bit_cast(double, bits);
        }
      };
      read(0, xa);
#pragma unroll
      for (int g0 = 0; g0 < BW; g0 += 2 * G) {
        if (g0 + G < BW) read(g0 + G, xb);
        __builtin_amdgcn_sched_barrier(0);
        add(g0, xa);
        if (g0 + 2 * G < BW) read(g0 + 2 * G, xa);
        __builtin_amdgcn_sched_barrier(0);
        if (g0 + G < BW) add(g0 + G, xb);
      }
      __builtin_amdgcn_sched_barrier(0);
      refill(s, j + D);  // (at the chunk's end: the loop's first wait is then for its own loads)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const double scale = 1.0 / sqrt((double)kSignNnz);
  if (row < n) {
#pragma unroll
    for (int p = 0; p < BW; ++p) Y[(int64_t)(t * BW + p) * ocs + blk_off(row, obs)] = acc[p] * scale;
  }
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

namespace {
template <int BW>
hapod_status sign_sketch_bw(const void* const* d_cols, const int64_t* d_rbs, const int64_t* d_rows, int64_t n, int64_t m,
                            int64_t full_rows, uint64_t seed, double* Y, int64_t ocs, int64_t obs,
                            hipStream_t stream) {
  const size_t lds = sizeof(double) * 2 * 2 * BW * kSketchRows;
  static bool attr = false;
  if (!attr) {
    HAPOD_HIP(hipFuncSetAttribute((const void*)sign_sketch_kernel<BW, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    HAPOD_HIP(hipFuncSetAttribute((const void*)sign_sketch_kernel<BW, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  const int64_t chunks = (m + BW - 1) / BW;
  const int64_t slices = (n + kSketchRows - 1) / kSketchRows;
  const int64_t fast = std::min(slices, std::max<int64_t>(full_rows, 0) / kSketchRows);
  if (slices > INT32_MAX) {
    set_error("sparse sign sketch: too many rows");
    return HAPOD_E_UNSUPPORTED;
  }
  const dim3 block(kSignNnz * 64);
  if (fast > 0) {
    hipLaunchKernelGGL((sign_sketch_kernel<BW, false>), dim3((unsigned)fast), block, lds, stream, d_cols, d_rbs,
                       d_rows, n, m, chunks, (int64_t)0, seed, Y, ocs, obs);
    HAPOD_HIP(hipGetLastError());
  }
  if (slices > fast) {
    hipLaunchKernelGGL((sign_sketch_kernel<BW, true>), dim3((unsigned)(slices - fast)), block, lds, stream, d_cols,
                       d_rbs, d_rows, n, m, chunks, fast, seed, Y, ocs, obs);
    HAPOD_HIP(hipGetLastError());
  }
  return HAPOD_OK;
}
}  // namespace

hapod_status launch_sign_sketch(const void* const* d_cols, const int64_t* d_rbs, const int64_t* d_rows, int64_t n,
                                int64_t m, int64_t full_rows, uint64_t seed, int64_t ell, double* Y, int64_t ocs,
                                int64_t obs, hipStream_t stream) {
  if (n <= 0 || m <= 0) return HAPOD_OK;
  switch (ell) {
    case 128: return sign_sketch_bw<16>(d_cols, d_rbs, d_rows, n, m, full_rows, seed, Y, ocs, obs, stream);
    case 256: return sign_sketch_bw<32>(d_cols, d_rbs, d_rows, n, m, full_rows, seed, Y, ocs, obs, stream);
    case 384: return sign_sketch_bw<48>(d_cols, d_rbs, d_rows, n, m, full_rows, seed, Y, ocs, obs, stream);
    case 512: return sign_sketch_bw<64>(d_cols, d_rbs, d_rows, n, m, full_rows, seed, Y, ocs, obs, stream);
    default:
      set_error("sparse sign sketch: ell must be 128, 256, 384 or 512");
      return HAPOD_E_UNSUPPORTED;
  }
}

hapod_status launch_transpose(const double* A, int64_t lda, int64_t m, double* T, int64_t ldt, hipStream_t stream) {
  if (m <= 0) return HAPOD_OK;
  const unsigned nb = (unsigned)((m + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, dim3(nb, nb), dim3(256), 0, stream, A, lda, m, T, ldt);
  HAPOD_HIP(hipGetLastError());
  return HAPOD_OK;
}

}  // namespace hapod
