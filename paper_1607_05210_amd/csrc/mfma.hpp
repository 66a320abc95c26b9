// CDNA4 (gfx950) MFMA helpers: operand types, the split-BF16 conversion and
// the lane layout of the 16x16 accumulator.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hapod {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));

// 16x16 MFMA accumulators.  Operand lanes: lane l supplies row (A) / column
// (B) index l % 16 and reduction slot l / 16.  Result lanes: lane l holds
// column l % 16; its register v holds
//   FP32 accumulators (f32 16x16x4, bf16 16x16x32): row 4 * (l / 16) + v,
//   FP64 accumulators (f64 16x16x4):                row (l / 16) + 4 * v.
template <class Acc> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<f4>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<d4>(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Split of FP32 values into BF16 parts, x = hi + lo + r with hi = bf16(x),
// lo = bf16(x - hi) (x - hi is exact in FP32), |r| <= 2^-16 |x|: two values
// at a time on gfx950's packed conversion (v_cvt_pk_bf16_f32: round to
// nearest, ties to even, the default mode; Inf stays Inf, NaN stays NaN).
// hi2 / lo2 hold the parts of a in the low and of b in the high 16 bits.
__device__ __forceinline__ void split_bf16x2(float a, float b, uint32_t& hi2, uint32_t& lo2) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef __bf16 b2v __attribute__((ext_vector_type(2)));
  const f2v x{a, b};
  const b2v h = __builtin_convertvector(x, b2v);
  const b2v l = __builtin_convertvector(x - __builtin_convertvector(h, f2v), b2v);
  hi2 = __builtin_bit_cast(uint32_t, h);
  lo2 = __builtin_bit_cast(uint32_t, l);
}

// eight values: the hi parts and the lo parts as MFMA operands
__device__ __forceinline__ void split_bf16x8(const float* x, bf8& hi, bf8& lo) {
  typedef __attribute__((ext_vector_type(4))) uint32_t u4v;
  u4v h, l;
  uint32_t hh[4], ll[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) split_bf16x2(x[2 * e], x[2 * e + 1], hh[e], ll[e]);
  h = u4v{hh[0], hh[1], hh[2], hh[3]};
  l = u4v{ll[0], ll[1], ll[2], ll[3]};
  hi = __builtin_bit_cast(bf8, h);
  lo = __builtin_bit_cast(bf8, l);
}

// Pointers into global memory (address space 1): loads through them become
// global_load instructions instead of generic flat loads.
template <class T> using gptr = const __attribute__((address_space(1))) T*;
template <class T> __device__ __forceinline__ gptr<T> as_global(const T* p) { return (gptr<T>)p; }

// Map a linear workgroup id to a work-item index so that each of the 8 XCDs
// (which receive workgroups round-robin) gets one contiguous range of items.
__device__ __forceinline__ int xcd_item(int bid, int nblk) {
  int q = nblk >> 3, r = nblk & 7;
  int x = bid & 7, i = bid >> 3;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace hapod
