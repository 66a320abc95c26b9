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

// IEEE-754 binary32 -> bfloat16, round to nearest, ties to even, written
// from the format definition (bf16 is the upper half of a binary32).
__device__ __forceinline__ uint16_t bf16_bits_rne(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  if ((u & 0x7f800000u) == 0x7f800000u) {       // Inf / NaN: truncate, keep NaN quiet
    uint16_t h = (uint16_t)(u >> 16);
    if (u & 0x007fffffu) h |= 0x0040u;
    return h;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi).
__device__ __forceinline__ void split_bf16x8(const float* x, bf8& hi, bf8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    uint16_t h = bf16_bits_rne(x[e]);
    float r = x[e] - bf16_bits_to_float(h);
    uint16_t l = bf16_bits_rne(r);
    hi[e] = __builtin_bit_cast(__bf16, h);
    lo[e] = __builtin_bit_cast(__bf16, l);
  }
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
