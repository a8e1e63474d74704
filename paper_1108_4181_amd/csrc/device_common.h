// Device helpers shared by the solver's kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace td {

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int out_row(int L) { return 4 * ((L >> 2) & 3) + (L >> 4); }
__device__ __forceinline__ int out_col(int L) { return L & 3; }

// Work-groups are handed to the 8 XCDs of the chip round-robin by blockIdx.  This
// maps blockIdx so that logical work items [x*per, (x+1)*per) run on XCD x, in
// order: consecutive logical items (the column tiles of one block row, which read
// the same matrix) then share that XCD's L2.  gridDim.x is a multiple of 8.
__device__ __forceinline__ int xcd_remap(int b, int grid) {
  const int per = grid >> 3;
  return (b & 7) * per + (b >> 3);
}
inline int grid_pad8(int total) { return (total + 7) & ~7; }

// rows per wave = 16*RT; waves per work-group = Mp / (16*RT)
inline int choose_rt(int Mp) {
  if (Mp >= 256 && Mp % 64 == 0) return 4;
  if (Mp >= 64 && Mp % 32 == 0) return 2;
  return 1;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// round-to-nearest-even float -> bfloat16 bits; NaN stays a quiet NaN
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int PREC> struct LP;
template <> struct LP<1> {   // float32
  using T = float;
  static constexpr int KG = 16;                    // k per group
  __device__ static T from_f(float v) { return v; }
  __device__ static void mma(f32x4& acc, const uint4& a, const uint4& b) {
    const f32x4 av = __builtin_bit_cast(f32x4, a);
    const f32x4 bv = __builtin_bit_cast(f32x4, b);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[u], acc, 0, 0, 0);
  }
};
template <> struct LP<2> {   // bfloat16
  using T = uint16_t;
  static constexpr int KG = 32;
  __device__ static T from_f(float v) { return f2bf(v); }
  __device__ static void mma(f32x4& acc, const uint4& a, const uint4& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   acc, 0, 0, 0);
  }
};

__device__ __forceinline__ int lp_xcd_remap(int b, int grid) {
  const int per = grid >> 3;
  return (b & 7) * per + (b >> 3);
}
inline int lp_pad8(int t) { return (t + 7) & ~7; }

}  // namespace td
