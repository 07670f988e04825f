// Vector loads of dense rows as FP32 registers, for FP32 and bfloat16 data.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace spc3d {

typedef uint16_t bf16_t;   // bfloat16 bit pattern

__device__ inline float bf16_to_f32(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest even; NaN stays NaN (quiet bit set, sign and upper payload
// kept).  Integer formulation: add 0x7FFF plus the lowest kept bit, truncate.
__device__ inline bf16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

// Load VEC consecutive elements starting at p (16-byte aligned when VEC*size
// is 16) into FP32 registers.
template <typename T, int VEC>
struct VecLoad;

template <>
struct VecLoad<float, 4> {
  static __device__ inline void load(const float* p, float (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};

template <>
struct VecLoad<float, 1> {
  static __device__ inline void load(const float* p, float (&o)[1]) { o[0] = *p; }
};

template <>
struct VecLoad<bf16_t, 8> {
  static __device__ inline void load(const bf16_t* p, float (&o)[8]) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = __uint_as_float(w[i] << 16);
      o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  }
};

template <>
struct VecLoad<bf16_t, 1> {
  static __device__ inline void load(const bf16_t* p, float (&o)[1]) { o[0] = bf16_to_f32(*p); }
};

}  // namespace spc3d

namespace spc3d {

// Raw 16-byte vectors (4 FP32 or 8 bfloat16), kept unconverted in registers
// while loads are in flight and converted at use.
template <typename T, int VEC>
struct Unpack;

template <>
struct Unpack<float, 4> {
  static __device__ inline void run(const uint4& r, float (&o)[4]) {
    o[0] = __uint_as_float(r.x); o[1] = __uint_as_float(r.y);
    o[2] = __uint_as_float(r.z); o[3] = __uint_as_float(r.w);
  }
};

template <>
struct Unpack<bf16_t, 8> {
  static __device__ inline void run(const uint4& r, float (&o)[8]) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = __uint_as_float(w[i] << 16);
      o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  }
};

}  // namespace spc3d
