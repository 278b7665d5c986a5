// Device-side helpers shared by the HIP kernels (CDNA4 / gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tok {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// 64-bit SplitMix64 output function on state x (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

// Two floats -> packed bf16 pair (a in the low half), round to nearest even
// (one v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// ---- fp8 e4m3 (OCP) with E8M0 block scales ---------------------------------
typedef __attribute__((ext_vector_type(8))) int i32x8;
constexpr float kFp8Max = 448.0f;

// Exponent e of the smallest power of two with amax * 2^-e <= 448 (0 for an
// all-zero block), clamped to the E8M0 range; the stored scale byte is e + 127.
__device__ __forceinline__ int fp8_block_exp(float amax) {
  if (!(amax > 0.f)) return 0;
  const uint32_t b = __float_as_uint(amax * (1.0f / kFp8Max));
  int e = (int)((b >> 23) & 255u) - 127;
  if (b & 0x7fffffu) e += 1;
  return e < -127 ? -127 : (e > 127 ? 127 : e);
}

// Four floats (already scaled into [-448, 448]) -> four e4m3 bytes, element 0 lowest.
__device__ __forceinline__ uint32_t pack_fp8x4(float a, float b, float c, float d) {
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, lo, true);
}

__device__ __forceinline__ float silu_f(float x) {
  return x * __builtin_amdgcn_rcpf(1.0f + __expf(-x));
}

}  // namespace tok
