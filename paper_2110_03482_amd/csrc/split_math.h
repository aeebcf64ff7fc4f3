// Device helpers of the split-precision matrix-core kernels (gfx950 v_mfma_f32_16x16x32_{f16,bf16}).
//
// An FP32 value v is carried as a half-precision head and tail, v = hi + lo with
// hi = half(v) and lo = half(v - hi); products are accumulated in FP32 as
//     A_hi B_hi + A_hi B_lo + A_lo B_hi
// (A_lo B_lo, about 2^-22 relative for FP16, is dropped).  Pairs of values travel packed in one
// 32-bit word, first value in the low half.  FP16 has a small range, so data operands carry a
// power-of-two scale per chunk (chunk_scale), exact and divided out after the products.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdd {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf162v __attribute__((ext_vector_type(2)));

// The 8-half operand type and the 16x16x32 product of one format (BF: bfloat16, else float16).
template <bool BF>
struct HalfMma;

template <>
struct HalfMma<false> {
  typedef half8 V8;
  __device__ static __forceinline__ floatx4 mfma(V8 a, V8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct HalfMma<true> {
  typedef bf16x8 V8;
  __device__ static __forceinline__ floatx4 mfma(V8 a, V8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// 1.0f in a scalar register whose value the compiler does not see.  In fma(h, -one, x) with a
// float16 h this keeps the mixed-precision form (v_fma_mix_f32 takes the half operand as it is
// packed) instead of the conversion and subtraction that the folded x - h would cost.
__device__ __forceinline__ float opaque_one() {
  float one;
  asm("s_mov_b32 %0, 1.0" : "=s"(one));
  return one;
}

// Head/tail split of a pair (x, y): hi = (half(x), half(y)), lo = (half(x - hi_x), half(y - hi_y)).
// The residuals x - hi_x are exact in float32 (hi_x holds the leading 11 or 8 bits of x).  MIX
// (float16): the residuals through v_fma_mix_f32; the same values, fewer instructions, though in
// some kernels more live registers (the single-chunk factorised kernel keeps it inside its
// register budget only with a launch bound of three waves per SIMD).
template <bool BF, bool MIX = true>
__device__ __forceinline__ void split_pair(float x, float y, uint32_t* hi, uint32_t* lo) {
  const float2v v = {x, y};
  if constexpr (BF) {
    const bf162v h = __builtin_convertvector(v, bf162v);
    const float2v hb = __builtin_convertvector(h, float2v);
    const float2v r = {x - hb[0], y - hb[1]};
    *hi = __builtin_bit_cast(uint32_t, h);
    *lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf162v));
  } else if constexpr (MIX) {
    const half2v h = __builtin_convertvector(v, half2v);
    const float one = opaque_one();
    const float2v r = {__builtin_fmaf((float)h[0], -one, x), __builtin_fmaf((float)h[1], -one, y)};
    *hi = __builtin_bit_cast(uint32_t, h);
    *lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, half2v));
  } else {
    const half2v h = __builtin_convertvector(v, half2v);
    const float2v hb = __builtin_convertvector(h, float2v);
    const float2v r = {x - hb[0], y - hb[1]};
    *hi = __builtin_bit_cast(uint32_t, h);
    *lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, half2v));
  }
}

// (x, y) -> (x, -y) and (x, y) -> (y, x) on packed half pairs (exact).
__device__ __forceinline__ uint32_t neg_hi(uint32_t w) { return w ^ 0x80000000u; }
__device__ __forceinline__ uint32_t swap16(uint32_t w) { return (w >> 16) | (w << 16); }

// Scale 2^(14 - ceil(log2 L1)) of a chunk whose input series have L1 norms <= L1 (float bits):
// |X| <= L1 keeps every scaled value below 2^14.  1 for an empty chunk.
__device__ __forceinline__ float chunk_scale(unsigned int l1bits) {
  const float l1 = __uint_as_float(l1bits);
  int ex = 0;
  (void)frexpf(l1, &ex);
  return l1 > 0.0f ? ldexpf(1.0f, 14 - ex) : 1.0f;
}

}  // namespace fdd
