// Device-side arithmetic shared by the gfx950 kernels: exact phases and sin/cos of a fraction
// of a turn.
//
// Phases are unsigned fixed-point fractions of a turn.  The phasor of Eq. 4 for bin f and
// delay tau is exp(+2 pi i f tau / L); its phase f*tau/L is only needed modulo one turn.  A
// 64-bit increment  inc = frac(tau / L) * 2^64  (exact for nearest-sample delays, where it is
// (d mod L) << (64 - log2 L)) gives the phase of bin f as the wrapping product inc * f, whose
// top 32 bits feed sincos_turn.  This keeps the argument exact however large f*tau becomes;
// float32 arithmetic on f*tau would lose all phase information at the paper's sizes.
//
// The planner tabulates, per (channel, DM), the increment and the unit phasor of one bin step
// (evaluated in float64 from all 64 bits), channel-major: entry (c, dm) = {inc.lo, inc.hi,
// cos, sin}.  A kernel seeds a run of bins with one 16-byte load and one sincos_turn, then
// walks the run by complex multiplication.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdd {

struct PhaseInc {
  uint32_t hi;  // top 32 bits of the 64-bit turn fraction
  uint32_t lo;  // next 32 bits
};

// Raw buffer loads: a wave-uniform base and byte count (a descriptor in scalar registers) and
// a per-lane 32-bit byte offset.  Offsets at or past the byte count read as zero, so a kernel
// can stage zeros for channels past the last one without branches or 64-bit address
// arithmetic.  The byte count saturates at 2^31 - 1: a window must be smaller than 2 GiB.
constexpr int kRawBufferWord3 = 0x00020000;   // descriptor word 3: untyped 32-bit data, no swizzle
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base, int64_t bytes) {
  const int n = bytes <= 0 ? 0 : (bytes >= 0x7fffffff ? 0x7fffffff : (int)bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, kRawBufferWord3);
}
__device__ __forceinline__ float4 load_f4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const f4v v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
  return make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ uint4 load_u4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const u4v v = __builtin_bit_cast(u4v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
  return make_uint4(v[0], v[1], v[2], v[3]);
}

// Top 32 bits of (inc * f) mod 2^64, for f < 2^32.
__device__ __forceinline__ uint32_t phase_at(PhaseInc inc, uint32_t f) {
  return inc.hi * f + __umulhi(inc.lo, f);
}

// sin and cos of 2 pi p / 2^32.  Reduction to the nearest quarter turn is exact in integer
// arithmetic; the remainder |y| <= pi/4 is evaluated with the Taylor series of sin to y^9 and
// of cos to y^10 (truncation below 2e-9), then rotated by the quarter turns.
__device__ __forceinline__ void sincos_turn(uint32_t p, float* s_out, float* c_out) {
  const uint32_t q = (p + 0x20000000u) >> 30;
  const int32_t r = (int32_t)(p - (q << 30));
  const float y = (float)r * 1.46291807926715968e-9f;   // 2 pi / 2^32
  const float y2 = y * y;
  float s = fmaf(y2, 2.75573192e-6f, -1.98412698e-4f);   // 1/9!, -1/7!
  s = fmaf(y2, s, 8.33333333e-3f);                        // 1/5!
  s = fmaf(y2, s, -1.66666667e-1f);                       // -1/3!
  s = fmaf(y2 * y, s, y);
  float c = fmaf(y2, -2.75573192e-7f, 2.48015873e-5f);   // -1/10!, 1/8!
  c = fmaf(y2, c, -1.38888889e-3f);                       // -1/6!
  c = fmaf(y2, c, 4.16666667e-2f);                        // 1/4!
  c = fmaf(y2, c, -0.5f);                                 // -1/2!
  c = fmaf(y2, c, 1.0f);
  const uint32_t qq = q & 3u;
  const float cs = (qq & 1u) ? s : c;
  const float sn = (qq & 1u) ? c : s;
  *c_out = (qq == 1u || qq == 2u) ? -cs : cs;
  *s_out = (qq >= 2u) ? -sn : sn;
}

// Phasor of bin f0 and of one bin step, from a table entry {inc.lo, inc.hi, cos, sin}.
__device__ __forceinline__ void seed_phasor(uint4 e, uint32_t f0, float2* w, float2* step) {
  const PhaseInc inc = {e.y, e.x};
  float s, c;
  sincos_turn(phase_at(inc, f0), &s, &c);
  *w = make_float2(c, s);
  *step = make_float2(__uint_as_float(e.z), __uint_as_float(e.w));
}

// sin and cos of 2 pi p / 2^32 from a 256-entry table of the phasors of k / 256 turn (nearest k)
// and the rotation by the remainder |y| <= pi / 256, whose sine and cosine are y - y^3 / 6 and
// 1 - y^2 / 2 to within 2e-12 and 1e-9.
__device__ __forceinline__ float2 turn_phasor_tab(uint32_t p, const float2* tab) {
  const uint32_t k = (p + 0x800000u) >> 24;
  const int32_t r = (int32_t)(p << 8) >> 8;             // p - k 2^24, in [-2^23, 2^23)
  const float y = (float)r * 1.46291807926715968e-9f;   // 2 pi / 2^32
  const float y2 = y * y;
  const float s = fmaf(y2 * y, -1.66666667e-1f, y);
  const float c = fmaf(y2, -0.5f, 1.0f);
  const float2 t = tab[k];
  return make_float2(fmaf(t.x, c, -t.y * s), fmaf(t.y, c, t.x * s));
}
// seed_phasor with the table form of sincos_turn.
__device__ __forceinline__ void seed_phasor_tab(uint4 e, uint32_t f0, const float2* tab, float2* w, float2* step) {
  const PhaseInc inc = {e.y, e.x};
  *w = turn_phasor_tab(phase_at(inc, f0), tab);
  *step = make_float2(__uint_as_float(e.z), __uint_as_float(e.w));
}
// Entry k of that table (k < 256), from sincos_turn.
__device__ __forceinline__ float2 turn_table_entry(uint32_t k) {
  float s, c;
  sincos_turn(k << 24, &s, &c);
  return make_float2(c, s);
}

// The same from a per-channel linear entry {inc0.lo, inc0.hi, d.lo, d.hi} for trial j: the
// increment is inc0 + j d (mod 2^64) and the step phasor is evaluated from its top 32 bits
// (truncation below 2^-32 of a turn).
__device__ __forceinline__ void seed_phasor_linear(uint4 e, uint32_t j, uint32_t f0, float2* w, float2* step) {
  const uint64_t inc = (((uint64_t)e.y << 32) | e.x) + (uint64_t)j * (((uint64_t)e.w << 32) | e.z);
  const PhaseInc pi = {(uint32_t)(inc >> 32), (uint32_t)inc};
  float s, c;
  sincos_turn(phase_at(pi, f0), &s, &c);
  *w = make_float2(c, s);
  sincos_turn(pi.hi, &s, &c);
  *step = make_float2(c, s);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

}  // namespace fdd
