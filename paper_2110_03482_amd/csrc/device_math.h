// Device-side arithmetic shared by the gfx950 kernels: exact phase reduction and sin/cos of a
// fraction of a turn.
//
// Phases are unsigned fixed-point fractions of a turn.  The phasor of Eq. 4 for bin f and
// delay tau is exp(+2 pi i f tau / L); its phase f*tau/L is only needed modulo one turn.  A
// 64-bit increment  inc = frac(tau / L) * 2^64  (exact for nearest-sample delays, where it is
// (d mod L) << (64 - log2 L)) gives the phase of bin f as the wrapping product inc * f, whose
// top 32 bits feed sincos_turn.  This keeps the argument exact however large f*tau becomes;
// float32 arithmetic on f*tau would lose all phase information at the paper's sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdd {

struct PhaseInc {
  uint32_t hi;  // top 32 bits of the 64-bit turn fraction
  uint32_t lo;  // next 32 bits
};

// Delay-mode codes (match fdd_delay_mode).
constexpr int kDelayExact = 0;
constexpr int kDelayRound = 1;

// Phase increment per Fourier bin for a delay of tau samples and transform length 2^log_len.
__device__ __forceinline__ PhaseInc phase_increment(double tau, int log_len, int mode) {
  PhaseInc r;
  if (mode == kDelayRound) {
    // nearest sample, halves up; the phase of bin f is (d f mod L) / L exactly
    double d = floor(tau + 0.5);
    double dm = d - ldexp(floor(ldexp(d, -log_len)), log_len);   // d mod L, exact
    r.hi = (uint32_t)dm << (32 - log_len);
    r.lo = 0u;
  } else {
    double v = ldexp(tau, -log_len);        // tau / L, exact
    double fr = v - floor(v);               // in [0, 1), exact
    double s = ldexp(fr, 32);               // < 2^32
    double h = floor(s);
    double rem = ldexp(s - h, 32);          // < 2^32, exact
    r.hi = (uint32_t)h;
    r.lo = (uint32_t)fmin(floor(rem), 4294967295.0);
  }
  return r;
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

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

}  // namespace fdd
