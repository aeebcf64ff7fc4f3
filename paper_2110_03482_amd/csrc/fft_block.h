// Workgroup-resident complex FFT for gfx950 (Stockham autosort, radix up to 32).
//
// A transform of N = 2^LOGN complex points is held in registers by T = N / E threads,
// E = 2^LOGE points each: thread t owns points t + T*q, q < E.  Every pass of radix R
// (R <= E) performs E/R butterflies per thread; butterfly j = t + T*b reads points
// j + r*N/R, which are exactly the thread's own points b + r*E/R, so loads never cross
// threads.  Only the scatter of a pass's outputs to their autosort positions
//     (j / Ns) * Ns * R + (j mod Ns) + r * Ns
// needs LDS.  After the last pass the outputs land back in the owner's registers in natural
// order, so the last pass needs no exchange.  The exchange moves real and imaginary parts in
// two rounds through an N-float buffer so that a 2^15-point transform fits in LDS.
//
// The radix-R butterfly is an in-register radix-2 decimation-in-frequency network whose
// twiddles are compile-time constants; its bit-reversed result is renamed back at no cost.
// Pass twiddles are evaluated in registers from their exact fixed-point angle (sincos_turn),
// which keeps long-latency loads out of the passes.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_math.h"

namespace fdd {

// exp(-2 pi i p / 2^32) (forward) or exp(+2 pi i p / 2^32) (INV).
template <bool INV>
__device__ __forceinline__ float2 turn_phasor(uint32_t p) {
  float s, c;
  sincos_turn(p, &s, &c);
  return make_float2(c, INV ? s : -s);
}

// ----------------------------------------------------------------------------- constexpr trig
// Taylor series evaluated in double at compile time, argument reduced to [-pi, pi].
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_reduce(double x) {
  while (x > kPi) x -= 2.0 * kPi;
  while (x < -kPi) x += 2.0 * kPi;
  return x;
}
constexpr double cx_sin(double x) {
  x = cx_reduce(x);
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) {
  x = cx_reduce(x);
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// exp(sign * 2 pi i m / R) as float constants.
template <int R, bool INV>
struct RootTable {
  float c[R];
  float s[R];
  constexpr RootTable() : c(), s() {
    for (int m = 0; m < R; ++m) {
      const double a = (INV ? 2.0 : -2.0) * kPi * m / R;
      c[m] = (float)cx_cos(a);
      s[m] = (float)cx_sin(a);
    }
  }
};

__device__ __forceinline__ float2 f2add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 f2sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// d * exp(sign * 2 pi i m / R) with the trivial factors 1 and -/+i special-cased.
template <int R, bool INV>
__device__ __forceinline__ float2 twiddle_const(float2 d, int m) {
  constexpr RootTable<R, INV> tab{};
  if (m == 0) return d;
  if (4 * m == R) return INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
  const float c = tab.c[m], s = tab.s[m];
  return make_float2(fmaf(d.x, c, -d.y * s), fmaf(d.x, s, d.y * c));
}

constexpr int cx_bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r = (r << 1) | ((v >> i) & 1);
  return r;
}
constexpr int cx_log2(int v) { return v <= 1 ? 0 : 1 + cx_log2(v >> 1); }

// In-place R-point DFT of a[0..R), sign -1 (forward) or +1 (INV), natural-order output.
template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2* a) {
#pragma unroll
  for (int half = R / 2; half >= 1; half >>= 1) {
#pragma unroll
    for (int s = 0; s < R; s += 2 * half) {
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const float2 u = a[s + i], w = a[s + i + half];
        a[s + i] = f2add(u, w);
        a[s + i + half] = twiddle_const<R, INV>(f2sub(u, w), i * (R / (2 * half)));
      }
    }
  }
  float2 t[R];
#pragma unroll
  for (int k = 0; k < R; ++k) t[k] = a[cx_bitrev(k, cx_log2(R))];
#pragma unroll
  for (int k = 0; k < R; ++k) a[k] = t[k];
}

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }

template <int LOGN>
struct LdsSize {
  static constexpr int floats = (1 << LOGN) + ((1 << LOGN) >> 5);
};

// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// d * exp(sign * 2 pi i M / D), sign -1 (forward) or +1 (INV), for compile-time M and D; the
// quarter turns are exact and the rest costs one complex multiplication by constants.
template <int M, int D, bool INV>
__device__ __forceinline__ float2 rotate_const(float2 d) {
  constexpr int m = M % D;
  if constexpr (m == 0) {
    return d;
  } else if constexpr (2 * m == D) {
    return make_float2(-d.x, -d.y);
  } else if constexpr (4 * m == D) {
    return INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
  } else if constexpr (4 * m == 3 * D) {
    return INV ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
  } else {
    constexpr double ang = (INV ? 2.0 : -2.0) * kPi * m / D;
    constexpr float c = (float)cx_cos(ang), s = (float)cx_sin(ang);
    return make_float2(fmaf(d.x, c, -d.y * s), fmaf(d.x, s, d.y * c));
  }
}

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

template <int LOGN, int LOGE, bool INV, int LOGRMAX = 4>
struct BlockFft {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 1 << LOGE;
  static constexpr int T = N / E;

  // Padded LDS index of point i; for T >= 32 the read side of an exchange reduces to
  // rd0 + q (T + T/32), rd0 = t + t/32.
  __device__ __forceinline__ static int read_index(int t, int q) {
    if constexpr (T >= 32) return t + (t >> 5) + q * (T + T / 32);
    else return lds_pad(t + T * q);
  }

  // One Stockham pass over sub-transform size Ns = 2^LOGNS; recursion runs the rest.
  template <int LOGNS>
  __device__ __forceinline__ static void pass(float2 (&v)[E], float* lds) {
    if constexpr (LOGNS < LOGN) {
      constexpr int LOGRC = LOGE < LOGRMAX ? LOGE : LOGRMAX;    // radix cap
      constexpr int LOGR = (LOGRC < LOGN - LOGNS) ? LOGRC : (LOGN - LOGNS);
      constexpr int R = 1 << LOGR;
      constexpr int NB = E / R;          // butterflies per thread
      constexpr int Ns = 1 << LOGNS;
      constexpr bool last = (LOGNS + LOGR == LOGN);
      const int t = threadIdx.x;
      // Pass twiddles.  Butterfly b = 0 .. NB-1 of thread t is j = t + T b, k = j mod Ns, and
      // scales its input r by w^r, w = exp(-/+ 2 pi i k / (Ns R)).  For Ns <= T every b has
      // k0 = t mod Ns; for Ns > T, k = t + T b' with b' = b mod (Ns / T), and the extra factor
      // exp(-/+ 2 pi i r T b' / (Ns R)) is a compile-time constant.  So only the twiddles of k0
      // are evaluated: w^(2^e) from the exact 32-bit fixed-point angle 2^e k0 / (Ns R) of a
      // turn, every other power as a product of those (w^r = w^(2^e) w^(r - 2^e), 2^e the top
      // bit of r): log2 R evaluations instead of R - 1, at most log2 R - 1 extra roundings.
      float2 tw[R];
      if constexpr (Ns > 1) {
        constexpr int SH = 32 - LOGNS - LOGR;
        const uint32_t k0 = (uint32_t)t & (uint32_t)(Ns - 1);
#pragma unroll
        for (int r = 1; r < R; r *= 2) tw[r] = turn_phasor<INV>((uint32_t)(r * k0) << SH);
#pragma unroll
        for (int r = 3; r < R; ++r) {
          if ((r & (r - 1)) == 0) continue;
          const int top = 1 << cx_log2(r);
          tw[r] = cmulf(tw[top], tw[r - top]);
        }
      }
      // butterflies in place: the outputs of butterfly b overwrite its inputs, slot b + r*NB
      static_for<0, NB>([&](auto bi) {
        constexpr int b = decltype(bi)::value;
        constexpr int BP = Ns > T ? b % (Ns / T) : 0;
        float2 a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = v[b + r * NB];
        if constexpr (Ns > 1) {
          static_for<1, R>([&](auto ri) {
            constexpr int r = decltype(ri)::value;
            a[r] = rotate_const<r * T * BP, Ns * R, INV>(cmulf(a[r], tw[r]));
          });
        }
        dft_reg<R, INV>(a);
#pragma unroll
        for (int r = 0; r < R; ++r) v[b + r * NB] = a[r];
      });
      // After the last pass the outputs already sit on the owner's points in natural order.
      if constexpr (!last) {
        // Output r of butterfly j goes to point base + r Ns, base = (j / Ns) Ns R + k.  For
        // power-of-two Ns and R the padding splits: pad(base + r Ns) = pad(base) + r Ns +
        // (r Ns) / 32, a compile-time offset per r.
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int j = t + T * b;
            const int k = j & (Ns - 1);
            const int base = ((j >> LOGNS) << (LOGNS + LOGR)) + k;
            const int pb = base + (base >> 5);
#pragma unroll
            for (int r = 0; r < R; ++r)
              lds[pb + r * Ns + ((r * Ns) >> 5)] = part ? v[b + r * NB].y : v[b + r * NB].x;
          }
          __syncthreads();
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const float val = lds[read_index(t, q)];
            if (part) v[q].y = val; else v[q].x = val;
          }
          __syncthreads();
        }
        pass<LOGNS + LOGR>(v, lds);
      }
    }
  }

  __device__ __forceinline__ static void run(float2 (&v)[E], float* lds) {
    pass<0>(v, lds);
  }

  // Calls fn(integral_constant q, Z[f], Z[(N - f) mod N]) for every owned point f = t + T q.
  // The partner point is owned by another thread; it is fetched through LDS in two rounds
  // (partners in the upper half of the index range, then in the lower half), so that only N/2
  // complex values are ever staged and no thread has to hold a second copy of its points.
  template <class Fn>
  __device__ __forceinline__ static void with_mirror(const float2 (&v)[E], float* lds, Fn fn) {
    float2* l2 = reinterpret_cast<float2*>(lds);
    const int t = threadIdx.x;
#pragma unroll
    for (int upper = 1; upper >= 0; --upper) {
#pragma unroll
      for (int q = 0; q < E; ++q)
        if ((q >= E / 2) == (upper != 0)) l2[t + T * q - upper * (N / 2)] = v[q];
      __syncthreads();
      static_for<0, E>([&](auto qi) {
        constexpr int q = decltype(qi)::value;
        const int m = (N - (t + T * q)) & (N - 1);
        if ((m >= N / 2) == (upper != 0)) fn(qi, v[q], l2[m - upper * (N / 2)]);
      });
      __syncthreads();
    }
  }

  // exp(-/+ 2 pi i f / (2N)) for the owned points f = t + T q: one evaluation at f = t, then a
  // constant rotation by T q / (2N) of a turn per q.
  template <int Q>
  __device__ __forceinline__ static float2 half_bin_phasor(float2 w0) {
    return rotate_const<T * Q, 2 * N, INV>(w0);
  }
  __device__ __forceinline__ static float2 half_bin_phasor_base() {
    return turn_phasor<INV>((uint32_t)threadIdx.x << (32 - LOGN - 1));
  }
};

}  // namespace fdd
