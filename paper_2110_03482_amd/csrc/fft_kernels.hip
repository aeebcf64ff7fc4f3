// Forward (real-to-complex) and inverse (complex-to-real) transforms of the dedispersion path,
// and the transpose/unpack of 8-bit time-major input.  gfx950, one workgroup per series.
//
// Forward (Eq. 3, Algorithm 1 preprocessing): series (c, k) holds input samples kS .. kS+L-1
// of channel c, zero beyond n_samp.  Its L real samples are packed as N = L/2 complex points
// z[j] = x[2j] + i x[2j+1], transformed with an N-point FFT, and split into the L/2+1 bins of
// the real transform:
//     X[f] = (Z[f] + conj Z[N-f]) / 2 - i exp(-2 pi i f / L) (Z[f] - conj Z[N-f]) / 2.
// 8-bit chunks lying wholly inside the data have the zero point 128 removed first; that is a
// pure DC offset, restored exactly after the inverse (DC phasors are 1 for every delay).
//
// Inverse (Eq. 6, postprocessing): the reverse split
//     Z[f] = A[f] + i B[f],  A = (Y[f] + conj Y[N-f]) / 2,  B = exp(+2 pi i f / L) (Y[f] - conj Y[N-f]) / 2
// with Im Y[0] = Im Y[N] = 0, an inverse N-point FFT scaled by 1/N, and x[2j] = Re z[j],
// x[2j+1] = Im z[j].  The scaling step of Algorithm 1 and the extraction of the S samples
// a chunk keeps (Sec. 2.2 discard rule) are fused into the store.
#include "fdd_internal.h"
#include "fft_block.h"

namespace fdd {

// ----------------------------------------------------------------------------- transpose

// uint8 [n_samp][n_chan] -> uint8 [n_chan][n_samp], 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_u8(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                      int64_t n_samp, int n_chan) {
  __shared__ uint8_t tile[64][65];
  const int64_t t0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = tid + 256 * e;
    const int i = idx >> 6, j = idx & 63;           // sample row i, channel j
    const int64_t t = t0 + i;
    const int c = c0 + j;
    tile[i][j] = (t < n_samp && c < n_chan) ? in[t * n_chan + c] : (uint8_t)0;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = tid + 256 * e;
    const int j = idx >> 6, i = idx & 63;           // channel j, sample i
    const int64_t t = t0 + i;
    const int c = c0 + j;
    if (t < n_samp && c < n_chan) out[(int64_t)c * n_samp + t] = tile[i][j];
  }
}

// The same for n_samp and n_chan multiples of 64, moving 4-byte words: a thread loads 4
// channels of one sample and stores 4 samples of one channel, gathered from the tile with byte
// permutes.
__global__ __launch_bounds__(256) void k_transpose_u8_w(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        int64_t n_samp, int n_chan) {
  __shared__ uint32_t tile[64][17];                 // [sample][4-channel word], padded row
  const int64_t t0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  const int64_t wrow = n_chan / 4;                  // words per input row
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 256 * e;
    const int i = idx >> 4, k = idx & 15;           // sample i, channel word k
    tile[i][k] = in[(t0 + i) * wrow + c0 / 4 + k];
  }
  __syncthreads();
  const int64_t wcol = n_samp / 4;                  // words per output row
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 256 * e;
    const int c = idx >> 4, g = idx & 15;           // channel c, samples 4g .. 4g + 3
    const int k = c >> 2, sh = 8 * (c & 3);
    const uint32_t b0 = (tile[4 * g][k] >> sh) & 0xffu;
    const uint32_t b1 = (tile[4 * g + 1][k] >> sh) & 0xffu;
    const uint32_t b2 = (tile[4 * g + 2][k] >> sh) & 0xffu;
    const uint32_t b3 = (tile[4 * g + 3][k] >> sh) & 0xffu;
    out[(int64_t)(c0 + c) * wcol + t0 / 4 + g] = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
  }
}

// ----------------------------------------------------------------------------- forward

// Sum over the workgroup (any size up to 1024); lds needs blockDim.x / 64 floats.
__device__ __forceinline__ float block_sum(float v, float* lds) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  float r = 0.0f;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) r += lds[i];
  __syncthreads();
  return r;
}

__global__ void k_zero_u32(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <int LOGN, int LOGE, bool U8>
__device__ __forceinline__ void r2c_body(const FftArgs& a, const int k, const int c) {
  using F = BlockFft<LOGN, LOGE, false>;
  constexpr int N = F::N, E = F::E, T = F::T;
  constexpr int64_t L = 2 * (int64_t)N;
  __shared__ float lds[LdsSize<LOGN>::floats];
  const uint8_t* __restrict__ in_u8 = a.in_u8;
  const float* __restrict__ in_f32 = a.in_f32;
  float2* __restrict__ X = a.X;
  const int64_t n_samp = a.n_samp, stride = a.stride, pitch = a.pitch;
  const int n_chunks = a.n_chunks;
  unsigned int* __restrict__ l1max = a.l1max;
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)k * stride;
  const float zp = (U8 && s0 + L <= n_samp) ? 128.0f : 0.0f;
  const int64_t rem64 = n_samp - s0;                           // samples of the series inside the data
  const int rem = rem64 < L ? (rem64 > 0 ? (int)rem64 : 0) : (int)L;
  float2 v[E];
  if constexpr (U8) {
    const uint8_t* src = in_u8 + (int64_t)c * n_samp + s0;
    if (rem == (int)L && ((uintptr_t)src & 1u) == 0) {
      // whole series, 2-byte aligned: one 16-bit load per point (x[2j] low byte, x[2j+1] high)
      const uint16_t* s16 = reinterpret_cast<const uint16_t*>(src);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const uint32_t w = s16[t + T * q];
        v[q] = make_float2((float)(w & 0xffu) - zp, (float)(w >> 8) - zp);
      }
    } else {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int s = 2 * (t + T * q);
        v[q].x = s < rem ? (float)src[s] - zp : 0.0f;
        v[q].y = s + 1 < rem ? (float)src[s + 1] - zp : 0.0f;
      }
    }
  } else {
    const float* src = in_f32 + (int64_t)c * n_samp + s0;
    if (rem == (int)L && ((uintptr_t)src & 7u) == 0) {
      const float2* s2 = reinterpret_cast<const float2*>(src);
#pragma unroll
      for (int q = 0; q < E; ++q) v[q] = s2[t + T * q];
    } else {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int s = 2 * (t + T * q);
        v[q].x = s < rem ? src[s] : 0.0f;
        v[q].y = s + 1 < rem ? src[s + 1] : 0.0f;
      }
    }
  }
  if (l1max != nullptr) {
    // |X[f]| <= sum_t |x[t]|: the series' L1 norm bounds every bin, which sets the
    // power-of-two data scale of the half-precision phasor sums
    float s1 = 0.0f;
#pragma unroll
    for (int q = 0; q < E; ++q) s1 += fabsf(v[q].x) + fabsf(v[q].y);
    s1 = block_sum(s1, lds);
    if (t == 0) atomicMax(l1max + k, __float_as_uint(s1));   // non-negative floats order as uints
  }
  F::run(v, lds);
  const int row_chunks = a.row_chunks > 0 ? a.row_chunks : n_chunks;   // chunks per row of X
  float2* dst = X + ((int64_t)c * row_chunks + k) * pitch;
  const float2 w0 = F::half_bin_phasor_base();                 // exp(-2 pi i t / L)
  F::with_mirror(v, lds, [&](auto qi, float2 zf, float2 zm) {
    constexpr int q = decltype(qi)::value;
    const int f = t + T * q;
    const float2 zc = make_float2(zm.x, -zm.y);                // conj Z[N - f]
    const float2 a = make_float2(0.5f * (zf.x + zc.x), 0.5f * (zf.y + zc.y));
    const float2 d = make_float2(0.5f * (zf.x - zc.x), 0.5f * (zf.y - zc.y));
    const float2 b = make_float2(d.y, -d.x);                   // -i d
    const float2 w = F::template half_bin_phasor<q>(w0);       // exp(-2 pi i f / L)
    dst[f] = make_float2(a.x + fmaf(w.x, b.x, -w.y * b.y), a.y + fmaf(w.x, b.y, w.y * b.x));
  });
  if (t == 0) dst[N] = make_float2(v[0].x - v[0].y, 0.0f);   // Nyquist bin
}

template <int LOGN, int LOGE, bool U8>
__global__ __launch_bounds__(1 << (LOGN - LOGE)) void k_r2c(FftArgs a) {
  r2c_body<LOGN, LOGE, U8>(a, blockIdx.x, blockIdx.y);
}

// Batched form: one workgroup per (beam, channel, chunk) series; all beams of the launch
// share L.
template <int LOGN, int LOGE, bool U8>
__global__ __launch_bounds__(1 << (LOGN - LOGE)) void k_r2c_grouped(Group<FftArgs> g) {
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (bid >= g.total) return;
  const int b = group_beam(g.prefix, g.n_beams, bid);
  const FftArgs a = g.beams[b];
  const int lid = bid - g.prefix[b];
  if (lid >= a.n_chunks * a.n_rows) return;
  r2c_body<LOGN, LOGE, U8>(a, lid % a.n_chunks, lid / a.n_chunks);
}

// ----------------------------------------------------------------------------- inverse

// INTER: Y is read as interleaved complex a.Yc (chunked DM-factorised phasor sums), else as the
// planes a.Yr, a.Yi.
template <int LOGN, int LOGE, bool INTER>
__device__ __forceinline__ void c2r_body(const FftArgs& a, const int k, const int dm) {
  using F = BlockFft<LOGN, LOGE, true>;
  constexpr int N = F::N, E = F::E, T = F::T;
  constexpr int64_t L = 2 * (int64_t)N;
  __shared__ float lds[LdsSize<LOGN>::floats];
  const float* __restrict__ Yr = a.Yr;
  const float* __restrict__ Yi = a.Yi;
  float* __restrict__ out = a.out;
  const int64_t n_samp = a.n_samp, stride = a.stride, keep = a.keep, pitch = a.pitch;
  const int n_chunks = a.n_chunks;
  const float add_full = a.add_full;
  const int t = threadIdx.x;
  const int row_chunks = a.row_chunks > 0 ? a.row_chunks : n_chunks;   // chunks per row of Y
  const int64_t row = ((int64_t)dm * row_chunks + k) * pitch;
  const float* yr = Yr + row;
  const float* yi = Yi + row;
  const float2* yc = a.Yc + row;
  const float scale = a.inv_n > 0.0f ? a.inv_n : 1.0f / (float)N;
  const float2 w0 = F::half_bin_phasor_base();                 // exp(+2 pi i t / L)
  // Bins are read in groups of QG points, double-buffered: the loads of group g + 1 are in
  // flight while group g is split, so the reads are not serialised on memory latency.
  constexpr int QG = E < 8 ? E : 8;
  constexpr int NG = E / QG;
  float2 bf[2][QG], bm[2][QG];                                 // Y[f], Y[N - f]
  auto load_group = [&](auto gi) {
    constexpr int g = decltype(gi)::value;
    static_for<0, QG>([&](auto ui) {
      constexpr int u = decltype(ui)::value;
      const int f = t + T * (g * QG + u);
      const int fm = N - f;                                    // in 1 .. N
      if constexpr (INTER) {
        bf[g & 1][u] = yc[f];
        bm[g & 1][u] = yc[fm];
      } else {
        bf[g & 1][u] = make_float2(yr[f], yi[f]);
        bm[g & 1][u] = make_float2(yr[fm], yi[fm]);
      }
    });
  };
  float2 v[E];
  load_group(std::integral_constant<int, 0>{});
  static_for<0, NG>([&](auto gi) {
    constexpr int g = decltype(gi)::value;
    if constexpr (g + 1 < NG) load_group(std::integral_constant<int, g + 1>{});
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, QG>([&](auto ui) {
      constexpr int u = decltype(ui)::value;
      constexpr int q = g * QG + u;
      const int f = t + T * q;
      float2 yf = bf[g & 1][u];
      float2 ym = make_float2(bm[g & 1][u].x, -bm[g & 1][u].y);   // conj Y[N - f]
      if constexpr (q == 0) {                                  // only q = 0 holds f = 0 (thread 0)
        yf.y = f == 0 ? 0.0f : yf.y;
        ym.y = f == 0 ? 0.0f : ym.y;
      }
      const float2 a = make_float2(0.5f * (yf.x + ym.x), 0.5f * (yf.y + ym.y));
      const float2 d = make_float2(0.5f * (yf.x - ym.x), 0.5f * (yf.y - ym.y));
      const float2 b = cmulf(F::template half_bin_phasor<q>(w0), d);   // exp(+2 pi i f / L) d
      v[q] = make_float2((a.x - b.y) * scale, (a.y + b.x) * scale);   // A + i B
    });
    __builtin_amdgcn_sched_barrier(0);
  });
  F::run(v, lds);
  const int64_t s0 = (int64_t)k * stride;
  const bool full = a.full_chunks >= 0 ? k < a.full_chunks : s0 + L <= n_samp;
  const float add = full ? add_full : 0.0f;
  float* dst = out + (int64_t)dm * n_samp + s0;
  const int lim = (int)((keep < n_samp - s0) ? keep : n_samp - s0);   // <= L
  // Points q < qfull lie below lim for every thread (2 T (q + 1) <= lim); point qfull is cut
  // per sample; later points are all past it.  The tests on q are uniform.
  const int qfull = lim / (2 * T);
  const bool al = ((uintptr_t)dst & 7u) == 0;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int s = 2 * (t + T * q);
    const float2 o = make_float2(v[q].x + add, v[q].y + add);
    if (q < qfull) {
      if (al) {
        *reinterpret_cast<float2*>(dst + s) = o;
      } else {
        dst[s] = o.x;
        dst[s + 1] = o.y;
      }
    } else if (q == qfull) {
      if (s < lim) dst[s] = o.x;
      if (s + 1 < lim) dst[s + 1] = o.y;
    }
  }
}

template <int LOGN, int LOGE, bool INTER>
__global__ __launch_bounds__(1 << (LOGN - LOGE)) void k_c2r(FftArgs a) {
  c2r_body<LOGN, LOGE, INTER>(a, blockIdx.x, blockIdx.y);
}

template <int LOGN, int LOGE>
__global__ __launch_bounds__(1 << (LOGN - LOGE)) void k_c2r_grouped(Group<FftArgs> g) {
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (bid >= g.total) return;
  const int b = group_beam(g.prefix, g.n_beams, bid);
  const FftArgs a = g.beams[b];
  const int lid = bid - g.prefix[b];
  if (lid >= a.n_chunks * a.n_rows) return;
  c2r_body<LOGN, LOGE, false>(a, lid % a.n_chunks, lid / a.n_chunks);
}

// ----------------------------------------------------------------------------- long transforms
//
// Transforms longer than one workgroup can hold (N = L/2 > 2^15 complex points) run as a
// sequence of global-memory Stockham passes, one radix-R butterfly per thread: butterfly j of
// a series reads points j + r N/R (consecutive threads, consecutive addresses), applies the
// twiddles exp(-/+ 2 pi i r k / (Ns R)), k = j mod Ns, and writes to the autosort positions
// (j / Ns) Ns R + k + r Ns.  The first forward pass loads real samples directly (packing
// x[2j] + i x[2j+1], zero point and zero padding as in k_r2c); the last inverse pass stores
// real samples directly (scaling, valid-sample extraction and zero-point restore as in k_c2r).

enum { kPassComplex = 0, kPassLoadF32 = 1, kPassLoadU8 = 2, kPassStoreReal = 3 };

template <int LOGR, bool INV, int MODE>
__global__ __launch_bounds__(256) void k_fft_pass(LongPassArgs a) {
  constexpr int R = 1 << LOGR;
  const int64_t nb = (int64_t)1 << (a.log_n - LOGR);     // butterflies per series
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= nb) return;
  const int series = blockIdx.y;                          // (row, chunk) = (series / n_chunks, % n_chunks)
  const int64_t Ns = (int64_t)1 << a.log_ns;
  const int64_t k = j & (Ns - 1);
  float2 v[R];
  if constexpr (MODE == kPassLoadF32 || MODE == kPassLoadU8) {
    const int row = series / a.n_chunks, chunk = series % a.n_chunks;
    const int64_t s0 = (int64_t)chunk * a.stride;
    const int64_t L = (int64_t)2 << a.log_n;
    float zp = 0.0f;
    float l1 = 0.0f;
    if constexpr (MODE == kPassLoadU8) zp = (s0 + L <= a.n_samp) ? 128.0f : 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t s = s0 + 2 * (j + r * nb);
      float x0 = 0.0f, x1 = 0.0f;
      if constexpr (MODE == kPassLoadU8) {
        const uint8_t* src = a.in_u8 + (int64_t)row * a.n_samp;
        if (s < a.n_samp) x0 = (float)src[s] - zp;
        if (s + 1 < a.n_samp) x1 = (float)src[s + 1] - zp;
      } else {
        const float* src = a.in_f32 + (int64_t)row * a.n_samp;
        if (s < a.n_samp) x0 = src[s];
        if (s + 1 < a.n_samp) x1 = src[s + 1];
      }
      l1 += fabsf(x0) + fabsf(x1);
      v[r] = make_float2(x0, x1);
    }
    if (a.l1sum != nullptr) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) l1 += __shfl_xor(l1, o, 64);
      if ((threadIdx.x & 63) == 0) atomicAdd(a.l1sum + series, l1);
    }
  } else {
    const float2* src = a.in + (int64_t)series * a.in_pitch;
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
  }
  if (a.log_ns > 0) {
    // exp(-/+ 2 pi i r k / (Ns R)): angle r k / (Ns R) of a turn, exact in 32-bit fixed point
    const int sh = 32 - a.log_ns - LOGR;
    constexpr int G = R > 8 ? 8 : R;
    float2 lo[G];
#pragma unroll
    for (int vv = 1; vv < G; ++vv) lo[vv] = turn_phasor<INV>((uint32_t)(vv * k) << sh);
#pragma unroll
    for (int u = 0; u < R / G; ++u) {
      float2 hi = make_float2(1.0f, 0.0f);
      if (u > 0) hi = turn_phasor<INV>((uint32_t)(u * G * k) << sh);
#pragma unroll
      for (int vv = 0; vv < G; ++vv) {
        const int r = u * G + vv;
        if (r == 0) continue;
        const float2 w = vv == 0 ? hi : (u == 0 ? lo[vv] : cmul(hi, lo[vv]));
        v[r] = cmul(v[r], w);
      }
    }
  }
  dft_reg<R, INV>(v);
  const int64_t base = ((j >> a.log_ns) << (a.log_ns + LOGR)) + k;
  if constexpr (MODE == kPassStoreReal) {
    // point m holds samples 2m and 2m + 1 of the chunk
    const int row = series / a.n_chunks, chunk = series % a.n_chunks;
    const int64_t s0 = (int64_t)chunk * a.stride;
    const int64_t L = (int64_t)2 << a.log_n;
    const float add = (s0 + L <= a.n_samp) ? a.add_full : 0.0f;
    const int64_t lim = (a.keep < a.n_samp - s0) ? a.keep : a.n_samp - s0;
    float* dst = a.out_real + (int64_t)row * a.n_samp + s0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t m = base + r * Ns;
      if (2 * m < lim) dst[2 * m] = v[r].x + add;
      if (2 * m + 1 < lim) dst[2 * m + 1] = v[r].y + add;
    }
  } else {
    float2* dst = a.out + (int64_t)series * a.out_pitch;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
  }
}

// Real-to-complex split of a long series: X[f] for f = 0 .. N from Z[f] and Z[N - f].
__global__ __launch_bounds__(256) void k_r2c_split(LongPassArgs a) {
  const int64_t N = (int64_t)1 << a.log_n;
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f > N) return;
  const int series = blockIdx.y;
  const float2* z = a.in + (int64_t)series * a.in_pitch;
  float2* x = a.out + (int64_t)series * a.out_pitch;
  const float2 zf = z[f & (N - 1)];
  const float2 zm = z[(N - f) & (N - 1)];
  const float2 zc = make_float2(zm.x, -zm.y);
  const float2 av = make_float2(0.5f * (zf.x + zc.x), 0.5f * (zf.y + zc.y));
  const float2 d = make_float2(0.5f * (zf.x - zc.x), 0.5f * (zf.y - zc.y));
  const float2 b = make_float2(d.y, -d.x);                                  // -i d
  const float2 w = turn_phasor<false>((uint32_t)f << (31 - a.log_n));        // exp(-2 pi i f / L)
  x[f] = make_float2(av.x + fmaf(w.x, b.x, -w.y * b.y), av.y + fmaf(w.x, b.y, w.y * b.x));
}

// Complex-to-real pre-split of a long series: Z[f] = A + i B from the planes of Y, scaled 1/N.
__global__ __launch_bounds__(256) void k_c2r_split(LongPassArgs a) {
  const int64_t N = (int64_t)1 << a.log_n;
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= N) return;
  const int series = blockIdx.y;
  const float* yr = a.yr + (int64_t)series * a.in_pitch;
  const float* yi = a.yi + (int64_t)series * a.in_pitch;
  const int64_t fm = N - f;
  const float2 yf = make_float2(yr[f], f == 0 ? 0.0f : yi[f]);
  const float2 ym = make_float2(yr[fm], fm == N ? 0.0f : -yi[fm]);       // conj Y[N - f]
  const float2 av = make_float2(0.5f * (yf.x + ym.x), 0.5f * (yf.y + ym.y));
  const float2 d = make_float2(0.5f * (yf.x - ym.x), 0.5f * (yf.y - ym.y));
  const float2 w = turn_phasor<true>((uint32_t)f << (31 - a.log_n));         // exp(+2 pi i f / L)
  const float2 b = cmul(w, d);
  const float scale = ldexpf(1.0f, -a.log_n);
  a.out[(int64_t)series * a.out_pitch + f] = make_float2((av.x - b.y) * scale, (av.y + b.x) * scale);
}

__global__ void k_l1_max(const float* l1sum, int n_rows, int n_chunks, unsigned int* l1max) {
  // l1max[k] = max over rows of l1sum[row * n_chunks + k]; one thread per chunk
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_chunks) return;
  float m = 0.0f;
  for (int r = 0; r < n_rows; ++r) m = fmaxf(m, l1sum[(int64_t)r * n_chunks + k]);
  l1max[k] = __float_as_uint(m);
}

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

namespace {
constexpr int kLongLogR = 4;

template <bool INV, int MODE>
hipError_t launch_pass(int logr, LongPassArgs a, hipStream_t st) {
  const int64_t nb = (int64_t)1 << (a.log_n - logr);
  const dim3 grid((unsigned)((nb + 255) / 256), (unsigned)a.n_series);
  switch (logr) {
    case 1: hipLaunchKernelGGL((k_fft_pass<1, INV, MODE>), grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_fft_pass<2, INV, MODE>), grid, dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_fft_pass<3, INV, MODE>), grid, dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_fft_pass<4, INV, MODE>), grid, dim3(256), 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_fft_pass<5, INV, MODE>), grid, dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// radices of the passes: radix 16, the remainder (1..5 bits) folded into the last pass
void pass_radices(int log_n, int* logr, int* n) {
  *n = 0;
  int left = log_n;
  while (left > 0) {
    int r = left >= 2 * kLongLogR ? kLongLogR : (left > 5 ? left - kLongLogR : left);
    logr[(*n)++] = r;
    left -= r;
  }
}
}  // namespace

// Forward real transform of every (row, chunk) series of length L = 2^(log_n + 1) into
// X [series][pitch] (bins 0 .. N); `work` holds one series-sized complex buffer per series.
hipError_t launch_r2c_long(const FftArgs& f, float2* work, float* l1sum, hipStream_t st) {
  LongPassArgs a;
  a.log_n = f.log_n;
  a.n_series = f.n_rows * f.n_chunks;
  a.n_chunks = f.n_chunks;
  a.stride = f.stride;
  a.n_samp = f.n_samp;
  a.in_u8 = f.in_u8;
  a.in_f32 = f.in_f32;
  int logr[16], np = 0;
  pass_radices(a.log_n, logr, &np);
  // ping-pong: the last pass must land in `work` so the split can write X
  float2* bufs[2] = {work, f.X};
  int cur = (np % 2 == 1) ? 0 : 1;          // buffer receiving pass 0's output
  hipError_t e = hipSuccess;
  if (f.l1max != nullptr) {
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((a.n_series + 255) / 256)), dim3(256), 0, st, l1sum,
                       (int64_t)a.n_series);
    a.l1sum = l1sum;
  }
  int log_ns = 0;
  for (int p = 0; p < np; ++p) {
    a.log_ns = log_ns;
    a.out = bufs[cur];
    a.out_pitch = cur == 0 ? ((int64_t)1 << a.log_n) : f.pitch;
    if (p == 0) {
      e = f.in_u8 != nullptr ? launch_pass<false, kPassLoadU8>(logr[p], a, st)
                             : launch_pass<false, kPassLoadF32>(logr[p], a, st);
      a.l1sum = nullptr;
    } else {
      e = launch_pass<false, kPassComplex>(logr[p], a, st);
    }
    if (e != hipSuccess) return e;
    a.in = bufs[cur];
    a.in_pitch = a.out_pitch;
    cur ^= 1;
    log_ns += logr[p];
  }
  if (f.l1max != nullptr)
    hipLaunchKernelGGL(k_l1_max, dim3((unsigned)((f.n_chunks + 63) / 64)), dim3(64), 0, st, l1sum, f.n_rows,
                       f.n_chunks, f.l1max);
  // final result is in work (pitch N); split into X
  a.in = work;
  a.in_pitch = (int64_t)1 << a.log_n;
  a.out = f.X;
  a.out_pitch = f.pitch;
  const int64_t nbins = ((int64_t)1 << a.log_n) + 1;
  hipLaunchKernelGGL(k_r2c_split, dim3((unsigned)((nbins + 255) / 256), (unsigned)a.n_series), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Inverse real transform of every (DM, chunk) series from the Y planes to the output.
hipError_t launch_c2r_long(const FftArgs& f, float2* work, float2* work2, hipStream_t st) {
  LongPassArgs a;
  a.log_n = f.log_n;
  a.n_series = f.n_rows * f.n_chunks;
  a.n_chunks = f.n_chunks;
  a.stride = f.stride;
  a.n_samp = f.n_samp;
  a.keep = f.keep;
  a.add_full = f.add_full;
  a.out_real = f.out;
  a.yr = f.Yr;
  a.yi = f.Yi;
  a.in_pitch = f.pitch;
  a.out = work;
  a.out_pitch = (int64_t)1 << a.log_n;
  const int64_t N = (int64_t)1 << a.log_n;
  hipLaunchKernelGGL(k_c2r_split, dim3((unsigned)((N + 255) / 256), (unsigned)a.n_series), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int logr[16], np = 0;
  pass_radices(a.log_n, logr, &np);
  float2* bufs[2] = {work, work2};
  int cur = 0;
  int log_ns = 0;
  for (int p = 0; p < np; ++p) {
    a.log_ns = log_ns;
    a.in = bufs[cur];
    a.in_pitch = N;
    a.out = bufs[cur ^ 1];
    a.out_pitch = N;
    e = (p == np - 1) ? launch_pass<true, kPassStoreReal>(logr[p], a, st)
                      : launch_pass<true, kPassComplex>(logr[p], a, st);
    if (e != hipSuccess) return e;
    cur ^= 1;
    log_ns += logr[p];
  }
  return hipSuccess;
}

// ----------------------------------------------------------------------------- launchers

namespace {
template <int LOGN>
constexpr int fft_loge() {
  return LOGN >= 15 ? 5 : (LOGN >= 12 ? 4 : 3);
}
// The inverse of 2^15 points spills less with 64 points in each of 512 threads (measured
// 8.61 -> 7.95 ms on 2048 x 21 series); the forward transform, which also unpacks and sums
// L1 norms, is faster with 32 points in each of 1024 threads.
template <int LOGN>
constexpr int fft_loge_inv() {
  return LOGN >= 15 ? 6 : fft_loge<LOGN>();
}

template <int LOGN>
hipError_t launch_r2c_n(const FftArgs& a, hipStream_t st) {
  constexpr int LOGE = fft_loge<LOGN>();
  dim3 grid((unsigned)a.n_chunks, (unsigned)a.n_rows);
  if (a.l1max != nullptr) {
    hipLaunchKernelGGL(k_zero_u32, dim3((a.n_chunks + 255) / 256), dim3(256), 0, st, a.l1max, a.n_chunks);
  }
  if (a.in_u8 != nullptr)
    hipLaunchKernelGGL((k_r2c<LOGN, LOGE, true>), grid, dim3(1 << (LOGN - LOGE)), 0, st, a);
  else
    hipLaunchKernelGGL((k_r2c<LOGN, LOGE, false>), grid, dim3(1 << (LOGN - LOGE)), 0, st, a);
  return hipGetLastError();
}

template <int LOGN>
hipError_t launch_r2c_grouped_n(bool u8, const Group<FftArgs>& g, hipStream_t st) {
  constexpr int LOGE = fft_loge<LOGN>();
  const dim3 grid = linear_grid(g.total);
  if (u8)
    hipLaunchKernelGGL((k_r2c_grouped<LOGN, LOGE, true>), grid, dim3(1 << (LOGN - LOGE)), 0, st, g);
  else
    hipLaunchKernelGGL((k_r2c_grouped<LOGN, LOGE, false>), grid, dim3(1 << (LOGN - LOGE)), 0, st, g);
  return hipGetLastError();
}

template <int LOGN>
hipError_t launch_c2r_grouped_n(const Group<FftArgs>& g, hipStream_t st) {
  constexpr int LOGE = fft_loge_inv<LOGN>();
  hipLaunchKernelGGL((k_c2r_grouped<LOGN, LOGE>), linear_grid(g.total), dim3(1 << (LOGN - LOGE)), 0, st, g);
  return hipGetLastError();
}

template <int LOGN>
hipError_t launch_c2r_n(const FftArgs& a, hipStream_t st) {
  constexpr int LOGE = fft_loge_inv<LOGN>();
  dim3 grid((unsigned)a.n_chunks, (unsigned)a.n_rows);
  if (a.Yc != nullptr)
    hipLaunchKernelGGL((k_c2r<LOGN, LOGE, true>), grid, dim3(1 << (LOGN - LOGE)), 0, st, a);
  else
    hipLaunchKernelGGL((k_c2r<LOGN, LOGE, false>), grid, dim3(1 << (LOGN - LOGE)), 0, st, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_zero_u32(unsigned int* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, (int)n);
  return hipGetLastError();
}

hipError_t launch_transpose_u8(const uint8_t* in, uint8_t* out, int64_t n_samp, int n_chan, hipStream_t st) {
  dim3 grid((unsigned)((n_samp + 63) / 64), (unsigned)((n_chan + 63) / 64));
  const bool words = n_samp % 64 == 0 && n_chan % 64 == 0 && ((uintptr_t)in & 3u) == 0 && ((uintptr_t)out & 3u) == 0;
  if (words)
    hipLaunchKernelGGL(k_transpose_u8_w, grid, dim3(256), 0, st, (const uint32_t*)in, (uint32_t*)out, n_samp, n_chan);
  else
    hipLaunchKernelGGL(k_transpose_u8, grid, dim3(256), 0, st, in, out, n_samp, n_chan);
  return hipGetLastError();
}

hipError_t launch_r2c(int log_n, const FftArgs& a, hipStream_t st) {
  switch (log_n) {
    case 5: return launch_r2c_n<5>(a, st);
    case 6: return launch_r2c_n<6>(a, st);
    case 7: return launch_r2c_n<7>(a, st);
    case 8: return launch_r2c_n<8>(a, st);
    case 9: return launch_r2c_n<9>(a, st);
    case 10: return launch_r2c_n<10>(a, st);
    case 11: return launch_r2c_n<11>(a, st);
    case 12: return launch_r2c_n<12>(a, st);
    case 13: return launch_r2c_n<13>(a, st);
    case 14: return launch_r2c_n<14>(a, st);
    case 15: return launch_r2c_n<15>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r(int log_n, const FftArgs& a, hipStream_t st) {
  switch (log_n) {
    case 5: return launch_c2r_n<5>(a, st);
    case 6: return launch_c2r_n<6>(a, st);
    case 7: return launch_c2r_n<7>(a, st);
    case 8: return launch_c2r_n<8>(a, st);
    case 9: return launch_c2r_n<9>(a, st);
    case 10: return launch_c2r_n<10>(a, st);
    case 11: return launch_c2r_n<11>(a, st);
    case 12: return launch_c2r_n<12>(a, st);
    case 13: return launch_c2r_n<13>(a, st);
    case 14: return launch_c2r_n<14>(a, st);
    case 15: return launch_c2r_n<15>(a, st);
    default: return hipErrorInvalidValue;
  }
}

int64_t fft_grouped_tiles(const FftArgs& a) { return (int64_t)a.n_chunks * a.n_rows; }

hipError_t launch_r2c_grouped(int log_n, bool u8, const Group<FftArgs>& g, hipStream_t st) {
  if (g.total <= 0) return hipSuccess;
  switch (log_n) {
    case 5: return launch_r2c_grouped_n<5>(u8, g, st);
    case 6: return launch_r2c_grouped_n<6>(u8, g, st);
    case 7: return launch_r2c_grouped_n<7>(u8, g, st);
    case 8: return launch_r2c_grouped_n<8>(u8, g, st);
    case 9: return launch_r2c_grouped_n<9>(u8, g, st);
    case 10: return launch_r2c_grouped_n<10>(u8, g, st);
    case 11: return launch_r2c_grouped_n<11>(u8, g, st);
    case 12: return launch_r2c_grouped_n<12>(u8, g, st);
    case 13: return launch_r2c_grouped_n<13>(u8, g, st);
    case 14: return launch_r2c_grouped_n<14>(u8, g, st);
    case 15: return launch_r2c_grouped_n<15>(u8, g, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r_grouped(int log_n, const Group<FftArgs>& g, hipStream_t st) {
  if (g.total <= 0) return hipSuccess;
  switch (log_n) {
    case 5: return launch_c2r_grouped_n<5>(g, st);
    case 6: return launch_c2r_grouped_n<6>(g, st);
    case 7: return launch_c2r_grouped_n<7>(g, st);
    case 8: return launch_c2r_grouped_n<8>(g, st);
    case 9: return launch_c2r_grouped_n<9>(g, st);
    case 10: return launch_c2r_grouped_n<10>(g, st);
    case 11: return launch_c2r_grouped_n<11>(g, st);
    case 12: return launch_c2r_grouped_n<12>(g, st);
    case 13: return launch_c2r_grouped_n<13>(g, st);
    case 14: return launch_c2r_grouped_n<14>(g, st);
    case 15: return launch_c2r_grouped_n<15>(g, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdd
