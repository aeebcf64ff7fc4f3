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
__global__ __launch_bounds__(1 << (LOGN - LOGE)) void k_r2c(
    const uint8_t* __restrict__ in_u8,   // [n_chan][n_samp] (transposed) or null
    const float* __restrict__ in_f32,    // [n_chan][n_samp] or null
    float2* __restrict__ X,              // [n_chan][n_chunks][pitch]
    const float2* __restrict__ twL,      // exp(-2 pi i j / L), j < L
    int64_t n_samp, int64_t stride, int64_t pitch, int n_chunks,
    unsigned int* __restrict__ l1max) {  // per chunk: max over channels of sum |x| (float bits), or null
  using F = BlockFft<LOGN, LOGE, false>;
  constexpr int N = F::N, E = F::E, T = F::T;
  constexpr int64_t L = 2 * (int64_t)N;
  __shared__ float lds[LdsSize<LOGN>::floats];
  const int t = threadIdx.x;
  const int k = blockIdx.x;
  const int c = blockIdx.y;
  const int64_t s0 = (int64_t)k * stride;
  const float zp = (U8 && s0 + L <= n_samp) ? 128.0f : 0.0f;
  float2 v[E];
  if constexpr (U8) {
    const uint8_t* src = in_u8 + (int64_t)c * n_samp;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t s = s0 + 2 * (int64_t)(t + T * q);
      v[q].x = s < n_samp ? (float)src[s] - zp : 0.0f;
      v[q].y = s + 1 < n_samp ? (float)src[s + 1] - zp : 0.0f;
    }
  } else {
    const float* src = in_f32 + (int64_t)c * n_samp;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t s = s0 + 2 * (int64_t)(t + T * q);
      v[q].x = s < n_samp ? src[s] : 0.0f;
      v[q].y = s + 1 < n_samp ? src[s + 1] : 0.0f;
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
  float2* dst = X + ((int64_t)c * n_chunks + k) * pitch;
  F::with_mirror(v, lds, [&](int q, float2 zf, float2 zm) {
    const int f = t + T * q;
    const float2 zc = make_float2(zm.x, -zm.y);                // conj Z[N - f]
    const float2 a = make_float2(0.5f * (zf.x + zc.x), 0.5f * (zf.y + zc.y));
    const float2 d = make_float2(0.5f * (zf.x - zc.x), 0.5f * (zf.y - zc.y));
    const float2 b = make_float2(d.y, -d.x);                   // -i d
    const float2 w = twL[f];                                   // exp(-2 pi i f / L)
    dst[f] = make_float2(a.x + fmaf(w.x, b.x, -w.y * b.y), a.y + fmaf(w.x, b.y, w.y * b.x));
  });
  if (t == 0) dst[N] = make_float2(v[0].x - v[0].y, 0.0f);   // Nyquist bin
}

// ----------------------------------------------------------------------------- inverse

template <int LOGN, int LOGE>
__global__ __launch_bounds__(1 << (LOGN - LOGE)) void k_c2r(
    const float* __restrict__ Yr, const float* __restrict__ Yi,   // [n_dm][n_chunks][pitch] planes
    float* __restrict__ out,                                      // [n_dm][n_samp]
    const float2* __restrict__ twL, int64_t n_samp, int64_t stride, int64_t keep, int64_t pitch,
    int n_chunks, float add_full) {
  using F = BlockFft<LOGN, LOGE, true>;
  constexpr int N = F::N, E = F::E, T = F::T;
  constexpr int64_t L = 2 * (int64_t)N;
  __shared__ float lds[LdsSize<LOGN>::floats];
  const int t = threadIdx.x;
  const int k = blockIdx.x;
  const int dm = blockIdx.y;
  const int64_t row = ((int64_t)dm * n_chunks + k) * pitch;
  const float* yr = Yr + row;
  const float* yi = Yi + row;
  const float scale = 1.0f / (float)N;
  float2 v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int f = t + T * q;
    const int fm = N - f;                                      // in 1 .. N
    const float2 yf = make_float2(yr[f], f == 0 ? 0.0f : yi[f]);
    const float2 ym = make_float2(yr[fm], fm == N ? 0.0f : -yi[fm]);   // conj Y[N - f]
    const float2 a = make_float2(0.5f * (yf.x + ym.x), 0.5f * (yf.y + ym.y));
    const float2 d = make_float2(0.5f * (yf.x - ym.x), 0.5f * (yf.y - ym.y));
    const float2 w = twL[f];                                   // exp(-2 pi i f / L); use conj
    const float2 b = make_float2(fmaf(w.x, d.x, w.y * d.y), fmaf(w.x, d.y, -w.y * d.x));
    v[q] = make_float2((a.x - b.y) * scale, (a.y + b.x) * scale);   // A + i B
    if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);      // bound loads in flight
  }
  F::run(v, lds);
  const int64_t s0 = (int64_t)k * stride;
  const float add = (s0 + L <= n_samp) ? add_full : 0.0f;
  float* dst = out + (int64_t)dm * n_samp + s0;
  const int64_t lim = (keep < n_samp - s0) ? keep : n_samp - s0;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int64_t s = 2 * (int64_t)(t + T * q);
    if (s < lim) dst[s] = v[q].x + add;
    if (s + 1 < lim) dst[s + 1] = v[q].y + add;
  }
}

// ----------------------------------------------------------------------------- launchers

namespace {
template <int LOGN>
constexpr int fft_loge() {
  return LOGN >= 15 ? 5 : (LOGN >= 12 ? 4 : 3);
}

template <int LOGN>
hipError_t launch_r2c_n(const FftArgs& a, hipStream_t st) {
  constexpr int LOGE = fft_loge<LOGN>();
  dim3 grid((unsigned)a.n_chunks, (unsigned)a.n_rows);
  if (a.l1max != nullptr) {
    hipLaunchKernelGGL(k_zero_u32, dim3((a.n_chunks + 255) / 256), dim3(256), 0, st, a.l1max, a.n_chunks);
  }
  if (a.in_u8 != nullptr)
    hipLaunchKernelGGL((k_r2c<LOGN, LOGE, true>), grid, dim3(1 << (LOGN - LOGE)), 0, st, a.in_u8, a.in_f32, a.X,
                       a.twL, a.n_samp, a.stride, a.pitch, a.n_chunks, a.l1max);
  else
    hipLaunchKernelGGL((k_r2c<LOGN, LOGE, false>), grid, dim3(1 << (LOGN - LOGE)), 0, st, a.in_u8, a.in_f32, a.X,
                       a.twL, a.n_samp, a.stride, a.pitch, a.n_chunks, a.l1max);
  return hipGetLastError();
}

template <int LOGN>
hipError_t launch_c2r_n(const FftArgs& a, hipStream_t st) {
  constexpr int LOGE = fft_loge<LOGN>();
  dim3 grid((unsigned)a.n_chunks, (unsigned)a.n_rows);
  hipLaunchKernelGGL((k_c2r<LOGN, LOGE>), grid, dim3(1 << (LOGN - LOGE)), 0, st, a.Yr, a.Yi, a.out, a.twL,
                     a.n_samp, a.stride, a.keep, a.pitch, a.n_chunks, a.add_full);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_transpose_u8(const uint8_t* in, uint8_t* out, int64_t n_samp, int n_chan, hipStream_t st) {
  dim3 grid((unsigned)((n_samp + 63) / 64), (unsigned)((n_chan + 63) / 64));
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

}  // namespace fdd
