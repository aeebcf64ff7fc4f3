// Brute-force time-domain dedispersion (Eq. 2) on the vector ALUs, the method the paper
// measures FDD against (Secs. 2.1 and 4.1), with the plan's nearest-sample delays:
//
//     y[dm, t] = sum_c x~[c, t + d[dm, c]],   d = floor(tau + 1/2),
//
// x~ being the input extended by zeros beyond n_samp, or, for single-chunk plans, zero-padded
// to L and periodic with period L (the circular convention of the single-chunk FDD).
//
// A workgroup owns DT = 8 trial DMs and TS consecutive output samples.  Per stage of KC
// channels it copies, for each channel, the input window [t0 + dmin, t0 + TS + dmax) of its DM
// tile into LDS, then each thread adds, for each of its 8 DMs, its samples at that DM's offset
// in the window.  Lane l owns the 4-sample groups (8-bit) or samples (float) l, l + 256, ...,
// so the lanes of a wave read consecutive LDS words (no bank conflicts) and the shift within a
// word is the same for the whole wave.  8-bit samples are added as packed 16-bit integers (a
// byte permute splits 4 samples into two 16-bit pairs; packed u16 adds), flushed into 32-bit
// integer sums every 256 channels (256 * 255 < 2^16), so 8-bit results are exact integer sums.
// Float input is summed in float32 in channel order.
#include "fdd_internal.h"

namespace fdd {

namespace {
constexpr int kDt = 8;          // DMs per workgroup

typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));

// Largest delay spread over the 8 DMs of a tile (per channel) that the windows hold: 504
// samples for fine DM grids; coarse grids take the WIDE shape with fewer channels per stage.
template <bool U8, bool WIDE>
struct TddShape {
  static constexpr int SPAN = WIDE ? 4088 : 504;
  static constexpr int TS = U8 ? 2048 : 1024;
  static constexpr int SPT = U8 ? 8 : 4;
  static constexpr int KC = U8 ? (WIDE ? 4 : 16) : (WIDE ? 2 : 8);
  static constexpr int WINW = U8 ? (TS + SPAN + 16) / 4 : TS + SPAN + 8;   // dwords (4 samples) or floats
};
}  // namespace

template <bool U8, bool WIDE>
__global__ __launch_bounds__(256) void k_tdd(TddArgs a) {
  using S = TddShape<U8, WIDE>;
  constexpr int TS = S::TS, SPT = S::SPT, KC = S::KC, WINW = S::WINW;
  __shared__ uint32_t win[KC * WINW];
  __shared__ int dl[KC][kDt];        // offset of each DM's samples in its channel's window
  __shared__ int sbase[KC];          // window start relative to t0 (a multiple of 4 for 8-bit data)

  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * TS;
  const int dm0 = blockIdx.y * kDt;
  const int64_t n = a.n_samp;
  const int64_t period = a.period;   // 0: zero extension
  const bool dword_rows = (n & 3) == 0;

  uint32_t acc16[U8 ? kDt : 1][U8 ? SPT / 2 : 1];   // 8-bit: packed u16 sums, per group (s0, s2) and (s1, s3)
  uint32_t acc32[U8 ? kDt : 1][U8 ? SPT : 1];
  float accf[U8 ? 1 : kDt][U8 ? 1 : SPT];
#pragma unroll
  for (int j = 0; j < kDt; ++j) {
    if constexpr (U8) {
#pragma unroll
      for (int s = 0; s < SPT / 2; ++s) acc16[j][s] = 0u;
#pragma unroll
      for (int s = 0; s < SPT; ++s) acc32[j][s] = 0u;
    } else {
#pragma unroll
      for (int s = 0; s < SPT; ++s) accf[j][s] = 0.0f;
    }
  }

  for (int cb = 0; cb < a.n_chan; cb += KC) {
    const int nc = a.n_chan - cb < KC ? a.n_chan - cb : KC;
    __syncthreads();                                 // the previous stage's windows are consumed
    if (tid < nc) {
      const int* drow = a.dtab + (int64_t)(cb + tid) * a.n_dm;
      int dmin = 0x7fffffff, d[kDt];
#pragma unroll
      for (int j = 0; j < kDt; ++j) {
        const int dm = dm0 + j < a.n_dm ? dm0 + j : a.n_dm - 1;
        d[j] = drow[dm];
        dmin = d[j] < dmin ? d[j] : dmin;
      }
      const int sb = U8 ? (dmin & ~3) : dmin;        // t0 is a multiple of 4
      sbase[tid] = sb;
#pragma unroll
      for (int j = 0; j < kDt; ++j) dl[tid][j] = d[j] - sb;
    }
    __syncthreads();
    for (int i = tid; i < nc * WINW; i += 256) {
      const int cl = i / WINW;
      const int w = i - cl * WINW;
      const uint8_t* row8 = a.in_u8 + (int64_t)(cb + cl) * n;
      const float* rowf = a.in_f32 + (int64_t)(cb + cl) * n;
      if constexpr (U8) {
        const int64_t p = t0 + sbase[cl] + 4 * (int64_t)w;         // multiple of 4
        const int64_t q = period ? p & (period - 1) : p;            // period: a power of two >= 64
        uint32_t v = 0u;
        if (dword_rows && q + 4 <= n) {
          v = *(const uint32_t*)(row8 + q);
        } else {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int64_t qb = period ? (p + b) & (period - 1) : p + b;
            if (qb < n) v |= (uint32_t)row8[qb] << (8 * b);
          }
        }
        win[cl * WINW + w] = v;
      } else {
        const int64_t p = t0 + sbase[cl] + w;
        const int64_t q = period ? p & (period - 1) : p;
        win[cl * WINW + w] = __float_as_uint(q < n ? rowf[q] : 0.0f);
      }
    }
    __syncthreads();
    for (int cl = 0; cl < nc; ++cl) {
      const uint32_t* wc = win + cl * WINW;
      int rels[kDt];
#pragma unroll
      for (int j = 0; j < kDt; ++j) rels[j] = __builtin_amdgcn_readfirstlane(dl[cl][j]);   // offset of DM j in the window
      if constexpr (U8) {
        // all window words of the channel first, then the arithmetic: the loads overlap
        uint32_t w0[kDt][SPT / 4], w1[kDt][SPT / 4];
#pragma unroll
        for (int j = 0; j < kDt; ++j)
#pragma unroll
          for (int g = 0; g < SPT / 4; ++g) {
            const int wi = tid + 256 * g + (rels[j] >> 2);
            w0[j][g] = wc[wi];
            w1[j][g] = wc[wi + 1];
          }
#pragma unroll
        for (int j = 0; j < kDt; ++j) {
          const uint32_t sh = (uint32_t)(rels[j] & 3);
#pragma unroll
          for (int g = 0; g < SPT / 4; ++g) {
            const uint32_t v = __builtin_amdgcn_alignbyte(w1[j][g], w0[j][g], sh);   // 4 samples
            const uint32_t pe = __builtin_amdgcn_perm(0u, v, 0x0c020c00u);            // (s0, s2)
            const uint32_t po = __builtin_amdgcn_perm(0u, v, 0x0c030c01u);            // (s1, s3)
            acc16[j][2 * g] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(ushort2v, acc16[j][2 * g]) +
                                                               __builtin_bit_cast(ushort2v, pe));
            acc16[j][2 * g + 1] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(ushort2v, acc16[j][2 * g + 1]) +
                                                                   __builtin_bit_cast(ushort2v, po));
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < kDt; ++j)
#pragma unroll
          for (int s = 0; s < SPT; ++s) accf[j][s] += __uint_as_float(wc[tid + 256 * s + rels[j]]);
      }
    }
    if constexpr (U8) {
      if (((cb + KC) & 255) == 0 || cb + KC >= a.n_chan) {         // at most 256 channels per u16 sum
#pragma unroll
        for (int j = 0; j < kDt; ++j) {
#pragma unroll
          for (int g = 0; g < SPT / 4; ++g) {
            acc32[j][4 * g + 0] += acc16[j][2 * g] & 0xffffu;
            acc32[j][4 * g + 2] += acc16[j][2 * g] >> 16;
            acc32[j][4 * g + 1] += acc16[j][2 * g + 1] & 0xffffu;
            acc32[j][4 * g + 3] += acc16[j][2 * g + 1] >> 16;
            acc16[j][2 * g] = 0u;
            acc16[j][2 * g + 1] = 0u;
          }
        }
      }
    }
  }

#pragma unroll
  for (int j = 0; j < kDt; ++j) {
    const int dm = dm0 + j;
    if (dm >= a.n_dm) continue;
    float* row = a.out + (int64_t)dm * n;
    if constexpr (U8) {
#pragma unroll
      for (int g = 0; g < SPT / 4; ++g) {
        const int64_t t = t0 + 4 * (tid + 256 * g);
        const float4 v = make_float4((float)acc32[j][4 * g], (float)acc32[j][4 * g + 1], (float)acc32[j][4 * g + 2],
                                     (float)acc32[j][4 * g + 3]);
        if (dword_rows && t + 4 <= n) {
          *(float4*)(row + t) = v;
        } else {
          if (t < n) row[t] = v.x;
          if (t + 1 < n) row[t + 1] = v.y;
          if (t + 2 < n) row[t + 2] = v.z;
          if (t + 3 < n) row[t + 3] = v.w;
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < SPT; ++s) {
        const int64_t t = t0 + tid + 256 * s;
        if (t < n) row[t] = accf[j][s];
      }
    }
  }
}

// ------------------------------------------------------------------------------- 8-bit, 32 DMs
//
// For fine DM grids one workgroup takes 32 DMs x 1024 samples, so every staged input byte
// serves 32 DMs instead of 8 (the input windows are otherwise re-read from the caches once per
// DM tile).  The window is stored four times, shifted by 0..3 bytes, so that a lane's 4
// samples at any offset are one aligned LDS word.  Sums stay in packed 16-bit registers and
// are added to the output in global memory every 256 channels (exact: integer partial sums
// below 2^24 in float32).
namespace {
constexpr int kDt64 = 32, kTs64 = 1024, kKc64 = 4, kSpan64 = 1016;
constexpr int kWin64 = (kTs64 + kSpan64 + 8) / 4;   // words per shifted copy
}  // namespace

__global__ __launch_bounds__(256) void k_tdd_u8_fine(TddArgs a) {
  __shared__ uint32_t win[kKc64][4][kWin64];
  __shared__ int rel[kKc64][kDt64];     // delays of the stage's channels for the tile's DMs
  __shared__ int sbase[kKc64];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kTs64;
  const int dm0 = blockIdx.y * kDt64;
  const int64_t n = a.n_samp;
  const int64_t period = a.period;
  const bool dword_rows = (n & 3) == 0;
  const int64_t t = t0 + 4 * tid;

  uint32_t acc[kDt64][2];               // packed u16 sums of samples (0, 2) and (1, 3)
#pragma unroll
  for (int j = 0; j < kDt64; ++j) acc[j][0] = acc[j][1] = 0u;

  for (int cb = 0; cb < a.n_chan; cb += kKc64) {
    const int nc = a.n_chan - cb < kKc64 ? a.n_chan - cb : kKc64;
    __syncthreads();
    if (tid < nc * kDt64) {                          // delays of the stage's channels and the tile's DMs
      const int cl = tid / kDt64, j = tid - (tid / kDt64) * kDt64;
      const int dm = dm0 + j < a.n_dm ? dm0 + j : a.n_dm - 1;
      rel[cl][j] = a.dtab[(int64_t)(cb + cl) * a.n_dm + dm];
    }
    __syncthreads();
    if (tid < nc) {
      int dmin = 0x7fffffff;
      for (int j = 0; j < kDt64; ++j) dmin = rel[tid][j] < dmin ? rel[tid][j] : dmin;
      sbase[tid] = dmin & ~3;
    }
    __syncthreads();
    for (int i = tid; i < nc * kWin64; i += 256) {
      const int cl = i / kWin64;
      const int w = i - cl * kWin64;
      const uint8_t* row = a.in_u8 + (int64_t)(cb + cl) * n;
      uint32_t v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t p = t0 + sbase[cl] + 4 * (int64_t)(w + h);
        const int64_t q = period ? p & (period - 1) : p;
        uint32_t x = 0u;
        if (dword_rows && q + 4 <= n) {
          x = *(const uint32_t*)(row + q);
        } else {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int64_t qb = period ? (p + b) & (period - 1) : p + b;
            if (qb < n) x |= (uint32_t)row[qb] << (8 * b);
          }
        }
        v[h] = x;
      }
      win[cl][0][w] = v[0];
      win[cl][1][w] = __builtin_amdgcn_alignbyte(v[1], v[0], 1u);
      win[cl][2][w] = __builtin_amdgcn_alignbyte(v[1], v[0], 2u);
      win[cl][3][w] = __builtin_amdgcn_alignbyte(v[1], v[0], 3u);
    }
    __syncthreads();
#pragma unroll 1
    for (int cl = 0; cl < nc; ++cl) {
      const int sb = __builtin_amdgcn_readfirstlane(sbase[cl]);
#pragma unroll
      for (int j = 0; j < kDt64; ++j) {
        const int r = __builtin_amdgcn_readfirstlane(rel[cl][j]) - sb;   // offset of DM j in the window
        const uint32_t v = win[cl][r & 3][tid + (r >> 2)];            // samples t .. t + 3
        const uint32_t pe = __builtin_amdgcn_perm(0u, v, 0x0c020c00u);   // (s0, s2)
        const uint32_t po = __builtin_amdgcn_perm(0u, v, 0x0c030c01u);   // (s1, s3)
        acc[j][0] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(ushort2v, acc[j][0]) + __builtin_bit_cast(ushort2v, pe));
        acc[j][1] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(ushort2v, acc[j][1]) + __builtin_bit_cast(ushort2v, po));
      }
    }
    const bool last = cb + kKc64 >= a.n_chan;
    if (((cb + kKc64) & 255) == 0 || last) {         // at most 256 channels per 16-bit sum
      const bool first = cb + kKc64 <= 256;
#pragma unroll
      for (int j = 0; j < kDt64; ++j) {
        const int dm = dm0 + j;
        const float4 s4 = make_float4((float)(acc[j][0] & 0xffffu), (float)(acc[j][1] & 0xffffu),
                                      (float)(acc[j][0] >> 16), (float)(acc[j][1] >> 16));
        acc[j][0] = acc[j][1] = 0u;
        if (dm >= a.n_dm) continue;
        float* dst = a.out + (int64_t)dm * n + t;
        if (dword_rows && t + 4 <= n) {
          float4 o = s4;
          if (!first) {
            const float4 prev = *(const float4*)dst;
            o = make_float4(prev.x + s4.x, prev.y + s4.y, prev.z + s4.z, prev.w + s4.w);
          }
          *(float4*)dst = o;
        } else {
          const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2)
            if (t + s2 < n) dst[s2] = first ? sv[s2] : dst[s2] + sv[s2];
        }
      }
    }
  }
}

int tdd_span_max() { return TddShape<true, true>::SPAN; }
int tdd_span64_max() { return kSpan64; }
int tdd_tile64() { return kDt64; }
int tdd_dm_tile() { return kDt; }

hipError_t launch_tdd(const TddArgs& a, int span, int span64, hipStream_t st) {
  const bool u8 = a.in_u8 != nullptr;
  if (u8 && span64 <= kSpan64) {
    const int64_t gx = (a.n_samp + kTs64 - 1) / kTs64;
    const int gy = (a.n_dm + kDt64 - 1) / kDt64;
    if (gx > 0x7fffffff || gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tdd_u8_fine, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, a);
    return hipGetLastError();
  }
  const bool wide = span > TddShape<true, false>::SPAN;
  if (span > TddShape<true, true>::SPAN) return hipErrorInvalidValue;
  const int ts = u8 ? TddShape<true, false>::TS : TddShape<false, false>::TS;
  const int64_t gx = (a.n_samp + ts - 1) / ts;
  const int gy = (a.n_dm + kDt - 1) / kDt;
  if (gx > 0x7fffffff || gy > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)gx, (unsigned)gy), block(256);
  if (u8) {
    if (wide) hipLaunchKernelGGL((k_tdd<true, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_tdd<true, false>), grid, block, 0, st, a);
  } else {
    if (wide) hipLaunchKernelGGL((k_tdd<false, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_tdd<false, false>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace fdd
