// Phasor sum on the half-precision matrix cores with split operands (precision form).
//
// Same contraction as the FP32 kernel (Eqs. 4 and 7, chunks batched per bin):
//     [Yr | Yi] = sum_c ( Wr [Xr | Xi] + Wi [-Xi | Xr] )
// written here as one real GEMM whose contraction index runs over (channel, cos/sin part):
// A[dm][2c + p] = (Wr, Wi)[p],  B[2c + p][n] = (cos operand, sin operand)[p] of column n.
// Both operands are split into a half-precision head and tail, v = hi + lo with
// hi = half(v) and lo = half(v - hi), and the product is accumulated in float32 as
//     A_hi B_hi + A_hi B_lo + A_lo B_hi      (A_lo B_lo, ~2^-22 relative, is dropped).
// FP16 has a small range, so every data column (chunk k) carries a power-of-two scale
// 2^(14 - ceil(log2 L1_k)), where L1_k is the largest L1 norm of chunk k's input series over
// the channels: |X| <= L1 keeps every scaled value below 2^14.  The scale is exact and is
// divided out in the epilogue.  BF16 needs no scale but uses it all the same.
//
// gfx950 v_mfma_f32_16x16x32_{f16,bf16}: lane l holds A[l % 16][8 (l / 16) .. +7] and
// B[8 (l / 16) .. +7][l % 16] (8 halves each) and D[4 (l / 16) + r][l % 16] in register r.
// A lane therefore generates the phasors of one DM and four consecutive channels; the B
// operand of a (bin, column) row is 16 channels x 2 parts = 32 halves, padded to 40 so that
// the 16-byte reads of eight consecutive lanes fall in distinct LDS banks.  The data operand
// of the next 16 channels is prefetched into registers while the current one is in use.
#include "device_math.h"
#include "fdd_internal.h"
#include "split_math.h"

namespace fdd {

namespace {
constexpr int kXcds = 8;
}  // namespace

// PRE: X already holds, per complex value, the split words {hi, lo} of the scaled (Re, Im)
// pair (k_split_x), so the staging only rearranges them.
// DESC: X through a descriptor over the stage's 16 channels (32-bit offsets; the window, 16 x
// x_chunks x pitch x 8 bytes, must stay below 2 GiB).
template <bool BF, int NT, int FB, bool PRE = false, bool DESC = false>
__device__ __forceinline__ void phasor_split_body(const PhasorArgs& a, const int bid, const int n_dmt,
                                                  const int n_bb,
    const int tid) {
  using H = HalfMma<BF>;
  typedef typename H::V8 V8;
  constexpr int KC = 16;                 // channels per LDS stage = one MFMA contraction step
  constexpr int NCOL = NT * 16;
  constexpr int ROWW = 20;               // 32-bit words per (bin, column) row: 16 channels + 4 padding
  // per-bin stride padded by 8 words: the four 16-lane groups of a staging store (bins f, f+2,
  // f+4, f+6) then land on alternating bank halves
  constexpr int BINW = NCOL * ROWW + 8;
  constexpr int PLANEW = FB * BINW;      // words per plane
  constexpr int PER = (KC * 8 * NT * (FB / 2) + 255) / 256;   // staged float4 per thread, N <= 8 NT
  __shared__ uint4 lhi[PLANEW / 4];
  __shared__ uint4 llo[PLANEW / 4];
  __shared__ float colscale[32];
  __shared__ float2 sctab[256];          // phasors of k / 256 turn, for the seeds

  const int xcd = bid % kXcds;
  const int slot = bid / kXcds;
  const int bb = (slot / n_dmt) * kXcds + xcd;
  const int dmt = slot % n_dmt;
  if (bb >= n_bb) return;                // uniform per workgroup, before any barrier
  const int fb0 = bb * FB;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int N = a.n_chunks;
  const int XC = a.x_chunks > 0 ? a.x_chunks : N;   // chunks per row of X and of Y
  const int YC = a.y_chunks > 0 ? a.y_chunks : N;
  const int nel = KC * N * (FB / 2);

  for (int i = tid; i < PLANEW / 4; i += 256) {
    lhi[i] = make_uint4(0u, 0u, 0u, 0u);
    llo[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (tid < N) colscale[tid] = chunk_scale(a.l1max[tid]);
  sctab[tid] = turn_table_entry((uint32_t)tid);
  uint32_t* whi = reinterpret_cast<uint32_t*>(lhi);
  uint32_t* wlo = reinterpret_cast<uint32_t*>(llo);

  // Staging: element e = (channel cl fastest, bin pair fp, chunk k) is the float4 of bins
  // (2 fp, 2 fp + 1) of (cb + cl, k); prefetched one stage ahead into registers.
  float4 pf[PER];
  auto fetch = [&](int cb) {
    if constexpr (DESC) {
      // channels past n_chan read as zeros; a slot that holds no element points past the window
      const int nc = min(KC, a.n_chan - cb);
      const __amdgpu_buffer_rsrc_t rx = raw_rsrc(a.X + (int64_t)cb * XC * a.pitch, (int64_t)nc * XC * a.pitch * 8);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        const int cl = e % KC;
        const int fp = (e / KC) % (FB / 2);
        const int k = e / (KC * (FB / 2));
        const uint32_t off = e < nel ? ((uint32_t)(cl * XC + k) * (uint32_t)a.pitch + (uint32_t)(fb0 + 2 * fp)) * 8u
                                     : 0xFFFFFFF0u;
        pf[q] = load_f4(rx, off);
      }
    } else {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        const int cl = e % KC;
        const int fp = (e / KC) % (FB / 2);
        const int k = e / (KC * (FB / 2));
        const int c = cb + cl;
        pf[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (e < nel && c < a.n_chan) pf[q] = *(const float4*)(a.X + ((int64_t)c * XC + k) * a.pitch + fb0 + 2 * fp);
      }
    }
  };
  auto deposit = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      if (e >= nel) continue;
      const int cl = e % KC;
      const int fp = (e / KC) % (FB / 2);
      const int k = e / (KC * (FB / 2));
      const float sk = colscale[k];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        uint32_t h, l;                                    // (Re, Im) of X, scaled and split
        if constexpr (PRE) {
          h = __float_as_uint(b ? pf[q].z : pf[q].x);
          l = __float_as_uint(b ? pf[q].w : pf[q].y);
        } else {
          split_pair<BF>((b ? pf[q].z : pf[q].x) * sk, (b ? pf[q].w : pf[q].y) * sk, &h, &l);
        }
        const int f = 2 * fp + b;
        const int w0 = f * BINW + k * ROWW + cl;          // column k: (Re, -Im)
        const int w1 = f * BINW + (k + N) * ROWW + cl;    // column k + N: (Im, Re)
        whi[w0] = neg_hi(h);
        wlo[w0] = neg_hi(l);
        whi[w1] = swap16(h);
        wlo[w1] = swap16(l);
      }
    }
  };

  int dm = dmt * 64 + wave * 16 + (lane & 15);
  if (dm >= a.n_dm) dm = a.n_dm - 1;             // its results are not stored
  const int cq = lane >> 4;

  floatx4 acc[FB][NT];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[f][nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

  // Phase-table entries of this lane's DM for the 4 channels it seeds, loaded one stage ahead so
  // that their latency is spent while the previous stage computes.  With two column tiles the
  // 16 extra registers would cost a wave of occupancy, so that shape loads them in the stage.
  // They come through a descriptor over the stage's 16 channels: the byte offsets are the same
  // in every stage, and channels past n_chan read as zero entries (against data staged as zeros).
  constexpr bool kAhead = NT != 2;
  uint32_t toff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) toff[q] = (uint32_t)(((4 * cq + q) * a.n_dm + dm) * 16);
  auto tab_rsrc = [&](int cb) {
    const int nc = min(KC, a.n_chan - cb);
    return raw_rsrc(a.ptab + (int64_t)cb * a.n_dm, (int64_t)nc * a.n_dm * 16);
  };
  uint4 tnext[4];
  {
    const __amdgpu_buffer_rsrc_t rt = tab_rsrc(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) tnext[q] = load_u4(rt, toff[q]);
  }
  __syncthreads();                               // colscale
  fetch(0);
  for (int cb = 0; cb < a.n_chan; cb += KC) {
    __syncthreads();                             // the previous stage's operands are consumed
    deposit();
    __syncthreads();

    // phasors of this lane's DM for channels cb + 4 cq .. + 3 (clamped channels: data staged as zeros)
    float2 w[4], st[4];
    if constexpr (!kAhead) {
      const __amdgpu_buffer_rsrc_t rt = tab_rsrc(cb);
#pragma unroll
      for (int q = 0; q < 4; ++q) tnext[q] = load_u4(rt, toff[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) seed_phasor_tab(tnext[q], (uint32_t)fb0, sctab, &w[q], &st[q]);
    if constexpr (kAhead) {
      const __amdgpu_buffer_rsrc_t rt = tab_rsrc(cb + KC);
#pragma unroll
      for (int q = 0; q < 4; ++q) tnext[q] = load_u4(rt, toff[q]);
    }
    if (cb + KC < a.n_chan) fetch(cb + KC);      // in flight while this stage computes
    const int rowbase = (lane & 15) * ROWW + 4 * cq;     // words
#pragma unroll
    for (int f = 0; f < FB; ++f) {
      uint32_t ah[4], al[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        split_pair<BF>(w[q].x, w[q].y, &ah[q], &al[q]);
        w[q] = cmul(w[q], st[q]);
      }
      const V8 Ahi = __builtin_bit_cast(V8, make_uint4(ah[0], ah[1], ah[2], ah[3]));
      const V8 Alo = __builtin_bit_cast(V8, make_uint4(al[0], al[1], al[2], al[3]));
      V8 Bhi[NT], Blo[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int at = (f * BINW + 16 * nt * ROWW + rowbase) / 4;
        Bhi[nt] = __builtin_bit_cast(V8, lhi[at]);
        Blo[nt] = __builtin_bit_cast(V8, llo[at]);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[f][nt] = H::mfma(Ahi, Bhi[nt], acc[f][nt]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[f][nt] = H::mfma(Ahi, Blo[nt], acc[f][nt]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[f][nt] = H::mfma(Alo, Bhi[nt], acc[f][nt]);
    }
  }

  if (a.P != nullptr) {
    // single chunk: column 0 = Re Y, column 1 = Im Y (lanes j = 0 and 1 of each group)
    const float inv = 1.0f / colscale[0];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int dmr = dmt * 64 + wave * 16 + 4 * (lane >> 4) + r;
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const float yr = acc[f][0][r] * inv + ((fb0 + f) == 0 ? a.dc_add : 0.0f);
        const float yi = __shfl_down(acc[f][0][r], 1, 64) * inv;
        if ((lane & 15) == 0 && dmr < a.n_dm && fb0 + f < a.n_pow_bins)
          a.P[(int64_t)dmr * a.n_pow_bins + fb0 + f] = fmaf(yr, yr, yi * yi);
      }
    }
    return;
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = 16 * nt + (lane & 15);
    if (n >= 2 * N) continue;
    const int k = n < N ? n : n - N;
    const float inv = 1.0f / colscale[k];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int dmr = dmt * 64 + wave * 16 + 4 * (lane >> 4) + r;
      if (dmr >= a.n_dm) continue;
      float* dst = (n < N ? a.Yr + ((int64_t)dmr * YC + n) * a.pitch
                          : a.Yi + ((int64_t)dmr * YC + (n - N)) * a.pitch) + fb0;
#pragma unroll
      for (int f = 0; f < FB; f += 4)
        *(float4*)(dst + f) = make_float4(acc[f][nt][r] * inv, acc[f + 1][nt][r] * inv, acc[f + 2][nt][r] * inv,
                                          acc[f + 3][nt][r] * inv);
    }
  }
}

// linear workgroup id; grids are 2-D only to keep each dimension below 2^32 work-items
__device__ __forceinline__ int linear_block_s() { return blockIdx.y * gridDim.x + blockIdx.x; }

template <bool BF, int NT, int FB, bool DESC>
__global__ __launch_bounds__(256, 2) void k_phasor_split(PhasorArgs a, int n_dmt, int n_bb) {
  phasor_split_body<BF, NT, FB, true, DESC>(a, linear_block_s(), n_dmt, n_bb, threadIdx.x);
}

// Scale and split X in place, once per call instead of once per DM tile: every complex value
// (Re, Im) of chunk k becomes the two words {hi, lo} of split2(Re s_k, Im s_k).  Two values
// per thread; rows are (channel, chunk) series of `pitch` bins.
template <bool BF>
__global__ __launch_bounds__(256) void k_split_x(float4* X, const unsigned int* l1max, int n_chunks, int64_t rows,
                                                 int64_t pitch) {
  const int64_t i = (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
  const int64_t per_row = pitch / 2;
  if (i >= rows * per_row) return;
  const float sk = chunk_scale(l1max[(i / per_row) % n_chunks]);
  const float4 v = X[i];
  uint32_t h0, l0, h1, l1;
  split_pair<BF>(v.x * sk, v.y * sk, &h0, &l0);
  split_pair<BF>(v.z * sk, v.w * sk, &h1, &l1);
  X[i] = make_float4(__uint_as_float(h0), __uint_as_float(l0), __uint_as_float(h1), __uint_as_float(l1));
}

// Batched form: the tiles of every beam of the group, one per workgroup or persistent.
template <bool BF, int NT, int FB, bool PERSIST>
__global__ __launch_bounds__(256, 2) void k_phasor_split_grouped(Group<PhasorArgs> g) {
  grouped_tiles<PERSIST>(g.counters, g.total, [&](int t, int tid) {
    const int b = group_beam(g.prefix, g.n_beams, t);
    const PhasorArgs a = PERSIST ? load_uniform(g.beams + b) : g.beams[b];
    phasor_split_body<BF, NT, FB>(a, t - g.prefix[b], a.n_dmt, a.n_bb, tid);
  });
}

bool phasor_split_supported(int n_chunks) { return n_chunks >= 1 && n_chunks <= 24; }

namespace {
template <bool BF, int FB, bool DESC>
hipError_t launch_split_fb(const PhasorArgs& a, hipStream_t st) {
  const int n_dmt = (a.n_dm + 63) / 64;
  const int n_bb = (a.n_bins + FB - 1) / FB;
  const int n_bb8 = (n_bb + kXcds - 1) / kXcds * kXcds;
  const int64_t blocks = (int64_t)n_dmt * n_bb8;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid = linear_grid(blocks), block(256);
  switch ((2 * a.n_chunks + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_phasor_split<BF, 1, FB, DESC>), grid, block, 0, st, a, n_dmt, n_bb); break;
    case 2: hipLaunchKernelGGL((k_phasor_split<BF, 2, FB, DESC>), grid, block, 0, st, a, n_dmt, n_bb); break;
    case 3: hipLaunchKernelGGL((k_phasor_split<BF, 3, FB, DESC>), grid, block, 0, st, a, n_dmt, n_bb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_phasor_split(const PhasorArgs& a, bool bf16, hipStream_t st) {
  if (!phasor_split_supported(a.n_chunks)) return hipErrorInvalidValue;
  if (a.P != nullptr && a.n_chunks != 1) return hipErrorInvalidValue;
  const int64_t xc = a.x_chunks > 0 ? a.x_chunks : a.n_chunks;
  if (16 * 8 * xc * a.pitch <= 0x7fffffff)
    return bf16 ? launch_split_fb<true, 8, true>(a, st) : launch_split_fb<false, 8, true>(a, st);
  return bf16 ? launch_split_fb<true, 8, false>(a, st) : launch_split_fb<false, 8, false>(a, st);
}

hipError_t launch_split_x(float2* X, const unsigned int* l1max, int n_chan, int n_chunks, int64_t pitch, bool bf16,
                          hipStream_t st) {
  if (X == nullptr || l1max == nullptr || n_chan < 1 || n_chunks < 1 || pitch % 2 != 0) return hipErrorInvalidValue;
  const int64_t n = (int64_t)n_chan * n_chunks * (pitch / 2);
  const dim3 grid = linear_grid((n + 255) / 256);
  if (bf16)
    hipLaunchKernelGGL(k_split_x<true>, grid, dim3(256), 0, st, (float4*)X, l1max, n_chunks,
                       (int64_t)n_chan * n_chunks, pitch);
  else
    hipLaunchKernelGGL(k_split_x<false>, grid, dim3(256), 0, st, (float4*)X, l1max, n_chunks,
                       (int64_t)n_chan * n_chunks, pitch);
  return hipGetLastError();
}

namespace {
constexpr int kSplitFb = 8;

template <bool BF, int NT, bool P>
hipError_t launch_split_grouped_nt(const Group<PhasorArgs>& g, hipStream_t st) {
  const void* k = (const void*)k_phasor_split_grouped<BF, NT, kSplitFb, P>;
  hipLaunchKernelGGL((k_phasor_split_grouped<BF, NT, kSplitFb, P>), grouped_grid(P, k, g.total), dim3(256), 0, st, g);
  return hipGetLastError();
}

template <bool BF>
hipError_t launch_split_grouped_bf(int nt, bool persist, const Group<PhasorArgs>& g, hipStream_t st) {
  switch (nt * 2 + (persist ? 1 : 0)) {
    case 2: return launch_split_grouped_nt<BF, 1, false>(g, st);
    case 3: return launch_split_grouped_nt<BF, 1, true>(g, st);
    case 4: return launch_split_grouped_nt<BF, 2, false>(g, st);
    case 5: return launch_split_grouped_nt<BF, 2, true>(g, st);
    case 6: return launch_split_grouped_nt<BF, 3, false>(g, st);
    case 7: return launch_split_grouped_nt<BF, 3, true>(g, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

int64_t phasor_split_tiles(PhasorArgs* a) {
  a->n_dmt = (a->n_dm + 63) / 64;
  a->n_bb = (a->n_bins + kSplitFb - 1) / kSplitFb;
  return (int64_t)a->n_dmt * ((a->n_bb + kXcds - 1) / kXcds * kXcds);
}

hipError_t launch_phasor_split_grouped(bool bf16, int nt, bool persist, const Group<PhasorArgs>& g,
                                       hipStream_t st) {
  if (g.total <= 0) return hipSuccess;
  return bf16 ? launch_split_grouped_bf<true>(nt, persist, g, st) : launch_split_grouped_bf<false>(nt, persist, g, st);
}

}  // namespace fdd
