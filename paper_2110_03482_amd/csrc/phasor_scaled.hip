// Power spectra with spin-frequency-scaled DMs (Sec. 2.3, Eq. 8) on the FP32 matrix cores.
//
// Eq. 8 lets the trial DM of a row scale as DM_f = DM_ref r / f across a range of spin
// frequencies f around a reference r: the phasor exp(+2 pi i f DM_f kappa_c / L) then equals
// exp(+2 pi i r DM_ref kappa_c / L) for every f of the range.  With blocks of 64 bins and the
// block's middle bin as r, the phasor sum of a block is one dense product
//     Ytilde[q, f] = sum_c W_r[q, c] X[c, f],   f in the block,
// over the rows q of a scaled DM grid, taken in the real form [Yr | Yi] = Wr [Xr | Xi] +
// Wi [-Xi | Xr] (128 columns: the block's 64 bins, real and imaginary parts).  Each phasor is
// generated once per block instead of once per bin.  A second kernel resamples the power
// |Ytilde|^2 linearly in DM back onto the trial grid: row q of bin f holds the DM
// DM'_q r / f, so trial DM_j sits at the fractional row (DM_j f / r - DM_0) / dDM.
//
// Work decomposition (v_mfma_f32_16x16x4_f32, 64-lane waves): a workgroup owns 64 scaled rows
// (4 waves x 16) and one block; channels stream through LDS 16 at a time, double-buffered;
// per 4-channel step lane l generates the phasor of (row l%16, channel l/16) at the reference
// bin from the 64-bit turn increments of its channel (one sincos_turn) and feeds its cos and
// sin to two sets of 8 products.  The power |Yr|^2 + |Yi|^2 of a bin sits in one lane (columns
// b and 64 + b are 4 tiles apart), so the epilogue writes it directly.  Workgroups are numbered
// so that the row tiles of one block run back to back on one XCD and share its L2.
#include "device_math.h"
#include "fdd_internal.h"
#include "split_math.h"

namespace fdd {

namespace {
constexpr int kXcds = 8;
constexpr int kKc = 16;                                  // channels per LDS stage
constexpr int kCols = 2 * kScaledBlock;                  // [Re | Im] of the block's bins
constexpr int kNt = kCols / 16;                          // column tiles
constexpr int kCst = kCols + 16;                         // per-channel LDS stride: the 4 channels of
                                                         // one product step fall in distinct banks
constexpr int kPlane = kKc * kCst;
constexpr int kPer = kKc * (kScaledBlock / 2) / 256;     // float4 staging loads per thread
static_assert(kPer * 256 == kKc * (kScaledBlock / 2), "staging must divide evenly");
}  // namespace

__global__ __launch_bounds__(256) void k_phasor_scaled_f32(ScaledArgs a, int n_rt) {
  __shared__ float bre2[2][kPlane];
  __shared__ float bim2[2][kPlane];
  const int bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int xcd = bid % kXcds;
  const int slot = bid / kXcds;
  const int bb = (slot / n_rt) * kXcds + xcd;
  const int rt = slot % n_rt;
  if (bb >= a.n_blocks) return;                          // uniform per workgroup, before any barrier
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int f0 = a.f_min + bb * kScaledBlock;
  const uint32_t ref = (uint32_t)(f0 + kScaledBlock / 2);

  // staging element e = tid + 256 j: channel e / 32 of the stage, bins 2 (e % 32) and + 1
  int ccl[kPer], cbin[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int e = tid + 256 * j;
    ccl[j] = e / (kScaledBlock / 2);
    cbin[j] = 2 * (e % (kScaledBlock / 2));
  }
  float4 pf[kPer];
  auto fetch = [&](int cb) {
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int c = cb + ccl[j];
      pf[j] = c < a.n_chan ? *(const float4*)(a.X + (int64_t)c * a.pitch + f0 + cbin[j])
                           : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  };
  auto deposit = [&](float* bre, float* bim) {
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i0 = ccl[j] * kCst + cbin[j];
      const float4 v = pf[j];                             // (re, im) of bins cbin, cbin + 1
      bre[i0] = v.x;
      bre[i0 + 1] = v.z;
      bre[i0 + kScaledBlock] = v.y;
      bre[i0 + kScaledBlock + 1] = v.w;
      bim[i0] = -v.y;
      bim[i0 + 1] = -v.w;
      bim[i0 + kScaledBlock] = v.x;
      bim[i0 + kScaledBlock + 1] = v.z;
    }
  };

  int q = rt * 64 + wave * 16 + (lane & 15);
  if (q >= a.n_rows) q = a.n_rows - 1;                   // a clamped row's results are not stored
  const uint64_t uq = (uint64_t)q;
  const int cq = lane >> 4;

  floatx4 acc[kNt];
#pragma unroll
  for (int nt = 0; nt < kNt; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

  fetch(0);
  deposit(bre2[0], bim2[0]);
  __syncthreads();
  int it = 0;
  for (int cb = 0; cb < a.n_chan; cb += kKc, ++it) {
    const float* bre = bre2[it & 1];
    const float* bim = bim2[it & 1];
    uint4 e[kKc / 4];
#pragma unroll
    for (int s = 0; s < kKc / 4; ++s) {
      int c = cb + 4 * s + cq;
      if (c >= a.n_chan) c = a.n_chan - 1;               // its data were staged as zeros
      e[s] = a.ctab[c];
    }
    if (cb + kKc < a.n_chan) fetch(cb + kKc);            // in flight while this stage computes
#pragma unroll
    for (int s = 0; s < kKc / 4; ++s) {
      const uint64_t inc_a = ((uint64_t)e[s].y << 32) | e[s].x;
      const uint64_t inc_d = ((uint64_t)e[s].w << 32) | e[s].z;
      const uint64_t inc = inc_a + uq * inc_d;           // turn fraction per bin of row q, mod 1
      const PhaseInc pi = {(uint32_t)(inc >> 32), (uint32_t)inc};
      float sn, cs;
      sincos_turn(phase_at(pi, ref), &sn, &cs);
      const int cl = 4 * s + cq;
      const float* pr = bre + cl * kCst + (lane & 15);
      const float* pm = bim + cl * kCst + (lane & 15);
#pragma unroll
      for (int nt = 0; nt < kNt; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(cs, pr[16 * nt], acc[nt], 0, 0, 0);
#pragma unroll
      for (int nt = 0; nt < kNt; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sn, pm[16 * nt], acc[nt], 0, 0, 0);
    }
    {
      // Scheduling only: keep two B-operand reads (ds_read2, two MFMAs each) in flight ahead
      // of the matrix instructions instead of waiting for each read right before its MFMAs.
      constexpr int kReads = (kKc / 4) * kNt;
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);      // DS reads
#pragma unroll
      for (int i = 0; i < kReads - 2; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);    // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
    }
    // the other buffer was last read in the previous stage, which every wave has left
    if (cb + kKc < a.n_chan) deposit(bre2[(it + 1) & 1], bim2[(it + 1) & 1]);
    __syncthreads();
  }

  // D[i][j] of a 16x16 tile sits in lane 16 (i / 4) + j, register i % 4; tile nt holds the real
  // parts of bins 16 nt .. and tile nt + 4 their imaginary parts.
#pragma unroll
  for (int nt = 0; nt < kNt / 2; ++nt) {
    const int bin = 16 * nt + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 64 + wave * 16 + 4 * (lane >> 4) + r;
      if (row >= a.n_rows) continue;
      const float yr = acc[nt][r], yi = acc[nt + kNt / 2][r];
      a.Q[(int64_t)row * a.q_pitch + (int64_t)bb * kScaledBlock + bin] = fmaf(yr, yr, yi * yi);
    }
  }
}

// The same block products on the half-precision matrix cores, operands split into head and
// tail (A_hi B_hi + A_hi B_lo + A_lo B_hi in FP32), from X already scaled and split in place
// (launch_split_x).  K = 32 per product = 16 channels x (cos, sin): lane l holds the four
// phasors of row l % 16 and channels 4 (l / 16) .. + 3 as packed (cos, sin) head and tail
// pairs, and reads its B operand (the same four channels of column l % 16 of a tile) with one
// 16-byte LDS load per tile and plane.
template <bool BF>
__global__ __launch_bounds__(256) void k_phasor_scaled_split(ScaledArgs a, int n_rt, const unsigned int* l1max) {
  using H = HalfMma<BF>;
  typedef typename H::V8 V8;
  constexpr int KC = 16;                                  // channels per stage = one product's K
  constexpr int ROWW = 20;                                // words per column: 16 channels + 4 padding
  constexpr int PLANEW = kCols * ROWW;
  __shared__ uint4 lhi2[2][PLANEW / 4];
  __shared__ uint4 llo2[2][PLANEW / 4];
  const int bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int xcd = bid % kXcds;
  const int slot = bid / kXcds;
  const int bb = (slot / n_rt) * kXcds + xcd;
  const int rt = slot % n_rt;
  if (bb >= a.n_blocks) return;                          // uniform per workgroup, before any barrier
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int f0 = a.f_min + bb * kScaledBlock;
  const uint32_t ref = (uint32_t)(f0 + kScaledBlock / 2);
  const float inv = 1.0f / chunk_scale(l1max[0]);

  // staging element e = tid + 256 j: channel e / 32 of the stage, bins 2 (e % 32) and + 1;
  // X holds the split words {hi, lo} of each scaled (Re, Im) pair
  constexpr int PER = KC * (kScaledBlock / 2) / 256;
  int ccl[PER], cbin[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    ccl[j] = e / (kScaledBlock / 2);
    cbin[j] = 2 * (e % (kScaledBlock / 2));
  }
  uint4 pf[PER];
  auto fetch = [&](int cb) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int c = cb + ccl[j];
      pf[j] = c < a.n_chan ? *(const uint4*)(a.X + (int64_t)c * a.pitch + f0 + cbin[j]) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto deposit = [&](uint32_t* whi, uint32_t* wlo) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const uint32_t h = b ? pf[j].z : pf[j].x;
        const uint32_t l = b ? pf[j].w : pf[j].y;
        const int w0 = (cbin[j] + b) * ROWW + ccl[j];                  // column bin: (Re, -Im)
        const int w1 = (kScaledBlock + cbin[j] + b) * ROWW + ccl[j];   // column 64 + bin: (Im, Re)
        whi[w0] = neg_hi(h);
        wlo[w0] = neg_hi(l);
        whi[w1] = swap16(h);
        wlo[w1] = swap16(l);
      }
    }
  };

  int q = rt * 64 + wave * 16 + (lane & 15);
  if (q >= a.n_rows) q = a.n_rows - 1;                   // a clamped row's results are not stored
  const uint64_t uq = (uint64_t)q;
  const int cq = lane >> 4;

  floatx4 acc[kNt];
#pragma unroll
  for (int nt = 0; nt < kNt; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

  fetch(0);
  deposit(reinterpret_cast<uint32_t*>(lhi2[0]), reinterpret_cast<uint32_t*>(llo2[0]));
  __syncthreads();
  int it = 0;
  for (int cb = 0; cb < a.n_chan; cb += KC, ++it) {
    uint4 e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int c = cb + 4 * cq + k;
      if (c >= a.n_chan) c = a.n_chan - 1;               // its data were staged as zeros
      e[k] = a.ctab[c];
    }
    if (cb + KC < a.n_chan) fetch(cb + KC);              // in flight while this stage computes
    uint32_t ah[4], al[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t inc_a = ((uint64_t)e[k].y << 32) | e[k].x;
      const uint64_t inc_d = ((uint64_t)e[k].w << 32) | e[k].z;
      const uint64_t inc = inc_a + uq * inc_d;
      const PhaseInc pi = {(uint32_t)(inc >> 32), (uint32_t)inc};
      float sn, cs;
      sincos_turn(phase_at(pi, ref), &sn, &cs);
      split_pair<BF>(cs, sn, &ah[k], &al[k]);
    }
    const V8 Ahi = __builtin_bit_cast(V8, make_uint4(ah[0], ah[1], ah[2], ah[3]));
    const V8 Alo = __builtin_bit_cast(V8, make_uint4(al[0], al[1], al[2], al[3]));
    const uint4* bhi = lhi2[it & 1];
    const uint4* blo = llo2[it & 1];
    const int base = ((lane & 15) * ROWW + 4 * cq) / 4;
#pragma unroll
    for (int nt = 0; nt < kNt; ++nt) {
      const V8 Bh = __builtin_bit_cast(V8, bhi[base + 16 * nt * ROWW / 4]);
      const V8 Bl = __builtin_bit_cast(V8, blo[base + 16 * nt * ROWW / 4]);
      acc[nt] = H::mfma(Ahi, Bh, acc[nt]);
      acc[nt] = H::mfma(Ahi, Bl, acc[nt]);
      acc[nt] = H::mfma(Alo, Bh, acc[nt]);
    }
    // the other buffer was last read in the previous stage, which every wave has left
    if (cb + KC < a.n_chan)
      deposit(reinterpret_cast<uint32_t*>(lhi2[(it + 1) & 1]), reinterpret_cast<uint32_t*>(llo2[(it + 1) & 1]));
    __syncthreads();
  }

#pragma unroll
  for (int nt = 0; nt < kNt / 2; ++nt) {
    const int bin = 16 * nt + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 64 + wave * 16 + 4 * (lane >> 4) + r;
      if (row >= a.n_rows) continue;
      const float yr = acc[nt][r] * inv, yi = acc[nt + kNt / 2][r] * inv;
      a.Q[(int64_t)row * a.q_pitch + (int64_t)bb * kScaledBlock + bin] = fmaf(yr, yr, yi * yi);
    }
  }
}

// Linear resampling in DM: trial j at bin f reads the two scaled rows around
// s* = (DM_j f / r - DM_0) / dDM.  A thread takes four consecutive bins (one block, one r) of
// kResampleRows consecutive trials, whose scaled rows overlap, so each row comes from memory
// about once.  s* is linear in f within a block: s* = f DM_j / (r dDM) - DM_0 / dDM.
constexpr int kResampleRows = 8;

__global__ __launch_bounds__(256) void k_scaled_resample(ResampleArgs a) {
  const int j0 = (int)blockIdx.y * kResampleRows;
  const int64_t fb = (int64_t)a.f_min + 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  if (fb >= a.n_pow_bins) return;
  const int64_t col0 = fb - a.f_min;
  const int64_t ref = a.f_min + col0 / kScaledBlock * kScaledBlock + kScaledBlock / 2;
  const double off = a.dm0 / a.step;
  for (int jj = 0; jj < kResampleRows; ++jj) {
    const int j = j0 + jj;
    if (j >= a.n_dm) break;
    const double slope = a.dms[j] / ((double)ref * a.step);
    float out[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      out[i] = 0.0f;
      if (fb + i >= a.n_pow_bins) continue;
      const double ss = fma(slope, (double)(fb + i), -off);
      const double fl = floor(ss);
      int64_t q0 = (int64_t)fl + kScaledHalo;
      double w = ss - fl;
      if (q0 < 0) {                                        // outside the planned halo: clamp
        q0 = 0;
        w = 0.0;
      } else if (q0 > a.n_rows - 2) {
        q0 = a.n_rows - 2;
        w = 1.0;
      }
      const float* src = a.Q + q0 * a.q_pitch + col0 + i;
      const float wf = (float)w;
      out[i] = fmaf(wf, src[a.q_pitch], (1.0f - wf) * src[0]);
    }
    float* dst = a.P + (int64_t)j * a.n_pow_bins + fb;
    if (fb + 4 <= a.n_pow_bins) {
      *(float4*)dst = make_float4(out[0], out[1], out[2], out[3]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (fb + i < a.n_pow_bins) dst[i] = out[i];
    }
  }
}

hipError_t launch_phasor_scaled(const ScaledArgs& a, int precision, const unsigned int* l1max, hipStream_t st) {
  if (a.n_blocks <= 0) return hipSuccess;
  if (a.n_rows < 2 || a.n_chan < 1 || a.X == nullptr || a.Q == nullptr || a.ctab == nullptr ||
      a.q_pitch < (int64_t)a.n_blocks * kScaledBlock || (precision != FDD_FP32 && l1max == nullptr))
    return hipErrorInvalidValue;
  const int n_rt = (a.n_rows + 63) / 64;
  const int64_t n_bb8 = ((int64_t)a.n_blocks + kXcds - 1) / kXcds * kXcds;
  const int64_t blocks = (int64_t)n_rt * n_bb8;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid = linear_grid(blocks);
  if (precision == FDD_FP32)
    hipLaunchKernelGGL(k_phasor_scaled_f32, grid, dim3(256), 0, st, a, n_rt);
  else if (precision == FDD_FP16_SPLIT)
    hipLaunchKernelGGL(k_phasor_scaled_split<false>, grid, dim3(256), 0, st, a, n_rt, l1max);
  else
    hipLaunchKernelGGL(k_phasor_scaled_split<true>, grid, dim3(256), 0, st, a, n_rt, l1max);
  return hipGetLastError();
}

hipError_t launch_scaled_resample(const ResampleArgs& a, hipStream_t st) {
  const int64_t bins = (int64_t)a.n_pow_bins - a.f_min;
  if (bins <= 0) return hipSuccess;
  if (a.n_dm < 1 || a.n_dm > 65535 || a.n_rows < 2 || a.Q == nullptr || a.P == nullptr || a.dms == nullptr ||
      !(a.step > 0.0))
    return hipErrorInvalidValue;
  const int64_t gx = (bins + 4 * 256 - 1) / (4 * 256);
  if (gx > 0x7fffffff || (a.n_pow_bins - a.f_min) % 4 != 0) return hipErrorInvalidValue;
  const unsigned gy = (unsigned)((a.n_dm + kResampleRows - 1) / kResampleRows);
  hipLaunchKernelGGL(k_scaled_resample, dim3((unsigned)gx, gy), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace fdd
