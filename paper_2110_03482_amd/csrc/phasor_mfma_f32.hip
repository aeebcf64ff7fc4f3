// Phasor sum as a dense complex contraction on the FP32 matrix cores (Eqs. 4 and 7).
//
// For every spin-frequency bin f the phasor sum over time chunks k is a matrix product
//     Y[dm, k] = sum_c W[dm, c] X[c, k],   W[dm, c] = exp(+2 pi i f tau[dm, c] / L),
// the matrix-vector product of Sec. 2.3 batched over the overlap-save chunks.  It is
// written as a real product with twice the columns:
//     [Yr | Yi] = Wr [Xr | Xi] + Wi [-Xi | Xr],
// so the phasor (A) operand carries cos or sin only, and the data (B) operand has 2N columns
// (N chunks), padded to NT*16.
//
// Work decomposition (gfx950, v_mfma_f32_16x16x4_f32, 64-lane waves):
//  - a workgroup owns 64 DMs (4 waves x 16) and FB = 16 consecutive bins, all chunks;
//  - channels stream through LDS in groups of KC = 8: the group's data for the 16 bins is
//    read from HBM once (128-byte runs along f) and rearranged into the two B planes
//    [c][f][column] (cos-part and sin-part operands);
//  - per 4-channel step, lane l generates the phasor of (DM l%16, channel l/16) for the 16
//    bins: exact 64-bit phase at the first bin and one bin step via sincos_turn, then 15
//    complex multiplications.  Its cos feeds the first MFMA set and its sin the second, so
//    no phasor is computed twice;
//  - accumulators live in registers: 16 bins x NT tiles x 4 floats per lane;
//  - the epilogue writes, per lane, 16 consecutive bins of one (DM, chunk) row of the Yr or
//    Yi plane (float4 stores).
// Workgroups are numbered so that the DM tiles of one bin block run back to back on the same
// XCD (hardware dispatches workgroup i to XCD i mod 8), so the bin block's data is served
// from that XCD's L2 after the first read.
#include "device_math.h"
#include "fdd_internal.h"

namespace fdd {

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kFB = 16;     // bins per workgroup
constexpr int kKC = 8;      // channels per LDS stage
constexpr int kDmTile = 64; // DMs per workgroup
constexpr int kXcds = 8;
}  // namespace

template <int NT>
__global__ __launch_bounds__(256) void k_phasor_mfma_f32(PhasorArgs a, int n_dmt, int n_bb) {
  constexpr int NCOL = NT * 16;
  // per-channel stride padded by 16 floats so that the four channels read by one MFMA step
  // fall in distinct LDS banks
  constexpr int CST = kFB * NCOL + 16;
  constexpr int PLANE = kKC * CST;
  __shared__ float bre[PLANE];
  __shared__ float bim[PLANE];

  const int bid = blockIdx.x;
  const int xcd = bid % kXcds;
  const int slot = bid / kXcds;
  const int bb = (slot / n_dmt) * kXcds + xcd;
  const int dmt = slot % n_dmt;
  if (bb >= n_bb) return;                     // uniform per workgroup, before any barrier
  const int fb0 = bb * kFB;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int N = a.n_chunks;
  const int ncol = 2 * N;

  // zero once: padding columns (>= 2N) are never written by the staging below
  for (int i = tid; i < PLANE; i += 256) {
    bre[i] = 0.0f;
    bim[i] = 0.0f;
  }

  const int dm = dmt * kDmTile + wave * 16 + (lane & 15);
  const double dmv = a.dms[dm < a.n_dm ? dm : a.n_dm - 1];
  const int cq = lane >> 4;

  floatx4 acc[kFB][NT];
#pragma unroll
  for (int f = 0; f < kFB; ++f)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[f][nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

  for (int cb = 0; cb < a.n_chan; cb += kKC) {
    __syncthreads();
    // stage X[cb .. cb+KC)[0 .. N)[fb0 .. fb0+16) into the two operand planes
    const int nel = kKC * N * (kFB / 2);
    for (int e = tid; e < nel; e += 256) {
      const int fp = e % (kFB / 2);
      const int k = (e / (kFB / 2)) % N;
      const int cl = e / ((kFB / 2) * N);
      const int c = cb + cl;
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (c < a.n_chan) v = *(const float4*)(a.X + ((int64_t)c * N + k) * a.pitch + fb0 + 2 * fp);
      const int i0 = cl * CST + 2 * fp * NCOL;
      const int i1 = i0 + NCOL;
      bre[i0 + k] = v.x;
      bim[i0 + k] = -v.y;
      bre[i0 + k + N] = v.y;
      bim[i0 + k + N] = v.x;
      bre[i1 + k] = v.z;
      bim[i1 + k] = -v.w;
      bre[i1 + k + N] = v.w;
      bim[i1 + k + N] = v.z;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kKC / 4; ++s) {
      const int cl = 4 * s + cq;
      int c = cb + cl;
      if (c >= a.n_chan) c = a.n_chan - 1;      // its data were staged as zeros
      const PhaseInc inc = phase_increment(dmv * a.kappa[c], a.log_len, a.mode);
      float sn, cs;
      sincos_turn(phase_at(inc, (uint32_t)fb0), &sn, &cs);
      float2 w = make_float2(cs, sn);
      sincos_turn(inc.hi, &sn, &cs);
      const float2 step = make_float2(cs, sn);
      float wr[kFB], wi[kFB];
#pragma unroll
      for (int f = 0; f < kFB; ++f) {
        wr[f] = w.x;
        wi[f] = w.y;
        w = cmul(w, step);
      }
      const float* pr = bre + cl * CST + (lane & 15);
      const float* pi = bim + cl * CST + (lane & 15);
#pragma unroll
      for (int f = 0; f < kFB; ++f)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[f][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wr[f], pr[f * NCOL + 16 * nt], acc[f][nt], 0, 0, 0);
#pragma unroll
      for (int f = 0; f < kFB; ++f)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[f][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wi[f], pi[f * NCOL + 16 * nt], acc[f][nt], 0, 0, 0);
    }
  }

  // D[i][j] of a 16x16 tile sits in lane 16*(i/4) + j, register i%4.
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = 16 * nt + (lane & 15);
    if (n >= ncol) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int dmr = dmt * kDmTile + wave * 16 + 4 * (lane >> 4) + r;
      if (dmr >= a.n_dm) continue;
      float* dst = (n < N ? a.Yr + ((int64_t)dmr * N + n) * a.pitch
                          : a.Yi + ((int64_t)dmr * N + (n - N)) * a.pitch) + fb0;
#pragma unroll
      for (int f = 0; f < kFB; f += 4)
        *(float4*)(dst + f) = make_float4(acc[f][nt][r], acc[f + 1][nt][r], acc[f + 2][nt][r], acc[f + 3][nt][r]);
    }
  }
}

bool phasor_mfma_f32_supported(int n_chunks) { return n_chunks >= 3 && n_chunks <= 24; }

hipError_t launch_phasor_mfma_f32(const PhasorArgs& a, hipStream_t st) {
  if (!phasor_mfma_f32_supported(a.n_chunks)) return hipErrorInvalidValue;
  const int n_dmt = (a.n_dm + kDmTile - 1) / kDmTile;
  const int n_bb = (a.n_bins + kFB - 1) / kFB;
  const int n_bb8 = (n_bb + kXcds - 1) / kXcds * kXcds;
  const int64_t blocks = (int64_t)n_dmt * n_bb8;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const int nt = (2 * a.n_chunks + 15) / 16;
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_phasor_mfma_f32<1>), dim3((unsigned)blocks), dim3(256), 0, st, a, n_dmt, n_bb); break;
    case 2: hipLaunchKernelGGL((k_phasor_mfma_f32<2>), dim3((unsigned)blocks), dim3(256), 0, st, a, n_dmt, n_bb); break;
    case 3: hipLaunchKernelGGL((k_phasor_mfma_f32<3>), dim3((unsigned)blocks), dim3(256), 0, st, a, n_dmt, n_bb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fdd
