// Phasor sum on the vector ALUs (Eqs. 4 and 7), any number of chunks, FP32.
//
//     Y[dm, k, f] = sum_c X[c, k, f] * exp(+2 pi i f tau[dm, c] / L)
//
// For one spin-frequency bin this is a matrix-vector product per chunk (Sec. 2.3); with a
// single chunk nothing is shared along the chunk axis, so this kernel is the path for the
// single-transform workloads, and the fallback for any shape.  Each thread owns one DM and
// FV consecutive bins.  Per channel it reads the exact 64-bit phase increment of its delay and
// the step phasor from the planner's table, evaluates the phasor of its first bin with
// sincos_turn, and walks the remaining bins by complex multiplication (at most FV-1 steps, so the recurrence error stays
// at a few float32 ulps).  Threads of a block that share bins read the same data from L1.
//
// With P set, the epilogue writes power spectra |Y|^2 for bins below L/2 (Sec. 5) instead of
// the complex result.
#include "device_math.h"
#include "fdd_internal.h"

namespace fdd {

namespace {
constexpr int kBinThreads = 64;   // threads along bins per block
constexpr int kDmThreads = 4;     // threads along DMs per block
}

template <int FV, int NK>
__device__ __forceinline__ void phasor_valu_body(const PhasorArgs& a, const int bx, const int by, const int bz) {
  const int tx = threadIdx.x % kBinThreads;
  const int ty = threadIdx.x / kBinThreads;
  const int f0 = (bx * kBinThreads + tx) * FV;
  const int dm = by * kDmThreads + ty;
  const int k0 = bz * NK;
  if (dm >= a.n_dm || f0 >= a.n_bins) return;   // no barriers in this kernel
  float2 acc[NK][FV];
#pragma unroll
  for (int kk = 0; kk < NK; ++kk)
#pragma unroll
    for (int i = 0; i < FV; ++i) acc[kk][i] = make_float2(0.0f, 0.0f);

  int nk = a.n_chunks - k0;
  if (nk > NK) nk = NK;
  for (int c = 0; c < a.n_chan; ++c) {
    float2 w, step;
    seed_phasor(a.ptab[(int64_t)c * a.n_dm + dm], (uint32_t)f0, &w, &step);
    const float2* xr = a.X + ((int64_t)c * a.n_chunks + k0) * a.pitch + f0;
#pragma unroll
    for (int i = 0; i < FV; ++i) {
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        if (kk < nk) {
          const float2 x = xr[(int64_t)kk * a.pitch + i];
          acc[kk][i].x = fmaf(w.x, x.x, fmaf(-w.y, x.y, acc[kk][i].x));
          acc[kk][i].y = fmaf(w.x, x.y, fmaf(w.y, x.x, acc[kk][i].y));
        }
      }
      w = cmul(w, step);
    }
  }

  if (a.P != nullptr) {
    if (f0 == 0) acc[0][0].x += a.dc_add;
#pragma unroll
    for (int i = 0; i < FV; ++i) {
      const int f = f0 + i;
      if (f < a.n_pow_bins)
        a.P[(int64_t)dm * a.n_pow_bins + f] = fmaf(acc[0][i].x, acc[0][i].x, acc[0][i].y * acc[0][i].y);
    }
    return;
  }
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    if (kk < nk) {
      const int64_t row = ((int64_t)dm * a.n_chunks + k0 + kk) * a.pitch;
#pragma unroll
      for (int i = 0; i < FV; ++i) {
        const int f = f0 + i;
        if (f < a.n_bins) {
          a.Yr[row + f] = acc[kk][i].x;
          a.Yi[row + f] = acc[kk][i].y;
        }
      }
    }
  }
}

template <int FV, int NK>
__global__ __launch_bounds__(256) void k_phasor_valu(PhasorArgs a) {
  phasor_valu_body<FV, NK>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Batched form: tile t of beam b is block (t mod n_bb, (t / n_bb) mod n_dmt, t / (n_bb n_dmt))
// of that beam's own launch.
template <int FV, int NK>
__global__ __launch_bounds__(256) void k_phasor_valu_grouped(Group<PhasorArgs> g) {
  const int t = blockIdx.y * gridDim.x + blockIdx.x;
  if (t >= g.total) return;
  const int b = group_beam(g.prefix, g.n_beams, t);
  const PhasorArgs& a = g.beams[b];
  const int lt = t - g.prefix[b];
  phasor_valu_body<FV, NK>(a, lt % a.n_bb, (lt / a.n_bb) % a.n_dmt, lt / (a.n_bb * a.n_dmt));
}

namespace {
constexpr int kFv = 16;
}

int64_t phasor_valu_tiles(PhasorArgs* a, int nk) {
  a->n_bb = (a->n_bins + kBinThreads * kFv - 1) / (kBinThreads * kFv);
  a->n_dmt = (a->n_dm + kDmThreads - 1) / kDmThreads;
  return (int64_t)a->n_bb * a->n_dmt * ((a->n_chunks + nk - 1) / nk);
}

hipError_t launch_phasor_valu_grouped(int nk, const Group<PhasorArgs>& g, hipStream_t st) {
  if (g.total <= 0) return hipSuccess;
  const dim3 grid = linear_grid(g.total), block(kBinThreads * kDmThreads);
  if (nk == 1) hipLaunchKernelGGL((k_phasor_valu_grouped<kFv, 1>), grid, block, 0, st, g);
  else if (nk == 4) hipLaunchKernelGGL((k_phasor_valu_grouped<kFv, 4>), grid, block, 0, st, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_phasor_valu(const PhasorArgs& a, hipStream_t st) {
  constexpr int FV = kFv;
  dim3 block(kBinThreads * kDmThreads);
  const unsigned gx = (unsigned)((a.n_bins + kBinThreads * FV - 1) / (kBinThreads * FV));
  const unsigned gy = (unsigned)((a.n_dm + kDmThreads - 1) / kDmThreads);
  if (a.n_chunks == 1 || a.P != nullptr) {
    hipLaunchKernelGGL((k_phasor_valu<FV, 1>), dim3(gx, gy, 1), block, 0, st, a);
  } else {
    constexpr int NK = 4;
    const unsigned gz = (unsigned)((a.n_chunks + NK - 1) / NK);
    hipLaunchKernelGGL((k_phasor_valu<FV, NK>), dim3(gx, gy, gz), block, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace fdd
