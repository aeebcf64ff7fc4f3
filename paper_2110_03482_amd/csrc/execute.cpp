// Stage sequencing of fdd_execute / fdd_power_spectrum (Algorithm 1 without host copies:
// inputs and outputs are device resident, so there is nothing to overlap with PCIe).
#include "fdd_internal.h"

using namespace fdd;

namespace {

fdd_status check_ready(fdd_plan_t p, const void* in, const float* out) {
  if (p == nullptr) return fail(FDD_E_INVALID, "null plan");
  if (p->dry_run) return fail(FDD_E_INVALID, "a dry-run plan cannot execute");
  if (in == nullptr || out == nullptr) return fail(FDD_E_INVALID, "null input or output");
  if (p->d_ws == nullptr) return fail(FDD_E_WORKSPACE, "no workspace attached");
  return FDD_OK;
}

// Record stage boundary i (0..4) of the current call into the profiling ring.
void mark(fdd_plan_t p, int i, hipStream_t st) {
  if (p->prof_depth == 0 || p->prof_calls >= p->prof_depth) return;
  const size_t slot = (size_t)p->prof_calls * 5 + (size_t)i;
  p->ev_ok[slot] = hipEventRecord(p->ev[slot], st) == hipSuccess;
  if (i == 4) ++p->prof_calls;
}

fdd_status forward(fdd_plan_t p, const void* in, hipStream_t st) {
  const fdd_plan_desc& d = p->desc;
  FftArgs f;
  if (d.input == FDD_IN_U8_TIME_MAJOR) {
    uint8_t* xt = p->d_ws + p->ws.xt;
    hipError_t e = launch_transpose_u8((const uint8_t*)in, xt, d.n_samp, d.n_chan, st);
    if (e != hipSuccess) return hip_fail(e, "transpose launch");
    f.in_u8 = xt;
  } else {
    f.in_f32 = (const float*)in;
  }
  mark(p, 1, st);
  f.X = (float2*)(p->d_ws + p->ws.X);
  f.twL = (const float2*)(p->d_ws + p->ws.tw);
  f.n_samp = d.n_samp;
  f.stride = p->S;
  f.pitch = p->pitch;
  f.n_chunks = (int)p->n_chunks;
  f.n_rows = d.n_chan;
  if (d.precision != FDD_FP32) f.l1max = (unsigned int*)(p->d_ws + p->ws.scale);
  f.log_n = p->log_len - 1;
  hipError_t e = f.log_n > kMaxBlockLogN
                     ? launch_r2c_long(f, (float2*)(p->d_ws + p->ws.Z), (float*)(p->d_ws + p->ws.l1), st)
                     : launch_r2c(f.log_n, f, st);
  if (e != hipSuccess) return hip_fail(e, "forward FFT launch");
  mark(p, 2, st);
  return FDD_OK;
}

PhasorArgs phasor_args(fdd_plan_t p) {
  PhasorArgs a;
  a.X = (const float2*)(p->d_ws + p->ws.X);
  a.ptab = (const uint4*)(p->d_ws + p->ws.ptab);
  a.l1max = (const unsigned int*)(p->d_ws + p->ws.scale);
  a.n_dm = p->desc.n_dm;
  a.n_chan = p->desc.n_chan;
  a.n_chunks = (int)p->n_chunks;
  a.pitch = p->pitch;
  a.n_bins = (int)p->n_bins;
  a.n_pow_bins = (int)(p->L / 2);
  a.log_len = p->log_len;
  a.tile_variant = p->tile_variant;
  if (p->fac_fine > 0) {
    a.n_coarse = p->fac_coarse;
    a.n_fine = p->fac_fine;
    a.vtab = a.ptab + (size_t)p->desc.n_chan * (size_t)p->fac_coarse;
  }
  return a;
}

}  // namespace

extern "C" {

fdd_status fdd_execute(fdd_plan_t p, const void* in, float* out, void* stream) {
  fdd_status s = check_ready(p, in, out);
  if (s != FDD_OK) return s;
  if (p->desc.flags & FDD_PLAN_POWER_ONLY) return fail(FDD_E_UNSUPPORTED, "the plan was made for power spectra only");
  hipStream_t st = (hipStream_t)stream;
  mark(p, 0, st);
  s = forward(p, in, st);
  if (s != FDD_OK) return s;
  PhasorArgs a = phasor_args(p);
  a.Yr = (float*)(p->d_ws + p->ws.Yr);
  a.Yi = (float*)(p->d_ws + p->ws.Yi);
  hipError_t e;
  if (p->fac_fine > 0) e = launch_phasor_fac(a, p->desc.precision, st);
  else if (p->kernel == "mfma_f32") e = launch_phasor_mfma_f32(a, st);
  else if (p->kernel == "mfma_f16_split") e = launch_phasor_split(a, false, st);
  else if (p->kernel == "mfma_bf16_split") e = launch_phasor_split(a, true, st);
  else e = launch_phasor_valu(a, st);
  if (e != hipSuccess) return hip_fail(e, "phasor-sum launch");
  mark(p, 3, st);
  FftArgs f;
  f.Yr = a.Yr;
  f.Yi = a.Yi;
  f.out = out;
  f.twL = (const float2*)(p->d_ws + p->ws.tw);
  f.n_samp = p->desc.n_samp;
  f.stride = p->S;
  f.keep = p->desc.single_chunk ? p->desc.n_samp : p->S;
  f.pitch = p->pitch;
  f.n_chunks = (int)p->n_chunks;
  f.n_rows = p->desc.n_dm;
  f.add_full = p->desc.input == FDD_IN_U8_TIME_MAJOR ? 128.0f * (float)p->desc.n_chan : 0.0f;
  f.log_n = p->log_len - 1;
  e = f.log_n > kMaxBlockLogN
          ? launch_c2r_long(f, (float2*)(p->d_ws + p->ws.Z), (float2*)(p->d_ws + p->ws.Yr), st)
          : launch_c2r(f.log_n, f, st);
  if (e != hipSuccess) return hip_fail(e, "inverse FFT launch");
  mark(p, 4, st);
  return FDD_OK;
}

fdd_status fdd_tdd_execute(fdd_plan_t p, const void* in, float* out, void* stream) {
  fdd_status s = check_ready(p, in, out);
  if (s != FDD_OK) return s;
  if (p->tdd_span > tdd_span_max())
    return fail(FDD_E_UNSUPPORTED, "nearest-sample delays of neighbouring DMs differ by " + std::to_string(p->tdd_span) +
                                       " samples; the time-domain kernel takes at most " + std::to_string(tdd_span_max()));
  const fdd_plan_desc& d = p->desc;
  hipStream_t st = (hipStream_t)stream;
  mark(p, 0, st);
  TddArgs a;
  if (d.input == FDD_IN_U8_TIME_MAJOR) {
    uint8_t* xt = p->d_ws + p->ws.xt;
    hipError_t e = launch_transpose_u8((const uint8_t*)in, xt, d.n_samp, d.n_chan, st);
    if (e != hipSuccess) return hip_fail(e, "transpose launch");
    a.in_u8 = xt;
  } else {
    a.in_f32 = (const float*)in;
  }
  mark(p, 1, st);
  mark(p, 2, st);
  a.out = out;
  a.dtab = (const int*)(p->d_ws + p->ws.dtab);
  a.n_samp = d.n_samp;
  a.period = d.single_chunk ? p->L : 0;
  a.n_chan = d.n_chan;
  a.n_dm = d.n_dm;
  hipError_t e = launch_tdd(a, p->tdd_span, p->tdd_span64, st);
  if (e != hipSuccess) return hip_fail(e, "time-domain launch");
  mark(p, 3, st);
  mark(p, 4, st);
  return FDD_OK;
}

fdd_status fdd_power_spectrum(fdd_plan_t p, const void* in, float* out, void* stream) {
  fdd_status s = check_ready(p, in, out);
  if (s != FDD_OK) return s;
  if (!p->desc.single_chunk) return fail(FDD_E_UNSUPPORTED, "power spectra need a single-chunk plan");
  hipStream_t st = (hipStream_t)stream;
  mark(p, 0, st);
  s = forward(p, in, st);
  if (s != FDD_OK) return s;
  PhasorArgs a = phasor_args(p);
  a.P = out;
  // the forward transform removed the 8-bit zero point from a chunk filling the whole
  // transform; the removed offset sits in bin 0 only, with phasor 1
  if (p->desc.input == FDD_IN_U8_TIME_MAJOR && p->desc.n_samp == p->L)
    a.dc_add = 128.0f * (float)p->L * (float)p->desc.n_chan;
  hipError_t e;
  if (p->fac_fine > 0) e = launch_phasor_fac(a, p->desc.precision, st);
  else if (p->kernel == "mfma_f16_split") e = launch_phasor_split(a, false, st);
  else if (p->kernel == "mfma_bf16_split") e = launch_phasor_split(a, true, st);
  else e = launch_phasor_valu(a, st);
  if (e != hipSuccess) return hip_fail(e, "phasor-sum launch");
  mark(p, 3, st);
  mark(p, 4, st);
  return FDD_OK;
}

}  // extern "C"
