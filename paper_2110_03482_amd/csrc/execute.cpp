// Stage sequencing of fdd_execute / fdd_power_spectrum (Algorithm 1 without host copies:
// inputs and outputs are device resident, so there is nothing to overlap with PCIe).
#include <algorithm>
#include <mutex>
#include <string>

#include "fdd_internal.h"

using namespace fdd;

// The static scratch of fdd_execute_noalloc (see scratch_address below for how host code reaches it).
static constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

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
  if (p->lin) a.ltab = (const uint4*)(p->d_ws + p->ws.ltab);
  if (p->fac_fine > 0) {
    a.n_coarse = p->fac_coarse;
    a.n_fine = p->fac_fine;
    a.vtab = a.ptab + (size_t)p->desc.n_chan * (size_t)p->fac_coarse;
  }
  return a;
}

// The phasor-sum arguments of one segment: its block of the phase table, its Y rows, and the
// bins 0 .. L/(2d) its shortened inverse reads (all bins for power spectra).
PhasorArgs segment_args(fdd_plan_t p, const PhasorArgs& all, const Segment& sg, bool power) {
  PhasorArgs a = all;
  a.ptab = all.ptab + sg.tab;
  a.lin_j0 = sg.j0;
  a.n_dm = sg.n;
  const size_t rows = (size_t)sg.j0 * (size_t)p->n_chunks * (size_t)p->pitch;
  if (power) {
    a.P = all.P + (size_t)sg.j0 * (size_t)all.n_pow_bins;
  } else {
    a.Yr = all.Yr + rows;
    a.Yi = all.Yi + rows;
    if (all.Yc != nullptr) a.Yc = all.Yc + rows;
    a.n_bins = (int)(p->L / sg.factor / 2 + 1);
  }
  return a;
}

// The direct matrix-core phasor sums (Eq. 7 batched over the overlap-save chunks), one launch
// per chunk group.
hipError_t launch_direct(fdd_plan_t p, const PhasorArgs& a, hipStream_t st) {
  const int ng = chunk_groups(a.n_chunks);
  for (int g = 0; g < ng; ++g) {
    const PhasorArgs t = chunk_group_args(a, g);
    const hipError_t e = p->kernel == "mfma_f32" ? launch_phasor_mfma_f32(t, st)
                                                 : launch_phasor_split(t, p->kernel == "mfma_bf16_split", st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The direct split kernels read X as split words: convert it once for all segments.
hipError_t presplit(fdd_plan_t p, hipStream_t st) {
  if (p->fac_fine > 0 || (p->kernel != "mfma_f16_split" && p->kernel != "mfma_bf16_split")) return hipSuccess;
  return launch_split_x((float2*)(p->d_ws + p->ws.X), (const unsigned int*)(p->d_ws + p->ws.scale),
                        p->desc.n_chan, (int)p->n_chunks, p->pitch, p->kernel == "mfma_bf16_split", st);
}

// Static scratch of fdd_execute_noalloc: the workspace of plans that execute without any
// device allocation.  One array per device, shared by every call on that device, for the whole
// process.  Host code reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in, not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// The scratch's device address on the current device, looked up once per device.
fdd_status scratch_address(uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(FDD_E_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = (uint8_t*)ptr;
  }
  *out = g_scratch[dev];
  return FDD_OK;
}

fdd_status execute_body(fdd_plan_t p, const void* in, float* out, hipStream_t st);

// Chunks k whose input samples [kS, kS + L) all lie inside the data.
int full_chunks(fdd_plan_t p) {
  const int64_t n = p->desc.n_samp;
  if (n < p->L) return 0;
  return (int)std::min<int64_t>((n - p->L) / p->S + 1, p->n_chunks);
}

}  // namespace

extern "C" {

fdd_status fdd_execute(fdd_plan_t p, const void* in, float* out, void* stream) {
  fdd_status s = check_ready(p, in, out);
  if (s != FDD_OK) return s;
  if (p->desc.flags & FDD_PLAN_POWER_ONLY) return fail(FDD_E_UNSUPPORTED, "the plan was made for power spectra only");
  return execute_body(p, in, out, (hipStream_t)stream);
}

fdd_status fdd_execute_noalloc(fdd_plan_t p, const void* in, float* out, void* stream) {
  if (p == nullptr) return fail(FDD_E_INVALID, "null plan");
  if (in == nullptr || out == nullptr) return fail(FDD_E_INVALID, "null input or output");
  if (p->desc.flags & FDD_PLAN_POWER_ONLY) return fail(FDD_E_UNSUPPORTED, "the plan was made for power spectra only");
  if (p->ws.total > kNoallocScratchBytes)
    return fail(FDD_E_UNSUPPORTED, "the plan's workspace (" + std::to_string(p->ws.total) +
                                       " bytes) exceeds the static scratch of " + std::to_string(kNoallocScratchBytes) +
                                       " bytes of fdd_execute_noalloc");
  uint8_t* ws = nullptr;
  fdd_status s = scratch_address(&ws);
  if (s != FDD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = upload_tables_async(p, ws, st);
  if (e != hipSuccess) return hip_fail(e, "table upload into the static scratch");
  uint8_t* const own = p->d_ws;
  p->d_ws = ws;                            // the kernels address the workspace through the plan
  s = execute_body(p, in, out, st);
  p->d_ws = own;
  return s;
}

}  // extern "C"

namespace {

fdd_status execute_body(fdd_plan_t p, const void* in, float* out, hipStream_t st) {
  fdd_status s;
  mark(p, 0, st);
  s = forward(p, in, st);
  if (s != FDD_OK) return s;
  PhasorArgs all = phasor_args(p);
  all.Yr = (float*)(p->d_ws + p->ws.Yr);
  all.Yi = (float*)(p->d_ws + p->ws.Yi);
  if (p->facw_nt > 0) all.Yc = (float2*)(p->d_ws + p->ws.Yr);   // both planes' memory, interleaved
  hipError_t e = presplit(p, st);
  if (e != hipSuccess) return hip_fail(e, "split launch");
  for (const Segment& sg : p->segs) {
    const PhasorArgs a = segment_args(p, all, sg, false);
    if (p->facw_nt > 0) e = launch_phasor_facw(a, p->desc.precision, p->facw_nt, st);
    else if (p->fac_fine > 0) e = launch_phasor_fac(a, p->desc.precision, st);
    else if (p->kernel == "mfma_f32" || p->kernel == "mfma_f16_split" || p->kernel == "mfma_bf16_split")
      e = launch_direct(p, a, st);
    else e = launch_phasor_valu(a, st);
    if (e != hipSuccess) return hip_fail(e, "phasor-sum launch");
  }
  mark(p, 3, st);
  for (const Segment& sg : p->segs) {
    const PhasorArgs a = segment_args(p, all, sg, false);
    int lg = 0;
    while ((1 << lg) < sg.factor) ++lg;
    FftArgs f;
    f.Yr = a.Yr;
    f.Yi = a.Yi;
    f.Yc = a.Yc;
    f.out = out + sg.out_off;
    f.twL = (const float2*)(p->d_ws + (sg.factor == 1 ? p->ws.tw : sg.tw));
    f.n_samp = sg.n_out;
    f.stride = p->S / sg.factor;
    f.keep = p->desc.single_chunk ? sg.n_out : p->S / sg.factor;
    f.pitch = p->pitch;
    f.n_chunks = (int)p->n_chunks;
    f.n_rows = sg.n;
    f.add_full = p->desc.input == FDD_IN_U8_TIME_MAJOR ? 128.0f * (float)p->desc.n_chan : 0.0f;
    f.log_n = p->log_len - 1 - lg;
    if (sg.factor > 1) {               // length L/d, scaled by 1/L; zero point by full-length chunks
      f.inv_n = 2.0f / (float)p->L;
      f.full_chunks = full_chunks(p);
    }
    e = f.log_n > kMaxBlockLogN
            ? launch_c2r_long(f, (float2*)(p->d_ws + p->ws.Z), (float2*)(p->d_ws + p->ws.Yr), st)
            : launch_c2r(f.log_n, f, st);
    if (e != hipSuccess) return hip_fail(e, "inverse FFT launch");
  }
  mark(p, 4, st);
  return FDD_OK;
}

}  // namespace

extern "C" {

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
  PhasorArgs all = phasor_args(p);
  all.P = out;
  // the forward transform removed the 8-bit zero point from a chunk filling the whole
  // transform; the removed offset sits in bin 0 only, with phasor 1
  if (p->desc.input == FDD_IN_U8_TIME_MAJOR && p->desc.n_samp == p->L)
    all.dc_add = 128.0f * (float)p->L * (float)p->desc.n_chan;
  hipError_t e = presplit(p, st);
  if (e != hipSuccess) return hip_fail(e, "split launch");
  for (const Segment& sg : p->segs) {
    const PhasorArgs a = segment_args(p, all, sg, true);
    if (p->fac_fine > 0) e = launch_phasor_fac(a, p->desc.precision, st);
    else if (p->kernel == "mfma_f16_split") e = launch_phasor_split(a, false, st);
    else if (p->kernel == "mfma_bf16_split") e = launch_phasor_split(a, true, st);
    else e = launch_phasor_valu(a, st);
    if (e != hipSuccess) return hip_fail(e, "phasor-sum launch");
  }
  mark(p, 3, st);
  mark(p, 4, st);
  return FDD_OK;
}

fdd_status fdd_power_spectrum_scaled(fdd_plan_t p, const void* in, float* out, void* stream) {
  fdd_status s = check_ready(p, in, out);
  if (s != FDD_OK) return s;
  if (!p->scaled) return fail(FDD_E_UNSUPPORTED, "the plan was not made with FDD_PLAN_SCALED_DM");
  hipStream_t st = (hipStream_t)stream;
  mark(p, 0, st);
  s = forward(p, in, st);
  if (s != FDD_OK) return s;
  const int prec = p->desc.precision;
  const bool split = prec != FDD_FP32;
  // low bins, exact as fdd_power_spectrum; their tiles end at f_min, a multiple of 64.  The
  // direct split kernels read X split in place, the others read plain X: order the launches
  // so that every kernel sees the form it reads.
  const bool low_reads_split = p->fac_fine == 0 && (p->kernel == "mfma_f16_split" || p->kernel == "mfma_bf16_split");
  auto low_bins = [&]() -> hipError_t {
    if (p->sc_fmin <= 0) return hipSuccess;
    PhasorArgs all = phasor_args(p);
    all.P = out;
    if (p->desc.input == FDD_IN_U8_TIME_MAJOR && p->desc.n_samp == p->L)
      all.dc_add = 128.0f * (float)p->L * (float)p->desc.n_chan;
    for (const Segment& sg : p->segs) {
      PhasorArgs a = segment_args(p, all, sg, true);
      a.n_bins = p->sc_fmin;
      hipError_t e;
      if (p->fac_fine > 0) e = launch_phasor_fac(a, prec, st);
      else if (p->kernel == "mfma_f16_split") e = launch_phasor_split(a, false, st);
      else if (p->kernel == "mfma_bf16_split") e = launch_phasor_split(a, true, st);
      else e = launch_phasor_valu(a, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  float2* X = (float2*)(p->d_ws + p->ws.X);
  const unsigned int* l1max = (const unsigned int*)(p->d_ws + p->ws.scale);
  hipError_t e = hipSuccess;
  if (!low_reads_split) e = low_bins();
  if (e != hipSuccess) return hip_fail(e, "phasor-sum launch");
  if (split || low_reads_split) {
    e = launch_split_x(X, l1max, p->desc.n_chan, (int)p->n_chunks, p->pitch, prec == FDD_BF16_SPLIT, st);
    if (e != hipSuccess) return hip_fail(e, "split launch");
  }
  if (low_reads_split) e = low_bins();
  if (e != hipSuccess) return hip_fail(e, "phasor-sum launch");
  ScaledArgs g;
  g.X = X;
  g.ctab = (const uint4*)(p->d_ws + p->ws.ctab);
  g.Q = (float*)(p->d_ws + p->ws.Q);
  g.n_chan = p->desc.n_chan;
  g.n_rows = p->desc.n_dm + 2 * kScaledHalo;
  g.n_blocks = p->sc_blocks;
  g.f_min = p->sc_fmin;
  g.pitch = p->pitch;
  g.q_pitch = (int64_t)p->sc_blocks * kScaledBlock;
  e = launch_phasor_scaled(g, prec, l1max, st);
  if (e != hipSuccess) return hip_fail(e, "scaled-DM phasor-sum launch");
  ResampleArgs r;
  r.Q = g.Q;
  r.P = out;
  r.dms = (const double*)(p->d_ws + p->ws.dmv);
  r.dm0 = p->grid_dm0;
  r.step = p->grid_step;
  r.n_dm = p->desc.n_dm;
  r.n_rows = g.n_rows;
  r.f_min = p->sc_fmin;
  r.n_pow_bins = (int)(p->L / 2);
  r.q_pitch = g.q_pitch;
  e = launch_scaled_resample(r, st);
  if (e != hipSuccess) return hip_fail(e, "DM resampling launch");
  mark(p, 3, st);
  mark(p, 4, st);
  return FDD_OK;
}

}  // extern "C"
