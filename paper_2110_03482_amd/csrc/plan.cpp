// Host planner and C ABI of the Fourier-domain dedispersion library.
//
// The planner validates a descriptor, forms the float64 delay per unit DM of every channel
// (Eq. 1 divided by the sampling time), sizes the overlap-save chunking (Sec. 2.2: at least
// the maximum delay is discarded at the end of every transformed series), builds the
// twiddle table and lays out one workspace.  Execution enqueues, on one stream and without
// host synchronisation, the stages of Algorithm 1: transpose/unpack (8-bit input only),
// forward FFT per channel and chunk, phasor sum, and either the inverse FFT with scaling and
// discard, or power spectra.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>

#include "fdd_internal.h"

namespace fdd {

namespace {
thread_local std::string g_last_error;

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool mul_ok(size_t a, size_t b, size_t* out) {
  if (a != 0 && b > std::numeric_limits<size_t>::max() / a) return false;
  *out = a * b;
  return true;
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

fdd_status fail(fdd_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

fdd_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return FDD_E_DEVICE;
}

// Eq. 1 in samples per unit DM; the operation order is part of the ABI contract.
static double kappa_of(double f_mhz, double ref_mhz, double tsamp_s) {
  const double inv_f2 = 1.0 / (f_mhz * f_mhz);
  const double inv_ref2 = 1.0 / (ref_mhz * ref_mhz);
  return (FDD_K_DM * (inv_f2 - inv_ref2)) / tsamp_s;
}

// Per (channel, DM): the 64-bit phase increment per Fourier bin, frac(tau / L) 2^64 (exact
// (d mod L) << (64 - log2 L) for nearest-sample delays), and the unit phasor of one bin step,
// exp(+2 pi i inc / 2^64), evaluated in float64.  Channel-major, so that the DM lanes of a
// kernel read consecutive entries.
static void phase_rows(const fdd_plan_s* p, const double* dms, size_t nd, std::vector<uint4>* out) {
  const size_t nc = p->kappa.size();
  out->resize(nc * nd);
  const int lg = p->log_len;
  for (size_t c = 0; c < nc; ++c) {
    for (size_t m = 0; m < nd; ++m) {
      const double tau = dms[m] * p->kappa[c];
      uint32_t hi = 0, lo = 0;
      if (p->desc.delay_mode == FDD_DELAY_ROUND) {
        const double d = std::floor(tau + 0.5);
        const double dl = d - std::ldexp(std::floor(std::ldexp(d, -lg)), lg);   // d mod L, exact
        hi = (uint32_t)dl << (32 - lg);
      } else {
        const double v = std::ldexp(tau, -lg);
        const double fr = v - std::floor(v);
        const double s = std::ldexp(fr, 32);
        const double h = std::floor(s);
        const double rem = std::ldexp(s - h, 32);
        hi = (uint32_t)h;
        lo = (uint32_t)std::min(std::floor(rem), 4294967295.0);
      }
      const double ang = 2.0 * M_PI * (std::ldexp((double)hi, -32) + std::ldexp((double)lo, -64));
      uint4 e;
      e.x = lo;
      e.y = hi;
      float cs = (float)std::cos(ang), sn = (float)std::sin(ang);
      std::memcpy(&e.z, &cs, 4);
      std::memcpy(&e.w, &sn, 4);
      (*out)[c * nd + m] = e;
    }
  }
}

void phase_table(const fdd_plan_s* p, std::vector<uint4>* out) { phase_rows(p, p->dms.data(), p->dms.size(), out); }

void phase_table_rows(const fdd_plan_s* p, int j0, int n, std::vector<uint4>* out) {
  phase_rows(p, p->dms.data() + j0, (size_t)n, out);
}

// DM-factorised tables: coarse trials DM_0 + a B dDM (channel-major [n_chan][A]) followed by
// fine offsets b dDM ([n_chan][B]); the delays of trial a B + b add up to DM_j kappa_c.
void factor_tables(const fdd_plan_s* p, int fine, int coarse, double dm0, double step, std::vector<uint4>* out) {
  std::vector<double> cdm((size_t)coarse), fdm((size_t)fine);
  for (int a = 0; a < coarse; ++a) cdm[(size_t)a] = dm0 + (double)a * fine * step;
  for (int b = 0; b < fine; ++b) fdm[(size_t)b] = (double)b * step;
  std::vector<uint4> tb;
  phase_rows(p, cdm.data(), cdm.size(), out);
  phase_rows(p, fdm.data(), fdm.size(), &tb);
  out->insert(out->end(), tb.begin(), tb.end());
}

// A DM list DM_j = DM_0 + j dDM (to 1e-12 of the largest DM), as numpy.linspace makes it.  The
// kernels that use the grid form delays from DM_0 and dDM: a deviation of 1e-12 DM_max moves a
// phase by at most 1e-12 pi tau_max radians (5e-8 at tau_max = 15000 samples).
bool uniform_grid(const std::vector<double>& dms, double* dm0, double* step) {
  const size_t n = dms.size();
  if (n < 2) return false;
  *dm0 = dms[0];
  *step = (dms[n - 1] - dms[0]) / (double)(n - 1);
  if (!(*step > 0.0)) return false;
  double big = 0.0;
  for (double v : dms) big = std::max(big, std::fabs(v));
  const double tol = 1e-12 * big;
  for (size_t j = 0; j < n; ++j)
    if (std::fabs(dms[j] - (*dm0 + (double)j * *step)) > tol) return false;
  return true;
}

void twiddle_table(int64_t L, std::vector<float2>* out) {
  out->resize((size_t)L);
  for (int64_t j = 0; j < L; ++j) {
    // exp(-2 pi i j / L), evaluated in float64
    const double a = -2.0 * M_PI * (double)j / (double)L;
    (*out)[(size_t)j] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
}

// frac(tau / L) as a 64-bit turn fraction {lo, hi} (any sign of tau), evaluated in float64.
static void turn_fraction(double tau, int lg, uint32_t* lo, uint32_t* hi) {
  const double v = std::ldexp(tau, -lg);
  const double fr = v - std::floor(v);
  const double s = std::ldexp(fr, 32);
  const double h = std::floor(s);
  *hi = (uint32_t)std::min(h, 4294967295.0);
  *lo = (uint32_t)std::min(std::floor(std::ldexp(s - h, 32)), 4294967295.0);
}

// Scaled-DM increments per channel: row q of the scaled grid has the delay
// (DM_0 + (q - halo) dDM) kappa_c, i.e. the turn fraction per bin inc_a + q inc_d.
static void scaled_table(const fdd_plan_s* p, std::vector<uint4>* out) {
  out->resize(p->kappa.size());
  const double first = p->grid_dm0 - (double)kScaledHalo * p->grid_step;
  for (size_t c = 0; c < p->kappa.size(); ++c) {
    uint4 e;
    turn_fraction(first * p->kappa[c], p->log_len, &e.x, &e.y);
    turn_fraction(p->grid_step * p->kappa[c], p->log_len, &e.z, &e.w);
    (*out)[c] = e;
  }
}

// Linear increments per channel for exact delays on a uniform grid DM_j = DM_0 + j dDM: the turn
// fraction per bin of trial j is inc0 + j d (mod 2^64), with inc0 from DM_0 kappa_c and d from
// dDM kappa_c (Eq. 1 is linear in DM).
static void linear_table(const fdd_plan_s* p, std::vector<uint4>* out) {
  out->resize(p->kappa.size());
  for (size_t c = 0; c < p->kappa.size(); ++c) {
    uint4 e;
    turn_fraction(p->grid_dm0 * p->kappa[c], p->log_len, &e.x, &e.y);
    turn_fraction(p->grid_step * p->kappa[c], p->log_len, &e.z, &e.w);
    (*out)[c] = e;
  }
}

// Nearest-sample delays d = floor(tau + 1/2) of every (channel, DM), channel-major.
static void delay_table(const fdd_plan_s* p, std::vector<int>* out) {
  const size_t nc = p->kappa.size(), nd = p->dms.size();
  out->resize(nc * nd);
  for (size_t c = 0; c < nc; ++c)
    for (size_t m = 0; m < nd; ++m) (*out)[c * nd + m] = (int)std::floor(p->dms[m] * p->kappa[c] + 0.5);
}

// The plan's small tables (twiddles, phase and delay tables, scaled-DM tables), computed once on
// the host at plan time and kept with the plan: each is (workspace byte offset, bytes).
static void build_host_tables(fdd_plan_s* p) {
  const WorkspaceLayout& w = p->ws;
  p->htabs.clear();
  auto keep = [&](size_t off, const void* src, size_t bytes) {
    std::vector<uint8_t> b(bytes);
    std::memcpy(b.data(), src, bytes);
    p->htabs.emplace_back(off, std::move(b));
  };
  std::vector<float2> tw;
  twiddle_table(p->L, &tw);
  keep(w.tw, tw.data(), tw.size() * sizeof(float2));
  for (const Segment& sg : p->segs) {
    if (sg.factor == 1) continue;
    twiddle_table(p->L / sg.factor, &tw);   // several segments may share a factor: same bytes
    keep(sg.tw, tw.data(), tw.size() * sizeof(float2));
  }
  std::vector<uint4> tab;
  if (p->fac_fine > 0) {
    factor_tables(p, p->fac_fine, p->fac_coarse, p->fac_dm0, p->fac_step, &tab);
  } else {
    std::vector<uint4> part;
    for (const Segment& sg : p->segs) {
      phase_table_rows(p, sg.j0, sg.n, &part);
      tab.insert(tab.end(), part.begin(), part.end());
    }
  }
  keep(w.ptab, tab.data(), tab.size() * sizeof(uint4));
  std::vector<int> dt;
  delay_table(p, &dt);
  keep(w.dtab, dt.data(), w.dtab_bytes);
  if (p->scaled) {
    std::vector<uint4> ct;
    scaled_table(p, &ct);
    keep(w.ctab, ct.data(), w.ctab_bytes);
    keep(w.dmv, p->dms.data(), w.dmv_bytes);
  }
  if (p->lin) {
    std::vector<uint4> lt;
    linear_table(p, &lt);
    keep(w.ltab, lt.data(), w.ltab_bytes);
  }
}

static fdd_status upload_tables(fdd_plan_s* p) {
  for (const auto& t : p->htabs) {
    const hipError_t e = hipMemcpy(p->d_ws + t.first, t.second.data(), t.second.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan tables)");
  }
  return FDD_OK;
}

hipError_t upload_tables_async(const fdd_plan_s* p, uint8_t* dst, hipStream_t st) {
  for (const auto& t : p->htabs) {
    const hipError_t e = hipMemcpyAsync(dst + t.first, t.second.data(), t.second.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static fdd_status layout(fdd_plan_s* p) {
  WorkspaceLayout& w = p->ws;
  const fdd_plan_desc& d = p->desc;
  size_t off = 0, tmp = 0;
  auto put = [&](size_t* at, size_t bytes) {
    *at = off;
    off = align_up(off + bytes);
  };
  // twiddles: L entries, then one table of L/d entries per distinct factor d > 1
  {
    std::vector<std::pair<int, size_t>> at;   // factor -> byte offset within the region
    size_t tb = align_up((size_t)p->L * sizeof(float2));
    for (Segment& sg : p->segs) {
      if (sg.factor == 1) continue;
      size_t o = 0;
      bool seen = false;
      for (const auto& pr : at)
        if (pr.first == sg.factor) {
          o = pr.second;
          seen = true;
        }
      if (!seen) {
        o = tb;
        at.push_back({sg.factor, o});
        tb = align_up(tb + (size_t)(p->L / sg.factor) * sizeof(float2));
      }
      sg.tw = o;                                // made absolute below
    }
    w.tw_bytes = tb;
  }
  put(&w.tw, w.tw_bytes);
  for (Segment& sg : p->segs)
    if (sg.factor != 1) sg.tw += w.tw;
  const size_t rows_tab = std::max((size_t)d.n_dm, (size_t)p->fac_coarse + (size_t)p->fac_fine);
  if (!mul_ok((size_t)d.n_chan * rows_tab, sizeof(uint4), &w.ptab_bytes))
    return fail(FDD_E_NOMEM, "phase table size overflows");
  put(&w.ptab, w.ptab_bytes);
  w.scale_bytes = (size_t)p->n_chunks * sizeof(float);
  put(&w.scale, w.scale_bytes);
  if (d.input == FDD_IN_U8_TIME_MAJOR) {
    if (!mul_ok((size_t)d.n_chan, (size_t)d.n_samp, &w.xt_bytes)) return fail(FDD_E_NOMEM, "input size overflows");
    put(&w.xt, w.xt_bytes);
  }
  size_t rows = 0;
  if (!mul_ok((size_t)d.n_chan, (size_t)p->n_chunks, &rows) || !mul_ok(rows, (size_t)p->pitch, &tmp) ||
      !mul_ok(tmp, sizeof(float2), &w.X_bytes))
    return fail(FDD_E_NOMEM, "Fourier-domain input size overflows");
  put(&w.X, w.X_bytes);
  const bool power_only = (d.flags & FDD_PLAN_POWER_ONLY) != 0;
  if (!power_only) {
    if (!mul_ok((size_t)d.n_dm, (size_t)p->n_chunks, &rows) || !mul_ok(rows, (size_t)p->pitch, &tmp) ||
        !mul_ok(tmp, sizeof(float), &w.Y_bytes))
      return fail(FDD_E_NOMEM, "Fourier-domain output size overflows");
    put(&w.Yr, w.Y_bytes);
    put(&w.Yi, w.Y_bytes);
  }
  if (p->log_len - 1 > kMaxBlockLogN) {
    // long transforms: one complex work buffer, sized for the forward (channels) and, unless
    // power only, the inverse (DMs) series; the inverse's second buffer is the spent Y memory
    const size_t series = (size_t)(power_only ? d.n_chan : std::max(d.n_chan, d.n_dm)) * (size_t)p->n_chunks;
    if (!mul_ok(series, (size_t)(p->L / 2) * sizeof(float2), &w.Z_bytes))
      return fail(FDD_E_NOMEM, "work buffer size overflows");
    put(&w.Z, w.Z_bytes);
    w.l1_bytes = (size_t)d.n_chan * (size_t)p->n_chunks * sizeof(float);
    put(&w.l1, w.l1_bytes);
  }
  if (!mul_ok((size_t)d.n_chan * (size_t)d.n_dm, sizeof(int), &w.dtab_bytes))
    return fail(FDD_E_NOMEM, "delay table size overflows");
  put(&w.dtab, w.dtab_bytes);
  if (p->lin) {
    w.ltab_bytes = (size_t)d.n_chan * sizeof(uint4);
    put(&w.ltab, w.ltab_bytes);
  }
  if (p->scaled) {
    w.ctab_bytes = (size_t)d.n_chan * sizeof(uint4);
    put(&w.ctab, w.ctab_bytes);
    w.dmv_bytes = (size_t)d.n_dm * sizeof(double);
    put(&w.dmv, w.dmv_bytes);
    const size_t rows = (size_t)d.n_dm + 2 * kScaledHalo;
    if (!mul_ok(rows * (size_t)p->sc_blocks * kScaledBlock, sizeof(float), &w.Q_bytes))
      return fail(FDD_E_NOMEM, "scaled-DM buffer size overflows");
    put(&w.Q, w.Q_bytes);
  }
  w.total = off;
  return FDD_OK;
}

}  // namespace fdd

using namespace fdd;

extern "C" {

const char* fdd_version(void) { return "fdd-gfx950 0.1"; }

const char* fdd_status_string(fdd_status s) {
  switch (s) {
    case FDD_OK: return "ok";
    case FDD_E_INVALID: return "invalid argument";
    case FDD_E_OVERLAP: return "overlap does not cover the maximum delay";
    case FDD_E_UNSUPPORTED: return "unsupported configuration";
    case FDD_E_NOMEM: return "out of memory";
    case FDD_E_DEVICE: return "device error";
    case FDD_E_WORKSPACE: return "workspace missing or too small";
  }
  return "unknown status";
}

const char* fdd_last_error(void) { return g_last_error.c_str(); }

fdd_status fdd_dispersion_delays(int32_t n_chan, const double* freqs, double ref, double tsamp, double dm,
                                 double* tau_out) {
  if (n_chan < 1 || freqs == nullptr || tau_out == nullptr) return fail(FDD_E_INVALID, "null or empty arguments");
  if (!(tsamp > 0.0) || !(ref > 0.0) || !std::isfinite(dm)) return fail(FDD_E_INVALID, "bad tsamp, reference or DM");
  for (int32_t c = 0; c < n_chan; ++c) tau_out[c] = dm * kappa_of(freqs[c], ref, tsamp);
  return FDD_OK;
}

fdd_status fdd_smearing_factors(int32_t n_chan, const double* freqs, double tsamp, int32_t n_dm, const double* dm,
                                int32_t max_factor, int32_t* out) {
  if (n_chan < 1 || n_dm < 0 || freqs == nullptr || (n_dm > 0 && (dm == nullptr || out == nullptr)))
    return fail(FDD_E_INVALID, "null or empty arguments");
  if (!(tsamp > 0.0) || !std::isfinite(tsamp)) return fail(FDD_E_INVALID, "tsamp must be finite and > 0");
  if (max_factor < 1 || (max_factor & (max_factor - 1)) != 0) return fail(FDD_E_INVALID, "max_factor must be a power of two >= 1");
  std::vector<double> f(freqs, freqs + n_chan);
  for (double v : f)
    if (!(v > 0.0) || !std::isfinite(v)) return fail(FDD_E_INVALID, "channel frequencies must be finite and > 0");
  std::sort(f.begin(), f.end());
  double w = 0.0;
  for (size_t c = 1; c < f.size(); ++c) {
    const double g = f[c] - f[c - 1];
    if (g > 0.0 && (w == 0.0 || g < w)) w = g;
  }
  // Eq. 1 across the lowest channel, per unit DM, in samples
  double per_dm = 0.0;
  if (w > 0.0 && f[0] - 0.5 * w > 0.0) {
    const double lo = f[0] - 0.5 * w, hi = f[0] + 0.5 * w;
    per_dm = FDD_K_DM * (1.0 / (lo * lo) - 1.0 / (hi * hi)) / tsamp;
  }
  for (int32_t m = 0; m < n_dm; ++m) {
    if (!(dm[m] >= 0.0) || !std::isfinite(dm[m])) return fail(FDD_E_INVALID, "DMs must be finite and >= 0");
    const double sm = dm[m] * per_dm;
    int32_t d = 1;
    while (d < max_factor && 2.0 * d <= sm) d *= 2;
    out[m] = d;
  }
  return FDD_OK;
}

fdd_status fdd_plan(const fdd_plan_desc* desc, fdd_plan_t* out) {
  if (desc == nullptr || out == nullptr) return fail(FDD_E_INVALID, "null descriptor or output");
  *out = nullptr;
  const fdd_plan_desc& d = *desc;
  if (d.n_chan < 1 || d.n_dm < 1 || d.n_samp < 1) return fail(FDD_E_INVALID, "n_chan, n_dm and n_samp must be >= 1");
  if (d.chan_freq_mhz == nullptr || d.dm == nullptr) return fail(FDD_E_INVALID, "null frequency or DM array");
  if (!(d.tsamp_s > 0.0) || !std::isfinite(d.tsamp_s)) return fail(FDD_E_INVALID, "tsamp must be finite and > 0");
  if (!(d.ref_freq_mhz > 0.0) || !std::isfinite(d.ref_freq_mhz)) return fail(FDD_E_INVALID, "bad reference frequency");
  if (d.input != FDD_IN_U8_TIME_MAJOR && d.input != FDD_IN_F32_CHAN_MAJOR) return fail(FDD_E_INVALID, "bad input kind");
  if (d.precision < FDD_FP32 || d.precision > FDD_BF16_SPLIT) return fail(FDD_E_INVALID, "bad precision");
  if (d.delay_mode != FDD_DELAY_EXACT && d.delay_mode != FDD_DELAY_ROUND) return fail(FDD_E_INVALID, "bad delay mode");
  const int64_t L = d.chunk_len;
  if (L < 64 || (L & (L - 1)) != 0) return fail(FDD_E_INVALID, "chunk_len must be a power of two >= 64");
  if (L > (int64_t(1) << 22)) return fail(FDD_E_UNSUPPORTED, "chunk_len above 2^22 is not supported");
  for (int32_t c = 0; c < d.n_chan; ++c) {
    const double f = d.chan_freq_mhz[c];
    if (!(f > 0.0) || !std::isfinite(f)) return fail(FDD_E_INVALID, "channel frequencies must be finite and > 0");
    if (f > d.ref_freq_mhz) return fail(FDD_E_INVALID, "a channel lies above the reference frequency (negative delay)");
  }
  for (int32_t m = 0; m < d.n_dm; ++m) {
    const double v = d.dm[m];
    if (!(v >= 0.0) || !std::isfinite(v)) return fail(FDD_E_INVALID, "DMs must be finite and >= 0");
  }
  int32_t max_ds = 1;
  if (d.downsample != nullptr) {
    for (int32_t m = 0; m < d.n_dm; ++m) {
      const int32_t f = d.downsample[m];
      if (f < 1 || (f & (f - 1)) != 0 || (int64_t)f * 64 > L)
        return fail(FDD_E_INVALID, "down-sampling factors must be powers of two from 1 to chunk_len/64");
      max_ds = std::max(max_ds, f);
    }
    if (max_ds > 1 && (d.flags & FDD_PLAN_POWER_ONLY))
      return fail(FDD_E_INVALID, "down-sampling shortens the inverse transform; a power-only plan has none");
    if (max_ds > 1 && L > (int64_t(1) << (kMaxBlockLogN + 1)))
      return fail(FDD_E_UNSUPPORTED, "down-sampled output needs chunk_len <= 2^16");
  }

  fdd_plan_s* p = new (std::nothrow) fdd_plan_s();
  if (p == nullptr) return fail(FDD_E_NOMEM, "host allocation failed");
  p->desc = d;
  p->freqs.assign(d.chan_freq_mhz, d.chan_freq_mhz + d.n_chan);
  p->dms.assign(d.dm, d.dm + d.n_dm);
  p->ds.assign((size_t)d.n_dm, 1);
  if (d.downsample != nullptr) p->ds.assign(d.downsample, d.downsample + d.n_dm);
  p->desc.chan_freq_mhz = p->freqs.data();
  p->desc.dm = p->dms.data();
  p->desc.downsample = p->ds.data();
  p->kappa.resize((size_t)d.n_chan);
  double kmax = 0.0, dmax = 0.0;
  for (int32_t c = 0; c < d.n_chan; ++c) {
    p->kappa[(size_t)c] = kappa_of(p->freqs[(size_t)c], d.ref_freq_mhz, d.tsamp_s);
    kmax = std::max(kmax, p->kappa[(size_t)c]);
  }
  for (int32_t m = 0; m < d.n_dm; ++m) dmax = std::max(dmax, p->dms[(size_t)m]);
  // tau = DM * kappa is monotone in both factors (both >= 0), so this is the largest delay.
  p->max_tau = dmax * kmax;
  p->L = L;
  p->log_len = 0;
  while ((int64_t(1) << p->log_len) < L) ++p->log_len;
  p->n_bins = L / 2 + 1;
  p->pitch = (p->n_bins + 63) / 64 * 64;
  const int64_t need = (int64_t)std::ceil(p->max_tau);
  if (d.single_chunk) {
    if (d.n_samp > L) {
      delete p;
      return fail(FDD_E_INVALID, "single-chunk mode needs n_samp <= chunk_len");
    }
    p->S = L;
    p->D = 0;
    p->n_chunks = 1;
  } else {
    p->D = d.overlap > 0 ? d.overlap : need;
    if (p->D < need) {
      delete p;
      return fail(FDD_E_OVERLAP, "overlap " + std::to_string(d.overlap) + " is shorter than ceil(max delay) = " +
                                     std::to_string(need));
    }
    if (p->D >= L) {
      delete p;
      return fail(FDD_E_OVERLAP, "overlap must be shorter than chunk_len; use a longer chunk");
    }
    // every down-sampled chunk keeps S/d whole output samples
    if ((L - p->D) % max_ds != 0) {
      if (d.overlap > 0) {
        delete p;
        return fail(FDD_E_INVALID, "chunk_len - overlap must be a multiple of the largest down-sampling factor " +
                                       std::to_string(max_ds));
      }
      p->D = L - (L - p->D) / max_ds * max_ds;
      if (p->D >= L) {
        delete p;
        return fail(FDD_E_OVERLAP, "no kept stride is a multiple of the largest down-sampling factor; use a longer chunk");
      }
    }
    p->S = L - p->D;
    p->n_chunks = (d.n_samp + p->S - 1) / p->S;
  }
  // runs of equal down-sampling factors, their output rows and phase-table blocks
  for (int32_t m = 0; m < d.n_dm;) {
    Segment sg;
    sg.j0 = m;
    sg.factor = p->ds[(size_t)m];
    while (m < d.n_dm && p->ds[(size_t)m] == sg.factor) ++m;
    sg.n = m - sg.j0;
    sg.n_out = (d.n_samp + sg.factor - 1) / sg.factor;
    sg.out_off = p->out_total;
    sg.tab = (size_t)d.n_chan * (size_t)sg.j0;
    p->out_total += (int64_t)sg.n * sg.n_out;
    p->segs.push_back(sg);
  }
  if (p->segs.size() > 256) {
    delete p;
    return fail(FDD_E_UNSUPPORTED, "more than 256 runs of equal down-sampling factors; sort the DMs by factor");
  }
  p->n_valid = d.n_samp - need > 0 ? d.n_samp - need : 0;
  if (p->n_chunks > 65535 || d.n_dm > 65535 * 4 || d.n_chan > 65535) {
    delete p;
    return fail(FDD_E_UNSUPPORTED, "grid dimension limit exceeded");
  }
  // direct matrix-core kernels, over chunk groups of at most kDirectMaxChunks when there are more
  p->kernel = (d.precision == FDD_FP32 && phasor_mfma_f32_supported(chunk_group_max((int)p->n_chunks)) &&
               phasor_mfma_f32_window_ok(p->n_chunks, p->pitch))
                  ? "mfma_f32" : "valu";
  // tuning override of the matrix-core tile shape
  if (const char* tv = std::getenv("FDD_TILE_VARIANT")) {
    const int v = std::atoi(tv);
    if (v >= 0 && v <= 4) p->tile_variant = v;
  }
  if (d.precision == FDD_FP16_SPLIT || d.precision == FDD_BF16_SPLIT)
    p->kernel = !phasor_split_supported(chunk_group_max((int)p->n_chunks)) ? ""
                : d.precision == FDD_FP16_SPLIT ? "mfma_f16_split" : "mfma_bf16_split";
  // DM factorisation: exact delays on a uniform DM grid, few chunks (where the direct kernels
  // leave most matrix-core columns empty).  FDD_FACTOR=0 disables it, FDD_FACTOR=all extends
  // it to every chunk count the factorised kernels take.
  {
    const char* fe = std::getenv("FDD_FACTOR");
    const bool off = fe != nullptr && std::strcmp(fe, "0") == 0;
    const bool all = fe != nullptr && std::strcmp(fe, "all") == 0;
    const int fine = phasor_fac_fine((int)p->n_chunks);
    double dm0 = 0.0, step = 0.0;
    if (!off && d.delay_mode == FDD_DELAY_EXACT && fine > 0 && (all || p->n_chunks <= 2) && max_ds == 1 &&
        uniform_grid(p->dms, &dm0, &step)) {
      p->fac_fine = fine;
      p->fac_coarse = (d.n_dm + fine - 1) / fine;
      p->fac_dm0 = dm0;
      p->fac_step = step;
      p->kernel = d.precision == FDD_FP32 ? "fac_f32" : d.precision == FDD_FP16_SPLIT ? "fac_f16_split" : "fac_bf16_split";
    }
    // Overlap-save plans: the chunked factorised kernels, in which every coarse phasor serves
    // 2 B N matrix-core columns instead of the direct kernels' 2 N.  They need the inverse's
    // interleaved Y (so not for power-only plans) and a one-workgroup inverse transform.
    // FDD_FACTOR=direct keeps the direct kernels.  In FP32 the direct matrix-core kernel is
    // the faster one on the paper-shaped workload (its phasor generation is a small share of
    // the FP32 products), so FP32 plans take the chunked factorised kernel only with
    // FDD_FACTOR=wide.
    const bool direct = fe != nullptr && std::strcmp(fe, "direct") == 0;
    const bool wide = fe != nullptr && std::strcmp(fe, "wide") == 0;
    if (!off && !direct && (d.precision != FDD_FP32 || wide) && p->fac_fine == 0 && d.delay_mode == FDD_DELAY_EXACT &&
        !d.single_chunk && max_ds == 1 &&
        !(d.flags & FDD_PLAN_POWER_ONLY) && p->log_len - 1 <= kMaxBlockLogN && p->n_chunks >= 3 &&
        uniform_grid(p->dms, &dm0, &step)) {
      const FacwChoice ch = facw_choose(d.n_dm, (int)p->n_chunks);
      if (ch.fine > 0 && ch.eff >= 0.7) {
        p->fac_fine = ch.fine;
        p->fac_coarse = ch.coarse;
        p->facw_nt = ch.nt;
        p->fac_dm0 = dm0;
        p->fac_step = step;
        p->kernel = d.precision == FDD_FP32 ? "facw_f32" : d.precision == FDD_FP16_SPLIT ? "facw_f16_split"
                                                                                          : "facw_bf16_split";
      }
    }
  }
  if (p->kernel.empty()) {
    delete p;
    return fail(FDD_E_UNSUPPORTED, "no phasor-sum kernel takes this plan");
  }
  // FDD_PHASE_TABLE=linear: the direct FP32 kernel on a uniform grid with exact delays derives
  // each trial's increment from two per-channel values instead of reading the [n_chan][n_dm]
  // phase table.  That removes the table's re-reads from memory but adds one sin/cos
  // evaluation per seed; on the paper-shaped workload the kernel is bound by instruction issue,
  // not by those reads, and the table is the faster of the two.
  {
    const char* pt = std::getenv("FDD_PHASE_TABLE");
    double dm0 = 0.0, step = 0.0;
    if (p->kernel == "mfma_f32" && d.delay_mode == FDD_DELAY_EXACT && pt != nullptr && std::strcmp(pt, "linear") == 0 &&
        uniform_grid(p->dms, &dm0, &step)) {
      p->lin = true;
      p->grid_dm0 = dm0;
      p->grid_step = step;
    }
  }
  // spin-frequency-scaled DMs (Eq. 8): first block whose rows stay within the halo
  if (d.flags & FDD_PLAN_SCALED_DM) {
    double dm0 = 0.0, step = 0.0;
    const char* why = nullptr;
    if (!d.single_chunk) why = "scaled DMs need a single-chunk plan";
    else if (d.delay_mode != FDD_DELAY_EXACT) why = "scaled DMs need exact delays";
    else if (L < 2 * kScaledBlock) why = "scaled DMs need chunk_len >= 128";
    else if (d.n_dm > 65535) why = "scaled DMs take at most 65535 trial DMs";
    else if (!uniform_grid(p->dms, &dm0, &step)) why = "scaled DMs need a uniform DM list (DM_0 + j dDM, n_dm >= 2)";
    if (why != nullptr) {
      delete p;
      return fail(FDD_E_UNSUPPORTED, why);
    }
    p->scaled = true;
    p->grid_dm0 = dm0;
    p->grid_step = step;
    double big = 0.0;
    for (double v : p->dms) big = std::max(big, std::fabs(v));
    // block starting at b (reference r = b + 32): rows move by at most big * 32 / (r dDM)
    const double rmin = 32.0 * big / ((double)(kScaledHalo - 1) * step);
    const double b = std::ceil(std::max(0.0, rmin - kScaledBlock / 2) / kScaledBlock) * kScaledBlock;
    const int64_t half = L / 2;
    // the first block always runs exactly: it holds bin 0 and its 8-bit zero-point restore
    p->sc_fmin = (int)std::min<double>(std::max(b, (double)kScaledBlock), (double)half);
    p->sc_blocks = (int)((half - p->sc_fmin + kScaledBlock - 1) / kScaledBlock);
  }
  // spread of the nearest-sample delays over the DM tiles of the time-domain kernels
  for (int tile : {tdd_dm_tile(), tdd_tile64()}) {
    int span = 0;
    for (int32_t c = 0; c < d.n_chan; ++c)
      for (int32_t m0 = 0; m0 < d.n_dm; m0 += tile) {
        double lo = 1e300, hi = -1e300;
        for (int32_t m = m0; m < std::min(d.n_dm, m0 + tile); ++m) {
          const double dd = std::floor(p->dms[(size_t)m] * p->kappa[(size_t)c] + 0.5);
          lo = std::min(lo, dd);
          hi = std::max(hi, dd);
        }
        span = std::max(span, (int)std::min(hi - lo, 2e9));
      }
    (tile == tdd_dm_tile() ? p->tdd_span : p->tdd_span64) = span;
  }
  fdd_status st = layout(p);
  if (st != FDD_OK) {
    delete p;
    return st;
  }
  p->dry_run = (d.flags & FDD_PLAN_DRY_RUN) != 0;
  build_host_tables(p);
  if (!p->dry_run && !(d.flags & FDD_PLAN_EXTERNAL_WORKSPACE)) {
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, p->ws.total);
    if (e != hipSuccess) {
      delete p;
      (void)hipGetLastError();
      return fail(FDD_E_NOMEM, std::string("hipMalloc(workspace): ") + hipGetErrorString(e));
    }
    p->d_ws = (uint8_t*)mem;
    p->ws_owned = true;
    st = upload_tables(p);
    if (st != FDD_OK) {
      (void)hipFree(mem);
      delete p;
      return st;
    }
  }
  *out = p;
  return FDD_OK;
}

fdd_status fdd_plan_info(fdd_plan_t p, fdd_plan_geometry* g) {
  if (p == nullptr || g == nullptr) return fail(FDD_E_INVALID, "null plan or output");
  g->chunk_len = p->L;
  g->stride = p->S;
  g->overlap = p->D;
  g->n_chunks = p->n_chunks;
  g->n_bins = p->n_bins;
  g->bins_padded = p->pitch;
  g->max_delay = p->max_tau;
  g->n_valid = p->n_valid;
  g->workspace_bytes = p->ws.total;
  g->out_samples = p->out_total;
  g->n_segments = (int32_t)p->segs.size();
  g->scaled_min_bin = p->scaled ? p->sc_fmin : 0;
  return FDD_OK;
}

fdd_status fdd_plan_output_offsets(fdd_plan_t p, int64_t* off) {
  if (p == nullptr || off == nullptr) return fail(FDD_E_INVALID, "null plan or output");
  for (const Segment& sg : p->segs)
    for (int i = 0; i < sg.n; ++i) off[sg.j0 + i] = sg.out_off + (int64_t)i * sg.n_out;
  off[p->desc.n_dm] = p->out_total;
  return FDD_OK;
}

fdd_status fdd_plan_delays(fdd_plan_t p, double* tau) {
  if (p == nullptr || tau == nullptr) return fail(FDD_E_INVALID, "null plan or output");
  const size_t nc = p->kappa.size();
  for (size_t m = 0; m < p->dms.size(); ++m)
    for (size_t c = 0; c < nc; ++c) tau[m * nc + c] = p->dms[m] * p->kappa[c];
  return FDD_OK;
}

const char* fdd_plan_kernel(fdd_plan_t p) { return p == nullptr ? "" : p->kernel.c_str(); }

fdd_status fdd_plan_factors(fdd_plan_t p, int32_t* fine, int32_t* coarse, int32_t* col_tiles) {
  if (p == nullptr) return fail(FDD_E_INVALID, "null plan");
  if (fine != nullptr) *fine = p->fac_fine;
  if (coarse != nullptr) *coarse = p->fac_coarse;
  if (col_tiles != nullptr) *col_tiles = p->facw_nt;
  return FDD_OK;
}

fdd_status fdd_set_workspace(fdd_plan_t p, void* mem, size_t bytes) {
  if (p == nullptr || mem == nullptr) return fail(FDD_E_INVALID, "null plan or workspace");
  if (p->dry_run) return fail(FDD_E_INVALID, "dry-run plans cannot take a workspace");
  if (bytes < p->ws.total) return fail(FDD_E_WORKSPACE, "workspace too small: need " + std::to_string(p->ws.total));
  if (((uintptr_t)mem % kAlign) != 0) return fail(FDD_E_INVALID, "workspace must be 256-byte aligned");
  if (p->ws_owned) {
    (void)hipFree(p->d_ws);
    p->ws_owned = false;
  }
  p->d_ws = (uint8_t*)mem;
  return upload_tables(p);
}

fdd_status fdd_destroy(fdd_plan_t p) {
  if (p == nullptr) return FDD_OK;
  if (p->ws_owned) (void)hipFree(p->d_ws);
  for (auto& e : p->ev)
    if (e != nullptr) (void)hipEventDestroy(e);
  delete p;
  return FDD_OK;
}

fdd_status fdd_profile_enable(fdd_plan_t p, int32_t depth) {
  if (p == nullptr || depth < 0) return fail(FDD_E_INVALID, "null plan or negative depth");
  if (p->dry_run) return fail(FDD_E_INVALID, "dry-run plan");
  for (auto& e : p->ev)
    if (e != nullptr) (void)hipEventDestroy(e);
  p->ev.assign((size_t)depth * 5, nullptr);
  p->ev_ok.assign((size_t)depth * 5, 0);
  for (auto& e : p->ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      p->prof_depth = 0;
      return hip_fail(r, "hipEventCreate");
    }
  }
  p->prof_depth = depth;
  p->prof_calls = 0;
  return FDD_OK;
}

fdd_status fdd_profile_read(fdd_plan_t p, float ms[4], int32_t* n_calls) {
  if (p == nullptr || ms == nullptr) return fail(FDD_E_INVALID, "null plan or output");
  for (int i = 0; i < 4; ++i) ms[i] = 0.0f;
  if (n_calls != nullptr) *n_calls = 0;
  if (p->prof_depth == 0) return fail(FDD_E_INVALID, "profiling is not enabled");
  const int64_t n = p->prof_calls < p->prof_depth ? p->prof_calls : p->prof_depth;
  double acc[4] = {0, 0, 0, 0};
  for (int64_t c = 0; c < n; ++c) {
    hipEvent_t* e = &p->ev[(size_t)c * 5];
    const char* ok = &p->ev_ok[(size_t)c * 5];
    for (int i = 0; i < 4; ++i) {
      if (!ok[i] || !ok[i + 1]) continue;
      hipError_t r = hipEventSynchronize(e[i + 1]);
      if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
      float t = 0.0f;
      r = hipEventElapsedTime(&t, e[i], e[i + 1]);
      if (r != hipSuccess) return hip_fail(r, "hipEventElapsedTime");
      acc[i] += t;
    }
  }
  for (int i = 0; i < 4; ++i) ms[i] = n > 0 ? (float)(acc[i] / (double)n) : 0.0f;
  if (n_calls != nullptr) *n_calls = (int32_t)n;
  p->prof_calls = 0;
  std::fill(p->ev_ok.begin(), p->ev_ok.end(), 0);
  return FDD_OK;
}

}  // extern "C"
