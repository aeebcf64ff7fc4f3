// Internal declarations shared by the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fdd.h"

namespace fdd {

struct FftArgs {
  const uint8_t* in_u8 = nullptr;   // forward: transposed 8-bit input
  const float* in_f32 = nullptr;    // forward: float input
  float2* X = nullptr;              // forward output
  const float* Yr = nullptr;        // inverse input planes
  const float* Yi = nullptr;
  const float2* Yc = nullptr;       // inverse input as interleaved complex [row][pitch] (instead of
                                    // the planes), written by the DM-factorised chunked kernels
  float* out = nullptr;             // inverse output [n_rows][n_samp]
  const float2* twL = nullptr;
  int64_t n_samp = 0;
  int64_t stride = 0;
  int64_t keep = 0;                 // samples kept per chunk
  int64_t pitch = 0;                // bins per row of X / Y
  int n_chunks = 0;
  int n_rows = 0;                   // channels (forward) or DMs (inverse)
  int row_chunks = 0;               // chunks per row of X / Y when several series share the rows
                                    // (beams stacked along the chunk axis); 0 = n_chunks
  float add_full = 0.0f;            // constant restored in chunks wholly inside the data
  int full_chunks = -1;             // inverse: chunks 0 .. full_chunks-1 lie wholly inside the data
                                    // (-1: decide from n_samp and the transform length)
  float inv_n = 0.0f;               // inverse: scale applied after the half-length transform
                                    // (0: 1 / (L/2), i.e. 1/L overall; shortened inverses use 2/L_full)
  unsigned int* l1max = nullptr;    // forward: per-chunk max L1 norm (float bits), or null
  int log_n = 0;                    // log2 of the complex points per series (L / 2)
};

// Arguments of the global-memory passes of long transforms.
struct LongPassArgs {
  const float2* in = nullptr;
  float2* out = nullptr;
  int64_t in_pitch = 0, out_pitch = 0;   // complex points between series
  const uint8_t* in_u8 = nullptr;        // first forward pass: real input
  const float* in_f32 = nullptr;
  float* out_real = nullptr;             // last inverse pass: real output [row][n_samp]
  const float* yr = nullptr;             // inverse pre-split: Y planes
  const float* yi = nullptr;
  float* l1sum = nullptr;                // per-series L1 norm accumulation, or null
  int log_n = 0, log_ns = 0;
  int n_series = 0, n_chunks = 1;
  int64_t stride = 0, n_samp = 0, keep = 0;
  float add_full = 0.0f;
};

struct PhasorArgs {
  const float2* X = nullptr;        // [n_chan][n_chunks][pitch]
  float* Yr = nullptr;              // [n_dm][n_chunks][pitch] (null for power spectra)
  float* Yi = nullptr;
  float* P = nullptr;               // [n_dm][n_pow_bins] power spectra, or null
  float2* Yc = nullptr;             // [n_dm][n_chunks][pitch] interleaved complex (chunked DM-factorised kernels)
  const uint4* ptab = nullptr;      // [n_chan][n_dm] {inc.lo, inc.hi, step cos, step sin}
  const unsigned int* l1max = nullptr; // [n_chunks] max over channels of the series L1 norm (float bits)
  int n_dm = 0;
  int n_chan = 0;
  int n_chunks = 0;
  int64_t pitch = 0;
  int n_bins = 0;                   // L/2 + 1
  int n_pow_bins = 0;               // L/2
  int log_len = 0;                  // log2 L
  float dc_add = 0.0f;              // added to Re Y at bin 0 before power (8-bit zero point)
  int tile_variant = 0;             // matrix-core tile shape (0 = default)
  int n_dmt = 0, n_bb = 0;          // grouped launches: DM tiles and bin blocks of this beam
  // DM-factorised kernels (uniform DM grid, exact delays): trial a*n_fine + b has the delay
  // tau_coarse[a] + tau_fine[b]; ptab then holds [n_chan][n_coarse] and vtab [n_chan][n_fine]
  const uint4* vtab = nullptr;
  int n_coarse = 0;
  int n_fine = 0;
  // Chunk tiling of the direct matrix-core kernels: chunks per row of X and of the Y planes
  // (0: n_chunks).  A launch over chunks k0 .. k0 + n_chunks - 1 of a wider plan has X, Yr, Yi
  // and l1max offset by k0 chunks and these set to the plan's chunk count.
  int x_chunks = 0;
  int y_chunks = 0;
  // Exact delays on a uniform DM grid (direct FP32 kernel): the increment of trial j is
  // inc0_c + (j + lin_j0) d_c (mod 2^64) from ltab[c] = {inc0.lo, inc0.hi, d.lo, d.hi}; ptab is
  // then not read.
  const uint4* ltab = nullptr;
  int lin_j0 = 0;
};

// Spin-frequency-scaled DMs (Eq. 8) for power spectra of one chunk.  Block b covers bins
// f_min + 64 b .. + 63 with reference bin r = f_min + 64 b + 32; row q of the scaled grid has
// DM'_q = DM_0 + (q - kScaledHalo) dDM and, at bin r, the phase increment inc_a + q inc_d
// (64-bit turn fractions per bin, per channel in ctab).
constexpr int kScaledBlock = 64;
constexpr int kScaledHalo = 32;
struct ScaledArgs {
  const float2* X = nullptr;        // [n_chan][pitch] forward spectra
  const uint4* ctab = nullptr;      // [n_chan] {inc_a.lo, inc_a.hi, inc_d.lo, inc_d.hi}
  float* Q = nullptr;               // [n_rows][q_pitch] |sum_c W X|^2 from bin f_min on
  int n_chan = 0;
  int n_rows = 0;                   // n_dm + 2 kScaledHalo
  int n_blocks = 0;
  int f_min = 0;
  int64_t pitch = 0;
  int64_t q_pitch = 0;              // n_blocks * kScaledBlock
};
struct ResampleArgs {
  const float* Q = nullptr;
  float* P = nullptr;               // [n_dm][n_pow_bins]
  const double* dms = nullptr;      // [n_dm] trial DMs
  double dm0 = 0.0, step = 0.0;     // the uniform grid DM_0 + j dDM
  int n_dm = 0;
  int n_rows = 0;
  int f_min = 0;
  int n_pow_bins = 0;
  int64_t q_pitch = 0;
};

// Brute-force time-domain dedispersion (Eq. 2) with nearest-sample delays.
struct TddArgs {
  const uint8_t* in_u8 = nullptr;   // channel-major 8-bit input [n_chan][n_samp], or
  const float* in_f32 = nullptr;    // channel-major float input [n_chan][n_samp]
  float* out = nullptr;             // [n_dm][n_samp]
  const int* dtab = nullptr;        // [n_chan][n_dm] delays in samples, floor(tau + 1/2)
  int64_t n_samp = 0;
  int64_t period = 0;               // L for single-chunk plans (circular), else 0 (zero extension)
  int n_chan = 0;
  int n_dm = 0;
};

// Grouped launch over several beams (the batched form): tiles [prefix[b], prefix[b+1]) belong
// to beam b, whose arguments are beams[b].  For the phasor sums each range is a multiple of 8
// long, so that a tile's beam-local id modulo 8 equals its global id modulo 8.
template <class Args>
struct Group {
  const Args* beams = nullptr;        // device array [n_beams]
  const int* prefix = nullptr;        // device array [n_beams + 1], ascending, prefix[0] = 0
  unsigned int* counters = nullptr;   // persistent launches: 8 ticket counters, zero at launch
  int n_beams = 0;
  int total = 0;                      // prefix[n_beams]
};

// Beam that owns tile `t`: the last b with prefix[b] <= t (binary search).
__device__ __forceinline__ int group_beam(const int* prefix, int n_beams, int t) {
  int lo = 0, hi = n_beams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Load a workgroup-uniform struct from device memory into scalar registers (dword by dword
// through readfirstlane), so that a beam's arguments cost no vector registers.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized struct expected");
  constexpr int kWords = (int)(sizeof(T) / 4);
  union U {
    T t;
    int w[kWords];
    __device__ U() {}
  } u;
  const int* src = reinterpret_cast<const int*>(p);
#pragma unroll
  for (int i = 0; i < kWords; ++i) u.w[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return u.t;
}

// Tile loops of the grouped phasor sums.  Non-persistent: one workgroup per tile, tile id =
// linear workgroup id (the hardware balances).  Persistent: workgroup p serves the tiles congruent to p modulo 8, claiming them
// one at a time from ticket counter p mod 8; the grid is a multiple of 8 workgroups, so every
// tile below `total` is claimed exactly once, each claim names a tile on the XCD that the
// hardware gives workgroup p (workgroups are dispatched round-robin over the 8 XCDs), and the
// tiles of one XCD are balanced dynamically.  Every workgroup leaves once its counter passes
// `total`.
template <bool PERSIST, class Body>
__device__ __forceinline__ void grouped_tiles(unsigned int* counters, int total, Body&& body) {
  if constexpr (!PERSIST) {
    const int t = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (t < total) body(t, (int)threadIdx.x);
    return;
  }
  __shared__ int ticket;
  const int xcd = (int)(blockIdx.x & 7u);
  for (;;) {
    __syncthreads();                          // the previous tile is done with LDS and `ticket`
    if (threadIdx.x == 0) ticket = (int)atomicAdd(counters + xcd, 1u) * 8 + xcd;
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(ticket);   // uniform: keeps beam arguments scalar
    if (t >= total) break;
    // the thread index reaches the body as an opaque value, so that nothing derived from it is
    // hoisted out of the loop and held in registers across tiles
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    body(t, tid);
  }
}

// Workgroups of a persistent launch: what fits on the device at once (at most `cap`), as a
// multiple of 8 and at least 8.
int persistent_blocks(const void* kernel, int threads, int64_t cap);


// A 1-D sequence of `blocks` workgroups laid out as a 2-D grid whose linear order
// (y * gridDim.x + x) is the sequence: the work-item count of one grid dimension must stay
// below 2^32.  Rows are multiples of 8 workgroups, so the linear id modulo 8 is the XCD.
inline dim3 linear_grid(int64_t blocks) {
  const int64_t row = int64_t(1) << 16;
  if (blocks <= row) return dim3((unsigned)blocks);
  return dim3((unsigned)row, (unsigned)((blocks + row - 1) / row));
}

// Grid of a grouped phasor launch: every tile (non-persistent) or what fits (persistent).
inline dim3 grouped_grid(bool persist, const void* kernel, int total) {
  return persist ? dim3((unsigned)persistent_blocks(kernel, 256, ((int64_t)total + 7) / 8 * 8))
                 : linear_grid(total);
}

hipError_t launch_zero_u32(unsigned int* p, int64_t n, hipStream_t st);
hipError_t launch_tdd(const TddArgs& a, int span, int span64, hipStream_t st);
int tdd_span_max();    // largest delay spread per channel over a tile of 8 DMs that the kernels take
int tdd_span64_max();  // the same over the larger DM tiles of the 8-bit kernel for fine grids
int tdd_tile64();      // DMs per tile of that kernel
int tdd_dm_tile();     // DMs per tile (8)
hipError_t launch_transpose_u8(const uint8_t* in, uint8_t* out, int64_t n_samp, int n_chan, hipStream_t st);
hipError_t launch_r2c(int log_n, const FftArgs& a, hipStream_t st);
hipError_t launch_c2r(int log_n, const FftArgs& a, hipStream_t st);
hipError_t launch_r2c_long(const FftArgs& a, float2* work, float* l1sum, hipStream_t st);
hipError_t launch_c2r_long(const FftArgs& a, float2* work, float2* work2, hipStream_t st);
constexpr int kMaxBlockLogN = 15;   // longest transform held by one workgroup: 2^15 complex points
hipError_t launch_phasor_valu(const PhasorArgs& a, hipStream_t st);
hipError_t launch_phasor_mfma_f32(const PhasorArgs& a, hipStream_t st);
// The single-plan split kernels read X as split words: call launch_split_x on X first (in
// place; X then no longer holds spectra).  The grouped split kernels read plain X.
hipError_t launch_phasor_split(const PhasorArgs& a, bool bf16, hipStream_t st);
hipError_t launch_split_x(float2* X, const unsigned int* l1max, int n_chan, int n_chunks, int64_t pitch, bool bf16,
                          hipStream_t st);
bool phasor_mfma_f32_supported(int n_chunks);
bool phasor_mfma_f32_window_ok(int64_t x_chunks, int64_t pitch);
bool phasor_split_supported(int n_chunks);

// Chunk tiling of the direct matrix-core kernels, which hold at most kDirectMaxChunks chunks
// (2 x 24 real columns) per workgroup: a plan with more chunks runs them over balanced chunk
// groups, group g covering chunks k0 .. k0 + cnt - 1.
constexpr int kDirectMaxChunks = 24;
inline int chunk_groups(int n_chunks) {
  return n_chunks <= kDirectMaxChunks ? 1 : (n_chunks + kDirectMaxChunks - 1) / kDirectMaxChunks;
}
inline int chunk_group_max(int n_chunks) {
  const int g = chunk_groups(n_chunks);
  return (n_chunks + g - 1) / g;
}
// The arguments of chunk group g of a (whole-plan) launch a: X, the Y planes and the chunk
// scales offset by k0 chunks, rows strided by the plan's chunk count.
inline PhasorArgs chunk_group_args(const PhasorArgs& a, int g) {
  const int n = a.n_chunks, ng = chunk_groups(n);
  if (ng == 1) return a;
  const int k0 = g * (n / ng) + (g < n % ng ? g : n % ng);
  const int cnt = n / ng + (g < n % ng ? 1 : 0);
  PhasorArgs t = a;
  const size_t off = (size_t)k0 * (size_t)a.pitch;
  t.n_chunks = cnt;
  t.x_chunks = n;
  t.y_chunks = n;
  t.X = a.X + off;
  if (a.Yr != nullptr) t.Yr = a.Yr + off;
  if (a.Yi != nullptr) t.Yi = a.Yi + off;
  if (a.l1max != nullptr) t.l1max = a.l1max + k0;
  return t;
}
// DM-factorised kernels: fine DMs per coarse row for n_chunks chunks (0 if not supported), and
// the launch (precision: fdd_precision) of a Y-plane or power-spectrum phasor sum.
int phasor_fac_fine(int n_chunks);
hipError_t launch_phasor_fac(const PhasorArgs& a, int precision, hipStream_t st);
int64_t phasor_fac_tiles(PhasorArgs* a, int precision);
hipError_t launch_phasor_fac_grouped(int precision, bool persist, const Group<PhasorArgs>& g, hipStream_t st);
// DM-factorised kernels for overlap-save plans: fine DMs B (8 or 16), coarse rows, and the
// number NT of 32-column tiles per column group (kFacwNtMin..kFacwNtMax) with the least
// estimated work for n_dm trials and n_chunks chunks; eff = useful share of the padded tiles.
// The launch writes interleaved complex Y (a.Yc).
struct FacwChoice {
  int fine = 0, coarse = 0, nt = 0;
  double eff = 0.0;
};
constexpr int kFacwNtMin = 4;
constexpr int kFacwNtMax = 7;
FacwChoice facw_choose(int n_dm, int n_chunks);
hipError_t launch_phasor_facw(const PhasorArgs& a, int precision, int nt, hipStream_t st);
// Spin-frequency-scaled DMs: the per-block matrix products and the resampling in DM.
// precision FDD_FP32: plain X; split precisions: X split in place by launch_split_x, and the
// per-chunk L1 maxima for the scale.
hipError_t launch_phasor_scaled(const ScaledArgs& a, int precision, const unsigned int* l1max, hipStream_t st);
hipError_t launch_scaled_resample(const ResampleArgs& a, hipStream_t st);

// Grouped launches of the batched form.  Tiles per beam (for the prefix sums) come from the
// *_tiles functions, which also fill a.n_dmt / a.n_bb where the kernel needs them.
hipError_t launch_r2c_grouped(int log_n, bool u8, const Group<FftArgs>& g, hipStream_t st);
hipError_t launch_c2r_grouped(int log_n, const Group<FftArgs>& g, hipStream_t st);
int64_t fft_grouped_tiles(const FftArgs& a);
int64_t phasor_mfma_f32_tiles(PhasorArgs* a, int variant);
hipError_t launch_phasor_mfma_f32_grouped(int nt, int variant, bool persist, const Group<PhasorArgs>& g,
                                          hipStream_t st);
int64_t phasor_split_tiles(PhasorArgs* a);
hipError_t launch_phasor_split_grouped(bool bf16, int nt, bool persist, const Group<PhasorArgs>& g,
                                       hipStream_t st);
int64_t phasor_valu_tiles(PhasorArgs* a, int nk);
hipError_t launch_phasor_valu_grouped(int nk, const Group<PhasorArgs>& g, hipStream_t st);
constexpr int kMfmaF32Variants = 5;

// Byte offsets of the workspace regions (256-byte aligned).
// A run of consecutive DMs that share one output down-sampling factor d.  Its phase table is
// its own [n_chan][n] block of the plan's table, its output rows follow each other from
// out_off, and its inverse transforms have length L/d with their own twiddle table.
struct Segment {
  int j0 = 0, n = 0;                  // DMs j0 .. j0 + n - 1
  int factor = 1;                     // d
  int64_t n_out = 0;                  // samples per output row, ceil(n_samp / d)
  int64_t out_off = 0;                // output sample where row j0 starts
  size_t tab = 0;                     // first phase-table entry of the segment
  size_t tw = 0;                      // workspace byte offset of its twiddles exp(-2 pi i j d / L), j < L/d
};

struct WorkspaceLayout {
  size_t tw = 0, tw_bytes = 0;        // float2 twiddles: L entries, then L/d for every other factor d
  size_t ptab = 0, ptab_bytes = 0;    // uint4 phase increments and step phasors, [n_chan][n] per segment
  size_t scale = 0, scale_bytes = 0;  // float [n_chunks]
  size_t xt = 0, xt_bytes = 0;        // transposed uint8 input
  size_t X = 0, X_bytes = 0;          // float2 [n_chan][n_chunks][pitch]
  size_t Yr = 0, Yi = 0, Y_bytes = 0; // float planes [n_dm][n_chunks][pitch] each (not for power-only plans)
  size_t Z = 0, Z_bytes = 0;          // long transforms: float2 [max(n_chan, n_dm) * n_chunks][L/2]
  size_t l1 = 0, l1_bytes = 0;        // long transforms: per-series L1 sums
  size_t dtab = 0, dtab_bytes = 0;    // int [n_chan][n_dm] nearest-sample delays (time-domain path)
  size_t ctab = 0, ctab_bytes = 0;    // scaled DMs: uint4 [n_chan] phase increments
  size_t ltab = 0, ltab_bytes = 0;    // linear phase increments: uint4 [n_chan] (uniform grid, exact delays)
  size_t dmv = 0, dmv_bytes = 0;      // scaled DMs: double [n_dm] trial DMs
  size_t Q = 0, Q_bytes = 0;          // scaled DMs: float [n_dm + 64][q_pitch]
  size_t total = 0;
};

}  // namespace fdd

struct fdd_plan_s {
  fdd_plan_desc desc{};                 // with pointers redirected to the copies below
  std::vector<double> freqs, dms, kappa;
  int log_len = 0;
  int64_t L = 0, S = 0, D = 0, n_chunks = 0, n_bins = 0, pitch = 0, n_valid = 0;
  double max_tau = 0.0;
  fdd::WorkspaceLayout ws;
  uint8_t* d_ws = nullptr;
  bool ws_owned = false;
  bool dry_run = false;
  std::string kernel = "valu";
  int tile_variant = 0;                 // FDD_TILE_VARIANT override
  // DM factorisation (uniform DM grid, exact delays): trial j = a * fac_fine + b
  int fac_fine = 0, fac_coarse = 0;     // 0: not factorised
  int facw_nt = 0;                      // > 0: the chunked factorised kernels with this many column tiles
  bool lin = false;                     // direct FP32 kernel with per-channel linear increments (ltab)
  int tdd_span = 0;                     // largest delay spread over 8 consecutive DMs (time-domain kernel)
  int tdd_span64 = 0;                   // ... over tdd_tile64() consecutive DMs
  double fac_dm0 = 0.0, fac_step = 0.0;
  // output down-sampling: the factor of every DM and the runs of equal factors (one segment
  // of factor 1 without down-sampling)
  std::vector<int32_t> ds;
  // the small tables on the host, uploaded into the workspace: (workspace byte offset, bytes)
  std::vector<std::pair<size_t, std::vector<uint8_t>>> htabs;
  std::vector<fdd::Segment> segs;
  int64_t out_total = 0;
  // spin-frequency-scaled DMs (FDD_PLAN_SCALED_DM)
  bool scaled = false;
  double grid_dm0 = 0.0, grid_step = 0.0;
  int sc_fmin = 0, sc_blocks = 0;
  // stage timing: a ring of `prof_depth` calls x 5 events
  int prof_depth = 0;
  int64_t prof_calls = 0;               // calls recorded since the last read
  std::vector<hipEvent_t> ev;
  std::vector<char> ev_ok;
};

namespace fdd {
// Planner tables (float64 on the host): twiddles exp(-2 pi i j / L), j < L, and the phase
// increments and step phasors of every (channel, DM), channel-major.
void twiddle_table(int64_t L, std::vector<float2>* out);
void phase_table(const fdd_plan_s* p, std::vector<uint4>* out);
// phase table of the DMs j0 .. j0 + n - 1 only, [n_chan][n]
void phase_table_rows(const fdd_plan_s* p, int j0, int n, std::vector<uint4>* out);
// DM factorisation: whether the DM list is DM_0 + j dDM (dDM > 0), and the coarse [n_chan][coarse]
// plus fine [n_chan][fine] phase tables of trial a * fine + b.
bool uniform_grid(const std::vector<double>& dms, double* dm0, double* step);
void factor_tables(const fdd_plan_s* p, int fine, int coarse, double dm0, double step, std::vector<uint4>* out);
// Enqueue the copies of the plan's host tables into a workspace at dst (same layout) on st.
hipError_t upload_tables_async(const fdd_plan_s* p, uint8_t* dst, hipStream_t st);
void set_error(const std::string& msg);
fdd_status fail(fdd_status s, const std::string& msg);
fdd_status hip_fail(hipError_t e, const char* what);
}  // namespace fdd
