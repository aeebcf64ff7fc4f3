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
//  - a workgroup owns 64 MW DMs (4 waves x 16 MW) and FB consecutive bins (FB = 8 for the
//    default tile), all chunks;
//  - channels stream through LDS in groups of KC (8 by default): the group's data for the FB
//    bins is read from HBM once (FB x 8-byte runs along f) and rearranged into the two B
//    planes [c][f][column] (cos-part and sin-part operands), double-buffered: the next group
//    is deposited into the other buffer right after the current one's products are issued,
//    so one barrier per group suffices;
//  - per 4-channel step, lane l generates the phasor of (DM l%16, channel l/16) for the
//    tile's bins: exact 64-bit phase of the first bin (planner table + sincos_turn), then
//    complex multiplications by the tabulated step phasor.  Its cos feeds the first MFMA set
//    and its sin the second, so no phasor is computed twice;
//  - accumulators live in registers: FB bins x NT tiles x 4 floats per lane and DM sub-tile;
//  - the epilogue writes, per lane, FB consecutive bins of one (DM, chunk) row of the Yr or
//    Yi plane (float4 stores).
// Workgroups are numbered so that the DM tiles of one bin block run back to back on the same
// XCD (hardware dispatches workgroup i to XCD i mod 8), so the bin block's data is served
// from that XCD's L2 after the first read.
#include <map>
#include <mutex>

#include "device_math.h"
#include "fdd_internal.h"

namespace fdd {

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kXcds = 8;
}  // namespace

// FB bins per workgroup, KC channels per LDS stage, NT 16-column tiles (2N <= 16 NT),
// MW 16-DM sub-tiles per wave (64 MW DMs per workgroup).  LIN: seeds from the per-channel linear
// increments (a.ltab) instead of the (channel, DM) phase table.
template <int NT, int FB, int KC, int MW, bool LIN = false>
__device__ __forceinline__ void phasor_mfma_f32_body(const PhasorArgs& a, const int bid, const int n_dmt,
                                                     const int n_bb,
    const int tid) {
  constexpr int kDmTile = 64 * MW;
  constexpr int NCOL = NT * 16;
  // per-channel stride padded by 16 floats so that the four channels read by one MFMA step
  // fall in distinct LDS banks
  constexpr int CST = FB * NCOL + 16;
  constexpr int PLANE = KC * CST;
  // staging elements (float4 = two bins of one (channel, chunk)) per thread, for N <= 8 NT
  constexpr int PER = (KC * 8 * NT * (FB / 2) + 255) / 256;
  __shared__ float bre2[2][PLANE];
  __shared__ float bim2[2][PLANE];
  // sin/cos table of the seeds (and, with LIN, of the step phasors), where its 2 KiB leave the
  // workgroups per CU unchanged
  constexpr int kLdsBase = 4 * PLANE * (int)sizeof(float);
  constexpr bool TAB = (163840 / (kLdsBase + 2048) == 163840 / kLdsBase);
  __shared__ float2 sctab[TAB ? 256 : 1];

  const int xcd = bid % kXcds;
  const int slot = bid / kXcds;
  const int bb = (slot / n_dmt) * kXcds + xcd;
  const int dmt = slot % n_dmt;
  if (bb >= n_bb) return;                     // uniform per workgroup, before any barrier
  const int fb0 = bb * FB;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int N = a.n_chunks;
  const int XC = a.x_chunks > 0 ? a.x_chunks : N;   // chunks per row of X and of Y
  const int YC = a.y_chunks > 0 ? a.y_chunks : N;
  const int nel = KC * N * (FB / 2);

  // zero once: padding columns (>= 2N) are never written by the staging below
  for (int i = tid; i < PLANE; i += 256) {
    bre2[0][i] = bre2[1][i] = 0.0f;
    bim2[0][i] = bim2[1][i] = 0.0f;
  }
  if constexpr (TAB) sctab[tid] = turn_table_entry((uint32_t)tid);

  // Staging map, fixed for all channel blocks: element e = tid + 256 j is the float4 of bins
  // (2 fp, 2 fp + 1) of chunk k of channel cl of the block.  The chunk varies fastest, so the
  // LDS stores of a wave fall in consecutive words of a bin row; bin pairs are 2 NCOL words
  // apart, a multiple of the 32 banks, and varying them first put 4 lanes on each bank.
  int goff[PER], loff[PER], ccl[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    const int k = e % N;
    const int fp = (e / N) % (FB / 2);
    const int cl = e / ((FB / 2) * N);
    goff[j] = k * (int)a.pitch + fb0 + 2 * fp;                 // in float2 units, within channel cl's row
    loff[j] = cl * CST + 2 * fp * NCOL + k;
    ccl[j] = e < nel ? cl : KC;                                 // KC marks "no element"
  }
  // Each group's X rows are read through a buffer descriptor over the rows of its KC channels
  // (channels past n_chan read as zeros), so an element's byte offset is the same in every
  // group; an element slot that holds nothing points past any window.  The window stays below
  // 2 GiB (KC XC pitch 8 bytes; checked by the planner).
  uint32_t xoff[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j)
    xoff[j] = ccl[j] < KC ? (uint32_t)(((int64_t)ccl[j] * XC * a.pitch + goff[j]) * 8) : 0xFFFFFFF0u;
  float4 pf[PER];
  auto fetch = [&](int cb) {
    const int nc = min(KC, a.n_chan - cb);
    const __amdgpu_buffer_rsrc_t rx = raw_rsrc(a.X + (int64_t)cb * XC * a.pitch, (int64_t)nc * XC * a.pitch * 8);
#pragma unroll
    for (int j = 0; j < PER; ++j) pf[j] = load_f4(rx, xoff[j]);
  };
  auto deposit = [&](float* bre, float* bim) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (ccl[j] >= KC) continue;
      const int i0 = loff[j];
      const int i1 = i0 + NCOL;
      const float4 v = pf[j];
      bre[i0] = v.x;
      bim[i0] = -v.y;
      bre[i0 + N] = v.y;
      bim[i0 + N] = v.x;
      bre[i1] = v.z;
      bim[i1] = -v.w;
      bre[i1 + N] = v.w;
      bim[i1 + N] = v.z;
    }
  };

  int dmi[MW];
#pragma unroll
  for (int m = 0; m < MW; ++m) {
    const int dm = dmt * kDmTile + (wave * MW + m) * 16 + (lane & 15);
    dmi[m] = dm < a.n_dm ? dm : a.n_dm - 1;   // a clamped row's results are not stored
  }
  const int cq = lane >> 4;

  floatx4 acc[MW][FB][NT];
#pragma unroll
  for (int m = 0; m < MW; ++m)
#pragma unroll
    for (int f = 0; f < FB; ++f)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[m][f][nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

  fetch(0);
  __syncthreads();                            // padding zeroed, table filled
  deposit(bre2[0], bim2[0]);
  __syncthreads();
  int it = 0;
  // Phase-table entries of the lane's (DM, channel) seeds (with LIN the channel's linear entry,
  // the same for every DM), through a descriptor over the group's KC channels like X: byte
  // offsets the same in every group, channels past n_chan read as zero entries (phasor 1, step
  // 0, against staged zeros).  Each entry is loaded for the next group as soon as its seed and
  // steps are formed, into the registers it leaves.
  uint32_t toff[KC / 4][MW];
#pragma unroll
  for (int s = 0; s < KC / 4; ++s)
#pragma unroll
    for (int m = 0; m < MW; ++m)
      toff[s][m] = LIN ? (uint32_t)((4 * s + cq) * 16) : (uint32_t)(((4 * s + cq) * a.n_dm + dmi[m]) * 16);
  auto tab_rsrc = [&](int cb) {
    const int nc = min(KC, a.n_chan - cb);
    if constexpr (LIN) return raw_rsrc(a.ltab + cb, (int64_t)nc * 16);
    else return raw_rsrc(a.ptab + (int64_t)cb * a.n_dm, (int64_t)nc * a.n_dm * 16);
  };
  uint4 tn[KC / 4][MW];
  {
    const __amdgpu_buffer_rsrc_t rt = tab_rsrc(0);
#pragma unroll
    for (int s = 0; s < KC / 4; ++s)
#pragma unroll
      for (int m = 0; m < MW; ++m) tn[s][m] = load_u4(rt, toff[s][m]);
  }
  for (int cb = 0; cb < a.n_chan; cb += KC, ++it) {
    const float* bre = bre2[it & 1];
    const float* bim = bim2[it & 1];
    const __amdgpu_buffer_rsrc_t rtn = tab_rsrc(cb + KC);
    if (cb + KC < a.n_chan) fetch(cb + KC);   // in flight while this block computes
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int cl = 4 * s + cq;                // channels past n_chan were staged as zeros
      const float* pr = bre + cl * CST + (lane & 15);
      const float* pi = bim + cl * CST + (lane & 15);
#pragma unroll
      for (int m = 0; m < MW; ++m) {
        float2 w, step;
        if constexpr (LIN && TAB) {            // seed_phasor_linear with table sin/cos
          const uint4 e = tn[s][m];
          const uint64_t inc = (((uint64_t)e.y << 32) | e.x) + (uint64_t)(uint32_t)(dmi[m] + a.lin_j0) * (((uint64_t)e.w << 32) | e.z);
          const PhaseInc pinc = {(uint32_t)(inc >> 32), (uint32_t)inc};
          w = turn_phasor_tab(phase_at(pinc, (uint32_t)fb0), sctab);
          step = turn_phasor_tab(pinc.hi, sctab);
        } else if constexpr (LIN) seed_phasor_linear(tn[s][m], (uint32_t)(dmi[m] + a.lin_j0), (uint32_t)fb0, &w, &step);
        else if constexpr (TAB) seed_phasor_tab(tn[s][m], (uint32_t)fb0, sctab, &w, &step);
        else seed_phasor(tn[s][m], (uint32_t)fb0, &w, &step);
        float wr[FB], wi[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          wr[f] = w.x;
          wi[f] = w.y;
          w = cmul(w, step);
        }
        tn[s][m] = load_u4(rtn, toff[s][m]);
#pragma unroll
        for (int f = 0; f < FB; ++f)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[m][f][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wr[f], pr[f * NCOL + 16 * nt], acc[m][f][nt], 0, 0, 0);
#pragma unroll
        for (int f = 0; f < FB; ++f)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[m][f][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wi[f], pi[f * NCOL + 16 * nt], acc[m][f][nt], 0, 0, 0);
      }
    }
    if constexpr (FB == 8 && MW == 1) {
      // Scheduling only: issue four B-operand reads (ds_read2, two MFMAs each) before the first
      // matrix instruction and one more after every two, so that three are in flight while a
      // pair of products waits for the oldest; left alone, the scheduler waits for each read
      // right before its two MFMAs.  (Two, five or six ahead measured slower; eight makes the
      // register allocator fall back to one.)  The other tile shapes lose occupancy to the
      // extra registers.
      constexpr int kReads = (KC / 4) * FB * NT;
      __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);      // DS reads
#pragma unroll
      for (int i = 0; i < kReads - 4; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);    // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
    }
    // the other buffer was last read in the previous group, which every wave has left
    if (cb + KC < a.n_chan) deposit(bre2[(it + 1) & 1], bim2[(it + 1) & 1]);
    __syncthreads();
  }

  // D[i][j] of a 16x16 tile sits in lane 16*(i/4) + j, register i%4.
#pragma unroll
  for (int m = 0; m < MW; ++m)
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = 16 * nt + (lane & 15);
    if (n >= 2 * N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int dmr = dmt * kDmTile + (wave * MW + m) * 16 + 4 * (lane >> 4) + r;
      if (dmr >= a.n_dm) continue;
      float* dst = (n < N ? a.Yr + ((int64_t)dmr * YC + n) * a.pitch
                          : a.Yi + ((int64_t)dmr * YC + (n - N)) * a.pitch) + fb0;
#pragma unroll
      for (int f = 0; f < FB; f += 4)
        *(float4*)(dst + f) =
            make_float4(acc[m][f][nt][r], acc[m][f + 1][nt][r], acc[m][f + 2][nt][r], acc[m][f + 3][nt][r]);
    }
  }
}

// linear workgroup id; grids are 2-D only to keep each dimension below 2^32 work-items
__device__ __forceinline__ int linear_block() { return blockIdx.y * gridDim.x + blockIdx.x; }

template <int NT, int FB, int KC, int MW, bool LIN>
__global__ __launch_bounds__(256) void k_phasor_mfma_f32(PhasorArgs a, int n_dmt, int n_bb) {
  phasor_mfma_f32_body<NT, FB, KC, MW, LIN>(a, linear_block(), n_dmt, n_bb, threadIdx.x);
}

// Batched form: the tiles of every beam of the group, one per workgroup or persistent.
template <int NT, int FB, int KC, int MW, bool PERSIST>
__global__ __launch_bounds__(256) void k_phasor_mfma_f32_grouped(Group<PhasorArgs> g) {
  grouped_tiles<PERSIST>(g.counters, g.total, [&](int t, int tid) {
    const int b = group_beam(g.prefix, g.n_beams, t);
    const PhasorArgs a = PERSIST ? load_uniform(g.beams + b) : g.beams[b];
    phasor_mfma_f32_body<NT, FB, KC, MW>(a, t - g.prefix[b], a.n_dmt, a.n_bb, tid);
  });
}

int persistent_blocks(const void* kernel, int threads, int64_t cap) {
  // resident workgroups per device, per kernel (queried once: launches may be under capture)
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int64_t> resident;
  int64_t n = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = resident.find({kernel, threads});
    if (it != resident.end()) {
      n = it->second;
    } else {
      int dev = 0, cus = 0, per_cu = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) == hipSuccess)
        n = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
      else
        n = 8;
      resident.emplace(std::make_pair(kernel, threads), n);
    }
  }
  if (n > cap) n = cap;
  n = n / 8 * 8;
  return n < 8 ? 8 : (int)n;
}

bool phasor_mfma_f32_supported(int n_chunks) { return n_chunks >= 3 && n_chunks <= 24; }

// The kernels read X through descriptors over the rows of 8 or 16 channels (x_chunks rows of
// pitch complex bins each), whose byte count must stay below 2^31.
bool phasor_mfma_f32_window_ok(int64_t x_chunks, int64_t pitch) { return 16 * 8 * x_chunks * pitch <= 0x7fffffff; }

namespace {
template <int FB, int KC, int MW, bool LIN>
hipError_t launch_tile_lin(const PhasorArgs& a, hipStream_t st) {
  const int n_dmt = (a.n_dm + 64 * MW - 1) / (64 * MW);
  const int n_bb = (a.n_bins + FB - 1) / FB;
  const int n_bb8 = (n_bb + kXcds - 1) / kXcds * kXcds;
  const int64_t blocks = (int64_t)n_dmt * n_bb8;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid = linear_grid(blocks), block(256);
  switch ((2 * a.n_chunks + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_phasor_mfma_f32<1, FB, KC, MW, LIN>), grid, block, 0, st, a, n_dmt, n_bb); break;
    case 2: hipLaunchKernelGGL((k_phasor_mfma_f32<2, FB, KC, MW, LIN>), grid, block, 0, st, a, n_dmt, n_bb); break;
    case 3: hipLaunchKernelGGL((k_phasor_mfma_f32<3, FB, KC, MW, LIN>), grid, block, 0, st, a, n_dmt, n_bb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int FB, int KC, int MW>
hipError_t launch_tile(const PhasorArgs& a, hipStream_t st) {
  return a.ltab != nullptr ? launch_tile_lin<FB, KC, MW, true>(a, st) : launch_tile_lin<FB, KC, MW, false>(a, st);
}
}  // namespace

// Tile variants (tuning): bins per workgroup x channels per LDS stage x DM sub-tiles per wave.
hipError_t launch_phasor_mfma_f32(const PhasorArgs& a, hipStream_t st) {
  if (!phasor_mfma_f32_supported(a.n_chunks) ||
      !phasor_mfma_f32_window_ok(a.x_chunks > 0 ? a.x_chunks : a.n_chunks, a.pitch))
    return hipErrorInvalidValue;
  switch (a.tile_variant) {
    case 1: return launch_tile<16, 8, 1>(a, st);
    case 2: return launch_tile<8, 16, 1>(a, st);
    case 3: return launch_tile<4, 8, 2>(a, st);
    case 4: return launch_tile<4, 16, 2>(a, st);
    default: return launch_tile<8, 8, 1>(a, st);
  }
}

namespace {
struct TileShape {
  int fb, mw;
};
constexpr TileShape kShapes[kMfmaF32Variants] = {{8, 1}, {16, 1}, {8, 1}, {4, 2}, {4, 2}};

template <int NT, int FB, int KC, int MW, bool P>
hipError_t launch_grouped_nt(const Group<PhasorArgs>& g, hipStream_t st) {
  const void* k = (const void*)k_phasor_mfma_f32_grouped<NT, FB, KC, MW, P>;
  hipLaunchKernelGGL((k_phasor_mfma_f32_grouped<NT, FB, KC, MW, P>), grouped_grid(P, k, g.total), dim3(256), 0, st,
                     g);
  return hipGetLastError();
}

template <int FB, int KC, int MW>
hipError_t launch_grouped_tile(int nt, bool persist, const Group<PhasorArgs>& g, hipStream_t st) {
  switch (nt * 2 + (persist ? 1 : 0)) {
    case 2: return launch_grouped_nt<1, FB, KC, MW, false>(g, st);
    case 3: return launch_grouped_nt<1, FB, KC, MW, true>(g, st);
    case 4: return launch_grouped_nt<2, FB, KC, MW, false>(g, st);
    case 5: return launch_grouped_nt<2, FB, KC, MW, true>(g, st);
    case 6: return launch_grouped_nt<3, FB, KC, MW, false>(g, st);
    case 7: return launch_grouped_nt<3, FB, KC, MW, true>(g, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

int64_t phasor_mfma_f32_tiles(PhasorArgs* a, int variant) {
  if (variant < 0 || variant >= kMfmaF32Variants) variant = 0;
  const TileShape sh = kShapes[variant];
  a->n_dmt = (a->n_dm + 64 * sh.mw - 1) / (64 * sh.mw);
  a->n_bb = (a->n_bins + sh.fb - 1) / sh.fb;
  return (int64_t)a->n_dmt * ((a->n_bb + kXcds - 1) / kXcds * kXcds);
}

// Same tile variants as launch_phasor_mfma_f32; nt = ceil(2 N / 16) of every beam in the group.
hipError_t launch_phasor_mfma_f32_grouped(int nt, int variant, bool persist, const Group<PhasorArgs>& g,
                                          hipStream_t st) {
  if (g.total <= 0) return hipSuccess;
  switch (variant) {
    case 1: return launch_grouped_tile<16, 8, 1>(nt, persist, g, st);
    case 2: return launch_grouped_tile<8, 16, 1>(nt, persist, g, st);
    case 3: return launch_grouped_tile<4, 8, 2>(nt, persist, g, st);
    case 4: return launch_grouped_tile<4, 16, 2>(nt, persist, g, st);
    default: return launch_grouped_tile<8, 8, 1>(nt, persist, g, st);
  }
}

}  // namespace fdd
