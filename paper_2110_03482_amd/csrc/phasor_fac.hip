// DM-factorised phasor sum on the matrix cores (Eqs. 4 and 7 for a uniform DM grid).
//
// With trial DMs DM_j = DM_0 + j dDM and exact (fractional) delays, Eq. 1 is linear in DM, so
// writing j = a B + b (a "coarse", b "fine") splits every delay exactly:
//     tau[j, c] = (DM_0 + a B dDM) kappa_c + (b dDM) kappa_c = tau_A[a, c] + tau_B[b, c],
// and the phasor of Eq. 4 factorises, W[j, c, f] = U[a, c, f] V[b, c, f].  Per bin f
//     Y[a B + b, k, f] = sum_c U[a, c, f] Z[c, (b, k), f],   Z[c, (b, k), f] = V[b, c, f] X[c, k, f],
// which is a matrix product [A x n_chan] x [n_chan x B N] even for a single chunk (N = 1),
// where the direct form is a matrix-vector product per bin (Sec. 2.3).  The fine index b
// fills the matrix-core columns that the chunk axis alone leaves empty, and only A + B
// phasors per channel and bin are generated instead of A B.  The product is taken in the
// real form of the other kernels, [Yr | Yi] = Ur [Zr | Zi] + Ui [-Zi | Zr]: 2 B N columns,
// B = 8 NT / N, so the NT column tiles are full.
//
// Nearest-sample delays do not add (round(x + y) != round(x) + round(y)), so these kernels
// serve exact delays only; the planner checks that the DM list is uniform.
//
// Work decomposition: a workgroup owns 64 coarse rows (4 waves x 16) and FB bins.  Per stage
// of channels it stages Z for every (channel, fine DM, chunk) of its bins in LDS: one thread
// per (channel, b, k) seeds V at the first bin from the planner's fine table and walks the
// bins by complex multiplication.  The coarse phasors U are generated per lane as in the
// direct kernels (one (coarse row, channel) per lane, exact seed, recurrence over the bins).
// The epilogue maps column (b, k, part) and coarse row a back to trial a B + b, and writes the
// Y planes or, for one chunk, power spectra |Y|^2 (Re and Im of a fine DM sit in the same lane:
// columns b and b + B are NT/2 tiles apart).
#include "device_math.h"
#include "fdd_internal.h"
#include "split_math.h"

namespace fdd {

namespace {
constexpr int kXcds = 8;
constexpr int kRows = 64;   // coarse rows per workgroup

// tile -> (bin block, coarse row tile).  Each XCD takes a contiguous range of bin blocks, in
// order, and the row tiles of one bin block back to back: neighbouring bin blocks share cache
// lines of X and of the output rows (a block covers only 16-32 bytes of a row), and on one XCD
// those partial lines meet in the same L2 instead of going to memory once per block.
struct TileXY {
  int bb, at;
};
__device__ __forceinline__ TileXY fac_tile(int bid, int n_at, int n_bb) {
  const int xcd = bid % kXcds;
  const int slot = bid / kXcds;
  const int per_xcd = (n_bb + kXcds - 1) / kXcds;
  return {xcd * per_xcd + slot / n_at, slot % n_at};
}
}  // namespace

// ------------------------------------------------------------------------------- FP32

// NT 16-column tiles (2 B N <= 16 NT), FB bins per workgroup, 8 channels per LDS stage.
template <int NT, int FB>
__device__ __forceinline__ void phasor_fac_f32_body(const PhasorArgs& a, const int bid, const int n_at,
                                                    const int n_bb, const int tid) {
  constexpr int KC = 8;
  constexpr int NCOL = NT * 16;
  constexpr int CST = FB * NCOL + 16;     // floats per channel: padding spreads the 4 channels of an MFMA step over banks
  constexpr int PLANE = KC * CST;
  static_assert(KC * NCOL / 2 <= 256, "one staging element per thread");
  __shared__ float bre[PLANE];
  __shared__ float bim[PLANE];

  const TileXY tl = fac_tile(bid, n_at, n_bb);
  if (tl.bb >= n_bb) return;                   // uniform per workgroup, before any barrier
  const int fb0 = tl.bb * FB;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int N = a.n_chunks;
  const int B = a.n_fine;
  const int A = a.n_coarse;
  const int BN = B * N;

  for (int i = tid; i < PLANE; i += 256) {     // columns >= 2 B N stay zero
    bre[i] = 0.0f;
    bim[i] = 0.0f;
  }

  // staging element of this thread: (channel cl of the stage, fine DM b, chunk k)
  const int s_cl = tid / BN;
  const int s_q = tid - s_cl * BN;             // column b N + k
  const int s_b = s_q / N;
  const int s_k = s_q - s_b * N;
  const bool stager = s_cl < KC;
  float4 pf[FB / 2];
  uint4 pv = make_uint4(0u, 0u, 0u, 0u);
  auto fetch = [&](int cb) {
    const int c = cb + s_cl;
    const bool ok = stager && c < a.n_chan;
    const float2* src = a.X + ((int64_t)(ok ? c : 0) * N + s_k) * a.pitch + fb0;
#pragma unroll
    for (int j = 0; j < FB / 2; ++j)
      pf[j] = ok ? *(const float4*)(src + 2 * j) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ok) pv = a.vtab[(int64_t)c * B + s_b];
  };
  auto deposit = [&]() {
    if (!stager) return;
    float2 v, st;
    seed_phasor(pv, (uint32_t)fb0, &v, &st);
    const int base = s_cl * CST + s_q;
#pragma unroll
    for (int j = 0; j < FB / 2; ++j) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float2 x = h ? make_float2(pf[j].z, pf[j].w) : make_float2(pf[j].x, pf[j].y);
        const float2 z = cmul(v, x);
        const int i0 = base + (2 * j + h) * NCOL;
        bre[i0] = z.x;
        bim[i0] = -z.y;
        bre[i0 + BN] = z.y;
        bim[i0 + BN] = z.x;
        v = cmul(v, st);
      }
    }
  };

  int arow = tl.at * kRows + wave * 16 + (lane & 15);
  if (arow >= A) arow = A - 1;                 // a clamped row's results are not stored
  const int cq = lane >> 4;

  floatx4 acc[FB][NT];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[f][nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

  fetch(0);
  for (int cb = 0; cb < a.n_chan; cb += KC) {
    __syncthreads();                           // the previous stage's operands are consumed
    deposit();
    __syncthreads();
    if (cb + KC < a.n_chan) fetch(cb + KC);    // in flight while this stage computes
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int cl = 4 * s + cq;
      int c = cb + cl;
      if (c >= a.n_chan) c = a.n_chan - 1;     // its data were staged as zeros
      float2 w, step;
      seed_phasor(a.ptab[(int64_t)c * A + arow], (uint32_t)fb0, &w, &step);
      float wr[FB], wi[FB];
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        wr[f] = w.x;
        wi[f] = w.y;
        w = cmul(w, step);
      }
      const float* pr = bre + cl * CST + (lane & 15);
      const float* pi = bim + cl * CST + (lane & 15);
#pragma unroll
      for (int f = 0; f < FB; ++f)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[f][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wr[f], pr[f * NCOL + 16 * nt], acc[f][nt], 0, 0, 0);
#pragma unroll
      for (int f = 0; f < FB; ++f)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[f][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wi[f], pi[f * NCOL + 16 * nt], acc[f][nt], 0, 0, 0);
    }
  }

  // D[i][j] of a 16x16 tile sits in lane 16 (i / 4) + j, register i % 4
  if (a.P != nullptr) {
    // one chunk, B = 8 NT: Re of fine DM b in column b (tiles < NT/2), Im in column b + B
#pragma unroll
    for (int nt = 0; nt < NT / 2; ++nt) {
      const int b = 16 * nt + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ar = tl.at * kRows + wave * 16 + 4 * (lane >> 4) + r;
        const int dm = ar * B + b;
        if (ar >= A || dm >= a.n_dm) continue;
        float p[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const float yr = acc[f][nt][r] + ((fb0 + f) == 0 ? a.dc_add : 0.0f);
          const float yi = acc[f][nt + NT / 2][r];
          p[f] = fmaf(yr, yr, yi * yi);
        }
        float* dst = a.P + (int64_t)dm * a.n_pow_bins + fb0;
        if (fb0 + FB <= a.n_pow_bins) {
#pragma unroll
          for (int f = 0; f < FB; f += 4) *(float4*)(dst + f) = make_float4(p[f], p[f + 1], p[f + 2], p[f + 3]);
        } else {
#pragma unroll
          for (int f = 0; f < FB; ++f)
            if (fb0 + f < a.n_pow_bins) dst[f] = p[f];
        }
      }
    }
    return;
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = 16 * nt + (lane & 15);
    if (n >= 2 * BN) continue;
    const bool im = n >= BN;
    const int q = im ? n - BN : n;
    const int b = q / N;
    const int k = q - b * N;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ar = tl.at * kRows + wave * 16 + 4 * (lane >> 4) + r;
      const int dm = ar * B + b;
      if (ar >= A || dm >= a.n_dm) continue;
      float* dst = (im ? a.Yi : a.Yr) + ((int64_t)dm * N + k) * a.pitch + fb0;
#pragma unroll
      for (int f = 0; f < FB; f += 4)
        *(float4*)(dst + f) =
            make_float4(acc[f][nt][r], acc[f + 1][nt][r], acc[f + 2][nt][r], acc[f + 3][nt][r]);
    }
  }
}

// ------------------------------------------------------------------------------- split FP16 / BF16
//
// As the direct split kernel: K = 32 per MFMA = 16 channels x (cos, sin) parts, operands split
// into head + tail, products hi.hi + hi.lo + lo.hi in FP32, every chunk scaled by a power of
// two 2^(14 - ceil(log2 L1_k)) (|Z| = |X| <= L1_k), divided out in the epilogue.

template <bool BF, int NT, int FB>
__device__ __forceinline__ void phasor_fac_split_body(const PhasorArgs& a, const int bid, const int n_at,
                                                      const int n_bb, const int tid) {
  using H = HalfMma<BF>;
  typedef typename H::V8 V8;
  constexpr int KC = 16;
  constexpr int NCOL = NT * 16;
  constexpr int ROWW = 20;                // words per (bin, column): 16 channels + 4 padding
  constexpr int BINW = NCOL * ROWW + 8;
  constexpr int PLANEW = FB * BINW;
  constexpr int PER = (KC * NCOL / 2 + 255) / 256;   // staging elements per thread
  __shared__ uint4 lhi[PLANEW / 4];
  __shared__ uint4 llo[PLANEW / 4];
  __shared__ float colscale[32];
  __shared__ float2 sctab[256];           // phasors of k / 256 turn, for the seeds

  const TileXY tl = fac_tile(bid, n_at, n_bb);
  if (tl.bb >= n_bb) return;
  const int fb0 = tl.bb * FB;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int N = a.n_chunks;
  const int B = a.n_fine;
  const int A = a.n_coarse;
  const int BN = B * N;
  const int nel = KC * BN;

  for (int i = tid; i < PLANEW / 4; i += 256) {
    lhi[i] = make_uint4(0u, 0u, 0u, 0u);
    llo[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (tid < N) colscale[tid] = chunk_scale(a.l1max[tid]);
  sctab[tid] = turn_table_entry((uint32_t)tid);
  uint32_t* whi = reinterpret_cast<uint32_t*>(lhi);
  uint32_t* wlo = reinterpret_cast<uint32_t*>(llo);

  // staging element e = tid + 256 j: channel cl = e % KC (fastest: consecutive LDS words),
  // column q = e / KC = b N + k.  X and the fine table are read through descriptors over the
  // stage's KC channels (channels past n_chan read as zeros), at byte offsets that are the same
  // in every stage; a slot that holds no element points past any window.
  float4 pf[PER][FB / 2];
  uint4 pv[PER];
  uint32_t xoff[PER], voff[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    const int cl = e % KC;
    const int q = e / KC;
    const int b = q / N;
    const int k = q - b * N;
    const bool ok = e < nel;
    xoff[j] = ok ? (uint32_t)((((int64_t)cl * N + k) * a.pitch + fb0) * 8) : 0xFFFFFFF0u;
    voff[j] = ok ? (uint32_t)((cl * B + b) * 16) : 0xFFFFFFF0u;
  }
  auto fetch = [&](int cb) {
    const int nc = min(KC, a.n_chan - cb);
    const __amdgpu_buffer_rsrc_t rx = raw_rsrc(a.X + (int64_t)cb * N * a.pitch, (int64_t)nc * N * a.pitch * 8);
    const __amdgpu_buffer_rsrc_t rv = raw_rsrc(a.vtab + (int64_t)cb * B, (int64_t)nc * B * 16);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
#pragma unroll
      for (int i = 0; i < FB / 2; ++i) pf[j][i] = load_f4(rx, xoff[j] + 16u * i);
      pv[j] = load_u4(rv, voff[j]);
    }
  };
  auto deposit = [&]() {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int e = tid + 256 * j;
      if (e >= nel) continue;
      const int cl = e % KC;
      const int q = e / KC;
      const int k = q - (q / N) * N;
      const float sk = colscale[k];
      float2 v, st;
      seed_phasor_tab(pv[j], (uint32_t)fb0, sctab, &v, &st);
#pragma unroll
      for (int i = 0; i < FB / 2; ++i) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float2 x = h ? make_float2(pf[j][i].z * sk, pf[j][i].w * sk)
                             : make_float2(pf[j][i].x * sk, pf[j][i].y * sk);
          const float2 z = cmul(v, x);
          uint32_t zh, zl;
          split_pair<BF>(z.x, z.y, &zh, &zl);
          const int f = 2 * i + h;
          const int w0 = f * BINW + q * ROWW + cl;          // column q: (Re, -Im)
          const int w1 = f * BINW + (q + BN) * ROWW + cl;   // column q + B N: (Im, Re)
          whi[w0] = neg_hi(zh);
          wlo[w0] = neg_hi(zl);
          whi[w1] = swap16(zh);
          wlo[w1] = swap16(zl);
          v = cmul(v, st);
        }
      }
    }
  };

  int arow = tl.at * kRows + wave * 16 + (lane & 15);
  if (arow >= A) arow = A - 1;
  const int cq = lane >> 4;

  floatx4 acc[FB][NT];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[f][nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

  __syncthreads();                                  // colscale
  fetch(0);
  for (int cb = 0; cb < a.n_chan; cb += KC) {
    __syncthreads();
    deposit();
    __syncthreads();
    if (cb + KC < a.n_chan) fetch(cb + KC);

    // coarse phasors of this lane's row for channels cb + 4 cq .. + 3 (channels past n_chan
    // read as zero entries, against data staged as zeros)
    float2 w[4], st[4];
    {
      const int nc = min(KC, a.n_chan - cb);
      const __amdgpu_buffer_rsrc_t rp = raw_rsrc(a.ptab + (int64_t)cb * A, (int64_t)nc * A * 16);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        seed_phasor_tab(load_u4(rp, (uint32_t)(((4 * cq + q) * A + arow) * 16)), (uint32_t)fb0, sctab, &w[q], &st[q]);
    }
    const int rowbase = (lane & 15) * ROWW + 4 * cq;
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
    const float inv = 1.0f / colscale[0];
#pragma unroll
    for (int nt = 0; nt < NT / 2; ++nt) {
      const int b = 16 * nt + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ar = tl.at * kRows + wave * 16 + 4 * (lane >> 4) + r;
        const int dm = ar * B + b;
        if (ar >= A || dm >= a.n_dm) continue;
        float p[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          const float yr = acc[f][nt][r] * inv + ((fb0 + f) == 0 ? a.dc_add : 0.0f);
          const float yi = acc[f][nt + NT / 2][r] * inv;
          p[f] = fmaf(yr, yr, yi * yi);
        }
        float* dst = a.P + (int64_t)dm * a.n_pow_bins + fb0;
        if (fb0 + FB <= a.n_pow_bins) {
#pragma unroll
          for (int f = 0; f < FB; f += 4) *(float4*)(dst + f) = make_float4(p[f], p[f + 1], p[f + 2], p[f + 3]);
        } else {
#pragma unroll
          for (int f = 0; f < FB; ++f)
            if (fb0 + f < a.n_pow_bins) dst[f] = p[f];
        }
      }
    }
    return;
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = 16 * nt + (lane & 15);
    if (n >= 2 * BN) continue;
    const bool im = n >= BN;
    const int q = im ? n - BN : n;
    const int b = q / N;
    const int k = q - b * N;
    const float inv = 1.0f / colscale[k];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ar = tl.at * kRows + wave * 16 + 4 * (lane >> 4) + r;
      const int dm = ar * B + b;
      if (ar >= A || dm >= a.n_dm) continue;
      float* dst = (im ? a.Yi : a.Yr) + ((int64_t)dm * N + k) * a.pitch + fb0;
#pragma unroll
      for (int f = 0; f < FB; f += 4)
        *(float4*)(dst + f) = make_float4(acc[f][nt][r] * inv, acc[f + 1][nt][r] * inv, acc[f + 2][nt][r] * inv,
                                          acc[f + 3][nt][r] * inv);
    }
  }
}

// ------------------------------------------------------------------------------- launches

namespace {
constexpr int kFacNt = 4;    // 64 columns: B = 32 / N fine DMs
constexpr int kFacFbF32 = 4;
constexpr int kFacFbSplit = 4;

__device__ __forceinline__ int fac_block() { return (int)(blockIdx.y * gridDim.x + blockIdx.x); }
}  // namespace

template <int NT, int FB>
__global__ __launch_bounds__(256) void k_phasor_fac_f32(PhasorArgs a, int n_at, int n_bb) {
  phasor_fac_f32_body<NT, FB>(a, fac_block(), n_at, n_bb, threadIdx.x);
}

template <bool BF, int NT, int FB>
__global__ __launch_bounds__(256, 3) void k_phasor_fac_split(PhasorArgs a, int n_at, int n_bb) {
  phasor_fac_split_body<BF, NT, FB>(a, fac_block(), n_at, n_bb, threadIdx.x);
}

// Batched form: one workgroup per tile of every beam of the group (a.n_dmt = coarse row tiles).
template <int NT, int FB, bool PERSIST>
__global__ __launch_bounds__(256) void k_phasor_fac_f32_grouped(Group<PhasorArgs> g) {
  grouped_tiles<PERSIST>(g.counters, g.total, [&](int t, int tid) {
    const int b = group_beam(g.prefix, g.n_beams, t);
    const PhasorArgs a = PERSIST ? load_uniform(g.beams + b) : g.beams[b];
    phasor_fac_f32_body<NT, FB>(a, t - g.prefix[b], a.n_dmt, a.n_bb, tid);
  });
}

template <bool BF, int NT, int FB, bool PERSIST>
__global__ __launch_bounds__(256, 2) void k_phasor_fac_split_grouped(Group<PhasorArgs> g) {
  grouped_tiles<PERSIST>(g.counters, g.total, [&](int t, int tid) {
    const int b = group_beam(g.prefix, g.n_beams, t);
    const PhasorArgs a = PERSIST ? load_uniform(g.beams + b) : g.beams[b];
    phasor_fac_split_body<BF, NT, FB>(a, t - g.prefix[b], a.n_dmt, a.n_bb, tid);
  });
}

int64_t phasor_fac_tiles(PhasorArgs* a, int precision) {
  const int fb = precision == FDD_FP32 ? kFacFbF32 : kFacFbSplit;
  a->n_dmt = (a->n_coarse + kRows - 1) / kRows;
  a->n_bb = (a->n_bins + fb - 1) / fb;
  return (int64_t)a->n_dmt * ((a->n_bb + kXcds - 1) / kXcds * kXcds);
}

namespace {
template <class K>
hipError_t launch_grouped(K kernel, bool persist, const Group<PhasorArgs>& g, hipStream_t st) {
  hipLaunchKernelGGL(kernel, grouped_grid(persist, (const void*)kernel, g.total), dim3(256), 0, st, g);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_phasor_fac_grouped(int precision, bool persist, const Group<PhasorArgs>& g, hipStream_t st) {
  if (g.total <= 0) return hipSuccess;
  if (precision == FDD_FP32)
    return persist ? launch_grouped(k_phasor_fac_f32_grouped<kFacNt, kFacFbF32, true>, true, g, st)
                   : launch_grouped(k_phasor_fac_f32_grouped<kFacNt, kFacFbF32, false>, false, g, st);
  if (precision == FDD_FP16_SPLIT)
    return persist ? launch_grouped(k_phasor_fac_split_grouped<false, kFacNt, kFacFbSplit, true>, true, g, st)
                   : launch_grouped(k_phasor_fac_split_grouped<false, kFacNt, kFacFbSplit, false>, false, g, st);
  return persist ? launch_grouped(k_phasor_fac_split_grouped<true, kFacNt, kFacFbSplit, true>, true, g, st)
                 : launch_grouped(k_phasor_fac_split_grouped<true, kFacNt, kFacFbSplit, false>, false, g, st);
}

int phasor_fac_fine(int n_chunks) { return n_chunks >= 1 && n_chunks <= 8 * kFacNt / 2 ? 8 * kFacNt / n_chunks : 0; }

hipError_t launch_phasor_fac(const PhasorArgs& a, int precision, hipStream_t st) {
  if (a.n_fine < 1 || 2 * a.n_fine * a.n_chunks > 16 * kFacNt || a.n_coarse < 1 || a.vtab == nullptr)
    return hipErrorInvalidValue;
  if (a.P != nullptr && (a.n_chunks != 1 || a.n_fine != 8 * kFacNt)) return hipErrorInvalidValue;
  const int fb = precision == FDD_FP32 ? kFacFbF32 : kFacFbSplit;
  const int n_at = (a.n_coarse + kRows - 1) / kRows;
  const int n_bb = (a.n_bins + fb - 1) / fb;
  const int n_bb8 = (n_bb + kXcds - 1) / kXcds * kXcds;
  const int64_t blocks = (int64_t)n_at * n_bb8;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid = linear_grid(blocks), block(256);
  if (precision == FDD_FP32)
    hipLaunchKernelGGL((k_phasor_fac_f32<kFacNt, kFacFbF32>), grid, block, 0, st, a, n_at, n_bb);
  else if (precision == FDD_FP16_SPLIT)
    hipLaunchKernelGGL((k_phasor_fac_split<false, kFacNt, kFacFbSplit>), grid, block, 0, st, a, n_at, n_bb);
  else
    hipLaunchKernelGGL((k_phasor_fac_split<true, kFacNt, kFacFbSplit>), grid, block, 0, st, a, n_at, n_bb);
  return hipGetLastError();
}

}  // namespace fdd
