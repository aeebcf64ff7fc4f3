// DM-factorised phasor sum for overlap-save plans (many chunks), on the matrix cores.
//
// Eqs. 4 and 7 with a uniform DM grid DM_j = DM_0 + j dDM and exact delays: Eq. 1 is linear in
// DM, so trial j = a B + b (a "coarse", b "fine") has the delay tau_A[a, c] + tau_B[b, c] and
// the phasor factorises, W[j, c, f] = U[a, c, f] V[b, c, f].  Per Fourier bin f
//     Y[a B + b, k, f] = sum_c U[a, c, f] Z[c, (k, b), f],   Z[c, (k, b), f] = V[b, c, f] X[c, k, f],
// a matrix product [A x n_chan] x [n_chan x B N].  With N chunks the direct product has 2N
// real columns per generated phasor (42 at 21 chunks); here every coarse phasor U serves
// 2 B N of them, so phasor generation (sin/cos, recurrence, head/tail split) drops from the
// main cost of the half-precision kernels to a fraction of the matrix work.
//
// Column order: q = k B + b (fine DM fastest).  The columns are cut into groups of Q = 16 NT;
// a workgroup owns one group, one block of FB bins and 128 coarse rows (4 waves x 32).  In the
// real form of the product, [Yr | Yi] = Ur [Zr | Zi] + Ui [-Zi | Zr], each 32-column tile t of a
// group holds the Re columns of q = 16 t .. 16 t + 15 (tile columns 0..15) and their Im
// columns (16..31), so that after one lane exchange a lane owns both parts of its outputs and
// writes them as complex pairs.
//
// Per stage of 16 channels the workgroup stages Z for its columns and bins in LDS (thread
// (channel slot cl, column j) covers column j of every tile; with B dividing 16 all its columns
// share one fine DM b, so one V phasor per thread and stage, seeded from the fine table), and
// each lane generates the coarse phasors U of its row (one seed from the coarse table per
// channel, a recurrence step per further bin).  LDS holds two stages: while the matrix cores
// work on one, the next one is staged, with one barrier per stage.
//
// Matrix cores: v_mfma_f32_32x32x16_{f16,bf16} (split precisions: head and tail of both operands,
// products hi.hi + hi.lo + lo.hi in float32) and v_mfma_f32_32x32x2_f32 (FP32).  Lane l supplies
// A[l % 32][K-slice l / 32] and B[K-slice l / 32][l % 32]; D[i][j] of a 32x32 tile sits in lane
// 32 (i / 4 % 2) + j, register 4 (i / 8) + i % 4.
//
// Output: Y as interleaved complex [n_dm][n_chunks][pitch] (Yc), FB bins = one 8 FB-byte
// store per (trial, chunk).  Nearest-sample delays do not add, so the planner uses these
// kernels for exact delays on uniform grids only.
#include "device_math.h"
#include "fdd_internal.h"
#include "split_math.h"

namespace fdd {

namespace {
constexpr int kWXcds = 8;
constexpr int kWRows = 128;   // coarse rows per workgroup
constexpr int kWKc = 16;      // channels per LDS stage
constexpr int kWFb = 2;       // bins per workgroup
constexpr int kWValuPerMfma = 7;   // vector instructions scheduled after each product (split kernels)

typedef float floatx16 __attribute__((ext_vector_type(16)));

template <bool BF>
struct HalfMma32;

template <>
struct HalfMma32<false> {
  typedef half8 V8;
  __device__ static __forceinline__ floatx16 mfma(V8 a, V8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct HalfMma32<true> {
  typedef bf16x8 V8;
  __device__ static __forceinline__ floatx16 mfma(V8 a, V8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

struct WTile {
  int bb, rt, g;
  bool ok;
};

// tile -> (bin block, coarse-row tile, column group).  Each XCD takes a contiguous range of
// tiles with the bin block fastest, so the workgroups resident on one XCD at a time cover
// neighbouring bins: they share the L2 lines of X and complete each other's partial lines of Y.
__device__ __forceinline__ WTile facw_tile(int n_bb, int n_rt, int n_g) {
  const int bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int64_t total = (int64_t)n_bb * n_rt * n_g;
  const int64_t per = (total + kWXcds - 1) / kWXcds;
  const int64_t t = (int64_t)(bid % kWXcds) * per + bid / kWXcds;
  WTile w;
  w.ok = t < total;
  w.bb = (int)(t % n_bb);
  const int64_t r = t / n_bb;
  w.rt = (int)(r % n_rt);
  w.g = (int)(r / n_rt);
  return w;
}

// Neither LDS reads nor matrix products may be scheduled across this point (VALU, scalar and
// memory-write work may): placed between a step's operand reads for two steps ahead and its
// products, it keeps the software pipeline's reads ahead of their use instead of letting the
// scheduler sink each read next to the product that needs it.
__device__ __forceinline__ void pin_lds_reads() {
  // VALU 0x002, SALU 0x004, VMEM 0x010/0x020/0x040, DS write 0x200, transcendental 0x400 may
  // cross; not 0x001 (every non-memory instruction, MFMA included), MFMA 0x008 or DS reads
  __builtin_amdgcn_sched_barrier(0x0676);
}

// Workgroup barrier that orders LDS accesses only: global loads in flight stay in flight (a
// full barrier would also wait for every outstanding load, among them the staging data of the
// stage after next).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Row of register r of a 32x32 accumulator in a lane of half h (= lane / 32).
__device__ __forceinline__ int acc_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Column-group geometry shared by both precisions.
struct ColGroup {
  int N, B, A, BN, lgB;
  int q0, kfirst, nks;
  int cl, jq, sb, kb, kstep;   // staging role of this thread
};

template <int NT>
__device__ __forceinline__ ColGroup facw_group(const PhasorArgs& a, const WTile& tl, int tid) {
  ColGroup g;
  g.N = a.n_chunks;
  g.B = a.n_fine;
  g.A = a.n_coarse;
  g.BN = g.B * g.N;
  g.lgB = g.B == 16 ? 4 : 3;
  g.q0 = tl.g * 16 * NT;
  g.kfirst = g.q0 >> g.lgB;
  const int qend = min(g.q0 + 16 * NT, g.BN);
  g.nks = ((qend - 1) >> g.lgB) - g.kfirst + 1;
  g.cl = tid & 15;
  g.jq = tid >> 4;
  const int qb = g.q0 + g.jq;          // this thread's column in tile 0; tile i adds 16
  g.sb = qb & (g.B - 1);               // B divides 16: the same fine DM in every tile
  g.kb = qb >> g.lgB;
  g.kstep = 16 >> g.lgB;
  return g;
}
}  // namespace

// ------------------------------------------------------------------------------- split FP16 / BF16

template <bool BF, int NT>
__global__ __launch_bounds__(256, 1) void k_phasor_facw_split(PhasorArgs a, int n_bb, int n_rt, int n_g) {
  using H = HalfMma32<BF>;
  typedef typename H::V8 V8;
  constexpr int FB = kWFb;
  constexpr int RW = 20;                     // words per (bin, tile, column): 16 channel slots + 4
  constexpr int PW = FB * NT * 32 * RW;      // words per plane
  __shared__ uint4 zs[2 * 2 * PW / 4];       // two stage buffers, each a head plane then a tail plane
  __shared__ float colscale[2 * NT + 2];     // power-of-two scales of the group's chunks
  __shared__ float2 sctab[256];              // phasors of k / 256 turn

  const WTile tl = facw_tile(n_bb, n_rt, n_g);
  if (!tl.ok) return;                        // uniform per workgroup, before any barrier
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, h = lane >> 5;
  const ColGroup g = facw_group<NT>(a, tl, tid);
  const uint32_t f0 = (uint32_t)(tl.bb * FB);
  if (tid < 2 * NT + 2) colscale[tid] = tid < g.nks ? chunk_scale(a.l1max[g.kfirst + tid]) : 1.0f;
  sctab[tid] = turn_table_entry((uint32_t)tid);

  // staging data of a stage, in registers: X of (channel cb + cl, chunk kb + i kstep), bins
  // f0, f0 + 1, and the fine-table entry of (channel, sb).  Each register is loaded again, for
  // the stage after next, as soon as it has been used, so that every load has a whole stage to
  // arrive (the stage barrier does not wait for global loads).
  float4 xr[NT];
  uint4 vr;
  // The stage's window of X (channels cb .. cb + 15) and of the fine table through buffer
  // descriptors: channels past n_chan read as zero, and so stage zeros (columns past B N read
  // other finite data, whose products land in output columns that are not stored).
  auto x_rsrc = [&](int cb) {
    const int nc = min(kWKc, a.n_chan - cb);
    return raw_rsrc(a.X + (int64_t)cb * g.N * a.pitch, (int64_t)nc * g.N * a.pitch * 8);
  };
  auto fetch_x = [&](__amdgpu_buffer_rsrc_t rx, int i) {
    // 24-bit products: rows < 2^24, 8 pitch < 2^24 for L <= 2^16
    xr[i] = load_f4(rx, __umul24((uint32_t)(g.cl * g.N + g.kb + i * g.kstep), (uint32_t)a.pitch * 8u) + f0 * 8u);
  };
  auto fetch_v = [&](int cb) {
    const int nc = min(kWKc, a.n_chan - cb);
    const __amdgpu_buffer_rsrc_t rv = raw_rsrc(a.vtab + (int64_t)cb * g.B, (int64_t)nc * g.B * 16);
    vr = load_u4(rv, (uint32_t)(g.cl * g.B + g.sb) * 16u);
  };
  auto fetch = [&](int cb) {
    fetch_v(cb);
    const __amdgpu_buffer_rsrc_t rx = x_rsrc(cb);
#pragma unroll
    for (int i = 0; i < NT; ++i) fetch_x(rx, i);
  };
  // Z of tile i (both bins), scaled, split and stored in the two column layouts
  float2 v0, v1;
  auto seed_v = [&]() {
    float2 vs;
    seed_phasor_tab(vr, f0, sctab, &v0, &vs);
    v1 = cmul(v0, vs);
  };
  auto deposit = [&](uint32_t* zw, int i) {
    const float sk = BF ? 1.0f : colscale[min(g.kb + i * g.kstep - g.kfirst, 2 * NT + 1)];
#pragma unroll
    for (int f = 0; f < FB; ++f) {
      float2 x = f ? make_float2(xr[i].z, xr[i].w) : make_float2(xr[i].x, xr[i].y);
      if constexpr (!BF) x = make_float2(x.x * sk, x.y * sk);   // BF16 has the range of FP32
      const float2 z = cmul(f ? v1 : v0, x);
      uint32_t zh, zl;
      split_pair<BF>(z.x, z.y, &zh, &zl);
      const int w = ((f * NT + i) * 32 + g.jq) * RW + g.cl;   // Re column: (Zr, -Zi)
      zw[w] = neg_hi(zh);
      zw[PW + w] = neg_hi(zl);
      zw[w + 16 * RW] = swap16(zh);                            // Im column: (Zi, Zr)
      zw[PW + w + 16 * RW] = swap16(zl);
    }
  };

  int arow = tl.rt * kWRows + wave * 32 + (lane & 31);
  if (arow >= g.A) arow = g.A - 1;           // a clamped row's results are not stored
  floatx16 acc[FB][NT];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[f][i][r] = 0.0f;

  // coarse-table entries of this lane's row for the stage's channels cb + 8 s + 4 h + u
  uint4 tn[8];
  // (channels past n_chan read as zero entries: phasor 1, against staged zeros)
  const __amdgpu_buffer_rsrc_t rp = raw_rsrc(a.ptab, (int64_t)a.n_chan * g.A * 16);
  auto fetch_u = [&](int cb, int s) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      tn[4 * s + u] = load_u4(rp, __umul24((uint32_t)(cb + 8 * s + 4 * h + u), (uint32_t)g.A * 16u) + (uint32_t)arow * 16u);
  };

  uint32_t* const zbase = reinterpret_cast<uint32_t*>(zs);
  const int n_st = (a.n_chan + kWKc - 1) / kWKc;
  V8 bh[2][NT], bl[2][NT];
  auto ldblk = [&](const uint32_t* zr, int blk, int r) {
    const int s = blk / FB, f = blk % FB;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int wo = ((f * NT + i) * 32 + (lane & 31)) * RW + 8 * s + 4 * h;
      bh[r][i] = __builtin_bit_cast(V8, *(const uint4*)(zr + wo));
      bl[r][i] = __builtin_bit_cast(V8, *(const uint4*)(zr + PW + wo));
    }
  };
  // coarse phasors: w / sp of K-step 0 (channels cb + 4 h + u), wn / spn of K-step 1
  float2 w[4], sp[4], wn[4], spn[4];
  V8 Ahi, Alo, Nhi, Nlo;                     // A operands of this block and of the next one
  auto split_next = [&](float2* wv, const float2* spv) {
    uint32_t ah[4], al[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      split_pair<BF>(wv[u].x, wv[u].y, &ah[u], &al[u]);
      wv[u] = cmul(wv[u], spv[u]);           // the next bin
    }
    Nhi = __builtin_bit_cast(V8, make_uint4(ah[0], ah[1], ah[2], ah[3]));
    Nlo = __builtin_bit_cast(V8, make_uint4(al[0], al[1], al[2], al[3]));
  };
  auto products = [&](int f, int r) {
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[f][i] = H::mfma(Ahi, bh[r][i], acc[f][i]);
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[f][i] = H::mfma(Ahi, bl[r][i], acc[f][i]);
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[f][i] = H::mfma(Alo, bh[r][i], acc[f][i]);
  };
  // Interleave of a block: every product followed by vector work, the next block's B operand
  // reads spread over the first 2 NT products.  The fence after it keeps each block's share of
  // the vector work (seeds, splits, staging) where the code puts it.
  auto interleave = [&](bool reads) {
#pragma unroll
    for (int i = 0; i < 3 * NT; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, kWValuPerMfma, 0);
      if (reads && i < 2 * NT) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  __syncthreads();                           // colscale
  fetch(0);
  fetch_u(0, 0);
  fetch_u(0, 1);
  seed_v();
#pragma unroll
  for (int i = 0; i < NT; ++i) deposit(zbase, i);
  fetch(kWKc);
#pragma unroll
  for (int u = 0; u < 4; ++u) seed_phasor_tab(tn[u], f0, sctab, &w[u], &sp[u]);
#pragma unroll
  for (int u = 0; u < 2; ++u) seed_phasor_tab(tn[4 + u], f0, sctab, &wn[u], &spn[u]);
  split_next(w, sp);
  Ahi = Nhi;
  Alo = Nlo;
  seed_v();
  fetch_v(2 * kWKc);
  fetch_u(kWKc, 0);
  // Per stage of 16 channels, four blocks (K-step s, bin f) of 3 NT products on the A operands
  // (coarse phasors, split) of one K-step and bin.  Software pipeline: each block splits the
  // next block's A operands, reads its B operands from LDS, and does a quarter of the seeding
  // and staging work of the next stage:
  //   block 0: seeds of K-step 1 (channels 2, 3 of the half), staging of tiles 0, 1
  //   block 1: seeds of the next stage's K-step 0 (channels 0, 1), tiles 2, 3
  //   block 2: the same for channels 2, 3, tiles 4, 5
  //   block 3: seeds of the next stage's K-step 1 (channels 0, 1), tile 6, the next V
  // Coarse-table entries are loaded right after their last use, two blocks or more ahead.
  for (int st = 0; st < n_st; ++st) {
    lds_barrier();                           // stage st staged; the other buffer no longer read
    const uint32_t* zr = zbase + (st & 1) * 2 * PW;
    uint32_t* zw = zbase + ((st + 1) & 1) * 2 * PW;
    const int cb = st * kWKc;
    const __amdgpu_buffer_rsrc_t rxn = x_rsrc(cb + 2 * kWKc);
    ldblk(zr, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    // block 0: K-step 0, bin f0
#pragma unroll
    for (int u = 2; u < 4; ++u) seed_phasor_tab(tn[4 + u], f0, sctab, &wn[u], &spn[u]);
    split_next(w, sp);                       // K-step 0, bin f0 + 1
    ldblk(zr, 1, 1);
#pragma unroll
    for (int i = 0; i < 2 && i < NT; ++i) {
      deposit(zw, i);
      fetch_x(rxn, i);
    }
    fetch_u(cb + kWKc, 1);                   // K-step 1 entries of the next stage (blocks 3 and 0)
    products(0, 0);
    interleave(true);
    Ahi = Nhi;
    Alo = Nlo;
    // block 1: K-step 0, bin f0 + 1
    split_next(wn, spn);                     // K-step 1, bin f0
#pragma unroll
    for (int u = 0; u < 2; ++u) seed_phasor_tab(tn[u], f0, sctab, &w[u], &sp[u]);
    ldblk(zr, 2, 0);
#pragma unroll
    for (int i = 2; i < 4 && i < NT; ++i) {
      deposit(zw, i);
      fetch_x(rxn, i);
    }
    products(1, 1);
    interleave(true);
    Ahi = Nhi;
    Alo = Nlo;
    // block 2: K-step 1, bin f0
    split_next(wn, spn);                     // K-step 1, bin f0 + 1
#pragma unroll
    for (int u = 2; u < 4; ++u) seed_phasor_tab(tn[u], f0, sctab, &w[u], &sp[u]);
    fetch_u(cb + 2 * kWKc, 0);               // K-step 0 entries of the stage after next
    ldblk(zr, 3, 1);
#pragma unroll
    for (int i = 4; i < 6 && i < NT; ++i) {
      deposit(zw, i);
      fetch_x(rxn, i);
    }
    products(0, 0);
    interleave(true);
    Ahi = Nhi;
    Alo = Nlo;
    // block 3: K-step 1, bin f0 + 1
    split_next(w, sp);                       // the next stage's K-step 0, bin f0
#pragma unroll
    for (int u = 0; u < 2; ++u) seed_phasor_tab(tn[4 + u], f0, sctab, &wn[u], &spn[u]);
#pragma unroll
    for (int i = 6; i < NT; ++i) {
      deposit(zw, i);
      fetch_x(rxn, i);
    }
    seed_v();                                // V of the stage after next, for the next deposits
    fetch_v(cb + 3 * kWKc);
    products(1, 1);
    interleave(false);
    Ahi = Nhi;
    Alo = Nlo;
  }

  // Epilogue: lane (column j < 16 of tile i) holds Re of column q = q0 + 16 i + j for the rows
  // of its registers, the lane 16 apart the Im parts.  One exchange gives each lane both parts
  // of half of the rows (registers r of a lane j < 16 with registers r of its partner, registers
  // r + 8 of a lane j >= 16 with those of its partner: v_permlane16_swap of the register pair
  // (r, r + 8)); the scale of chunk k is divided out.  (A select between acc[r] and acc[r + 8]
  // would be folded into a run-time register index, lowered as a chain of compares.)
  const int jj = lane & 31;
  const bool lo16 = jj < 16;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int q = g.q0 + 16 * i + (jj & 15);
    const int k = q >> g.lgB;
    const int b = q & (g.B - 1);
    const float inv = BF ? 1.0f : 1.0f / colscale[min(k - g.kfirst, 2 * NT + 1)];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float2 y[FB];
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(acc[f][i][r]),
                                                         __float_as_uint(acc[f][i][r + 8]), false, false);
        y[f] = make_float2(__uint_as_float(sw[0]) * inv, __uint_as_float(sw[1]) * inv);
      }
      const int ar = tl.rt * kWRows + wave * 32 + acc_row(lo16 ? r : r + 8, h);
      const int dm = ar * g.B + b;
      if (q < g.BN && ar < g.A && dm < a.n_dm)
        *(float4*)(a.Yc + ((int64_t)dm * g.N + k) * a.pitch + f0) = make_float4(y[0].x, y[0].y, y[1].x, y[1].y);
    }
  }
}

// ------------------------------------------------------------------------------- FP32
//
// K = 2 per product: lane half h supplies channel 2 s + h of K-step s, as cos (first product,
// B rows [Zr | Zi]) and sin (second product, B rows [-Zi | Zr]).  One phasor per lane and step.

template <int NT>
__global__ __launch_bounds__(256, 1) void k_phasor_facw_f32(PhasorArgs a, int n_bb, int n_rt, int n_g) {
  constexpr int FB = kWFb;
  constexpr int RW = 17;                     // words per (bin, tile, column): odd, so the 32 columns
                                             // of a 4-byte operand read fall in distinct banks
  constexpr int PW = FB * NT * 32 * RW;      // words per plane
  __shared__ float zs[2 * 2 * PW];           // two stage buffers, each a cos plane then a sin plane

  const WTile tl = facw_tile(n_bb, n_rt, n_g);
  if (!tl.ok) return;
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, h = lane >> 5;
  const ColGroup g = facw_group<NT>(a, tl, tid);
  const uint32_t f0 = (uint32_t)(tl.bb * FB);

  float4 xr[NT];
  uint4 vr;
  // The stage's window of X (channels cb .. cb + 15) and of the fine table through buffer
  // descriptors: channels past n_chan read as zero, and so stage zeros (columns past B N read
  // other finite data, whose products land in output columns that are not stored).
  auto fetch = [&](int cb) {
    const int nc = min(kWKc, a.n_chan - cb);
    const __amdgpu_buffer_rsrc_t rx = raw_rsrc(a.X + (int64_t)cb * g.N * a.pitch, (int64_t)nc * g.N * a.pitch * 8);
    const __amdgpu_buffer_rsrc_t rv = raw_rsrc(a.vtab + (int64_t)cb * g.B, (int64_t)nc * g.B * 16);
    vr = load_u4(rv, (uint32_t)(g.cl * g.B + g.sb) * 16u);
#pragma unroll
    for (int i = 0; i < NT; ++i)   // 24-bit products: rows < 2^24, 8 pitch < 2^24 for L <= 2^16
      xr[i] = load_f4(rx, __umul24((uint32_t)(g.cl * g.N + g.kb + i * g.kstep), (uint32_t)a.pitch * 8u) + f0 * 8u);
  };
  float2 v0, v1;
  auto seed_v = [&]() {
    float2 vs;
    seed_phasor(vr, f0, &v0, &vs);
    v1 = cmul(v0, vs);
  };
  auto deposit = [&](float* zw, int i) {
#pragma unroll
    for (int f = 0; f < FB; ++f) {
      const float2 x = f ? make_float2(xr[i].z, xr[i].w) : make_float2(xr[i].x, xr[i].y);
      const float2 z = cmul(f ? v1 : v0, x);
      const int w = ((f * NT + i) * 32 + g.jq) * RW + g.cl;
      zw[w] = z.x;                 // cos rows: Re column Zr, Im column Zi
      zw[w + 16 * RW] = z.y;
      zw[PW + w] = -z.y;           // sin rows: Re column -Zi, Im column Zr
      zw[PW + w + 16 * RW] = z.x;
    }
  };

  int arow = tl.rt * kWRows + wave * 32 + (lane & 31);
  if (arow >= g.A) arow = g.A - 1;
  floatx16 acc[FB][NT];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[f][i][r] = 0.0f;

  // coarse-table entries of this lane's row for the stage's channels cb + 2 s + h
  uint4 tn[8];
  const __amdgpu_buffer_rsrc_t rp = raw_rsrc(a.ptab, (int64_t)a.n_chan * g.A * 16);
  auto fetch_u = [&](int cb, int s) {
    tn[s] = load_u4(rp, __umul24((uint32_t)(cb + 2 * s + h), (uint32_t)g.A * 16u) + (uint32_t)arow * 16u);
  };

  const int n_st = (a.n_chan + kWKc - 1) / kWKc;
  fetch(0);
#pragma unroll
  for (int s = 0; s < 8; ++s) fetch_u(0, s);
  seed_v();
#pragma unroll
  for (int i = 0; i < NT; ++i) deposit(zs, i);
  fetch(kWKc);
  // As in the split kernel: one branch-free, software-pipelined sequence of steps (K-step s,
  // bin f, tile i) per stage, B operands read two steps ahead, the phasor of K-step s + 1 seeded
  // during K-step s, the next stage's staging spread over the steps.
  constexpr int NS = 8 * FB * NT;
  for (int st = 0; st < n_st; ++st) {
    __syncthreads();
    const float* zr = zs + (st & 1) * 2 * PW;
    float* zw = zs + ((st + 1) & 1) * 2 * PW;
    const int cb = st * kWKc;
    seed_v();
    float bc[3], bs[3];
    auto ldb = [&](int j, int r) {
      const int blk = j / NT, i = j % NT, s = blk / FB, f = blk % FB;
      const int wo = ((f * NT + i) * 32 + (lane & 31)) * RW + 2 * s + h;
      bc[r] = zr[wo];
      bs[r] = zr[PW + wo];
    };
    ldb(0, 0);
    ldb(1, 1);
    pin_lds_reads();
    float2 w, sp, wn, spn;
    seed_phasor(tn[0], f0, &w, &sp);
    fetch_u(cb + kWKc, 0);
    float cw = w.x, sw = w.y;
    // (nested so that each loop stays within the unroller's limits; j = s FB NT + jb)
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int jb = 0; jb < FB * NT; ++jb) {
      const int j = s * FB * NT + jb;
      const int i = jb % NT, f = jb / NT;
      if (i == 0 && j > 0) {
        if (f == 0) {                        // K-step s begins
          w = wn;
          sp = spn;
        } else {
          w = cmul(w, sp);
        }
        cw = w.x;
        sw = w.y;
      }
      if (i == 1 && f == 0 && s + 1 < 8) {   // seed the next K-step's phasor
        seed_phasor(tn[s + 1], f0, &wn, &spn);
        fetch_u(cb + kWKc, s + 1);
      }
      if (j + 2 < NS) ldb(j + 2, (j + 2) % 3);
      pin_lds_reads();
      const int r = j % 3;
      acc[f][i] = __builtin_amdgcn_mfma_f32_32x32x2f32(cw, bc[r], acc[f][i], 0, 0, 0);
      acc[f][i] = __builtin_amdgcn_mfma_f32_32x32x2f32(sw, bs[r], acc[f][i], 0, 0, 0);
      if (j % 16 == 7 && j / 16 < NT) deposit(zw, j / 16);
    }
    fetch((st + 2) * kWKc);
  }

  const int jj = lane & 31;
  const bool lo16 = jj < 16;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int q = g.q0 + 16 * i + (jj & 15);
    const int k = q >> g.lgB;
    const int b = q & (g.B - 1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float2 y[FB];
#pragma unroll
      for (int f = 0; f < FB; ++f) {   // the exchange of the split kernel's epilogue
        const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(acc[f][i][r]),
                                                         __float_as_uint(acc[f][i][r + 8]), false, false);
        y[f] = make_float2(__uint_as_float(sw[0]), __uint_as_float(sw[1]));
      }
      const int ar = tl.rt * kWRows + wave * 32 + acc_row(lo16 ? r : r + 8, h);
      const int dm = ar * g.B + b;
      if (q < g.BN && ar < g.A && dm < a.n_dm)
        *(float4*)(a.Yc + ((int64_t)dm * g.N + k) * a.pitch + f0) = make_float4(y[0].x, y[0].y, y[1].x, y[1].y);
    }
  }
}

// ------------------------------------------------------------------------------- host side

namespace {
struct FacwGrid {
  int n_bb, n_rt, n_g;
  int64_t blocks;
};

FacwGrid facw_grid(int n_bins, int n_coarse, int n_fine, int n_chunks, int nt) {
  FacwGrid g;
  g.n_bb = (n_bins + kWFb - 1) / kWFb;
  g.n_rt = (n_coarse + kWRows - 1) / kWRows;
  g.n_g = (n_fine * n_chunks + 16 * nt - 1) / (16 * nt);
  const int64_t total = (int64_t)g.n_bb * g.n_rt * g.n_g;
  g.blocks = (total + kWXcds - 1) / kWXcds * kWXcds;
  return g;
}

template <int NT>
hipError_t launch_facw_nt(const PhasorArgs& a, int precision, hipStream_t st) {
  const FacwGrid fg = facw_grid(a.n_bins, a.n_coarse, a.n_fine, a.n_chunks, NT);
  if (fg.blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid = linear_grid(fg.blocks), block(256);
  if (precision == FDD_FP32)
    hipLaunchKernelGGL((k_phasor_facw_f32<NT>), grid, block, 0, st, a, fg.n_bb, fg.n_rt, fg.n_g);
  else if (precision == FDD_FP16_SPLIT)
    hipLaunchKernelGGL((k_phasor_facw_split<false, NT>), grid, block, 0, st, a, fg.n_bb, fg.n_rt, fg.n_g);
  else
    hipLaunchKernelGGL((k_phasor_facw_split<true, NT>), grid, block, 0, st, a, fg.n_bb, fg.n_rt, fg.n_g);
  return hipGetLastError();
}
}  // namespace

FacwChoice facw_choose(int n_dm, int n_chunks) {
  // Time per workgroup tile by column-tile count nt = 4, 5, 6, 7, measured with the FP16 split
  // kernel on the paper-shaped bin and channel counts (ms per column group of 128 coarse rows
  // over all bins): the 7-tile shape is the fastest per tile (1.8 ms against 2.9-3.7), the
  // 4-tile one the cheapest per group.
  constexpr double kTileCost[kFacwNtMax - kFacwNtMin + 1] = {11.4, 15.7, 21.9, 12.7};
  constexpr double kFacwMinEff = 0.7;
  FacwChoice best;
  double best_cost = 0.0;
  for (int fine : {16, 8}) {
    const int coarse = (n_dm + fine - 1) / fine;
    for (int nt = kFacwNtMin; nt <= kFacwNtMax; ++nt) {
      const int64_t rt = (coarse + kWRows - 1) / kWRows;
      const int64_t grp = ((int64_t)fine * n_chunks + 16 * nt - 1) / (16 * nt);
      // useful (trial, chunk) pairs over the padded tile area (coarse rows x columns)
      const double eff = (double)n_dm * n_chunks / ((double)rt * kWRows * (double)grp * 16 * nt);
      const double cost = (double)rt * (double)grp * kTileCost[nt - kFacwNtMin];
      // shapes that pad more than 30 % of the tile area are not taken (the planner then keeps
      // the direct kernels when no shape is left)
      if (eff < kFacwMinEff) continue;
      if (best.fine == 0 || cost < best_cost) {
        best.fine = fine;
        best.coarse = coarse;
        best.nt = nt;
        best.eff = eff;
        best_cost = cost;
      }
    }
  }
  return best;
}

hipError_t launch_phasor_facw(const PhasorArgs& a, int precision, int nt, hipStream_t st) {
  if ((a.n_fine != 8 && a.n_fine != 16) || a.n_coarse < 1 || a.vtab == nullptr || a.Yc == nullptr ||
      a.P != nullptr || a.l1max == nullptr)
    return hipErrorInvalidValue;
  switch (nt) {
    case 4: return launch_facw_nt<4>(a, precision, st);
    case 5: return launch_facw_nt<5>(a, precision, st);
    case 6: return launch_facw_nt<6>(a, precision, st);
    case 7: return launch_facw_nt<7>(a, precision, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdd
