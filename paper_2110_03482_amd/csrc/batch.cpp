// Batched form: many beams (one plan each) dedispersed by grouped kernel launches.
//
// Sec. 3 of the paper processes channels and DMs in batches sized to the device memory and
// Sec. 5 proposes autotuning those parameters and processing beams observed together.  On
// MI355X one beam rarely fills the chip in every stage (a 256-channel, 2-chunk beam has only
// 512 forward transforms), so the batch runs each stage once for all beams of a memory wave:
//
//   zero counters -> [per wave: transpose (8-bit beams) -> grouped R2C per FFT length ->
//   grouped phasor sum per shape class -> grouped C2R per FFT length]
//
// Grouped kernels find their beam from a prefix sum over per-beam tile counts, so beams of
// any n_chan / n_samp / n_dm share a launch.  With FDD_BATCH_SHARE_PHASORS, beams observed with
// one set-up (same channels, DMs, sampling, FFT length and overlap) are stacked along the chunk
// axis into one phasor-sum problem: every phasor then serves the chunks of all of them (the
// Sec. 5 outlook of reusing phase rotations across beams), and single-chunk beams become
// matrix products with one column pair per beam.  The phasor sum of every shape class (precision,
// FFT length, chunk-column tiles) has several candidate kernels: the matrix-core tile shapes,
// one-workgroup-per-tile or persistent launches, and the DM-factorised kernels where the DM
// grid is uniform (the vector-ALU kernel serves the shapes matrix cores do not).  The autotuner
// times each candidate on the batch's own data on the first call and keeps the fastest, in
// memory and optionally in a JSON cache file.  The launch sequence is then captured into one
// HIP graph that every later call replays with a single launch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <sstream>

#include "fdd_internal.h"

using namespace fdd;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

enum Kind { kValu = 0, kMfmaF32 = 1, kSplitF16 = 2, kSplitBf16 = 3, kFac = 4 };

struct Choice {
  int kind = kValu;
  int variant = 0;       // matrix-core tile variant, chunks per thread of the VALU kernel, or the
                         // precision of a DM-factorised kernel
  bool persist = false;
  std::string name() const {
    char buf[64];
    switch (kind) {
      case kMfmaF32: std::snprintf(buf, sizeof buf, "mfma_f32/v%d/%s", variant, persist ? "persistent" : "grid"); break;
      case kSplitF16: std::snprintf(buf, sizeof buf, "mfma_f16_split/%s", persist ? "persistent" : "grid"); break;
      case kSplitBf16: std::snprintf(buf, sizeof buf, "mfma_bf16_split/%s", persist ? "persistent" : "grid"); break;
      case kFac: std::snprintf(buf, sizeof buf, "fac_%s/%s", variant == FDD_FP32 ? "f32" : variant == FDD_FP16_SPLIT ? "f16_split" : "bf16_split",
                               persist ? "persistent" : "grid"); break;
      default: std::snprintf(buf, sizeof buf, "valu/nk%d", variant); break;
    }
    return buf;
  }
};

struct Beam {
  fdd_plan_t plan = nullptr;
  int stack = 0;            // the phasor-sum problem this beam's chunks belong to
  int koff = 0;             // first chunk of this beam in its stack
  size_t xt = 0;            // transposed 8-bit input, offset in the stack's scratch
};

// One phasor-sum problem: a beam, or beams sharing a set-up stacked along the chunk axis.
struct Stack {
  std::vector<int> beams;
  const fdd_plan_s* rep = nullptr;   // a member plan (the set-up they share)
  int n_chunks = 0;                  // chunks of all members (matrix-core column pairs)
  int wave = 0;
  int cls = 0;                       // phasor shape class
  size_t tab = 0;                    // phase table (table arena)
  size_t ftab = 0;                   // DM-factorised tables (table arena), if fine > 0
  int fine = 0, coarse = 0;          // DM factorisation (0: DM list not uniform, or rounded delays)
  double dm0 = 0.0, step = 0.0;
  size_t tw = 0;                     // twiddles (table arena)
  size_t l1 = 0;                     // per-chunk L1 maxima (word index in the small arena), split only
  size_t X = 0, Yr = 0, Yi = 0;      // offsets in the stack's scratch
  size_t scratch = 0;                // base of the stack's scratch in the arena
  size_t bytes = 0;                  // size of the stack's scratch
};

struct Class {
  std::string key;
  int nt = 1;                 // 16-column tiles of the chunk axis (2 N columns)
  std::vector<Choice> cands;  // cands[0] is the single-plan choice
  std::vector<float> ms;      // measured per candidate (< 0: not timed)
  int choice = 0;
  bool settled = false;       // tuned, cached, or only one candidate
};

enum Stage { kTranspose = 0, kR2c = 1, kPhasor = 2, kC2r = 3 };

struct Launch {
  Stage stage = kR2c;
  int wave = 0;
  int log_n = 0;              // FFT stages: log2(L / 2)
  bool u8 = false;
  int cls = -1;               // phasor stage
  std::vector<int> beams;     // beams (transpose, FFT stages) or stacks (phasor stage)
  size_t args = 0, prefix = 0;   // descriptor buffer offsets
  size_t ctr = 0;             // phasor stage: word index of its 8 ticket counters
  int slots = 0;              // descriptors room: beams, or the stacks' chunk groups (phasor stage)
  int n_desc = 0;             // descriptors written for the current choice
  int total = 0;
};

// Process-wide autotune results, keyed by device architecture and shape class.
std::mutex g_tune_mu;
std::map<std::string, std::string> g_tune;

bool load_cache_file(const std::string& path, std::map<std::string, std::string>* out) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  // flat JSON object of string -> string; keys and values hold no quotes or escapes
  size_t i = 0;
  auto next_str = [&](std::string* v) {
    const size_t a = s.find('"', i);
    if (a == std::string::npos) return false;
    const size_t b = s.find('"', a + 1);
    if (b == std::string::npos) return false;
    *v = s.substr(a + 1, b - a - 1);
    i = b + 1;
    return true;
  };
  std::string k, v;
  while (next_str(&k) && next_str(&v)) (*out)[k] = v;
  return true;
}

bool save_cache_file(const std::string& path, const std::map<std::string, std::string>& m) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\n";
    size_t n = 0;
    for (const auto& kv : m) f << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++n < m.size() ? ",\n" : "\n");
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

struct fdd_batch_s {
  std::vector<Beam> beams;
  std::vector<Stack> stacks;
  std::vector<Class> classes;
  std::vector<Launch> launches;
  int n_waves = 0;
  uint32_t flags = 0;
  std::string cache_path, arch;
  uint8_t* d_tab = nullptr;
  size_t tab_bytes = 0;
  uint8_t* d_scr = nullptr;
  size_t scr_bytes = 0;
  unsigned int* d_small = nullptr;   // ticket counters, then L1 maxima; zeroed by every call
  size_t small_words = 0;
  uint8_t* d_desc = nullptr;
  std::vector<uint8_t> h_desc;
  std::vector<const void*> last_in;
  std::vector<float*> last_out;
  bool ready = false;                // descriptors and graph match last_in / last_out
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  hipEvent_t done = nullptr;         // recorded after every call's launches
  hipStream_t last_st = nullptr;     // stream of the last call
  bool launched = false;
};

namespace {

void release(fdd_batch_s* b) {
  if (b->exec != nullptr) (void)hipGraphExecDestroy(b->exec);
  if (b->graph != nullptr) (void)hipGraphDestroy(b->graph);
  if (b->cap != nullptr) (void)hipStreamDestroy(b->cap);
  if (b->done != nullptr) (void)hipEventDestroy(b->done);
  for (void* p : {(void*)b->d_tab, (void*)b->d_scr, (void*)b->d_small, (void*)b->d_desc})
    if (p != nullptr) (void)hipFree(p);
  b->exec = nullptr;
  b->graph = nullptr;
  b->cap = nullptr;
  b->done = nullptr;
}

const Choice& chosen(const fdd_batch_s* b, const Launch& l) {
  const Class& c = b->classes[(size_t)l.cls];
  return c.cands[(size_t)c.choice];
}

// Candidate kernels of the phasor sum for a plan's precision and chunk count; `fac` adds the
// DM-factorised kernels (uniform DM grid, exact delays).  cands[0] is what fdd_execute runs.
Class make_class(const fdd_plan_s* p, int N, bool fac, bool fac_default) {
  Class c;
  // the direct matrix-core kernels run over chunk groups of at most kDirectMaxChunks
  const int NG = chunk_group_max(N);
  c.nt = (2 * NG + 15) / 16;
  char key[112];
  const int prec = p->desc.precision;
  const char* fs = fac_default ? "+fac0" : fac ? "+fac" : "";
  if (prec == FDD_FP16_SPLIT || prec == FDD_BF16_SPLIT) {
    const int kind = prec == FDD_FP16_SPLIT ? kSplitF16 : kSplitBf16;
    std::snprintf(key, sizeof key, "%s/L%lld/nt%d%s", kind == kSplitF16 ? "f16split" : "bf16split",
                  (long long)p->L, c.nt, fs);
    c.cands.push_back({kind, 0, false});
    c.cands.push_back({kind, 0, true});
  } else if (N == 1) {
    std::snprintf(key, sizeof key, "fp32/L%lld/n1%s", (long long)p->L, fs);
    c.cands.push_back({kValu, 1, false});
  } else {
    // the single plan keeps these on the VALU (few chunks, or rows too long for the kernels'
    // 2 GiB descriptor window)
    const bool small = !phasor_mfma_f32_supported(NG) || !phasor_mfma_f32_window_ok(N, p->pitch);
    std::snprintf(key, sizeof key, "fp32/L%lld/%s%d%s", (long long)p->L, small ? "n" : "nt", small ? N : c.nt, fs);
    if (small) c.cands.push_back({kValu, 4, false});
    else
      for (int v = 0; v < kMfmaF32Variants; ++v)
        for (int per = 0; per < 2; ++per) c.cands.push_back({kMfmaF32, v, per == 1});
  }
  if (fac || fac_default) {
    const Choice g{kFac, prec, false}, q{kFac, prec, true};
    if (fac_default) c.cands.insert(c.cands.begin(), g);
    else c.cands.push_back(g);
    c.cands.push_back(q);
  }
  c.key = key;
  c.ms.assign(c.cands.size(), -1.0f);
  c.settled = c.cands.size() == 1;
  return c;
}

// Scratch bytes of one stack: its members' transposed 8-bit inputs, X and the two Y planes.
size_t stack_scratch(fdd_batch_s* b, Stack* sk) {
  const fdd_plan_s* p = sk->rep;
  size_t off = 0;
  for (int i : sk->beams) {
    Beam& bm = b->beams[(size_t)i];
    const fdd_plan_desc& d = bm.plan->desc;
    bm.xt = off;
    if (d.input == FDD_IN_U8_TIME_MAJOR) off = align_up(off + (size_t)d.n_chan * (size_t)d.n_samp);
  }
  sk->X = off;
  off = align_up(off + (size_t)p->desc.n_chan * (size_t)sk->n_chunks * (size_t)p->pitch * sizeof(float2));
  sk->Yr = off;
  const size_t yb = (size_t)p->desc.n_dm * (size_t)sk->n_chunks * (size_t)p->pitch * sizeof(float);
  off = align_up(off + yb);
  sk->Yi = off;
  off = align_up(off + yb);
  return off;
}

// Whether two plans share a set-up, so that their chunks can share phasors.
bool same_setup(const fdd_plan_s* x, const fdd_plan_s* y) {
  const fdd_plan_desc &a = x->desc, &c = y->desc;
  return a.n_chan == c.n_chan && a.n_dm == c.n_dm && a.ref_freq_mhz == c.ref_freq_mhz && a.tsamp_s == c.tsamp_s &&
         x->L == y->L && x->S == y->S && a.single_chunk == c.single_chunk && a.precision == c.precision &&
         a.delay_mode == c.delay_mode && x->freqs == y->freqs && x->dms == y->dms;
}

// Host copy of the launch descriptors for the given pointers and the current choices.
fdd_status fill(fdd_batch_s* b, const void* const* in, float* const* out) {
  std::fill(b->h_desc.begin(), b->h_desc.end(), 0);
  for (Launch& l : b->launches) {
    if (l.stage == kTranspose) continue;
    int64_t acc = 0;
    int* prefix = (int*)(b->h_desc.data() + l.prefix);
    int nd = 0;                                     // descriptors written
    for (size_t i = 0; i < l.beams.size(); ++i) {
      int64_t tiles = 0;
      if (l.stage == kPhasor) {
        const Stack& sk = b->stacks[(size_t)l.beams[i]];
        const fdd_plan_s* p = sk.rep;
        const fdd_plan_desc& d = p->desc;
        uint8_t* scr = b->d_scr + sk.scratch;
        PhasorArgs a;
        a.X = (const float2*)(scr + sk.X);
        a.Yr = (float*)(scr + sk.Yr);
        a.Yi = (float*)(scr + sk.Yi);
        a.ptab = (const uint4*)(b->d_tab + sk.tab);
        a.l1max = d.precision != FDD_FP32 ? b->d_small + sk.l1 : nullptr;
        a.n_dm = d.n_dm;
        a.n_chan = d.n_chan;
        a.n_chunks = sk.n_chunks;
        a.pitch = p->pitch;
        a.n_bins = (int)p->n_bins;
        a.n_pow_bins = (int)(p->L / 2);
        a.log_len = p->log_len;
        const Choice& ch = chosen(b, l);
        a.tile_variant = ch.kind == kMfmaF32 ? ch.variant : 0;
        if (ch.kind == kFac) {
          a.ptab = (const uint4*)(b->d_tab + sk.ftab);
          a.vtab = a.ptab + (size_t)d.n_chan * (size_t)sk.coarse;
          a.n_coarse = sk.coarse;
          a.n_fine = sk.fine;
          tiles = phasor_fac_tiles(&a, d.precision);
        } else if (ch.kind == kValu) {
          tiles = phasor_valu_tiles(&a, ch.variant);
        } else {
          // direct matrix-core kernels: one descriptor per chunk group
          const int ng = chunk_groups(a.n_chunks);
          for (int g = 0; g < ng; ++g) {
            PhasorArgs t = chunk_group_args(a, g);
            const int64_t tg = ch.kind == kMfmaF32 ? phasor_mfma_f32_tiles(&t, ch.variant) : phasor_split_tiles(&t);
            if (g + 1 == ng) {
              a = t;
              tiles = tg;
              break;
            }
            prefix[nd] = (int)acc;
            std::memcpy(b->h_desc.data() + l.args + (size_t)nd * sizeof(PhasorArgs), &t, sizeof t);
            ++nd;
            acc += tg;
            if (acc > std::numeric_limits<int>::max())
              return fail(FDD_E_UNSUPPORTED, "too many tiles in one grouped launch");
          }
        }
        prefix[nd] = (int)acc;
        std::memcpy(b->h_desc.data() + l.args + (size_t)nd * sizeof(PhasorArgs), &a, sizeof a);
        ++nd;
      } else {
        const Beam& bm = b->beams[(size_t)l.beams[i]];
        const Stack& sk = b->stacks[(size_t)bm.stack];
        const fdd_plan_s* p = bm.plan;
        const fdd_plan_desc& d = p->desc;
        uint8_t* scr = b->d_scr + sk.scratch;
        FftArgs f;
        f.twL = (const float2*)(b->d_tab + sk.tw);
        f.n_samp = d.n_samp;
        f.stride = p->S;
        f.pitch = p->pitch;
        f.n_chunks = (int)p->n_chunks;
        f.row_chunks = sk.n_chunks;
        f.log_n = p->log_len - 1;
        if (l.stage == kR2c) {
          if (d.input == FDD_IN_U8_TIME_MAJOR) f.in_u8 = scr + bm.xt;
          else f.in_f32 = (const float*)in[l.beams[i]];
          f.X = (float2*)(scr + sk.X) + (size_t)bm.koff * (size_t)p->pitch;
          f.n_rows = d.n_chan;
          f.l1max = d.precision != FDD_FP32 ? b->d_small + sk.l1 + bm.koff : nullptr;
        } else {
          f.Yr = (const float*)(scr + sk.Yr) + (size_t)bm.koff * (size_t)p->pitch;
          f.Yi = (const float*)(scr + sk.Yi) + (size_t)bm.koff * (size_t)p->pitch;
          f.out = out[l.beams[i]];
          f.keep = d.single_chunk ? d.n_samp : p->S;
          f.n_rows = d.n_dm;
          f.add_full = d.input == FDD_IN_U8_TIME_MAJOR ? 128.0f * (float)d.n_chan : 0.0f;
        }
        tiles = fft_grouped_tiles(f);
        prefix[nd] = (int)acc;
        std::memcpy(b->h_desc.data() + l.args + (size_t)nd * sizeof(FftArgs), &f, sizeof f);
        ++nd;
      }
      acc += tiles;
      if (acc > std::numeric_limits<int>::max()) return fail(FDD_E_UNSUPPORTED, "too many tiles in one grouped launch");
    }
    prefix[nd] = (int)acc;
    l.n_desc = nd;
    l.total = (int)acc;
  }
  return FDD_OK;
}

fdd_status upload(fdd_batch_s* b) {
  hipError_t e = hipMemcpy(b->d_desc, b->h_desc.data(), b->h_desc.size(), hipMemcpyHostToDevice);
  return e == hipSuccess ? FDD_OK : hip_fail(e, "hipMemcpy(batch descriptors)");
}

hipError_t enqueue_launch(fdd_batch_s* b, const Launch& l, const void* const* in, hipStream_t st) {
  switch (l.stage) {
    case kTranspose: {
      const Beam& bm = b->beams[(size_t)l.beams[0]];
      const fdd_plan_desc& d = bm.plan->desc;
      return launch_transpose_u8((const uint8_t*)in[l.beams[0]], b->d_scr + b->stacks[(size_t)bm.stack].scratch + bm.xt,
                                 d.n_samp, d.n_chan, st);
    }
    case kR2c:
    case kC2r: {
      Group<FftArgs> g;
      g.beams = (const FftArgs*)(b->d_desc + l.args);
      g.prefix = (const int*)(b->d_desc + l.prefix);
      g.n_beams = l.n_desc;
      g.total = l.total;
      return l.stage == kR2c ? launch_r2c_grouped(l.log_n, l.u8, g, st) : launch_c2r_grouped(l.log_n, g, st);
    }
    case kPhasor: {
      Group<PhasorArgs> g;
      g.beams = (const PhasorArgs*)(b->d_desc + l.args);
      g.prefix = (const int*)(b->d_desc + l.prefix);
      g.counters = b->d_small + l.ctr;
      g.n_beams = l.n_desc;
      g.total = l.total;
      const Choice& ch = chosen(b, l);
      const int nt = b->classes[(size_t)l.cls].nt;
      switch (ch.kind) {
        case kMfmaF32: return launch_phasor_mfma_f32_grouped(nt, ch.variant, ch.persist, g, st);
        case kSplitF16: return launch_phasor_split_grouped(false, nt, ch.persist, g, st);
        case kSplitBf16: return launch_phasor_split_grouped(true, nt, ch.persist, g, st);
        case kFac: return launch_phasor_fac_grouped(ch.variant, ch.persist, g, st);
        default: return launch_phasor_valu_grouped(ch.variant, g, st);
      }
    }
  }
  return hipErrorInvalidValue;
}

fdd_status enqueue_all(fdd_batch_s* b, const void* const* in, hipStream_t st) {
  hipError_t e = launch_zero_u32(b->d_small, (int64_t)b->small_words, st);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  for (const Launch& l : b->launches) {
    e = enqueue_launch(b, l, in, st);
    if (e != hipSuccess) return hip_fail(e, "grouped launch");
  }
  return FDD_OK;
}

// Time every candidate of every unsettled class on the beams of the first wave holding it:
// the wave's forward stages run once, then each candidate runs once to warm up and is timed
// (the best of three when a run is shorter than 50 ms).  A candidate whose warm-up is already
// kPrune times slower than the class's best timed run so far keeps its warm-up time and is
// not timed again.  Synchronises the stream.
constexpr float kPrune = 1.5f;

fdd_status autotune(fdd_batch_s* b, const void* const* in, float* const* out, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0 != nullptr) (void)hipEventDestroy(e0);
    return fail(FDD_E_DEVICE, "hipEventCreate failed");
  }
  fdd_status s = FDD_OK;
  auto check = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && s == FDD_OK) s = hip_fail(e, what);
    return s == FDD_OK;
  };
  for (int w = 0; w < b->n_waves && s == FDD_OK; ++w) {
    bool needed = false;
    for (const Launch& l : b->launches)
      if (l.wave == w && l.stage == kPhasor && !b->classes[(size_t)l.cls].settled) needed = true;
    if (!needed) continue;
    s = fill(b, in, out);
    if (s == FDD_OK) s = upload(b);
    if (s != FDD_OK) break;
    if (!check(launch_zero_u32(b->d_small, (int64_t)b->small_words, st), "zero launch")) break;
    for (const Launch& l : b->launches)
      if (l.wave == w && (l.stage == kTranspose || l.stage == kR2c))
        if (!check(enqueue_launch(b, l, in, st), "forward launch")) break;
    for (Launch& l : b->launches) {
      if (s != FDD_OK) break;
      if (l.wave != w || l.stage != kPhasor) continue;
      Class& c = b->classes[(size_t)l.cls];
      if (c.settled) continue;
      float lead = -1.0f;                                  // best timed run of the class so far
      for (size_t k = 0; k < c.cands.size() && s == FDD_OK; ++k) {
        c.choice = (int)k;
        s = fill(b, in, out);
        if (s == FDD_OK) s = upload(b);
        float best = -1.0f;
        for (int rep = 0; rep < 4 && s == FDD_OK; ++rep) {
          if (!check(launch_zero_u32(b->d_small + l.ctr, 8, st), "zero launch")) break;
          if (!check(hipEventRecord(e0, st), "hipEventRecord")) break;
          if (!check(enqueue_launch(b, l, in, st), "tuning launch")) break;
          if (!check(hipEventRecord(e1, st), "hipEventRecord")) break;
          if (!check(hipEventSynchronize(e1), "hipEventSynchronize")) break;
          float ms = 0.0f;
          if (!check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) break;
          if (rep == 0) {                                  // warm-up
            if (lead > 0.0f && ms > kPrune * lead) {       // clearly slower: keep the warm-up time
              best = ms;
              break;
            }
            continue;
          }
          if (best < 0.0f || ms < best) best = ms;
          if (rep == 1 && ms >= 50.0f) break;
        }
        c.ms[k] = best;
        if (best >= 0.0f && (lead < 0.0f || best < lead)) lead = best;
      }
      if (s != FDD_OK) break;
      int arg = 0;
      for (size_t k = 1; k < c.cands.size(); ++k)
        if (c.ms[k] >= 0.0f && (c.ms[(size_t)arg] < 0.0f || c.ms[k] < c.ms[(size_t)arg])) arg = (int)k;
      c.choice = arg;
      c.settled = true;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[b->arch + "|" + c.key] = c.cands[(size_t)arg].name();
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s == FDD_OK && !b->cache_path.empty()) {
    std::map<std::string, std::string> m;
    (void)load_cache_file(b->cache_path, &m);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      for (const auto& kv : g_tune) m[kv.first] = kv.second;
    }
    if (!save_cache_file(b->cache_path, m)) return fail(FDD_E_INVALID, "cannot write the autotune cache " + b->cache_path);
  }
  return s;
}

}  // namespace

extern "C" {

fdd_status fdd_batch_create(int32_t n, const fdd_plan_t* plans, const fdd_batch_desc* desc, fdd_batch_t* out) {
  if (out == nullptr) return fail(FDD_E_INVALID, "null output");
  *out = nullptr;
  if (n < 1 || plans == nullptr) return fail(FDD_E_INVALID, "a batch needs at least one plan");
  fdd_batch_desc dd{};
  if (desc != nullptr) dd = *desc;
  if (dd.reserved != 0 || (dd.flags & ~(FDD_BATCH_NO_GRAPH | FDD_BATCH_NO_AUTOTUNE | FDD_BATCH_SHARE_PHASORS)) != 0)
    return fail(FDD_E_INVALID, "unknown batch flags or nonzero reserved field");
  for (int32_t i = 0; i < n; ++i) {
    const fdd_plan_s* p = plans[i];
    if (p == nullptr) return fail(FDD_E_INVALID, "null plan in batch");
    if (p->dry_run) return fail(FDD_E_INVALID, "a dry-run plan cannot be batched");
    if (p->desc.flags & FDD_PLAN_POWER_ONLY) return fail(FDD_E_UNSUPPORTED, "power-only plans cannot be batched");
    if (p->log_len - 1 > kMaxBlockLogN) return fail(FDD_E_UNSUPPORTED, "batched beams need chunk_len <= 2^16");
    if (p->segs.size() != 1 || p->segs[0].factor != 1)
      return fail(FDD_E_UNSUPPORTED, "batched beams take no down-sampled output");
  }
  fdd_batch_s* b = new (std::nothrow) fdd_batch_s();
  if (b == nullptr) return fail(FDD_E_NOMEM, "host allocation failed");
  b->flags = dd.flags;
  if (dd.tune_cache != nullptr) b->cache_path = dd.tune_cache;
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete b;
    return fail(FDD_E_DEVICE, "no HIP device");
  }
  b->arch = prop.gcnArchName;
  std::map<std::string, std::string> cached;
  if (!b->cache_path.empty()) (void)load_cache_file(b->cache_path, &cached);

  // beams and stacks: with FDD_BATCH_SHARE_PHASORS, beams of one set-up fill stacks of up to
  // kMaxStackChunks chunks in order; otherwise every beam is a stack of its own
  constexpr int kMaxStackChunks = 24;
  b->beams.resize((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    Beam& bm = b->beams[(size_t)i];
    bm.plan = plans[i];
    int target = -1;
    if (dd.flags & FDD_BATCH_SHARE_PHASORS)
      for (size_t k = 0; k < b->stacks.size() && target < 0; ++k) {
        const Stack& sk = b->stacks[k];
        if (same_setup(sk.rep, bm.plan) && sk.n_chunks + bm.plan->n_chunks <= kMaxStackChunks) target = (int)k;
      }
    if (target < 0) {
      target = (int)b->stacks.size();
      b->stacks.emplace_back();
      b->stacks.back().rep = bm.plan;
    }
    Stack& sk = b->stacks[(size_t)target];
    bm.stack = target;
    bm.koff = sk.n_chunks;
    sk.n_chunks += (int)bm.plan->n_chunks;
    sk.beams.push_back(i);
  }

  // shape classes of the stacks (tuning state from the process cache or the file)
  std::map<std::string, int> class_of;
  for (Stack& sk : b->stacks) {
    const fdd_plan_s* p = sk.rep;
    const int fine = phasor_fac_fine(sk.n_chunks);
    if (p->desc.delay_mode == FDD_DELAY_EXACT && fine > 0 && uniform_grid(p->dms, &sk.dm0, &sk.step)) {
      sk.fine = fine;
      sk.coarse = (p->desc.n_dm + fine - 1) / fine;
    }
    // the kernel fdd_execute would pick: its own choice for a lone beam, the same rule for a stack
    const bool fac_default =
        sk.beams.size() == 1 ? p->fac_fine > 0 && p->facw_nt == 0 : (sk.fine > 0 && sk.n_chunks <= 2);
    Class c = make_class(p, sk.n_chunks, sk.fine > 0, fac_default);
    auto it = class_of.find(c.key);
    if (it == class_of.end()) {
      std::string name;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto t = g_tune.find(b->arch + "|" + c.key);
        if (t != g_tune.end()) name = t->second;
      }
      if (name.empty()) {
        auto t = cached.find(b->arch + "|" + c.key);
        if (t != cached.end()) name = t->second;
      }
      for (size_t k = 0; k < c.cands.size(); ++k)
        if (!name.empty() && c.cands[k].name() == name) {
          c.choice = (int)k;
          c.settled = true;
        }
      if (dd.flags & FDD_BATCH_NO_AUTOTUNE) {
        c.choice = 0;
        c.settled = true;
      }
      it = class_of.emplace(c.key, (int)b->classes.size()).first;
      b->classes.push_back(c);
    }
    sk.cls = it->second;
  }

  // table arena: one twiddle table per FFT length, phase tables per stack
  std::map<int64_t, size_t> tw_of;
  size_t off = 0;
  for (Stack& sk : b->stacks) {
    const fdd_plan_s* p = sk.rep;
    auto it = tw_of.find(p->L);
    if (it == tw_of.end()) {
      it = tw_of.emplace(p->L, off).first;
      off = align_up(off + (size_t)p->L * sizeof(float2));
    }
    sk.tw = it->second;
    sk.tab = off;
    off = align_up(off + (size_t)p->desc.n_chan * (size_t)p->desc.n_dm * sizeof(uint4));
    if (sk.fine > 0) {
      sk.ftab = off;
      off = align_up(off + (size_t)p->desc.n_chan * (size_t)(sk.coarse + sk.fine) * sizeof(uint4));
    }
  }
  b->tab_bytes = off;

  // memory waves: first-fit decreasing over the stacks' scratch sizes
  const int ns = (int)b->stacks.size();
  std::vector<int> order((size_t)ns);
  for (int i = 0; i < ns; ++i) {
    order[(size_t)i] = i;
    b->stacks[(size_t)i].bytes = stack_scratch(b, &b->stacks[(size_t)i]);
  }
  size_t limit = dd.scratch_limit;
  if (limit == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      release(b);
      delete b;
      return fail(FDD_E_DEVICE, "hipMemGetInfo failed");
    }
    limit = free_b / 4 * 3 > b->tab_bytes ? free_b / 4 * 3 - b->tab_bytes : 0;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->stacks[(size_t)x].bytes > b->stacks[(size_t)y].bytes; });
  std::vector<size_t> fill_of;
  for (int i : order) {
    Stack& sk = b->stacks[(size_t)i];
    if (sk.bytes > limit) {
      delete b;
      return fail(FDD_E_NOMEM, "the scratch of one beam or stack (" + std::to_string(sk.bytes) +
                                   " bytes) exceeds the scratch limit");
    }
    size_t w = 0;
    while (w < fill_of.size() && fill_of[w] + sk.bytes > limit) ++w;
    if (w == fill_of.size()) fill_of.push_back(0);
    sk.wave = (int)w;
    sk.scratch = fill_of[w];
    fill_of[w] += sk.bytes;
  }
  b->n_waves = (int)fill_of.size();
  b->scr_bytes = *std::max_element(fill_of.begin(), fill_of.end());

  // launches, wave by wave; grouped items ordered by decreasing work per tile (channels)
  size_t words = 0;
  for (int w = 0; w < b->n_waves; ++w) {
    std::vector<int> ws, wb;
    for (int i : order)
      if (b->stacks[(size_t)i].wave == w) ws.push_back(i);
    std::stable_sort(ws.begin(), ws.end(), [&](int x, int y) {
      return b->stacks[(size_t)x].rep->desc.n_chan > b->stacks[(size_t)y].rep->desc.n_chan;
    });
    for (int i : ws)
      for (int j : b->stacks[(size_t)i].beams) wb.push_back(j);
    for (int i : wb)
      if (b->beams[(size_t)i].plan->desc.input == FDD_IN_U8_TIME_MAJOR) {
        Launch l;
        l.stage = kTranspose;
        l.wave = w;
        l.beams = {i};
        b->launches.push_back(l);
      }
    auto grouped = [&](Stage stage, const std::vector<int>& items, auto key_of) {
      std::map<std::pair<int, int>, std::vector<int>> groups;
      for (int i : items) groups[key_of(i)].push_back(i);
      for (auto& g : groups) {
        Launch l;
        l.stage = stage;
        l.wave = w;
        l.beams = g.second;
        const fdd_plan_s* p = stage == kPhasor ? b->stacks[(size_t)g.second[0]].rep : b->beams[(size_t)g.second[0]].plan;
        l.log_n = p->log_len - 1;
        l.u8 = p->desc.input == FDD_IN_U8_TIME_MAJOR;
        if (stage == kPhasor) {
          l.cls = g.first.first;
          l.ctr = words;
          words += 8;
        }
        b->launches.push_back(l);
      }
    };
    grouped(kR2c, wb, [&](int i) {
      const fdd_plan_s* p = b->beams[(size_t)i].plan;
      return std::make_pair(p->log_len, p->desc.input == FDD_IN_U8_TIME_MAJOR ? 1 : 0);
    });
    grouped(kPhasor, ws, [&](int i) { return std::make_pair(b->stacks[(size_t)i].cls, 0); });
    grouped(kC2r, wb, [&](int i) { return std::make_pair(b->beams[(size_t)i].plan->log_len, 0); });
  }
  for (Stack& sk : b->stacks)
    if (sk.rep->desc.precision != FDD_FP32) {
      sk.l1 = words;
      words += (size_t)sk.n_chunks;
    }
  b->small_words = words;

  // descriptor buffer
  size_t doff = 0;
  for (Launch& l : b->launches) {
    if (l.stage == kTranspose) continue;
    const size_t each = l.stage == kPhasor ? sizeof(PhasorArgs) : sizeof(FftArgs);
    l.slots = 0;
    for (int i : l.beams) l.slots += l.stage == kPhasor ? chunk_groups(b->stacks[(size_t)i].n_chunks) : 1;
    l.args = doff;
    doff = align_up(doff + each * (size_t)l.slots);
    l.prefix = doff;
    doff = align_up(doff + sizeof(int) * ((size_t)l.slots + 1));
  }
  b->h_desc.assign(doff, 0);

  // device memory and tables
  auto alloc = [&](void** p, size_t bytes, const char* what) {
    hipError_t e = hipMalloc(p, bytes > 0 ? bytes : kAlign);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(FDD_E_NOMEM, std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
    }
    return FDD_OK;
  };
  fdd_status s = alloc((void**)&b->d_tab, b->tab_bytes, "batch tables");
  if (s == FDD_OK) s = alloc((void**)&b->d_scr, b->scr_bytes, "batch scratch");
  if (s == FDD_OK) s = alloc((void**)&b->d_small, b->small_words * sizeof(unsigned int), "batch counters");
  if (s == FDD_OK) s = alloc((void**)&b->d_desc, b->h_desc.size(), "batch descriptors");
  if (s == FDD_OK) {
    std::vector<uint8_t> tabs(b->tab_bytes, 0);
    for (const auto& kv : tw_of) {
      std::vector<float2> tw;
      twiddle_table(kv.first, &tw);
      std::memcpy(tabs.data() + kv.second, tw.data(), tw.size() * sizeof(float2));
    }
    for (const Stack& sk : b->stacks) {
      std::vector<uint4> tab;
      phase_table(sk.rep, &tab);
      std::memcpy(tabs.data() + sk.tab, tab.data(), tab.size() * sizeof(uint4));
      if (sk.fine > 0) {
        factor_tables(sk.rep, sk.fine, sk.coarse, sk.dm0, sk.step, &tab);
        std::memcpy(tabs.data() + sk.ftab, tab.data(), tab.size() * sizeof(uint4));
      }
    }
    hipError_t e = hipMemcpy(b->d_tab, tabs.data(), b->tab_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) s = hip_fail(e, "hipMemcpy(batch tables)");
  }
  if (s == FDD_OK && !(b->flags & FDD_BATCH_NO_GRAPH)) {
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) s = hip_fail(e, "hipStreamCreate");
  }
  if (s == FDD_OK) {
    hipError_t e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) s = hip_fail(e, "hipEventCreate");
  }
  if (s != FDD_OK) {
    release(b);
    delete b;
    return s;
  }
  *out = b;
  return FDD_OK;
}

fdd_status fdd_batch_execute(fdd_batch_t b, const void* const* in, float* const* out, void* stream) {
  if (b == nullptr || in == nullptr || out == nullptr) return fail(FDD_E_INVALID, "null batch, inputs or outputs");
  const size_t n = b->beams.size();
  for (size_t i = 0; i < n; ++i)
    if (in[i] == nullptr || out[i] == nullptr) return fail(FDD_E_INVALID, "null input or output of beam " + std::to_string(i));
  hipStream_t st = (hipStream_t)stream;
  // A call on another stream than the last one waits for it: the calls of a batch share the
  // descriptors and the ticket counters, and a chain of waits lets one event stand for all
  // earlier calls below.
  if (b->launched && st != b->last_st) {
    hipError_t e = hipStreamWaitEvent(st, b->done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  const bool same = b->ready && std::equal(in, in + n, b->last_in.begin()) && std::equal(out, out + n, b->last_out.begin());
  if (!same) {
    b->ready = false;
    // Earlier calls, on whichever stream, may still read the descriptors about to be rewritten.
    hipError_t e = b->launched ? hipEventSynchronize(b->done) : hipSuccess;
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    bool tune = false;
    for (const Class& c : b->classes) tune = tune || !c.settled;
    fdd_status s = tune ? autotune(b, in, out, st) : FDD_OK;
    if (s == FDD_OK) s = fill(b, in, out);
    if (s == FDD_OK) s = upload(b);
    if (s != FDD_OK) return s;
    if (!(b->flags & FDD_BATCH_NO_GRAPH)) {
      if (b->exec != nullptr) (void)hipGraphExecDestroy(b->exec);
      if (b->graph != nullptr) (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
      e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
      s = enqueue_all(b, in, b->cap);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(b->cap, &g);
      if (s != FDD_OK) {
        if (g != nullptr) (void)hipGraphDestroy(g);
        return s;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      b->graph = g;
      e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    }
    b->last_in.assign(in, in + n);
    b->last_out.assign(out, out + n);
    b->ready = true;
  }
  if (b->flags & FDD_BATCH_NO_GRAPH) {
    const fdd_status s = enqueue_all(b, in, st);
    if (s != FDD_OK) return s;
  } else {
    const hipError_t e = hipGraphLaunch(b->exec, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  const hipError_t e = hipEventRecord(b->done, st);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  b->last_st = st;
  b->launched = true;
  return FDD_OK;
}

fdd_status fdd_batch_info(fdd_batch_t b, int32_t* n_waves, size_t* scratch_bytes, size_t* table_bytes) {
  if (b == nullptr) return fail(FDD_E_INVALID, "null batch");
  if (n_waves != nullptr) *n_waves = b->n_waves;
  if (scratch_bytes != nullptr) *scratch_bytes = b->scr_bytes;
  if (table_bytes != nullptr) *table_bytes = b->tab_bytes;
  return FDD_OK;
}

fdd_status fdd_batch_describe(fdd_batch_t b, char* buf, size_t len, size_t* needed) {
  if (b == nullptr) return fail(FDD_E_INVALID, "null batch");
  std::ostringstream o;
  o << "{\"arch\": \"" << b->arch << "\", \"waves\": " << b->n_waves << ", \"scratch_bytes\": " << b->scr_bytes
    << ", \"table_bytes\": " << b->tab_bytes << ", \"graph\": " << ((b->flags & FDD_BATCH_NO_GRAPH) ? "false" : "true")
    << ",\n \"beams\": [";
  for (size_t i = 0; i < b->beams.size(); ++i) {
    const Stack& sk = b->stacks[(size_t)b->beams[i].stack];
    o << (i ? ", " : "") << "{\"stack\": " << b->beams[i].stack << ", \"first_chunk\": " << b->beams[i].koff
      << ", \"wave\": " << sk.wave << ", \"class\": " << sk.cls << "}";
  }
  o << "],\n \"stacks\": [";
  for (size_t i = 0; i < b->stacks.size(); ++i) {
    const Stack& sk = b->stacks[i];
    o << (i ? ", " : "") << "{\"beams\": " << sk.beams.size() << ", \"chunks\": " << sk.n_chunks
      << ", \"wave\": " << sk.wave << ", \"class\": " << sk.cls << ", \"scratch_bytes\": " << sk.bytes << "}";
  }
  o << "],\n \"classes\": [";
  for (size_t c = 0; c < b->classes.size(); ++c) {
    const Class& k = b->classes[c];
    o << (c ? ",\n  " : "\n  ") << "{\"key\": \"" << k.key << "\", \"choice\": \"" << k.cands[(size_t)k.choice].name()
      << "\", \"settled\": " << (k.settled ? "true" : "false") << ", \"candidates\": {";
    for (size_t j = 0; j < k.cands.size(); ++j)
      o << (j ? ", " : "") << "\"" << k.cands[j].name() << "\": " << (k.ms[j] >= 0.0f ? std::to_string(k.ms[j]) : "null");
    o << "}}";
  }
  o << "],\n \"launches\": [";
  static const char* names[] = {"transpose", "r2c", "phasor", "c2r"};
  for (size_t i = 0; i < b->launches.size(); ++i) {
    const Launch& l = b->launches[i];
    o << (i ? ", " : "") << "{\"stage\": \"" << names[l.stage] << "\", \"wave\": " << l.wave
      << (l.stage == kPhasor ? ", \"stacks\": " : ", \"beams\": ") << l.beams.size() << ", \"tiles\": " << l.total;
    if (l.stage == kPhasor) o << ", \"class\": " << l.cls;
    o << "}";
  }
  o << "]}";
  const std::string s = o.str();
  if (needed != nullptr) *needed = s.size() + 1;
  if (buf == nullptr || len < s.size() + 1) return fail(FDD_E_INVALID, "describe buffer too small");
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return FDD_OK;
}

fdd_status fdd_batch_destroy(fdd_batch_t b) {
  if (b == nullptr) return FDD_OK;
  release(b);
  delete b;
  return FDD_OK;
}

}  // extern "C"
