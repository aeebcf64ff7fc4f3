/*
 * fdd.h -- C ABI of the MI355X (gfx950) Fourier-domain dedispersion library.
 *
 * Method: Bassa et al., "Fourier-domain dedispersion" (arXiv:2110.03482), Sec. 2.2 and
 * Sec. 3.  For every channel c and trial DM, the dispersion delay (Eq. 1)
 *     tau[dm, c] = DM_dm * k_DM * (nu_c^-2 - nu_ref^-2) / t_samp      (samples)
 * is applied in the Fourier domain of time:
 *     X[c, k, f] = sum_t x[c, kS + t] exp(-2 pi i f t / L)             (Eq. 3, per chunk k)
 *     Y[dm, k, f] = sum_c X[c, k, f] exp(+2 pi i f tau[dm, c] / L)     (Eqs. 4 and 7)
 *     y[dm, kS + t] = (1/L) IDFT_L(Y[dm, k, .])[t],  t < S             (Eq. 6, wrap discarded)
 * or, without the inverse transform, power spectra |Y[dm, 0, f]|^2 (Sec. 5).
 *
 * Conventions fixed by this library (readings of the paper):
 *  - k_DM = FDD_K_DM.  nu_ref must be >= every channel frequency, so tau >= 0.
 *  - Output sample t of a DM sums input samples t + tau[dm, c] (lower frequencies arrive
 *    later and are advanced); hence the phasor sign +2 pi i above.
 *  - Delays are formed in float64 as kappa_c = (k_DM * (1/(nu_c*nu_c) - 1/(nu_ref*nu_ref)))
 *    / t_samp and tau = DM * kappa_c.  FDD_DELAY_ROUND uses d = floor(tau + 1/2) (Sec. 2.1,
 *    nearest sample), for which the result equals time-domain shift-and-sum (Eq. 2).
 *  - Chunked mode is overlap-save: chunk k covers input samples [kS, kS + L), zero beyond
 *    n_samp, and keeps its first S = L - D outputs; D >= ceil(max tau) (Sec. 2.2).
 *    Single-chunk mode zero-pads n_samp to L and is circular over L.
 *  - The inverse drops Im of bins 0 and L/2 and scales by 1/L.  Power spectra keep bins
 *    0 .. L/2-1 and are not normalised.
 *  - Down-sampled output (Sec. 2.2: where dispersive smearing spans several samples, the
 *    inverse transform is shortened).  A DM with factor d (a power of two) is inverted with a
 *    real transform of length M = L/d from bins 0 .. M/2 of Y, scaled by 1/L and with Im of
 *    bins 0 and M/2 dropped:
 *        z[dm, kS/d + m] = (1/L) [Re Y_0 + (-1)^m Re Y_{M/2}
 *                                 + 2 sum_{f=1}^{M/2-1} Re(Y_f exp(2 pi i f m / M))],  m < S/d,
 *    i.e. the series low-passed to |f| < M/2 (half weight at M/2) and sampled every d-th
 *    sample; the phasor sum of such a DM only visits bins 0 .. M/2.
 *
 * Memory and streams: every pointer named d_* is device memory owned by the caller.  All
 * device work is enqueued on the given stream (a hipStream_t; NULL = the null stream) and
 * nothing synchronises the host, except where stated.  A plan owns one workspace, so one
 * plan must not run concurrently on two streams; distinct plans are independent.
 *
 * Errors: every call returns an fdd_status.  Nothing throws across the ABI.  The text of the
 * most recent failure on the calling thread is available from fdd_last_error().
 */
#ifndef FDD_H
#define FDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Dispersion constant, MHz^2 pc^-1 cm^3 s (Eq. 1). */
#define FDD_K_DM 4.148808e3

typedef enum {
  FDD_OK = 0,
  FDD_E_INVALID = 1,      /* bad argument or descriptor field */
  FDD_E_OVERLAP = 2,      /* overlap shorter than the maximum delay, or not shorter than L */
  FDD_E_UNSUPPORTED = 3,  /* valid request this build does not implement */
  FDD_E_NOMEM = 4,        /* device allocation failed, or size overflow */
  FDD_E_DEVICE = 5,       /* a HIP call failed (detail in fdd_last_error) */
  FDD_E_WORKSPACE = 6     /* no workspace attached, or the attached one is too small */
} fdd_status;

typedef enum {
  FDD_IN_U8_TIME_MAJOR = 0,  /* uint8 [n_samp][n_chan] (packed 8-bit filterbank, Sec. 3) */
  FDD_IN_F32_CHAN_MAJOR = 1  /* float32 [n_chan][n_samp] */
} fdd_input_kind;

typedef enum {
  FDD_FP32 = 0,        /* phasor sum in float32 */
  FDD_FP16_SPLIT = 1,  /* hi/lo float16 phasors and data on MFMA, float32 accumulation (Sec. 5 outlook) */
  FDD_BF16_SPLIT = 2   /* hi/lo bfloat16 phasors and data on MFMA, float32 accumulation */
} fdd_precision;

typedef enum {
  FDD_DELAY_EXACT = 0, /* fractional delays, phase frac(f tau / L) (Eq. 4) */
  FDD_DELAY_ROUND = 1  /* delays rounded to the nearest sample (Eq. 2 equivalent) */
} fdd_delay_mode;

/* Plan flags. */
#define FDD_PLAN_DRY_RUN 1u             /* validate and size only; no device calls at all */
#define FDD_PLAN_EXTERNAL_WORKSPACE 2u  /* caller attaches the workspace with fdd_set_workspace */
#define FDD_PLAN_POWER_ONLY 4u          /* the plan will only compute power spectra: no inverse buffers */
#define FDD_PLAN_SCALED_DM 8u           /* also size the workspace for fdd_power_spectrum_scaled */

typedef struct {
  int32_t n_chan;               /* channels, >= 1 */
  const double* chan_freq_mhz;  /* host array [n_chan], any order, 0 < nu_c <= ref_freq_mhz; copied */
  double ref_freq_mhz;          /* nu_ref of Eq. 1 (the upper band edge) */
  double tsamp_s;               /* sampling time, > 0 */
  int32_t n_dm;                 /* trial DMs, >= 1 */
  const double* dm;             /* host array [n_dm], finite, >= 0 (pc cm^-3); copied */
  int64_t n_samp;               /* time samples per channel, >= 1 */
  int64_t chunk_len;            /* FFT length L: power of two, 2^6 .. 2^22 (above 2^16: multi-pass FFT) */
  int64_t overlap;              /* D = L - S; <= 0 picks ceil(max tau); ignored if single_chunk */
  int32_t single_chunk;         /* 1: one circular transform of length L >= n_samp */
  int32_t input;                /* fdd_input_kind */
  int32_t precision;            /* fdd_precision */
  int32_t delay_mode;           /* fdd_delay_mode */
  uint32_t flags;               /* FDD_PLAN_* */
  const int32_t* downsample;    /* host array [n_dm] of output down-sampling factors (powers of
                                   two, 1 .. chunk_len/64), or NULL for none; copied.  Factors
                                   above 1 need chunk_len <= 2^16 and a plan that inverts (not
                                   power-only); in chunked mode the kept stride S becomes a
                                   multiple of the largest factor (an automatic overlap is
                                   rounded up; an explicit one must already give that) */
} fdd_plan_desc;

typedef struct {
  int64_t chunk_len;        /* L */
  int64_t stride;           /* S = samples kept per chunk (L in single-chunk mode) */
  int64_t overlap;          /* D (0 in single-chunk mode) */
  int64_t n_chunks;         /* ceil(n_samp / S) */
  int64_t n_bins;           /* L/2 + 1 Fourier bins per chunk */
  int64_t bins_padded;      /* row pitch (in bins) of the Fourier-domain buffers */
  double max_delay;         /* max over (dm, c) of tau, samples */
  int64_t n_valid;          /* samples not touched by the end-of-series discard: n_samp - ceil(max tau) */
  size_t workspace_bytes;   /* device bytes a workspace for this plan must hold */
  int64_t out_samples;      /* float32 samples fdd_execute writes: sum over DMs of ceil(n_samp / d_dm)
                               (n_dm * n_samp without down-sampling) */
  int32_t n_segments;       /* runs of consecutive DMs with one down-sampling factor (1 without) */
  int64_t scaled_min_bin;   /* FDD_PLAN_SCALED_DM: first bin of the approximate region (0 otherwise) */
} fdd_plan_geometry;

typedef struct fdd_plan_s* fdd_plan_t;

/* Build a plan: validate the descriptor, copy the host arrays, compute the per-channel delay
 * per unit DM in float64 (Eq. 1: kappa_c = k_DM (nu_c^-2 - nu_ref^-2) / t_samp, tau = DM kappa_c)
 * and the chunk geometry of the Sec. 2.2 discard rule (every transformed series loses its last
 * ceil(max tau) samples to the cyclic wrap, so chunks advance by S = L - D with D >= ceil(max tau),
 * N_chunk = ceil(n_samp / S)).  Also tabulates, per (channel, DM), the exact 64-bit phase
 * increment frac(tau / L) 2^64 of Eq. 4 and picks the phasor-sum kernel.  Without
 * FDD_PLAN_EXTERNAL_WORKSPACE or FDD_PLAN_DRY_RUN it allocates its workspace on the current device.
 * Errors: FDD_E_INVALID, FDD_E_OVERLAP, FDD_E_UNSUPPORTED, FDD_E_NOMEM, FDD_E_DEVICE. */
fdd_status fdd_plan(const fdd_plan_desc* desc, fdd_plan_t* out);

/* Geometry (Sec. 2.2: L, S, D, N_chunk, bins L/2 + 1) and workspace size of a plan (host only). */
fdd_status fdd_plan_info(fdd_plan_t plan, fdd_plan_geometry* out);

/* Infrastructure (no passage of the paper): attach caller-owned device memory of at least
 * workspace_bytes (256-byte aligned) as the plan's workspace.  Synchronously uploads the plan's small tables into it.  The caller keeps
 * ownership and must keep it alive while the plan is used. */
fdd_status fdd_set_workspace(fdd_plan_t plan, void* d_workspace, size_t bytes);

/* Dedisperse (Sec. 2.2, Eqs. 3, 4, 7, 6 and the discard rule; Sec. 3 for the 8-bit transpose and
 * unpack): d_in is described by the plan's input kind; d_out is float32 [n_dm][n_samp]
 * (DM-major, Sec. 3), or with down-sampling the DM rows one after another, row dm holding
 * ceil(n_samp / d_dm) samples (offsets from fdd_plan_output_offsets).  Enqueued on `stream`;
 * does not synchronise.
 * Errors: FDD_E_INVALID (null pointers, dry-run plan), FDD_E_UNSUPPORTED (power-only plan),
 * FDD_E_WORKSPACE, FDD_E_DEVICE. */
fdd_status fdd_execute(fdd_plan_t plan, const void* d_in, float* d_out, void* stream);

/* For callers that cannot allocate device memory at execution time (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fdd_execute with the plan's
 * workspace in the library's static device scratch instead of the plan's own memory.  The plan
 * may be a dry-run plan (FDD_PLAN_DRY_RUN: no device memory at all); its workspace_bytes must be
 * at most 64 MiB (FDD_E_UNSUPPORTED otherwise).  The call enqueues on `stream` the upload of the
 * plan's tables (kept on the host since fdd_plan) into the scratch, then the same kernels as
 * fdd_execute; it calls no hipMalloc or hipFree.  The scratch is one 64 MiB array per device,
 * held until the process ends and shared by every call on that device: calls that overlap on one
 * device race with each other, so the caller orders them (one stream, or events).  Output and
 * errors as fdd_execute (a dry-run plan is accepted). */
fdd_status fdd_execute_noalloc(fdd_plan_t plan, const void* d_in, float* d_out, void* stream);

/* Infrastructure: start of every output row of fdd_execute, in float32 samples from d_out: offsets[dm] for
 * dm = 0 .. n_dm, offsets[n_dm] = out_samples (host array of n_dm + 1, written by the call). */
fdd_status fdd_plan_output_offsets(fdd_plan_t plan, int64_t* offsets);

/* Power spectra without the inverse transform (Sec. 5): d_out is float32 [n_dm][L/2],
 * |Y[dm, f]|^2 for f = 0 .. L/2-1 (down-sampling factors do not apply).  Single-chunk plans
 * only (FDD_E_UNSUPPORTED otherwise). */
fdd_status fdd_power_spectrum(fdd_plan_t plan, const void* d_in, float* d_out, void* stream);

/* Power spectra with spin-frequency-scaled DMs (Sec. 2.3, Eq. 8): an approximation, for plans
 * made with FDD_PLAN_SCALED_DM (single chunk, exact delays, a uniform DM list
 * DM_j = DM_0 + j dDM, n_dm >= 2).  Bins f >= f_min (geometry scaled_min_bin) are cut into
 * blocks of 64 with reference bin r = (first bin) + 32.  Within a block, row s of the scaled
 * grid (DM'_s = DM_0 + s dDM, s = -32 .. n_dm + 31) uses at bin f the DM DM'_s r / f, whose
 * phasor exp(+2 pi i r DM'_s kappa_c / L) does not depend on f, so the block's phasor sum is
 * one matrix product Q[s, f] = |sum_c W_r[s, c] X[c, f]|^2 (in the plan's precision: FP32, or
 * FP16/BF16 head+tail split).  The power at trial DM_j and bin
 * f is then resampled linearly in DM:
 *     s* = (DM_j f / r - DM_0) / dDM,  P[j, f] = (1 - w) Q[floor(s*), f] + w Q[floor(s*) + 1, f],
 * w = s* - floor(s*).  f_min is the smallest block start (at least 64) for which
 * |s* - j| <= 31 everywhere; bins below it are computed exactly as fdd_power_spectrum does.
 * Output float32 [n_dm][L/2].
 * Errors: FDD_E_UNSUPPORTED for a plan without FDD_PLAN_SCALED_DM; as fdd_power_spectrum. */
fdd_status fdd_power_spectrum_scaled(fdd_plan_t plan, const void* d_in, float* d_out, void* stream);

/* Brute-force time-domain dedispersion (Eq. 2), the method FDD is compared with (Sec. 4.1):
 *     d_out[dm][t] = sum_c x[c][t + d[dm][c]],   d = floor(tau + 1/2)   (the plan's delays)
 * with x extended by zeros beyond n_samp, or, in single-chunk plans, zero-padded to chunk_len
 * and periodic.  Same input and output layouts as fdd_execute; sums of 8-bit input are exact
 * integers.  Uses the plan's workspace (any plan, power-only included); the output is at full
 * time resolution whatever the plan's down-sampling factors.  FDD_E_UNSUPPORTED if the delays
 * of 8 consecutive DMs differ by more than 4088 samples in some channel. */
fdd_status fdd_tdd_execute(fdd_plan_t plan, const void* d_in, float* d_out, void* stream);

/* Infrastructure: release a plan and the workspace it allocated itself (never a caller-owned one). */
fdd_status fdd_destroy(fdd_plan_t plan);

/* Infrastructure, stage timing (the stage split of the runtime breakdown in Sec. 4.1).
 * fdd_profile_enable(plan, depth) with depth >= 1 makes fdd_execute /
 * fdd_power_spectrum record HIP events on their stream around each stage, for the first
 * `depth` calls after enabling or after the last read (depth 0 disables).  fdd_profile_read waits for the recorded events and
 * returns the mean milliseconds per call for [0] transpose/unpack, [1] forward FFT,
 * [2] phasor sum, [3] inverse FFT (0 for a stage that did not run), writes the number of
 * calls averaged to *n_calls (may be NULL), and starts a new recording. */
fdd_status fdd_profile_enable(fdd_plan_t plan, int32_t depth);
fdd_status fdd_profile_read(fdd_plan_t plan, float ms[4], int32_t* n_calls);

/* ------------------------------------------------------------------------------------------
 * Batched form: many beams (one plan each, of uneven n_chan / n_samp / n_dm) dedispersed
 * together.  Sec. 3 processes channels and DMs in batches sized to the device memory; Sec. 5
 * proposes autotuning such parameters to the data size and names beams observed at once as
 * work to be processed together.  Here every stage (transpose, forward FFT, phasor sum, inverse FFT) is one
 * grouped kernel launch over all beams of a memory wave, the whole sequence is captured once
 * into a HIP graph and replayed by one graph launch per call, and the phasor-sum kernel of
 * each shape class (precision, FFT length, chunk-column tiles) is chosen by an autotuner that
 * times every candidate tile shape and launch style on the first call.
 *
 * Ownership: the batch owns its tables, Fourier-domain scratch, descriptors, graph and tuning
 * results; it reads its plans' parameters at create time and never uses their workspaces
 * (create the plans with FDD_PLAN_EXTERNAL_WORKSPACE to spare the memory).  The plans must
 * stay alive while the batch exists.  Beams whose scratch (Fourier-domain input and output)
 * does not fit `scratch_limit` together run in successive waves that reuse one arena.
 * Results equal fdd_execute of each plan to float32 rounding; with FDD_BATCH_NO_AUTOTUNE and
 * without FDD_BATCH_SHARE_PHASORS the batch uses the kernels fdd_execute would use and the
 * results are bitwise identical.
 * ------------------------------------------------------------------------------------------ */
typedef struct fdd_batch_s* fdd_batch_t;

#define FDD_BATCH_NO_GRAPH 1u       /* enqueue the grouped launches directly (no graph capture) */
#define FDD_BATCH_NO_AUTOTUNE 2u    /* use the single-plan kernel choice for every class */
#define FDD_BATCH_SHARE_PHASORS 4u  /* stack beams of one set-up (channels, DMs, sampling, FFT length,
                                       overlap, precision, delay mode) along the chunk axis, up to
                                       24 chunks per stack, so that every phasor serves all of them
                                       (Sec. 5 outlook); the kernel choice then follows the stack */

typedef struct {
  uint32_t flags;          /* FDD_BATCH_* */
  int32_t reserved;        /* must be 0 */
  size_t scratch_limit;    /* bytes of Fourier-domain scratch; 0 = 3/4 of the free device memory */
  const char* tune_cache;  /* path of a JSON autotune cache (read at create, rewritten after
                              tuning), or NULL for an in-process cache only */
} fdd_batch_desc;

/* Group `n_plans` plans (host array) into a batch on the current device: validates that every
 * plan can run batched (not dry-run, not power-only, chunk_len <= 2^16, no down-sampling), plans the waves,
 * allocates the scratch, uploads the tables.
 * Errors: FDD_E_INVALID, FDD_E_UNSUPPORTED, FDD_E_NOMEM, FDD_E_DEVICE. */
fdd_status fdd_batch_create(int32_t n_plans, const fdd_plan_t* plans, const fdd_batch_desc* desc,
                            fdd_batch_t* out);

/* Dedisperse every beam: d_in[i] / d_out[i] (host arrays of device pointers) are beam i's
 * input and float32 [n_dm][n_samp] output, as for fdd_execute.  The first call (and a call
 * whose pointers differ from the previous call's) synchronises `stream`: it runs the
 * autotuner if needed, writes the launch descriptors and captures the graph.  Other calls
 * enqueue one graph launch and do not synchronise.  A call on another stream than the previous
 * call's makes that stream wait for the previous call (an event, no host wait), and a call that
 * rewrites the descriptors first waits on the host for every earlier call of the batch; calls
 * from several host threads at once race.  The batch records events on `stream`, so it is not
 * meant to be called inside a caller's stream capture.
 * Errors: FDD_E_INVALID, FDD_E_DEVICE. */
fdd_status fdd_batch_execute(fdd_batch_t batch, const void* const* d_in, float* const* d_out, void* stream);

/* Infrastructure: sizes of a batch -- memory waves, scratch bytes, table bytes (any output may be NULL). */
fdd_status fdd_batch_info(fdd_batch_t batch, int32_t* n_waves, size_t* scratch_bytes, size_t* table_bytes);

/* Infrastructure: JSON description of the waves, shape classes, tuning candidates (with measured ms) and the
 * chosen kernels, written NUL-terminated into buf[len]; *needed (may be NULL) receives the
 * size required.  FDD_E_INVALID if len is too small. */
fdd_status fdd_batch_describe(fdd_batch_t batch, char* buf, size_t len, size_t* needed);

/* Infrastructure: release the batch (not its plans). */
fdd_status fdd_batch_destroy(fdd_batch_t batch);

/* Host helpers. */
/* tau (samples) of every channel at one DM, Eq. 1, exactly as plans compute it. */
fdd_status fdd_dispersion_delays(int32_t n_chan, const double* chan_freq_mhz, double ref_freq_mhz,
                                 double tsamp_s, double dm, double* tau_out);
/* Down-sampling factors from intra-channel smearing (Sec. 2.2: time-domain pipelines
 * down-sample once the smearing exceeds native samples).  The smearing of a DM is the Eq. 1
 * delay across the lowest channel, k_DM DM ((nu_lo - w/2)^-2 - (nu_lo + w/2)^-2) / t_samp
 * samples, with nu_lo the lowest channel frequency and w the smallest spacing of adjacent
 * channel frequencies (0 for one channel); out[dm] is the largest power of two <= that
 * smearing, at least 1 and at most max_factor (a power of two >= 1).  Host only. */
fdd_status fdd_smearing_factors(int32_t n_chan, const double* chan_freq_mhz, double tsamp_s, int32_t n_dm,
                                const double* dm, int32_t max_factor, int32_t* out);
/* The plan's float64 delay table tau[n_dm][n_chan] of Eq. 1 (host copy). */
fdd_status fdd_plan_delays(fdd_plan_t plan, double* tau_out);
/* Infrastructure: name of the phasor-sum kernel family a plan selected ("valu", "mfma_f32", ...). */
const char* fdd_plan_kernel(fdd_plan_t plan);
/* Infrastructure: the DM factorisation a plan uses for a uniform grid with exact delays (Eq. 1 is
 * linear in DM, so trial a*fine + b has the delay of coarse trial a plus that of fine offset b
 * and the phasor of Eq. 4 factorises): fine trials per coarse row, coarse rows, and the number
 * of 32-column matrix-core tiles per column group of the chunked kernels (0 for the others).
 * All three are 0 for a plan that is not factorised.  Any output pointer may be NULL. */
fdd_status fdd_plan_factors(fdd_plan_t plan, int32_t* fine, int32_t* coarse, int32_t* col_tiles);

/* Infrastructure: text of a status code, and of the calling thread's most recent failure. */
const char* fdd_status_string(fdd_status s);
const char* fdd_last_error(void);
/* Infrastructure: library version string. */
const char* fdd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FDD_H */
