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
  float* out = nullptr;             // inverse output [n_rows][n_samp]
  const float2* twL = nullptr;
  int64_t n_samp = 0;
  int64_t stride = 0;
  int64_t keep = 0;                 // samples kept per chunk
  int64_t pitch = 0;                // bins per row of X / Y
  int n_chunks = 0;
  int n_rows = 0;                   // channels (forward) or DMs (inverse)
  float add_full = 0.0f;            // constant restored in chunks wholly inside the data
  unsigned int* l1max = nullptr;    // forward: per-chunk max L1 norm (float bits), or null
};

struct PhasorArgs {
  const float2* X = nullptr;        // [n_chan][n_chunks][pitch]
  float* Yr = nullptr;              // [n_dm][n_chunks][pitch] (null for power spectra)
  float* Yi = nullptr;
  float* P = nullptr;               // [n_dm][n_pow_bins] power spectra, or null
  const double* dms = nullptr;      // [n_dm]
  const double* kappa = nullptr;    // [n_chan] delay in samples per unit DM
  const unsigned int* l1max = nullptr; // [n_chunks] max over channels of the series L1 norm (float bits)
  int n_dm = 0;
  int n_chan = 0;
  int n_chunks = 0;
  int64_t pitch = 0;
  int n_bins = 0;                   // L/2 + 1
  int n_pow_bins = 0;               // L/2
  int log_len = 0;                  // log2 L
  int mode = 0;                     // fdd_delay_mode
  float dc_add = 0.0f;              // added to Re Y at bin 0 before power (8-bit zero point)
  int tile_variant = 0;             // matrix-core tile shape (0 = default)
};

hipError_t launch_transpose_u8(const uint8_t* in, uint8_t* out, int64_t n_samp, int n_chan, hipStream_t st);
hipError_t launch_r2c(int log_n, const FftArgs& a, hipStream_t st);
hipError_t launch_c2r(int log_n, const FftArgs& a, hipStream_t st);
hipError_t launch_phasor_valu(const PhasorArgs& a, hipStream_t st);
hipError_t launch_phasor_mfma_f32(const PhasorArgs& a, hipStream_t st);
hipError_t launch_phasor_split(const PhasorArgs& a, bool bf16, hipStream_t st);
bool phasor_mfma_f32_supported(int n_chunks);
bool phasor_split_supported(int n_chunks);

// Byte offsets of the workspace regions (256-byte aligned).
struct WorkspaceLayout {
  size_t tw = 0, tw_bytes = 0;        // float2 twiddles, L entries
  size_t dms = 0, dms_bytes = 0;      // double [n_dm]
  size_t kappa = 0, kappa_bytes = 0;  // double [n_chan]
  size_t scale = 0, scale_bytes = 0;  // float [n_chunks]
  size_t xt = 0, xt_bytes = 0;        // transposed uint8 input
  size_t X = 0, X_bytes = 0;          // float2 [n_chan][n_chunks][pitch]
  size_t Yr = 0, Yi = 0, Y_bytes = 0; // float planes [n_dm][n_chunks][pitch] each
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
  // stage timing: a ring of `prof_depth` calls x 5 events
  int prof_depth = 0;
  int64_t prof_calls = 0;               // calls recorded since the last read
  std::vector<hipEvent_t> ev;
  std::vector<char> ev_ok;
};

namespace fdd {
void set_error(const std::string& msg);
fdd_status fail(fdd_status s, const std::string& msg);
fdd_status hip_fail(hipError_t e, const char* what);
}  // namespace fdd
