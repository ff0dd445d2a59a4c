// host_state.h -- host-side state shared by the C ABI translation units:
// contexts, constellation handles, device selection, error reporting and the
// per-SNR scalars of the channel model.
#pragma once

#include "../../include/air.h"
#include "device_common.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

constexpr int kSmallDoubles = 32;

// air_sweep_noalloc: devices served and the size of its per-GPU scratch array
// (the second tier's lists, counts and gathered samples of one launch).
constexpr int kMaxDevices = 64;
constexpr size_t kNoAllocScratchBytes = (size_t)48 << 20;

struct air_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  double* partials = nullptr;    // kMaxSnrPerLaunch x 4 x kMaxGrid
  // Per-call words in two slots that calls use in turn: a call's final
  // kernel zeroes the other slot, so the next call starts without a fill.
  air::CallWords* calls = nullptr;
  air::CallWords* call = nullptr;  // the slot of the current (or last) call
  bool next_zeroed = true;         // the other slot is known to hold zeros
  int* sticky = nullptr;         // tx-range error seen since the last air_sync
  // second tier of the matrix-core path: per-wave tile lists and their counts
  unsigned long long* t2_list = nullptr;
  double* t2_partials = nullptr; // kMaxSnrPerLaunch x 4 x kMaxGrid
  int64_t t2_slots = 0;          // capacity of t2_list
  int64_t t2_counts = 0;         // capacity of t2_nitem
  // flagged samples per wave (capacity t2_counts), those samples gathered
  // per SNR point (capacity 32 t2_slots) and per-SNR totals
  unsigned int* t2_nitem = nullptr;
  uint32_t* t2_items = nullptr;
  unsigned int* t2_tot = nullptr; // kMaxSnrPerLaunch
  // device results of the chained calls (air_aux_rates): the noise-variance
  // estimates (D + 1) and one SNR point's statistics (4)
  double* small = nullptr;       // kSmallDoubles
  // optional timing of the demapping kernels (air_set_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev;    // start/stop pairs recorded since the last read
  size_t ev_used = 0;
};

struct air_const {
  air_ctx* ctx = nullptr;   // creating context (a constellation is only used with it)
  int device = 0;
  int M = 0, D = 0, m = 0;
  double es = 0.0;
  double* x64 = nullptr;   // M x D, label order
  float* x32 = nullptr;    // M x D, label order
  uint32_t* lab = nullptr; // label of original index j
  uint32_t* pos = nullptr; // original index of label l
  // matrix-core point records, label order: [M][nk][2][8] operand elements
  uint16_t* rec_f16 = nullptr;
  uint16_t* rec_bf16 = nullptr;
  bool f16_ok = false;     // coordinates and |x|^2 within the half-precision range
  double r2max = 0.0;      // largest |x|^2
};

namespace air {

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

inline air_status fail(air_ctx* ctx, air_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

inline air_status hip_fail(air_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, e == hipErrorOutOfMemory ? AIR_E_NOMEM : AIR_E_DEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

// A *_dev argument must be device (or managed) memory of the context's device.
inline bool is_device_ptr(const air_ctx* ctx, const void* p) {
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) return false;
  return at.device == ctx->device;
}

// Noise scalars of one SNR point: sigma^2 = Es / (D 10^(snr_db/10)) per real
// dimension, and the metric scale c = 1 / (2 sigma^2 ln 2) of the log2 terms.
inline void snr_scalars(const air_const* c, double snr_db, double& sigma, double& cc) {
  const double ln2 = 0.69314718055994530942;
  const double snr = std::pow(10.0, snr_db / 10.0);
  const double sigma2 = c->es / ((double)c->D * snr);
  sigma = std::sqrt(sigma2);
  cc = 1.0 / (2.0 * sigma2 * ln2);
}

// Scalars of a receiver metric with the noise variance given directly.
inline void sigma2_scalars(double sigma2, double& sigma, double& cc) {
  const double ln2 = 0.69314718055994530942;
  sigma = std::sqrt(sigma2);
  cc = 1.0 / (2.0 * sigma2 * ln2);
}

}  // namespace air
