// noalloc.hip -- air_sweep_noalloc: air_sweep for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc). The second tier's per-launch workspace --
// the first tier's per-wave lists and flagged counts, and the gathered
// flagged sample indices -- lives in one file-scope device array per GPU
// instead of the context's workspace, which air_sweep grows on demand.
#include "../../include/air.h"
#include "host_state.h"

#include <mutex>

namespace air {

// Defined in air_host.hip: the common driver with a caller-supplied second-tier workspace.
air_status run_sweep_scratch(air_ctx* ctx, const air_const* c, const void* Z, const uint32_t* tx, int64_t N,
                             const double* snr_db, int S, air_prec prec, double* stats, void* llr,
                             void* scratch, size_t scratch_bytes);

namespace {

// Every launch writes the parts of it that it reads before reading them, so
// nothing in it needs clearing between calls.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices];    // the array's device address on each GPU, once looked up

}  // namespace

// Looks up the array's address on `device` (current) once; called by
// air_create with that device selected.
hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();        // leave no error for the next runtime call
    return e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
  g_scratch[device] = ptr;
  return hipSuccess;
}

}  // namespace air

using namespace air;

extern "C" air_status air_sweep_noalloc(air_ctx* ctx, const air_const* c, const uint32_t* tx_dev,
                                        const void* Z_dev, int64_t N, const double* snr_db_host, int S,
                                        air_prec prec, double* stats_dev, void* llr_dev) {
  if (!ctx) return AIR_E_INVAL;
  if (!tx_dev || !stats_dev) return fail(ctx, AIR_E_INVAL, "tx_dev and stats_dev must not be null");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) ptr = g_scratch[ctx->device];
  }
  if (!ptr) return fail(ctx, AIR_E_DEVICE, "no-allocation scratch was not set up for this device");
  try {
    return run_sweep_scratch(ctx, c, Z_dev, tx_dev, N, snr_db_host, S, prec, stats_dev, llr_dev, ptr,
                             kNoAllocScratchBytes);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}
