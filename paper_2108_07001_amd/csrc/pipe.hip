// pipe.hip -- per-buffer streaming demapper (air_pipe_*).
//
// The paper's receiver moves buffers of ADC samples to the GPU by DMA, runs
// each buffer on its own processing stream and writes the demapped results
// back to host memory; it counts as real time because buffers are processed
// faster than they arrive (Section II). A pipe does the same for the demapping
// stage: the caller pushes host buffers of received symbols one after another
// and gets their LLRs back in host buffers. Each buffer takes three steps:
//
//   H2D copy (the slot's stream) -> demapping kernels (the context's stream)
//   -> D2H copy of the LLRs (the slot's stream)
//
// With `depth` slots the copies of one buffer overlap the kernels of another
// in both directions. The kernels of different buffers run one after another
// on the context's stream, so the context's workspace is never used by two
// launches at once, and every buffer's LLRs are bitwise those of air_llr on
// the same data. Host buffers that are pinned (hipHostMalloc) are copied
// directly; pageable ones go through pinned staging owned by the pipe (a
// host memcpy on the calling thread). All device and staging memory is
// allocated at creation.
#include "../../include/air.h"
#include "device_common.h"
#include "host_state.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace air;

namespace {

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t in_ready = nullptr, computed = nullptr, done = nullptr;
  void* d_in = nullptr;       // cap x D received symbols
  void* d_llr = nullptr;      // cap x m LLRs
  void* h_in = nullptr;       // pinned staging (pageable inputs)
  void* h_out = nullptr;      // pinned staging (pageable outputs)
  bool busy = false;          // work queued and not yet retired
  void* user_out = nullptr;   // where a staged output goes when retired
  size_t out_bytes = 0;
};

bool is_pinned_host(const void* p) {
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;                // pageable (unknown to the runtime)
  }
  return at.type == hipMemoryTypeHost;
}

}  // namespace

struct air_pipe {
  air_ctx* ctx = nullptr;
  const air_const* c = nullptr;
  int64_t cap = 0;
  air_prec prec = AIR_FP32;
  size_t tsz = 4;
  std::vector<Slot> slots;
  int64_t pushed = 0;
};

namespace {

void release(air_pipe* p) {
  for (Slot& s : p->slots) {
    if (s.st) (void)hipStreamSynchronize(s.st);
    (void)hipFree(s.d_in);
    (void)hipFree(s.d_llr);
    (void)hipHostFree(s.h_in);
    (void)hipHostFree(s.h_out);
    if (s.in_ready) (void)hipEventDestroy(s.in_ready);
    if (s.computed) (void)hipEventDestroy(s.computed);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.st) (void)hipStreamDestroy(s.st);
  }
  p->slots.clear();
}

// Waits for a slot's queued work and moves a staged output to its target.
air_status retire(air_pipe* p, Slot& s) {
  if (!s.busy) return AIR_OK;
  s.busy = false;
  const hipError_t e = hipEventSynchronize(s.done);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "pipe buffer completion");
  if (s.user_out) std::memcpy(s.user_out, s.h_out, s.out_bytes);
  s.user_out = nullptr;
  return AIR_OK;
}

}  // namespace

extern "C" {

air_status air_pipe_create(air_ctx* ctx, const air_const* c, int64_t max_symbols, int depth,
                           air_prec prec, air_pipe** out) {
  if (!ctx || !out) return AIR_E_INVAL;
  *out = nullptr;
  if (!c || c->ctx != ctx) return fail(ctx, AIR_E_INVAL, "constellation is null or from another context");
  if (max_symbols < 1) return fail(ctx, AIR_E_INVAL, "max_symbols must be >= 1");
  if (depth < 2 || depth > 8) return fail(ctx, AIR_E_INVAL, "depth must be 2..8");
  if (prec != AIR_FP32 && prec != AIR_FP64 && prec != AIR_FP16X3 && prec != AIR_BF16X3)
    return fail(ctx, AIR_E_INVAL, "unknown precision");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
  air_pipe* p = nullptr;
  try {
    p = new air_pipe();
    p->slots.resize((size_t)depth);
  } catch (...) {
    delete p;
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
  p->ctx = ctx;
  p->c = c;
  p->cap = max_symbols;
  p->prec = prec;
  p->tsz = prec == AIR_FP64 ? sizeof(double) : sizeof(float);
  const size_t in_b = (size_t)max_symbols * (size_t)c->D * p->tsz;
  const size_t out_b = (size_t)max_symbols * (size_t)c->m * p->tsz;
  hipError_t e = hipSuccess;
  for (Slot& s : p->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.in_ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.computed, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&s.d_in, in_b);
    if (e == hipSuccess) e = hipMalloc(&s.d_llr, out_b);
    if (e == hipSuccess) e = hipHostMalloc(&s.h_in, in_b, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s.h_out, out_b, hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    release(p);
    delete p;
    return hip_fail(ctx, e, "pipe allocation");
  }
  *out = p;
  return AIR_OK;
}

air_status air_pipe_push(air_pipe* p, const void* Y_host, int64_t N, double snr_db, void* llr_host) {
  if (!p) return AIR_E_INVAL;
  air_ctx* ctx = p->ctx;
  if (!Y_host || !llr_host) return fail(ctx, AIR_E_INVAL, "Y_host and llr_host must not be null");
  if (N < 1 || N > p->cap) return fail(ctx, AIR_E_INVAL, "N must be 1..max_symbols");
  if (!std::isfinite(snr_db)) return fail(ctx, AIR_E_INVAL, "SNR values must be finite");
  if (is_device_ptr(ctx, Y_host) || is_device_ptr(ctx, llr_host))
    return fail(ctx, AIR_E_INVAL, "pipe buffers are host memory (use air_llr for device buffers)");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
  Slot& s = p->slots[(size_t)(p->pushed % (int64_t)p->slots.size())];
  air_status st = retire(p, s);
  if (st != AIR_OK) return st;
  const size_t in_b = (size_t)N * (size_t)p->c->D * p->tsz;
  const size_t out_b = (size_t)N * (size_t)p->c->m * p->tsz;
  const void* src = Y_host;
  if (!is_pinned_host(Y_host)) {
    std::memcpy(s.h_in, Y_host, in_b);
    src = s.h_in;
  }
  const bool out_pinned = is_pinned_host(llr_host);
  hipError_t e = hipMemcpyAsync(s.d_in, src, in_b, hipMemcpyHostToDevice, s.st);
  if (e == hipSuccess) e = hipEventRecord(s.in_ready, s.st);
  if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, s.in_ready, 0);
  if (e != hipSuccess) return hip_fail(ctx, e, "pipe input copy");
  st = air_llr(ctx, p->c, s.d_in, N, snr_db, p->prec, s.d_llr);
  if (st != AIR_OK) return st;
  e = hipEventRecord(s.computed, ctx->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s.st, s.computed, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_pinned ? llr_host : s.h_out, s.d_llr, out_b, hipMemcpyDeviceToHost, s.st);
  if (e == hipSuccess) e = hipEventRecord(s.done, s.st);
  if (e != hipSuccess) return hip_fail(ctx, e, "pipe output copy");
  s.busy = true;
  s.user_out = out_pinned ? nullptr : llr_host;
  s.out_bytes = out_b;
  ++p->pushed;
  return AIR_OK;
}

air_status air_pipe_wait(air_pipe* p) {
  if (!p) return AIR_E_INVAL;
  DeviceGuard g(p->ctx->device);
  if (!g.ok) return fail(p->ctx, AIR_E_DEVICE, "cannot select the context's device");
  const int64_t n = (int64_t)p->slots.size();
  air_status first = AIR_OK;
  for (int64_t k = 0; k < n; ++k) {          // oldest first
    const air_status st = retire(p, p->slots[(size_t)((p->pushed + k) % n)]);
    if (first == AIR_OK) first = st;
  }
  if (first != AIR_OK) return first;
  return air_sync(p->ctx);
}

void air_pipe_destroy(air_pipe* p) {
  if (!p) return;
  DeviceGuard g(p->ctx->device);
  release(p);
  delete p;
}

}  // extern "C"
