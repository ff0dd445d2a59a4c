// air_host.hip -- the C ABI of libair (include/air.h): contexts, constellation
// upload, argument validation, per-SNR scalars, kernel dispatch and the
// fixed-order FP64 reduction of per-block partial sums into MI / GMI / SE.
#include "../../include/air.h"
#include "device_common.h"
#include "host_state.h"
#include "mfma_wide.h"
#include "hd_kernels.h"
#include "aux_kernels.h"

#include <cmath>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

namespace air {

// Vector-kernel launchers, one per (type, D), defined in vec_inst_*.hip
// (arguments: launch, grid, where, max-log form, part: 0 the first tier, 1
// the FP32 second tier).
using VecFn = hipError_t (*)(const DemapArgs&, int, const Launch&, bool, int);
#define AIR_DECL(tag, D) hipError_t launch_vec_##tag##_d##D(const DemapArgs&, int, const Launch&, bool, int);
#define AIR_DECL_ALL(tag)                                                                        \
  AIR_DECL(tag, 1) AIR_DECL(tag, 2) AIR_DECL(tag, 3) AIR_DECL(tag, 4) AIR_DECL(tag, 5)          \
  AIR_DECL(tag, 6) AIR_DECL(tag, 7) AIR_DECL(tag, 8) AIR_DECL(tag, 9) AIR_DECL(tag, 10)         \
  AIR_DECL(tag, 11) AIR_DECL(tag, 12) AIR_DECL(tag, 13) AIR_DECL(tag, 14) AIR_DECL(tag, 15)     \
  AIR_DECL(tag, 16)
AIR_DECL_ALL(f32)
AIR_DECL_ALL(f64)
#undef AIR_DECL_ALL
#undef AIR_DECL

#define AIR_FN(tag, D) launch_vec_##tag##_d##D
static const VecFn kVecF32[kMaxD + 1] = {
    nullptr, AIR_FN(f32, 1), AIR_FN(f32, 2), AIR_FN(f32, 3), AIR_FN(f32, 4), AIR_FN(f32, 5),
    AIR_FN(f32, 6), AIR_FN(f32, 7), AIR_FN(f32, 8), AIR_FN(f32, 9), AIR_FN(f32, 10),
    AIR_FN(f32, 11), AIR_FN(f32, 12), AIR_FN(f32, 13), AIR_FN(f32, 14), AIR_FN(f32, 15),
    AIR_FN(f32, 16)};
static const VecFn kVecF64[kMaxD + 1] = {
    nullptr, AIR_FN(f64, 1), AIR_FN(f64, 2), AIR_FN(f64, 3), AIR_FN(f64, 4), AIR_FN(f64, 5),
    AIR_FN(f64, 6), AIR_FN(f64, 7), AIR_FN(f64, 8), AIR_FN(f64, 9), AIR_FN(f64, 10),
    AIR_FN(f64, 11), AIR_FN(f64, 12), AIR_FN(f64, 13), AIR_FN(f64, 14), AIR_FN(f64, 15),
    AIR_FN(f64, 16)};
#undef AIR_FN

// Hard-decision launchers, one per D, defined in hd_inst.hip.
using HdFn = hipError_t (*)(const HdArgs&, int, hipStream_t);
#define AIR_DECL(D) hipError_t launch_hd_d##D(const HdArgs&, int, hipStream_t);
AIR_DECL(1) AIR_DECL(2) AIR_DECL(3) AIR_DECL(4) AIR_DECL(5) AIR_DECL(6) AIR_DECL(7) AIR_DECL(8)
AIR_DECL(9) AIR_DECL(10) AIR_DECL(11) AIR_DECL(12) AIR_DECL(13) AIR_DECL(14) AIR_DECL(15) AIR_DECL(16)
#undef AIR_DECL
static const HdFn kHd[kMaxD + 1] = {
    nullptr, launch_hd_d1, launch_hd_d2, launch_hd_d3, launch_hd_d4, launch_hd_d5, launch_hd_d6,
    launch_hd_d7, launch_hd_d8, launch_hd_d9, launch_hd_d10, launch_hd_d11, launch_hd_d12,
    launch_hd_d13, launch_hd_d14, launch_hd_d15, launch_hd_d16};

// Matrix-core hard-decision launchers, one per D, defined in hd_mfma_inst.hip.
using HdMfmaFn = hipError_t (*)(const HdArgs&, const void*, float, int, hipStream_t);
#define AIR_DECL(D) hipError_t launch_hd_mfma_d##D(const HdArgs&, const void*, float, int, hipStream_t);
AIR_DECL(1) AIR_DECL(2) AIR_DECL(3) AIR_DECL(4) AIR_DECL(5) AIR_DECL(6) AIR_DECL(7) AIR_DECL(8)
AIR_DECL(9) AIR_DECL(10) AIR_DECL(11) AIR_DECL(12) AIR_DECL(13) AIR_DECL(14) AIR_DECL(15) AIR_DECL(16)
#undef AIR_DECL
static const HdMfmaFn kHdMfma[kMaxD + 1] = {
    nullptr, launch_hd_mfma_d1, launch_hd_mfma_d2, launch_hd_mfma_d3, launch_hd_mfma_d4, launch_hd_mfma_d5,
    launch_hd_mfma_d6, launch_hd_mfma_d7, launch_hd_mfma_d8, launch_hd_mfma_d9, launch_hd_mfma_d10,
    launch_hd_mfma_d11, launch_hd_mfma_d12, launch_hd_mfma_d13, launch_hd_mfma_d14, launch_hd_mfma_d15,
    launch_hd_mfma_d16};

// Matrix-core launchers, one per (operand type, D), defined in mfma_inst_*.hip.
using MfmaFn = hipError_t (*)(const DemapArgs&, const void*, int, const Launch&, int);
#define AIR_DECL(tag, D) hipError_t launch_mfma_##tag##_d##D(const DemapArgs&, const void*, int, const Launch&, int);
#define AIR_DECL_ALL(tag)                                                                        \
  AIR_DECL(tag, 1) AIR_DECL(tag, 2) AIR_DECL(tag, 3) AIR_DECL(tag, 4) AIR_DECL(tag, 5)          \
  AIR_DECL(tag, 6) AIR_DECL(tag, 7) AIR_DECL(tag, 8) AIR_DECL(tag, 9) AIR_DECL(tag, 10)         \
  AIR_DECL(tag, 11) AIR_DECL(tag, 12) AIR_DECL(tag, 13) AIR_DECL(tag, 14) AIR_DECL(tag, 15)     \
  AIR_DECL(tag, 16)
AIR_DECL_ALL(f16)
AIR_DECL_ALL(bf16)
#undef AIR_DECL_ALL
#undef AIR_DECL
#define AIR_FN(tag, D) launch_mfma_##tag##_d##D
static const MfmaFn kMfmaF16[kMaxD + 1] = {
    nullptr, AIR_FN(f16, 1), AIR_FN(f16, 2), AIR_FN(f16, 3), AIR_FN(f16, 4), AIR_FN(f16, 5),
    AIR_FN(f16, 6), AIR_FN(f16, 7), AIR_FN(f16, 8), AIR_FN(f16, 9), AIR_FN(f16, 10),
    AIR_FN(f16, 11), AIR_FN(f16, 12), AIR_FN(f16, 13), AIR_FN(f16, 14), AIR_FN(f16, 15),
    AIR_FN(f16, 16)};
static const MfmaFn kMfmaBF16[kMaxD + 1] = {
    nullptr, AIR_FN(bf16, 1), AIR_FN(bf16, 2), AIR_FN(bf16, 3), AIR_FN(bf16, 4), AIR_FN(bf16, 5),
    AIR_FN(bf16, 6), AIR_FN(bf16, 7), AIR_FN(bf16, 8), AIR_FN(bf16, 9), AIR_FN(bf16, 10),
    AIR_FN(bf16, 11), AIR_FN(bf16, 12), AIR_FN(bf16, 13), AIR_FN(bf16, 14), AIR_FN(bf16, 15),
    AIR_FN(bf16, 16)};
#undef AIR_FN

// Grid of a matrix-core launch: 4 waves per block, one pair of 32-sample
// tiles (64 samples) per wave and round.
static int mfma_grid(int64_t N) {
  const int64_t pairs = ((N + 31) / 32 + 1) / 2;
  const int64_t g = (pairs + 3) / 4;
  return (int)(g < kMaxGrid ? g : kMaxGrid);
}

// Grid of a vector-kernel launch: one sample per thread and round. Sets of
// M >= 32 points take up to kMaxGrid blocks; for the small sets, whose
// samples are cheap, the per-block reductions weigh more and 1024 blocks
// measured faster (2-D QAM-4 buffers of 2^20 symbols: 1536 blocks, 25 %
// slower).
static int vec_grid(int64_t N, int M = 0) {
  const int64_t cap = M >= 32 ? kMaxGrid : 1024;
  const int64_t g = (N + kBlock - 1) / kBlock;
  return (int)(g < cap ? g : cap);
}

// Fixed-order reduction of the per-block partials of one launch: block s
// reduces SNR point s; wave q of it sums quantity q over the demapping blocks
// (lane l takes blocks l, l + 64, ...; then a fixed butterfly), so the result
// does not depend on timing. stats[4 s + q] = MI, GMI, SE_MI, SE_GMI; NaN if
// a tx index was invalid. Block 0 folds this call's error into the sticky word
// and zeroes the next call's words.
__global__ __launch_bounds__(256) void finish_kernel(const double* __restrict__ partials,
                                                     const double* __restrict__ t2_partials,
                                                     int nblocks, int nblocks2, int64_t N, int M, int m,
                                                     double* stats, const CallWords* call,
                                                     CallWords* next, int* sticky, int no_mi) {
  __shared__ double sums[4];
  const int s = blockIdx.x;
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double t = 0.0;
  // each lane's blocks (at most kMaxGrid / 64 = 24 per list) loaded at once,
  // then added in block order
  constexpr int kPer = kMaxGrid / 64;
  const double* p = partials + ((int64_t)s * 4 + q) * nblocks;
  double v[kPer], v2[kPer];
  const double* p2 = t2_partials ? t2_partials + ((int64_t)s * 4 + q) * nblocks2 : nullptr;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    v[i] = lane + 64 * i < nblocks ? p[lane + 64 * i] : 0.0;
    v2[i] = p2 && lane + 64 * i < nblocks2 ? p2[lane + 64 * i] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) t += v[i];
#pragma unroll
  for (int i = 0; i < kPer; ++i) t += v2[i];
  t = wave_sum(t);
  if (lane == 0) sums[q] = t;
  __syncthreads();
  const int bad = call->err;
  if (threadIdx.x == 0) {
    if (stats) {
      const double n = (double)N;
      const double su = sums[0], sv = sums[1], suu = sums[2], svv = sums[3];
      double mi = log2((double)M) - su / n;
      double gmi = (double)m - sv / n;
      double se_mi = __builtin_nan(""), se_gmi = __builtin_nan("");
      if (N > 1) {
        const double vu = (suu - su * su / n) / (n - 1.0);
        const double vv = (svv - sv * sv / n) / (n - 1.0);
        se_mi = sqrt((vu > 0.0 ? vu : 0.0) / n);
        se_gmi = sqrt((vv > 0.0 ? vv : 0.0) / n);
      }
      if (no_mi) mi = se_mi = __builtin_nan("");       // max-log: no symbol-wise MI
      if (bad) mi = gmi = se_mi = se_gmi = __builtin_nan("");
      stats[4 * s + 0] = mi;
      stats[4 * s + 1] = gmi;
      stats[4 * s + 2] = se_mi;
      stats[4 * s + 3] = se_gmi;
    }
    if (s == 0) {
      if (bad) atomicOr(sticky, bad);
      clear_call_words(next);
    }
  }
}

// Folds a call's tx-range error into the sticky word and zeroes the next
// call's words (calls without a reduction kernel of their own).
__global__ void fold_error_kernel(const CallWords* call, CallWords* next, int* sticky) {
  if (threadIdx.x == 0) {
    if (call->err) atomicOr(sticky, call->err);
    clear_call_words(next);
  }
}

// noalloc.hip: looks up the no-allocation scratch array's address on a device.
hipError_t noalloc_scratch_init(int device);

}  // namespace air

using namespace air;

namespace {

int bits_of(int M) {
  int m = 0;
  while ((1 << m) < M) ++m;
  return m;
}

// Round-to-nearest-even conversions of a double to half / bfloat16 bits.
uint16_t to_f16_bits(double v) {
  _Float16 h = (_Float16)v;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}
double from_f16_bits(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (double)h;
}
uint16_t to_bf16_bits(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double from_bf16_bits(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// Point side of the matrix-core K slots for one point x (length D), as
// operand bits, q = |x|^2, every part rounded to nearest even (hi = round(v),
// lo = round(v - hi); bfloat16: mid = round(v - hi), lo = round(v - hi - mid)):
//  slot for slot, half precision: [x_hi | x_lo | x_hi | q_hi, q_lo, q_hi | 1],
//    bfloat16: [x_hi | x_mid | x_lo | x_hi | x_mid | x_hi |
//               q_hi, q_mid, q_lo, q_hi, q_mid, q_hi | 1];
//  shared chunks, half precision: [x_hi | q_hi, q_lo | 1 | x_lo],
//    bfloat16: [x_hi | q_hi, q_mid, q_lo | 1 | x_mid | x_lo];
// then zeros to whole chunks. The 1 multiplies the sample side's shift.
void point_record(const double* x, int D, bool bf, uint16_t* out) {
  const int kp = 16 * mfma_nk(D, bf);
  auto cv = [bf](double v) { return bf ? to_bf16_bits(v) : to_f16_bits(v); };
  auto back = [bf](uint16_t b) { return bf ? from_bf16_bits(b) : from_f16_bits(b); };
  for (int k = 0; k < kp; ++k) out[k] = 0;
  double q = 0.0;
  for (int d = 0; d < D; ++d) q += x[d] * x[d];
  // parts[level]: hi, (mid,) lo
  auto split = [&](double v, uint16_t* parts) {
    parts[0] = cv(v);
    const double r = v - back(parts[0]);
    if (bf) {
      parts[1] = cv(r);
      parts[2] = cv(r - back(parts[1]));
    } else {
      parts[1] = cv(r);
    }
  };
  uint16_t qp[3];
  split(q, qp);
  if (shared_chunks(D, bf)) {
    const int L = split_levels(bf);
    for (int d = 0; d < D; ++d) {
      uint16_t xp[3];
      split(x[d], xp);
      out[d] = xp[0];
      if (bf) {
        out[D + 4 + d] = xp[1];
        out[2 * D + 4 + d] = xp[2];
      } else {
        out[D + 3 + d] = xp[1];
      }
    }
    for (int l = 0; l <= L; ++l) out[D + l] = qp[l];
  } else if (bf) {
    for (int d = 0; d < D; ++d) {
      uint16_t xp[3];
      split(x[d], xp);
      out[d] = xp[0];
      out[D + d] = xp[1];
      out[2 * D + d] = xp[2];
      out[3 * D + d] = xp[0];
      out[4 * D + d] = xp[1];
      out[5 * D + d] = xp[0];
    }
    out[6 * D] = qp[0];
    out[6 * D + 1] = qp[1];
    out[6 * D + 2] = qp[2];
    out[6 * D + 3] = qp[0];
    out[6 * D + 4] = qp[1];
    out[6 * D + 5] = qp[0];
  } else {
    for (int d = 0; d < D; ++d) {
      uint16_t xp[3];
      split(x[d], xp);
      out[d] = xp[0];
      out[D + d] = xp[1];
      out[2 * D + d] = xp[0];
    }
    out[3 * D] = qp[0];
    out[3 * D + 1] = qp[1];
    out[3 * D + 2] = qp[0];
  }
  out[shift_slot(D, bf)] = cv(1.0);
}

// Per-SNR scalars of one launch.
// With `aux`, the values are the noise variances of the receiver's Gaussian
// metric (auxiliary channel) instead of SNR points.
void fill_snr(SnrTable& t, const air_const* c, const double* snr_db, int S, bool aux) {
  for (int s = 0; s < S; ++s) {
    if (aux) sigma2_scalars(snr_db[s], t.sigma[s], t.c[s]);
    else snr_scalars(c, snr_db[s], t.sigma[s], t.c[s]);
    t.sigmaf[s] = (float)t.sigma[s];
    t.cf[s] = (float)t.c[s];
  }
}

// Second-tier workspace: `slots` list entries and `counts` per-wave counters;
// grows on demand and is kept, so repeated calls of one size allocate nothing.
void free_t2(air_ctx* ctx) {
  (void)hipFree(ctx->t2_list);
  (void)hipFree(ctx->t2_nitem);
  (void)hipFree(ctx->t2_items);
  ctx->t2_list = nullptr;
  ctx->t2_nitem = nullptr;
  ctx->t2_items = nullptr;
  ctx->t2_slots = ctx->t2_counts = 0;
}

air_status ensure_t2(air_ctx* ctx, int64_t slots, int64_t counts) {
  if (slots <= ctx->t2_slots && counts <= ctx->t2_counts) return AIR_OK;
  (void)hipStreamSynchronize(ctx->stream);
  free_t2(ctx);
  hipError_t e = hipMalloc(&ctx->t2_list, sizeof(unsigned long long) * slots);
  if (e == hipSuccess) e = hipMalloc(&ctx->t2_nitem, sizeof(unsigned int) * counts);
  // every slot lists one 32-sample tile, so an SNR point's gathered samples
  // fit in 32 entries per slot of that point
  if (e == hipSuccess) e = hipMalloc(&ctx->t2_items, sizeof(uint32_t) * 32 * slots);
  if (e != hipSuccess) {
    free_t2(ctx);
    return hip_fail(ctx, e, "second-tier workspace");
  }
  ctx->t2_slots = slots;
  ctx->t2_counts = counts;
  return AIR_OK;
}

// The words of a new call: the slot that the previous call's final kernel
// zeroed or, when that kernel was not issued (a call that failed part-way), a
// slot zeroed here. *next receives the slot this call's final kernel zeroes.
hipError_t begin_call(air_ctx* ctx, CallWords** next) {
  CallWords* cur = ctx->call == ctx->calls ? ctx->calls + 1 : ctx->calls;
  *next = cur == ctx->calls ? ctx->calls + 1 : ctx->calls;
  ctx->call = cur;
  const bool zeroed = ctx->next_zeroed;
  ctx->next_zeroed = false;
  return zeroed ? hipSuccess : hipMemsetAsync(cur, 0, sizeof(CallWords), ctx->stream);
}

bool prec_ok(air_prec p) { return p == AIR_FP64 || p == AIR_FP32 || p == AIR_BF16X3 || p == AIR_FP16X3; }

// Common driver of air_llr / air_mi_gmi / air_sweep.
// With `scratch` (scratch_bytes of device memory), the second tier's lists,
// counts and gathered samples of each launch are carved from it instead of
// the context's workspace, no timing events are created, and each launch
// takes as many SNR points as fit (air_sweep_noalloc): nothing is allocated.
air_status run(air_ctx* ctx, const air_const* c, const void* in, const uint32_t* tx, int64_t N,
               const double* snr_db, int S, int sweep, air_prec prec, double* stats, void* llr,
               bool aux = false, bool maxlog = false, void* scratch = nullptr, size_t scratch_bytes = 0) {
  if (!ctx) return AIR_E_INVAL;
  if (!c || c->ctx != ctx) return fail(ctx, AIR_E_INVAL, "constellation is null or from another context");
  if (!in) return fail(ctx, AIR_E_INVAL, sweep ? "Z_dev is null" : "Y_dev is null");
  if (N < 1) return fail(ctx, AIR_E_INVAL, "N must be >= 1");
  if (S < 1 || !snr_db) return fail(ctx, AIR_E_INVAL, "need at least one SNR point");
  if (!prec_ok(prec)) return fail(ctx, AIR_E_INVAL, "unknown precision");
  for (int s = 0; s < S; ++s) {
    if (!std::isfinite(snr_db[s])) return fail(ctx, AIR_E_INVAL, "SNR values must be finite");
    if (aux && !(snr_db[s] > 0.0)) return fail(ctx, AIR_E_INVAL, "sigma2_aux must be positive and finite");
  }
  if (prec == AIR_FP16X3 && !c->f16_ok)
    return fail(ctx, AIR_E_UNSUPPORTED, "constellation coordinates exceed the half-precision range");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
  if (!is_device_ptr(ctx, in)) return fail(ctx, AIR_E_INVAL, "input block is not device memory of this context");
  if (tx && !is_device_ptr(ctx, tx)) return fail(ctx, AIR_E_INVAL, "tx_dev is not device memory of this context");
  if (stats && !is_device_ptr(ctx, stats)) return fail(ctx, AIR_E_INVAL, "stats_dev is not device memory of this context");
  if (llr && !is_device_ptr(ctx, llr)) return fail(ctx, AIR_E_INVAL, "llr_dev is not device memory of this context");

  const bool fp64 = prec == AIR_FP64;
  const size_t tsz = fp64 ? sizeof(double) : sizeof(float);
  // matrix-core tiles hold 16 or 32 points; smaller sets run the FP32 vector kernel
  const bool mfma = (prec == AIR_FP16X3 || prec == AIR_BF16X3) && c->M >= 16;
  const int grid = mfma ? mfma_grid(N) : vec_grid(N, c->M);
  const VecFn vfn = fp64 ? kVecF64[c->D] : kVecF32[c->D];
  const MfmaFn mfn = prec == AIR_BF16X3 ? kMfmaBF16[c->D] : kMfmaF16[c->D];
  const void* rec = prec == AIR_BF16X3 ? (const void*)c->rec_bf16 : (const void*)c->rec_f16;
  DemapArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.tx = tx;
  a.partials = ctx->partials;
  a.xl = fp64 ? (const void*)c->x64 : (const void*)c->x32;
  a.lab = c->lab;
  a.N = N;
  a.llr_stride_s = N * (int64_t)c->m;
  a.M = c->M;
  a.m = c->m;
  a.D = c->D;
  a.sweep = sweep;
  // the FP32 vector kernel's exact form (AIR_FP32, and the matrix-core
  // precisions on sets of fewer than 16 points) also has a second tier
  const bool vec_t2 = !mfma && !fp64 && !maxlog;
  int snr_per_launch = kMaxSnrPerLaunch;
  if (mfma || vec_t2) {
    // per (SNR point, wave) a run of list slots, one per sample tile the wave
    // owns (matrix cores: pairs of tiles dealt out to the waves; vector
    // kernel: two tiles per wave and round, every slot written)
    const int64_t ntiles = (N + 31) / 32;
    const int64_t waves = (int64_t)grid * 4;
    const int64_t npairs = (ntiles + 1) / 2;
    const int64_t stride = (int64_t)grid * kBlock;
    const int64_t tpw = mfma ? 2 * ((npairs + waves - 1) / waves) : 2 * ((N + stride - 1) / stride);
    // tile indices, sample indices (with the padding of the last tile pair)
    // and per-SNR sample counts of the two tiers are 32-bit
    if (N > ((int64_t)1 << 32) - 128) return fail(ctx, AIR_E_UNSUPPORTED, "N too large for one call");
    if (scratch) {
      // per SNR point of a launch: list slots (8 bytes), flagged counts per
      // wave (4) and 32 gathered sample indices per slot (4 each); three
      // parts, each starting on a 256-byte boundary
      const int64_t per_snr = waves * tpw * 8 + waves * 4 + waves * tpw * 32 * 4;
      const int64_t avail = (int64_t)scratch_bytes - 3 * 256;
      const int64_t fit = avail > 0 ? avail / per_snr : 0;
      if (fit < 1)
        return fail(ctx, AIR_E_INVAL, "N too large for air_sweep_noalloc: one SNR point needs " +
                                          std::to_string(per_snr) + " bytes of its " +
                                          std::to_string(scratch_bytes) + "-byte scratch");
      snr_per_launch = (int)(fit < kMaxSnrPerLaunch ? fit : kMaxSnrPerLaunch);
      const int64_t sl = snr_per_launch;
      auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
      char* base = static_cast<char*>(scratch);
      a.t2_list = reinterpret_cast<unsigned long long*>(base);
      a.t2_nitem = reinterpret_cast<unsigned int*>(base + up(sl * waves * tpw * 8));
      a.t2_items = reinterpret_cast<uint32_t*>(base + up(sl * waves * tpw * 8) + up(sl * waves * 4));
    } else {
      const int64_t sl = S < kMaxSnrPerLaunch ? S : kMaxSnrPerLaunch;
      const air_status st = ensure_t2(ctx, sl * waves * tpw, sl * waves);
      if (st != AIR_OK) return st;
      a.t2_list = ctx->t2_list;
      a.t2_nitem = ctx->t2_nitem;
      a.t2_items = ctx->t2_items;
    }
    a.t2_partials = ctx->t2_partials;
    a.t2_tpw = (int)tpw;
    a.t2_cap = waves * tpw * 32;
    a.t2_tot = ctx->t2_tot;
  }
  CallWords* next = nullptr;
  hipError_t e = begin_call(ctx, &next);
  if (e != hipSuccess) return hip_fail(ctx, e, "clear call words");
  a.err = &ctx->call->err;
  a.recomputed = &ctx->call->recomputed;
  a.exact = &ctx->call->exact;
  for (int s0 = 0; s0 < S; s0 += snr_per_launch) {
    const int ns = (S - s0 < snr_per_launch) ? S - s0 : snr_per_launch;
    a.S = ns;
    fill_snr(a.snr, c, snr_db + s0, ns, aux);
    a.llr = llr ? (void*)((char*)llr + (size_t)s0 * N * c->m * tsz) : nullptr;
    // timed: the demapping kernel's dispatch itself sets the two events; they
    // serve timing only, so they skip the system-scope fence (a cache
    // write-back that idles the stream around the kernel: 5.8 -> 2.3 us per
    // 8-PSK^2 step)
    Launch lt{ctx->stream, nullptr, nullptr};
    if (ctx->timing && !scratch) {
      if (ctx->ev_used + 2 > ctx->ev.size()) {
        for (int k = 0; k < 2; ++k) {
          hipEvent_t ev;
          e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
          if (e != hipSuccess) return hip_fail(ctx, e, "timing event");
          ctx->ev.push_back(ev);
        }
      }
      lt.start = ctx->ev[ctx->ev_used];
      lt.stop = ctx->ev[ctx->ev_used + 1];
      ctx->ev_used += 2;
    }
    e = mfma ? mfn(a, rec, grid, lt, maxlog ? 2 : 0) : vfn(a, grid, lt, maxlog, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "demapping kernel launch");
    const bool tier2 = (mfma && !maxlog) || vec_t2;
    if (tier2) {
      const Launch l2{ctx->stream, nullptr, nullptr};
      e = mfma ? mfn(a, rec, grid, l2, 1) : vfn(a, grid, l2, false, 1);
      if (e != hipSuccess) return hip_fail(ctx, e, "second-tier launch");
    }
    hipLaunchKernelGGL(finish_kernel, dim3(ns), dim3(256), 0, ctx->stream, ctx->partials,
                       tier2 ? ctx->t2_partials : nullptr, grid, t2_grid(grid), N, c->M, c->m,
                       stats ? stats + 4 * s0 : nullptr, ctx->call, next, ctx->sticky, maxlog ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "reduction kernel launch");
  }
  ctx->next_zeroed = true;
  ctx->err.clear();
  return AIR_OK;
}

}  // namespace

namespace air {

// The sweep with a caller-supplied second-tier workspace (noalloc.hip).
air_status run_sweep_scratch(air_ctx* ctx, const air_const* c, const void* Z, const uint32_t* tx, int64_t N,
                             const double* snr_db, int S, air_prec prec, double* stats, void* llr,
                             void* scratch, size_t scratch_bytes) {
  return run(ctx, c, Z, tx, N, snr_db, S, 1, prec, stats, llr, false, false, scratch, scratch_bytes);
}

}  // namespace air

namespace {

// Driver of air_hard_decide / air_hard_sweep.
air_status run_hd(air_ctx* ctx, const air_const* c, const float* in, const uint32_t* tx, int64_t N,
                  const double* snr_db, int S, int sweep, uint32_t* decided, uint64_t* counts) {
  if (!ctx) return AIR_E_INVAL;
  if (!c || c->ctx != ctx) return fail(ctx, AIR_E_INVAL, "constellation is null or from another context");
  if (!in) return fail(ctx, AIR_E_INVAL, sweep ? "Z_dev is null" : "Y_dev is null");
  if (N < 1) return fail(ctx, AIR_E_INVAL, "N must be >= 1");
  if (S < 1) return fail(ctx, AIR_E_INVAL, "need at least one SNR point");
  if (counts && !tx) return fail(ctx, AIR_E_INVAL, "error counts need tx_dev");
  if (sweep)
    for (int s = 0; s < S; ++s)
      if (!std::isfinite(snr_db[s])) return fail(ctx, AIR_E_INVAL, "SNR values must be finite");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
  if (!is_device_ptr(ctx, in)) return fail(ctx, AIR_E_INVAL, "input block is not device memory of this context");
  if (tx && !is_device_ptr(ctx, tx)) return fail(ctx, AIR_E_INVAL, "tx_dev is not device memory of this context");
  if (decided && !is_device_ptr(ctx, decided))
    return fail(ctx, AIR_E_INVAL, "decided_dev is not device memory of this context");
  if (counts && !is_device_ptr(ctx, counts))
    return fail(ctx, AIR_E_INVAL, "counts_dev is not device memory of this context");
  HdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.tx = tx;
  a.xl = c->x32;
  a.lab = c->lab;
  a.pos = c->pos;
  a.N = N;
  a.M = c->M;
  a.sweep = sweep;
  CallWords* next = nullptr;
  hipError_t e = begin_call(ctx, &next);
  a.err = &ctx->call->err;
  if (e == hipSuccess && counts)
    e = hipMemsetAsync(counts, 0, sizeof(uint64_t) * 2 * (size_t)S, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "clear counters");
  // Matrix cores for M >= 32 when the coordinates are of moderate range
  // (max |x| in [1/16, 64]: the error bound of the product tiles holds), the
  // vector kernel otherwise; both decide as the FP32 procedure does.
  const bool on_mfma = c->M >= 32 && c->f16_ok && c->r2max >= 0x1p-8 && c->r2max <= 0x1p12;
  const int grid = on_mfma ? mfma_grid(N) : vec_grid(N, c->M);
  for (int s0 = 0; s0 < S; s0 += kMaxSnrPerLaunch) {
    const int ns = (S - s0 < kMaxSnrPerLaunch) ? S - s0 : kMaxSnrPerLaunch;
    a.S = ns;
    for (int s = 0; s < ns; ++s) {
      double sigma = 0.0, cc = 0.0;
      if (sweep) snr_scalars(c, snr_db[s0 + s], sigma, cc);
      a.sigma[s] = (float)sigma;
    }
    a.decided = decided ? decided + (size_t)s0 * N : nullptr;
    a.counts = counts ? reinterpret_cast<unsigned long long*>(counts) + 2 * s0 : nullptr;
    e = on_mfma ? kHdMfma[c->D](a, c->rec_f16, (float)c->r2max, grid, ctx->stream)
                : kHd[c->D](a, grid, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hard-decision kernel launch");
  }
  // a tx-range error is reported by air_sync like the demapping calls'
  hipLaunchKernelGGL(fold_error_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->call, next, ctx->sticky);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "error fold launch");
  ctx->next_zeroed = true;
  ctx->err.clear();
  return AIR_OK;
}

// Driver of air_noise_var.
air_status run_noise_var(air_ctx* ctx, const air_const* c, const void* Y, const uint32_t* tx,
                         int64_t N, air_prec prec, double* var) {
  if (!ctx) return AIR_E_INVAL;
  if (!c || c->ctx != ctx) return fail(ctx, AIR_E_INVAL, "constellation is null or from another context");
  if (!Y || !tx || !var) return fail(ctx, AIR_E_INVAL, "Y_dev, tx_dev and var_dev must not be null");
  if (N < 1) return fail(ctx, AIR_E_INVAL, "N must be >= 1");
  if (!prec_ok(prec)) return fail(ctx, AIR_E_INVAL, "unknown precision");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
  if (!is_device_ptr(ctx, Y)) return fail(ctx, AIR_E_INVAL, "Y_dev is not device memory of this context");
  if (!is_device_ptr(ctx, tx)) return fail(ctx, AIR_E_INVAL, "tx_dev is not device memory of this context");
  if (!is_device_ptr(ctx, var)) return fail(ctx, AIR_E_INVAL, "var_dev is not device memory of this context");
  CallWords* next = nullptr;
  hipError_t e = begin_call(ctx, &next);
  if (e != hipSuccess) return hip_fail(ctx, e, "clear call words");
  const int grid = vec_grid(N);     // <= kMaxGrid: D x grid partials fit the workspace
  if (prec == AIR_FP64)
    hipLaunchKernelGGL(noise_var_kernel<double>, dim3(grid), dim3(kBlock), 0, ctx->stream,
                       static_cast<const double*>(Y), tx, c->lab, c->x64, N, c->M, c->D, ctx->partials,
                       &ctx->call->err);
  else
    hipLaunchKernelGGL(noise_var_kernel<float>, dim3(grid), dim3(kBlock), 0, ctx->stream,
                       static_cast<const float*>(Y), tx, c->lab, c->x64, N, c->M, c->D, ctx->partials,
                       &ctx->call->err);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "noise estimate launch");
  hipLaunchKernelGGL(noise_var_finish, dim3(1), dim3(64), 0, ctx->stream, ctx->partials, grid, c->D, N,
                     var, &ctx->call->err, next, ctx->sticky);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "noise estimate reduction launch");
  ctx->next_zeroed = true;
  ctx->err.clear();
  return AIR_OK;
}

}  // namespace

extern "C" {

air_status air_create(air_ctx** out, int device, void* hip_stream) {
  if (!out) return AIR_E_INVAL;
  *out = nullptr;
  try {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return AIR_E_INVAL;
    DeviceGuard g(device);
    if (!g.ok) return AIR_E_DEVICE;
    air_ctx* ctx = new air_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    hipError_t e = hipMalloc(&ctx->partials, sizeof(double) * kMaxGrid * kMaxSnrPerLaunch * 4);
    if (e == hipSuccess) e = hipMalloc(&ctx->t2_partials, sizeof(double) * kMaxGrid * kMaxSnrPerLaunch * 4);
    if (e == hipSuccess) e = hipMalloc(&ctx->t2_tot, sizeof(unsigned int) * kMaxSnrPerLaunch);
    if (e == hipSuccess) e = hipMalloc(&ctx->calls, 2 * sizeof(CallWords));
    if (e == hipSuccess) e = hipMalloc(&ctx->sticky, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&ctx->small, sizeof(double) * kSmallDoubles);
    if (e == hipSuccess) e = hipMemset(ctx->calls, 0, 2 * sizeof(CallWords));
    ctx->call = ctx->calls;
    if (e == hipSuccess) e = hipMemset(ctx->sticky, 0, sizeof(int));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    // the no-allocation entry point's scratch on this device (looked up once
    // per device; if that fails, air_sweep_noalloc reports it)
    if (e == hipSuccess) (void)noalloc_scratch_init(device);
    if (e != hipSuccess) {
      air_destroy(ctx);
      return e == hipErrorOutOfMemory ? AIR_E_NOMEM : AIR_E_DEVICE;
    }
    *out = ctx;
    return AIR_OK;
  } catch (...) {
    return AIR_E_NOMEM;
  }
}

void air_destroy(air_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(ctx->partials);
  (void)hipFree(ctx->calls);
  (void)hipFree(ctx->sticky);
  free_t2(ctx);
  (void)hipFree(ctx->t2_partials);
  (void)hipFree(ctx->t2_tot);
  (void)hipFree(ctx->small);
  for (hipEvent_t ev : ctx->ev) (void)hipEventDestroy(ev);
  delete ctx;
}

air_status air_set_stream(air_ctx* ctx, void* hip_stream) {
  if (!ctx) return AIR_E_INVAL;
  // the next call reuses the workspace and call words of the work already
  // issued, so that work finishes first
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
  const hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "synchronize the previous stream");
  ctx->stream = (hipStream_t)hip_stream;
  return AIR_OK;
}

const char* air_last_error(const air_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

air_status air_sync(air_ctx* ctx) {
  if (!ctx) return AIR_E_INVAL;
  try {
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronize");
    int sticky = 0;
    e = hipMemcpy(&sticky, ctx->sticky, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "read device error word");
    if (sticky) {
      const int zero = 0;
      e = hipMemcpy(ctx->sticky, &zero, sizeof(int), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(ctx, e, "clear device error word");
      return fail(ctx, AIR_E_RANGE, "a transmitted index >= M was seen; affected statistics are NaN");
    }
    return AIR_OK;
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_const_create(air_ctx* ctx, const double* X, const uint32_t* labels, int M, int D,
                            air_const** out) {
  if (!ctx) return AIR_E_INVAL;
  if (!out) return fail(ctx, AIR_E_INVAL, "out is null");
  *out = nullptr;
  if (!X || !labels) return fail(ctx, AIR_E_INVAL, "X_host and labels_host must not be null");
  if (M < 2 || M > 4096 || (M & (M - 1)) != 0)
    return fail(ctx, AIR_E_INVAL, "M must be a power of two in [2, 4096]");
  if (D < 1 || D > kMaxD) return fail(ctx, AIR_E_INVAL, "D must be in [1, 16]");
  try {
    std::vector<int> pos(M, -1);
    for (int j = 0; j < M; ++j) {
      if (labels[j] >= (uint32_t)M || pos[labels[j]] >= 0)
        return fail(ctx, AIR_E_INVAL, "labels must be a bijection onto {0..M-1}");
      pos[labels[j]] = j;
    }
    for (int64_t i = 0; i < (int64_t)M * D; ++i)
      if (!std::isfinite(X[i])) return fail(ctx, AIR_E_INVAL, "X must be finite");
    // label order: row l holds the point whose label is l
    std::vector<double> x64((size_t)M * D);
    std::vector<float> x32((size_t)M * D);
    double es = 0.0;
    for (int l = 0; l < M; ++l) {
      double e = 0.0;
      for (int d = 0; d < D; ++d) {
        const double v = X[(size_t)pos[l] * D + d];
        x64[(size_t)l * D + d] = v;
        x32[(size_t)l * D + d] = (float)v;
        e += v * v;
      }
      es += e;
    }
    es /= (double)M;
    if (!(es > 0.0)) return fail(ctx, AIR_E_INVAL, "constellation has zero energy");
    const int kp = 16 * mfma_nk(D, false);
    const int kpb = 16 * mfma_nk(D, true);
    std::vector<uint16_t> r16((size_t)M * kp), rbf((size_t)M * kpb);
    bool f16_ok = true;
    for (int l = 0; l < M; ++l) {
      double q = 0.0;
      for (int d = 0; d < D; ++d) {
        const double v = x64[(size_t)l * D + d];
        q += v * v;
        f16_ok &= std::fabs(v) < 60000.0;
      }
      f16_ok &= q < 60000.0;
      point_record(&x64[(size_t)l * D], D, false, &r16[(size_t)l * kp]);
      point_record(&x64[(size_t)l * D], D, true, &rbf[(size_t)l * kpb]);
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
    air_const* c = new air_const();
    c->ctx = ctx;
    c->device = ctx->device;
    c->M = M;
    c->D = D;
    c->m = bits_of(M);
    c->es = es;
    c->f16_ok = f16_ok;
    for (int l = 0; l < M; ++l) {
      double q = 0.0;
      for (int d = 0; d < D; ++d) q += x64[(size_t)l * D + d] * x64[(size_t)l * D + d];
      c->r2max = q > c->r2max ? q : c->r2max;
    }
    hipError_t e = hipMalloc(&c->x64, sizeof(double) * M * D);
    if (e == hipSuccess) e = hipMalloc(&c->x32, sizeof(float) * M * D);
    if (e == hipSuccess) e = hipMalloc(&c->lab, sizeof(uint32_t) * M);
    if (e == hipSuccess) e = hipMalloc(&c->pos, sizeof(uint32_t) * M);
    if (e == hipSuccess) e = hipMalloc(&c->rec_f16, sizeof(uint16_t) * M * kp);
    if (e == hipSuccess) e = hipMalloc(&c->rec_bf16, sizeof(uint16_t) * M * kpb);
    if (e == hipSuccess) e = hipMemcpy(c->rec_f16, r16.data(), sizeof(uint16_t) * M * kp, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->rec_bf16, rbf.data(), sizeof(uint16_t) * M * kpb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->x64, x64.data(), sizeof(double) * M * D, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->x32, x32.data(), sizeof(float) * M * D, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->lab, labels, sizeof(uint32_t) * M, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      std::vector<uint32_t> posu(pos.begin(), pos.end());
      e = hipMemcpy(c->pos, posu.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      air_const_destroy(c);
      return hip_fail(ctx, e, "constellation upload");
    }
    *out = c;
    ctx->err.clear();
    return AIR_OK;
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

void air_const_destroy(air_const* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipFree(c->x64);
  (void)hipFree(c->x32);
  (void)hipFree(c->lab);
  (void)hipFree(c->pos);
  (void)hipFree(c->rec_f16);
  (void)hipFree(c->rec_bf16);
  delete c;
}

int air_const_bits(const air_const* c) { return c ? c->m : 0; }

air_status air_llr(air_ctx* ctx, const air_const* c, const void* Y_dev, int64_t N, double snr_db,
                   air_prec prec, void* llr_dev) {
  if (ctx && !llr_dev) return fail(ctx, AIR_E_INVAL, "llr_dev is null");
  try {
    return run(ctx, c, Y_dev, nullptr, N, &snr_db, 1, 0, prec, nullptr, llr_dev);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_mi_gmi(air_ctx* ctx, const air_const* c, const void* Y_dev, const uint32_t* tx_dev,
                      int64_t N, double snr_db, air_prec prec, double* stats_dev, void* llr_dev) {
  if (ctx && (!tx_dev || !stats_dev)) return fail(ctx, AIR_E_INVAL, "tx_dev and stats_dev must not be null");
  try {
    return run(ctx, c, Y_dev, tx_dev, N, &snr_db, 1, 0, prec, stats_dev, llr_dev);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_llr_aux(air_ctx* ctx, const air_const* c, const void* Y_dev, int64_t N, double sigma2_aux,
                       air_prec prec, void* llr_dev) {
  if (ctx && !llr_dev) return fail(ctx, AIR_E_INVAL, "llr_dev is null");
  try {
    return run(ctx, c, Y_dev, nullptr, N, &sigma2_aux, 1, 0, prec, nullptr, llr_dev, true);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_mi_gmi_aux(air_ctx* ctx, const air_const* c, const void* Y_dev, const uint32_t* tx_dev,
                          int64_t N, double sigma2_aux, air_prec prec, double* stats_dev, void* llr_dev) {
  if (ctx && (!tx_dev || !stats_dev)) return fail(ctx, AIR_E_INVAL, "tx_dev and stats_dev must not be null");
  try {
    return run(ctx, c, Y_dev, tx_dev, N, &sigma2_aux, 1, 0, prec, stats_dev, llr_dev, true);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_aux_rates(air_ctx* ctx, const air_const* c, const void* Y_dev, const uint32_t* tx_dev,
                         int64_t N, air_prec prec, double* var_host, double* rates_host) {
  if (ctx && !rates_host) return fail(ctx, AIR_E_INVAL, "rates_host is null");
  try {
    if (!ctx) return AIR_E_INVAL;
    if (!c || c->ctx != ctx) return fail(ctx, AIR_E_INVAL, "constellation is null or from another context");
    static_assert(kMaxD + 1 + 4 <= kSmallDoubles, "small device buffer too small");
    double* var_dev = ctx->small;
    double* stats_dev = ctx->small + (kMaxD + 1);
    air_status st = run_noise_var(ctx, c, Y_dev, tx_dev, N, prec, var_dev);
    if (st != AIR_OK) return st;
    DeviceGuard g(ctx->device);
    double var[kMaxD + 1];
    // the estimate is needed on the host to form the metric's scale
    hipError_t e = hipMemcpyAsync(var, var_dev, sizeof(double) * (c->D + 1), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "read the noise estimate");
    if (var_host)
      for (int d = 0; d <= c->D; ++d) var_host[d] = var[d];
    const double s2 = var[c->D];
    if (!(s2 > 0.0) || !std::isfinite(s2)) {
      for (int i = 0; i < 7; ++i) rates_host[i] = std::nan("");
      rates_host[0] = s2;
      const air_status se = air_sync(ctx);   // reports a tx-range error
      return se != AIR_OK ? se : fail(ctx, AIR_E_RANGE, "noise estimate is zero or not finite");
    }
    st = run(ctx, c, Y_dev, tx_dev, N, &s2, 1, 0, prec, stats_dev, nullptr, true);
    if (st != AIR_OK) return st;
    double stats[4];
    e = hipMemcpyAsync(stats, stats_dev, sizeof(stats), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "read the rates");
    rates_host[0] = s2;
    for (int i = 0; i < 4; ++i) rates_host[1 + i] = stats[i];
    st = air_ngmi(stats, 1, c->m, rates_host + 5);
    if (st != AIR_OK) return fail(ctx, st, "NGMI");
    return air_sync(ctx);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_llr_maxlog(air_ctx* ctx, const air_const* c, const void* Y_dev, int64_t N, double snr_db,
                          air_prec prec, void* llr_dev) {
  if (ctx && !llr_dev) return fail(ctx, AIR_E_INVAL, "llr_dev is null");
  try {
    return run(ctx, c, Y_dev, nullptr, N, &snr_db, 1, 0, prec, nullptr, llr_dev, false, true);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_gmi_maxlog(air_ctx* ctx, const air_const* c, const void* Y_dev, const uint32_t* tx_dev,
                          int64_t N, double snr_db, air_prec prec, double* stats_dev, void* llr_dev) {
  if (ctx && (!tx_dev || !stats_dev)) return fail(ctx, AIR_E_INVAL, "tx_dev and stats_dev must not be null");
  try {
    return run(ctx, c, Y_dev, tx_dev, N, &snr_db, 1, 0, prec, stats_dev, llr_dev, false, true);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_sweep_maxlog(air_ctx* ctx, const air_const* c, const uint32_t* tx_dev, const void* Z_dev,
                            int64_t N, const double* snr_db_host, int S, air_prec prec, double* stats_dev,
                            void* llr_dev) {
  if (ctx && (!tx_dev || !stats_dev)) return fail(ctx, AIR_E_INVAL, "tx_dev and stats_dev must not be null");
  try {
    return run(ctx, c, Z_dev, tx_dev, N, snr_db_host, S, 1, prec, stats_dev, llr_dev, false, true);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_noise_var(air_ctx* ctx, const air_const* c, const void* Y_dev, const uint32_t* tx_dev,
                         int64_t N, air_prec prec, double* var_dev) {
  try {
    return run_noise_var(ctx, c, Y_dev, tx_dev, N, prec, var_dev);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_sweep(air_ctx* ctx, const air_const* c, const uint32_t* tx_dev, const void* Z_dev,
                     int64_t N, const double* snr_db_host, int S, air_prec prec, double* stats_dev,
                     void* llr_dev) {
  if (ctx && (!tx_dev || !stats_dev)) return fail(ctx, AIR_E_INVAL, "tx_dev and stats_dev must not be null");
  try {
    return run(ctx, c, Z_dev, tx_dev, N, snr_db_host, S, 1, prec, stats_dev, llr_dev);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_hard_decide(air_ctx* ctx, const air_const* c, const float* Y_dev, const uint32_t* tx_dev,
                           int64_t N, uint32_t* decided_dev, uint64_t* counts_dev) {
  try {
    return run_hd(ctx, c, Y_dev, tx_dev, N, nullptr, 1, 0, decided_dev, counts_dev);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

air_status air_hard_sweep(air_ctx* ctx, const air_const* c, const uint32_t* tx_dev, const float* Z_dev,
                          int64_t N, const double* snr_db_host, int S, uint64_t* counts_dev,
                          uint32_t* decided_dev) {
  if (ctx && (!tx_dev || !counts_dev || !snr_db_host))
    return fail(ctx, AIR_E_INVAL, "tx_dev, counts_dev and snr_db_host must not be null");
  try {
    return run_hd(ctx, c, Z_dev, tx_dev, N, snr_db_host, S, 1, decided_dev, counts_dev);
  } catch (...) {
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
}

// erfc^-1 by Newton steps on g(x) = ln erfc(x) - ln v, which is concave and
// decreasing: after the first step every iterate lies right of the root and
// they decrease monotonically onto it (quadratically near it).
double air_q_factor_db(double ber) {
  if (!(ber > 0.0 && ber < 0.5)) return std::nan("");
  const double lv = std::log(2.0 * ber);
  double x = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double e = std::erfc(x);
    const double g = std::log(e) - lv;
    const double dg = -1.1283791670955126 * std::exp(-x * x) / e;
    const double step = g / dg;
    x -= step;
    if (std::fabs(step) <= 1e-15 * std::fabs(x)) break;
  }
  return 20.0 * std::log10(std::sqrt(2.0) * x);
}

int64_t air_last_exact(air_ctx* ctx) {
  if (!ctx) return -1;
  DeviceGuard g(ctx->device);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return -1;
  CallWords w;
  if (hipMemcpy(&w, ctx->call, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return (int64_t)w.exact;
}

int64_t air_last_recomputed(air_ctx* ctx) {
  if (!ctx) return -1;
  DeviceGuard g(ctx->device);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return -1;
  CallWords w;
  if (hipMemcpy(&w, ctx->call, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return (int64_t)w.recomputed;
}

air_status air_set_timing(air_ctx* ctx, int enable) {
  if (!ctx) return AIR_E_INVAL;
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  return AIR_OK;
}

air_status air_kernel_time(air_ctx* ctx, double* total_ms, int64_t* launches) {
  if (!ctx) return AIR_E_INVAL;
  if (!total_ms || !launches) return fail(ctx, AIR_E_INVAL, "null output pointer");
  DeviceGuard g(ctx->device);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronize");
  double t = 0.0;
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]);
    if (e != hipSuccess) return hip_fail(ctx, e, "event elapsed time");
    t += ms;
  }
  *total_ms = t;
  *launches = (int64_t)(ctx->ev_used / 2);
  ctx->ev_used = 0;
  return AIR_OK;
}

}  // extern "C"
