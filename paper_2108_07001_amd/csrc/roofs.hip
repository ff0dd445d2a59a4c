// roofs.hip -- microbenchmarks of the rates that bound the demapping path on
// this device (air_measure_roofs): the transcendental pipe (v_exp_f32 alone,
// and exp2 / log2 alternating), FP32 FMA, whether transcendentals issue
// alongside FMAs, the half-precision and bfloat16 matrix cores, and a plain
// device copy through HBM.
//
// Every kernel runs a fixed number of independent dependency chains per lane
// (enough to cover each unit's latency) over many waves, and is timed with
// HIP events after one untimed warm-up launch; a rate is the number of
// results (or flops, or bytes) the launch produced over its time.
#include "../../include/air.h"
#include "host_state.h"

#include <hip/hip_runtime.h>

namespace air {
namespace {

constexpr int kChains = 8;           // independent chains per lane
constexpr int kRoofBlocks = 256 * 8; // 8 blocks of 256 threads per CU
constexpr int kRoofIters = 1024;

// v_exp_f32 only: x <- 2^(-x) stays in [0.5, 1] (the negation is an operand
// modifier, not an instruction).
__global__ __launch_bounds__(256) void roof_exp(float* out, float seed) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * (float)(threadIdx.x + c);
  for (int i = 0; i < kRoofIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// exp2 and log2 in turn: x <- log2(2^x) stays at x.
__global__ __launch_bounds__(256) void roof_explog(float* out, float seed) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * (float)(threadIdx.x + c);
  for (int i = 0; i < kRoofIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(x[c]);
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_logf(x[c]);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// K FP32 FMA chains per exp chain (K = 0: FMAs only are not this kernel; see
// roof_fma). y <- y * a + b stays bounded for |a| < 1.
template <int K>
__global__ __launch_bounds__(256) void roof_exp_fma(float* out, float seed, float a, float b) {
  float x[kChains], y[kChains * K];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = seed + 0.01f * (float)(threadIdx.x + c);
#pragma unroll
  for (int c = 0; c < kChains * K; ++c) y[c] = seed + 0.02f * (float)(threadIdx.x + c);
  for (int i = 0; i < kRoofIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      x[c] = __builtin_amdgcn_exp2f(-x[c]);
#pragma unroll
      for (int k = 0; k < K; ++k) y[c * K + k] = __builtin_fmaf(y[c * K + k], a, b);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
#pragma unroll
  for (int c = 0; c < kChains * K; ++c) s += y[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// FP32 FMA only (non-packed: the library is built without packed FP32).
__global__ __launch_bounds__(256) void roof_fma(float* out, float seed, float a, float b) {
  float y[2 * kChains];
#pragma unroll
  for (int c = 0; c < 2 * kChains; ++c) y[c] = seed + 0.02f * (float)(threadIdx.x + c);
  for (int i = 0; i < kRoofIters; ++i) {
#pragma unroll
    for (int c = 0; c < 2 * kChains; ++c) y[c] = __builtin_fmaf(y[c], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 2 * kChains; ++c) s += y[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef _Float16 rh8 __attribute__((ext_vector_type(8)));
typedef __bf16 rb8 __attribute__((ext_vector_type(8)));
typedef float rf16 __attribute__((ext_vector_type(16)));

// 32x32x16 matrix-core products, four independent accumulator chains per wave.
template <bool BF>
__global__ __launch_bounds__(256) void roof_mfma(float* out, float seed) {
  rf16 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
  const float v = seed * (float)(threadIdx.x & 7) * 1e-3f;
  if constexpr (BF) {
    rb8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (__bf16)(v + (float)e * 1e-3f);
      b[e] = (__bf16)(v - (float)e * 1e-3f);
    }
    for (int i = 0; i < kRoofIters; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    }
  } else {
    rh8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (_Float16)(v + (float)e * 1e-3f);
      b[e] = (_Float16)(v - (float)e * 1e-3f);
    }
    for (int i = 0; i < kRoofIters; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[c][e];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Plain copy, 16 bytes per thread and step, grid-stride.
__global__ __launch_bounds__(256) void roof_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                 int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Seconds of one launch of `f` (the second of two launches; the first warms up).
template <typename F>
hipError_t time_launch(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F f, double& sec) {
  f();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipEventRecord(e0, st);
  if (e != hipSuccess) return e;
  f();
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  sec = (double)ms * 1e-3;
  return e;
}

}  // namespace
}  // namespace air

using namespace air;

extern "C" air_status air_measure_roofs(air_ctx* ctx, air_roofs* out) {
  if (!ctx || !out) return AIR_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
  const hipStream_t st = ctx->stream;
  const int64_t threads = (int64_t)kRoofBlocks * 256;
  const int64_t copy_elems = (int64_t)1 << 26;          // 1 GiB of float4
  float* sink = nullptr;
  float4* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&sink, sizeof(float) * threads);
  if (e == hipSuccess) e = hipMalloc(&buf, sizeof(float4) * 2 * copy_elems);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(buf, 0, sizeof(float4) * 2 * copy_elems, st);
  const dim3 grid(kRoofBlocks), block(256);
  const double lanes = (double)threads;
  double sec = 0.0;
  if (e == hipSuccess)
    e = time_launch(st, e0, e1, [&] { hipLaunchKernelGGL(roof_exp, grid, block, 0, st, sink, 0.5f); }, sec);
  if (e == hipSuccess) out->exp_per_s = lanes * kChains * kRoofIters / sec;
  if (e == hipSuccess)
    e = time_launch(st, e0, e1, [&] { hipLaunchKernelGGL(roof_explog, grid, block, 0, st, sink, 0.5f); }, sec);
  if (e == hipSuccess) out->explog_per_s = lanes * kChains * 2 * kRoofIters / sec;
  if (e == hipSuccess)
    e = time_launch(st, e0, e1, [&] { hipLaunchKernelGGL(roof_fma, grid, block, 0, st, sink, 0.5f, 0.999f, 1e-3f); },
                    sec);
  if (e == hipSuccess) out->fma_per_s = lanes * 2 * kChains * kRoofIters / sec;
  // exp + K FMAs per chain step: seconds per exp-chain step against the sum of
  // the two units' separate times for the same work
  double t1 = 0.0, t2 = 0.0, t4 = 0.0;
  if (e == hipSuccess)
    e = time_launch(st, e0, e1,
                    [&] { hipLaunchKernelGGL(roof_exp_fma<1>, grid, block, 0, st, sink, 0.5f, 0.999f, 1e-3f); }, t1);
  if (e == hipSuccess)
    e = time_launch(st, e0, e1,
                    [&] { hipLaunchKernelGGL(roof_exp_fma<2>, grid, block, 0, st, sink, 0.5f, 0.999f, 1e-3f); }, t2);
  if (e == hipSuccess)
    e = time_launch(st, e0, e1,
                    [&] { hipLaunchKernelGGL(roof_exp_fma<4>, grid, block, 0, st, sink, 0.5f, 0.999f, 1e-3f); }, t4);
  if (e == hipSuccess) {
    const double n_exp = lanes * kChains * kRoofIters;
    const double t_exp = n_exp / out->exp_per_s, t_fma = n_exp / out->fma_per_s;
    out->exp_fma_ratio[0] = t1 / (t_exp + 1.0 * t_fma);
    out->exp_fma_ratio[1] = t2 / (t_exp + 2.0 * t_fma);
    out->exp_fma_ratio[2] = t4 / (t_exp + 4.0 * t_fma);
  }
  const double mfma_flops = 2.0 * 32 * 32 * 16 * 4 * kRoofIters * (double)(kRoofBlocks * 4);
  if (e == hipSuccess)
    e = time_launch(st, e0, e1, [&] { hipLaunchKernelGGL(roof_mfma<false>, grid, block, 0, st, sink, 0.5f); }, sec);
  if (e == hipSuccess) out->mfma_f16_flops = mfma_flops / sec;
  if (e == hipSuccess)
    e = time_launch(st, e0, e1, [&] { hipLaunchKernelGGL(roof_mfma<true>, grid, block, 0, st, sink, 0.5f); }, sec);
  if (e == hipSuccess) out->mfma_bf16_flops = mfma_flops / sec;
  if (e == hipSuccess)
    e = time_launch(st, e0, e1,
                    [&] { hipLaunchKernelGGL(roof_copy, dim3(256 * 16), block, 0, st, buf, buf + copy_elems, copy_elems); },
                    sec);
  if (e == hipSuccess) out->copy_bytes_per_s = 2.0 * sizeof(float4) * (double)copy_elems / sec;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(ctx, e, "roof microbenchmarks");
  return AIR_OK;
}
