// hd_kernels.h -- hard decisions: the constellation point nearest to each
// received point, and symbol / bit error counts against the transmitted
// points (the paper's receiver demaps hard decisions and reports the BER,
// Section II and III).
//
// One sample per lane. The constellation is walked in label order in
// unrolled groups of G points whose FP32 coordinates are uniform across the
// wave (scalar loads). The distance is accumulated over the dimensions with
// fused multiply-adds, acc = fma(y_d - x_d, y_d - x_d, acc) from 0, all in
// FP32, and a strictly smaller distance replaces the best point, so ties go
// to the lower label. The SNR loop is outermost; error counts are exact
// integers (per-lane counters, a wave sum, then one atomic add per block and
// SNR point: integer sums do not depend on their order).
#pragma once
#include "device_common.h"

namespace air {

struct HdArgs {
  const float* in;            // N x D received points, or unit noise (sweep)
  const uint32_t* tx;         // N transmitted indices (X rows), or nullptr
  const float* xl;            // M x D coordinates in label order
  const uint32_t* lab;        // label of X row j
  const uint32_t* pos;        // X row of label l
  uint32_t* decided;          // [S][N] decided X rows, or nullptr
  unsigned long long* counts; // [S][2]: symbol errors, bit errors (zeroed by the host)
  int* err;                   // set when a transmitted index >= M is seen
  int64_t N;
  int M, S, sweep;
  float sigma[kMaxSnrPerLaunch];
};

template <int D, int G>
__global__ __launch_bounds__(kBlock) void hd_kernel(const HdArgs a) {
  __shared__ unsigned long long part[kBlock / 64][2];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int M = a.M;
  const int NG = M / G;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const float* __restrict__ xl = a.xl;
  for (int s = 0; s < a.S; ++s) {
    unsigned int se = 0, be = 0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.N; n += stride) {
      int tl = -1;
      const uint32_t t = a.tx ? a.tx[n] : 0u;
      if (a.tx) {
        if (t >= (uint32_t)M) {
          if (s == 0) atomicOr(a.err, 1);
          tl = -2;
        } else {
          tl = (int)a.lab[t];
        }
      }
      float y[D];
      const float* __restrict__ in = a.in + n * D;
      if (a.sweep) {
        const int lt = tl >= 0 ? tl : 0;
#pragma unroll
        for (int d = 0; d < D; ++d) y[d] = __builtin_fmaf(a.sigma[s], in[d], xl[lt * D + d]);
      } else {
#pragma unroll
        for (int d = 0; d < D; ++d) y[d] = in[d];
      }
      int best = 0;
      float bd = __builtin_inff();
      for (int g = 0; g < NG; ++g) {
        const float* __restrict__ xg = xl + (int64_t)g * (G * D);
#pragma unroll
        for (int i = 0; i < G; ++i) {
          float acc = 0.0f;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const float df = y[d] - xg[i * D + d];
            acc = __builtin_fmaf(df, df, acc);
          }
          const bool better = acc < bd;
          bd = better ? acc : bd;
          best = better ? g * G + i : best;
        }
      }
      if (a.decided) a.decided[(int64_t)s * a.N + n] = a.pos[best];
      if (tl >= 0 && best != tl) {
        se += 1;
        be += (unsigned int)__builtin_popcount((unsigned)(best ^ tl));
      }
    }
    const double ws = wave_sum((double)se), wb = wave_sum((double)be);
    if (lane == 0) {
      part[wave][0] = (unsigned long long)ws;
      part[wave][1] = (unsigned long long)wb;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      unsigned long long t = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w][threadIdx.x];
      if (a.counts && t) atomicAdd(a.counts + 2 * s + threadIdx.x, t);
    }
    __syncthreads();
  }
}

template <int D>
hipError_t launch_hd_d(const HdArgs& a, int grid, hipStream_t st) {
  switch (a.M >= 16 ? 16 : a.M) {
    case 2: hipLaunchKernelGGL((hd_kernel<D, 2>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 4: hipLaunchKernelGGL((hd_kernel<D, 4>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 8: hipLaunchKernelGGL((hd_kernel<D, 8>), dim3(grid), dim3(kBlock), 0, st, a); break;
    default: hipLaunchKernelGGL((hd_kernel<D, 16>), dim3(grid), dim3(kBlock), 0, st, a); break;
  }
  return hipGetLastError();
}

}  // namespace air
