// aux_kernels.h -- noise variance estimate with known transmitted points,
// for a receiver that models the channel as Gaussian with an estimated
// variance (auxiliary channel). The paper measures a real link, where the
// receiver does not know the noise statistics, and lists the normalised GMI
// among its acronyms; the estimate is the maximum-likelihood one with known
// means: s_d^2 = (1/N) sum_n (y_nd - x_{t_n},d)^2 per real dimension, and
// their mean as the isotropic estimate.
//
// One sample per lane, FP64 squares of the residuals (the received value
// widened to FP64 minus the FP64 coordinate), per-lane sums, a wave sum,
// per-wave values added in wave order, one partial per block and dimension,
// then noise_var_finish adds the block partials in a fixed order: the result
// does not depend on timing. HBM-bound: N D sizeof(T) + 4 N bytes read.
#pragma once
#include "device_common.h"

namespace air {

template <typename T>
__global__ __launch_bounds__(kBlock) void noise_var_kernel(const T* __restrict__ y,
                                                           const uint32_t* __restrict__ tx,
                                                           const uint32_t* __restrict__ lab,
                                                           const double* __restrict__ xl, int64_t N,
                                                           int M, int D, double* __restrict__ partials,
                                                           int* err) {
  __shared__ double wsum[kBlock / 64][kMaxD];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  double acc[kMaxD];
#pragma unroll
  for (int d = 0; d < kMaxD; ++d) acc[d] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
    const uint32_t t = tx[n];
    if (t >= (uint32_t)M) {
      atomicOr(err, 1);
      continue;
    }
    const double* __restrict__ x = xl + (int64_t)lab[t] * D;
    const T* __restrict__ yn = y + n * D;
#pragma unroll
    for (int d = 0; d < kMaxD; ++d)
      if (d < D) {
        const double e = (double)yn[d] - x[d];
        acc[d] = __builtin_fma(e, e, acc[d]);
      }
  }
#pragma unroll
  for (int d = 0; d < kMaxD; ++d)
    if (d < D) {
      const double w = wave_sum(acc[d]);
      if (lane == 0) wsum[wave][d] = w;
    }
  __syncthreads();
  if (threadIdx.x < D) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += wsum[w][threadIdx.x];
    partials[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

// One wave: dimension d's block partials (lane l takes blocks l, l + 64, ...,
// then a fixed butterfly); var[d] = sum / N, var[D] = the mean of the D
// values. NaN everywhere if a transmitted index was out of range; the error
// is folded into the sticky word. Lane 0 zeroes the next call's words.
__global__ __launch_bounds__(64) void noise_var_finish(const double* __restrict__ partials, int nblocks,
                                                       int D, int64_t N, double* __restrict__ var,
                                                       const int* err, CallWords* next, int* sticky) {
  const int lane = threadIdx.x;
  const bool bad = *err != 0;
  double all = 0.0;
  for (int d = 0; d < D; ++d) {
    double t = 0.0;
    for (int b = lane; b < nblocks; b += 64) t += partials[(int64_t)d * nblocks + b];
    t = wave_sum(t) / (double)N;
    all += t;
    if (lane == 0) var[d] = bad ? __builtin_nan("") : t;
  }
  if (lane == 0) {
    var[D] = bad ? __builtin_nan("") : all / (double)D;
    if (bad) atomicOr(sticky, 1);
    clear_call_words(next);
  }
}

}  // namespace air
