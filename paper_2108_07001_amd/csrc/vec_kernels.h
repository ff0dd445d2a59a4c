// vec_kernels.h -- vector-ALU demapping kernels (AIR_FP32 and AIR_FP64).
//
// One received sample per lane. The constellation is walked in label order
// in groups of G points (G = min(M, 16), compile time), so that the label
// bits below log2 G are the position i inside a group and the bits above are
// the group index g (uniform across the wave, so its coordinates come in
// through scalar loads). Per point: D direct differences, one FMA for the
// shifted exponent, one exp2. The 2m bit-side sums and the total are formed
// without per-point side bookkeeping:
//  * R[i] accumulates the terms at group position i over all groups; the low
//    label bits' sides are folded out of R once per sample;
//  * each group's total enters a binary-counter tree over the group index,
//    which hands the totals of the two children of every completed node to
//    the two sides of that level's label bit.
// Every sum over a sample's points is then formed once, in a fixed order.
//
// ML: the max-log form with the same structure, maxima of the exponents in
// place of sums of the terms; LLR = ln 2 (max side 0 - max side 1), the GMI
// term is the BMD rate of those LLRs taken as exact; no sum can starve, so
// the exact path is never needed.
#pragma once
#include "device_common.h"

namespace air {

template <int G> struct Log2G;
template <> struct Log2G<2> { static constexpr int v = 1; };
template <> struct Log2G<4> { static constexpr int v = 2; };
template <> struct Log2G<8> { static constexpr int v = 3; };
template <> struct Log2G<16> { static constexpr int v = 4; };

template <typename T, int N>
__device__ __forceinline__ T tree_sum(const T (&e)[N]) {
  // pairwise sum of e[0..N) (N a power of two)
  T buf[N];
#pragma unroll
  for (int i = 0; i < N; ++i) buf[i] = e[i];
#pragma unroll
  for (int w = N / 2; w >= 1; w >>= 1) {
#pragma unroll
    for (int i = 0; i < w; ++i) buf[i] = buf[2 * i] + buf[2 * i + 1];
  }
  return buf[0];
}

template <bool ML, typename T>
__device__ __forceinline__ T vcmb(T x, T y) {
  if constexpr (ML) return x > y ? x : y;
  else return x + y;
}

template <bool ML, typename T, int N>
__device__ __forceinline__ T tree_cmb(const T (&e)[N]) {
  if constexpr (!ML) {
    return tree_sum<T, N>(e);
  } else {
    T buf[N];
#pragma unroll
    for (int i = 0; i < N; ++i) buf[i] = e[i];
#pragma unroll
    for (int w = N / 2; w >= 1; w >>= 1) {
#pragma unroll
      for (int i = 0; i < w; ++i) buf[i] = vcmb<true>(buf[2 * i], buf[2 * i + 1]);
    }
    return buf[0];
  }
}

template <typename T, int D, int G, bool ML = false>
__global__ __launch_bounds__(kBlock) void demap_vec(const DemapArgs a, const T* __restrict__ xl) {
  constexpr int LG = Log2G<G>::v;
  constexpr int NL = kMaxBits - LG;
  extern __shared__ double acc_lds[];  // [waves][S][4]
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const int S = a.S;
  for (int i = threadIdx.x; i < waves * S * 4; i += blockDim.x) acc_lds[i] = 0.0;
  __syncthreads();

  const int M = a.M, m = a.m;
  const int NG = M / G;
  const int ngb = m - LG;
  const T K = Real<T>::shift(m);
  T* __restrict__ llr = static_cast<T*>(a.llr);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t rounds = (a.N + stride - 1) / stride;
  unsigned int slow_items = 0;   // items this lane sent through the exact path

  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t n = r * stride + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = n < a.N;
    int tl = -1;  // label of the transmitted point; -2 marks an invalid index
    if (valid && a.tx) {
      const uint32_t t = a.tx[n];
      if (t >= (uint32_t)M) {
        atomicOr(a.err, 1);
        tl = -2;
      } else {
        tl = (int)a.lab[t];
      }
    }
    for (int s = 0; s < S; ++s) {
      double su = 0.0, sv = 0.0;
      T* lout = (llr && valid) ? llr + (int64_t)s * a.llr_stride_s + n * m : nullptr;
      if (valid && tl != -2) {
        const T c = Real<T>::c(a.snr, s);
        T y[D];
        load_point<T, D>(a, n, tl, Real<T>::sigma(a.snr, s), y);

        const T z0 = ML ? -Real<T>::inf() : T(0);
        T R[G];
        T hi0[NL], hi1[NL], node[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) { hi0[l] = z0; hi1[l] = z0; node[l] = z0; }
        T total = z0;
        for (int g = 0; g < NG; ++g) {
          const T* __restrict__ xg = xl + (int64_t)g * (G * D);
          T e[G];
#pragma unroll
          for (int i = 0; i < G; ++i) {
            const T ai = Real<T>::fma(-c, sqdist<T, D>(y, xg + i * D), K);
            e[i] = ML ? ai : Real<T>::exp2(ai);
          }
          if (g == 0) {
#pragma unroll
            for (int i = 0; i < G; ++i) R[i] = e[i];
          } else {
#pragma unroll
            for (int i = 0; i < G; ++i) R[i] = vcmb<ML>(R[i], e[i]);
          }
          T carry = tree_cmb<ML, T, G>(e);
          bool placed = false;
#pragma unroll
          for (int l = 0; l < NL; ++l) {
            if (!placed && l < ngb) {
              if ((g >> l) & 1) {
                hi0[l] = vcmb<ML>(hi0[l], node[l]);
                hi1[l] = vcmb<ML>(hi1[l], carry);
                carry = vcmb<ML>(node[l], carry);
              } else {
                node[l] = carry;
                placed = true;
              }
            }
          }
          if (!placed) total = carry;  // the last group closes every level
        }

        T side[2 * kMaxBits];
#pragma unroll
        for (int i = 0; i < 2 * kMaxBits; ++i) side[i] = 0;
#pragma unroll
        for (int k = 0; k < LG; ++k) {
          T s0 = z0, s1 = z0;
#pragma unroll
          for (int i = 0; i < G; ++i) {
            if ((i >> k) & 1) s1 = vcmb<ML>(s1, R[i]);
            else s0 = vcmb<ML>(s0, R[i]);
          }
          side[2 * k] = s0;
          side[2 * k + 1] = s1;
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          if (l < ngb) {
            side[2 * (LG + l)] = hi0[l];
            side[2 * (LG + l) + 1] = hi1[l];
          }
        }
        if constexpr (ML) {
          (void)total;
          T v = 0;
#pragma unroll
          for (int k = 0; k < kMaxBits; ++k)
            if (k < m) {
              const T lam = side[2 * k] - side[2 * k + 1];
              if (lout) lout[k] = Real<T>::ln2() * lam;
              if (tl >= 0) {
                const T x = ((tl >> k) & 1) ? lam : -lam;      // log2(1 + 2^x)
                const T ax = x < T(0) ? -x : x;
                v += (x > T(0) ? x : T(0)) + Real<T>::log2(T(1) + Real<T>::exp2(-ax));
              }
            }
          if (tl >= 0) sv = (double)v;
        } else {
          T arg_t = 0;
          if (tl >= 0) arg_t = Real<T>::fma(-c, sqdist<T, D>(y, xl + (int64_t)tl * D), K);
          T u = 0, v = 0;
          slow_items += finish_item<T, D>(exact_args<T>(a, s), n, tl, total, side, arg_t, lout, u, v) ? 1u : 0u;
          if (tl >= 0) {
            su = (double)u;
            sv = (double)v;
          }
        }
      } else if (lout) {
        for (int k = 0; k < m; ++k) lout[k] = Real<T>::nan();
      }
      const double w0 = wave_sum(su), w1 = wave_sum(sv);
      const double w2 = wave_sum(su * su), w3 = wave_sum(sv * sv);
      if (lane == 0) {
        double* acc = acc_lds + ((int64_t)wave * S + s) * 4;
        acc[0] += w0;
        acc[1] += w1;
        acc[2] += w2;
        acc[3] += w3;
      }
    }
  }
  // one count per wave: same-address atomics from every item would serialise
  const double wslow = wave_sum((double)slow_items);
  if (lane == 0 && wslow > 0.0) {
    atomicAdd(a.recomputed, (unsigned long long)wslow);
    atomicAdd(a.exact, (unsigned long long)wslow);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S * 4; i += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < waves; ++w) t += acc_lds[w * S * 4 + i];
    a.partials[(int64_t)i * gridDim.x + blockIdx.x] = t;
  }
}

template <typename T, int D, int G>
hipError_t launch_vec_one(const DemapArgs& a, int grid, const Launch& l, bool ml) {
  const uint32_t shmem = (uint32_t)(sizeof(double) * (kBlock / 64) * a.S * 4);
  if (ml)
    launch_kernel(l, demap_vec<T, D, G, true>, dim3(grid), dim3(kBlock), shmem, a, static_cast<const T*>(a.xl));
  else
    launch_kernel(l, demap_vec<T, D, G, false>, dim3(grid), dim3(kBlock), shmem, a, static_cast<const T*>(a.xl));
  return hipGetLastError();
}

// ml: the max-log form.
template <typename T, int D>
hipError_t launch_vec_td(const DemapArgs& a, int grid, const Launch& l, bool ml) {
  switch (a.M >= 16 ? 16 : a.M) {
    case 2: return launch_vec_one<T, D, 2>(a, grid, l, ml);
    case 4: return launch_vec_one<T, D, 4>(a, grid, l, ml);
    case 8: return launch_vec_one<T, D, 8>(a, grid, l, ml);
    default: return launch_vec_one<T, D, 16>(a, grid, l, ml);
  }
}

}  // namespace air
