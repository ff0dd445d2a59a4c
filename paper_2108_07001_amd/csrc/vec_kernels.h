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
//
// FP32 (exact form) runs in two tiers like the matrix-core path: an item with
// a starved entry is not finished in the first tier's sums but listed
// (tier2_list.h), and demap_vec_t2 re-forms it with every term in an FP64
// frame, 2^(a + K64) = ldexp(exp2(frac a), floor a + K64), which widens the
// window from ~150 to ~1300 nats of |LLR|; only what still starves there
// takes the exact path. FP64 needs no second tier (its fixed shift already
// spans ~1000 log2 units) and finishes starved items on the exact path.
#pragma once
#include "device_common.h"
#include "tier2_list.h"

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
  // FP32 exact form: starved items go to the second tier (demap_vec_t2)
  constexpr bool T2 = !ML && sizeof(T) == 4;
  extern __shared__ double acc_lds[];  // [waves][S][4], then (T2) flagged counts [waves][S]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int waves = blockDim.x >> 6;
  const int S = a.S;
  unsigned int* nflag_lds = reinterpret_cast<unsigned int*>(acc_lds + waves * S * 4);
  for (int i = threadIdx.x; i < waves * S * 4; i += blockDim.x) acc_lds[i] = 0.0;
  if (T2)
    for (int i = threadIdx.x; i < waves * S; i += blockDim.x) nflag_lds[i] = 0u;
  __syncthreads();
  const int64_t wstride = (int64_t)gridDim.x * waves;   // waves of the launch
  const int64_t wgid = (int64_t)blockIdx.x * waves + wave;

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
      bool need2 = false;            // T2: a starved entry, finished by the second tier
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
        } else if constexpr (T2) {
          // every sum is finite and >= 0 for finite inputs, so the smallest
          // decides; without LLRs (a uniform choice per call) only the total
          // and the transmitted point's sides count (the other sides enter
          // nothing but the total; lanes without a transmitted label are not
          // live then)
          T smin = total;
          if (llr) {
#pragma unroll
            for (int i = 0; i < 2 * kMaxBits; ++i)
              if (i < 2 * m) smin = __builtin_fminf(smin, side[i]);
          } else {
#pragma unroll
            for (int k = 0; k < kMaxBits; ++k)
              if (k < m) smin = __builtin_fminf(smin, ((tl >> k) & 1) ? side[2 * k + 1] : side[2 * k]);
          }
          need2 = !(smin >= Real<T>::starve(m));
          if (!need2) {
            T arg_t = 0;
            if (tl >= 0) arg_t = Real<T>::fma(-c, sqdist<T, D>(y, xl + (int64_t)tl * D), K);
            T u = 0, v = 0;
            finish_fast<T>(m, tl, total, side, arg_t, lout, u, v);
            if (tl >= 0) {
              su = (double)u;
              sv = (double)v;
            }
          }
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
      if constexpr (T2) {
        // the wave's 64 samples are the 32-sample tiles 2 q and 2 q + 1
        // (q = first sample / 64); both entries are written, empty masks too,
        // so every slot of this (SNR point, wave) run holds this call's entry
        const unsigned long long bm = __ballot(need2);
        if (lane == 0) {
          const int64_t tile = (r * stride + (int64_t)blockIdx.x * blockDim.x + wave * 64) >> 5;
          unsigned long long* slot = a.t2_list + ((int64_t)s * wstride + wgid) * a.t2_tpw + 2 * r;
          slot[0] = ((bm & 0xffffffffull) << 32) | (unsigned long long)(uint32_t)tile;
          slot[1] = (bm & 0xffffffff00000000ull) | (unsigned long long)(uint32_t)(tile + 1);
          nflag_lds[wave * S + s] += (unsigned int)__builtin_popcountll(bm);
        }
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
  // (T2: the second tier counts the items it finishes)
  const double wslow = wave_sum((double)slow_items);
  if (lane == 0 && wslow > 0.0) {
    atomicAdd(a.recomputed, (unsigned long long)wslow);
    atomicAdd(a.exact, (unsigned long long)wslow);
  }
  if (T2)
    for (int s = lane; s < S; s += 64) a.t2_nitem[(int64_t)s * wstride + wgid] = nflag_lds[wave * S + s];
  __syncthreads();
  for (int i = threadIdx.x; i < S * 4; i += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < waves; ++w) t += acc_lds[w * S * 4 + i];
    a.partials[(int64_t)i * gridDim.x + blockIdx.x] = t;
  }
}

// Second tier of the FP32 vector kernel. The first tier's flagged samples,
// gathered per SNR point (t2_collect) and numbered as one sequence of
// 64-sample tiles (each point's run padded to a multiple of 64, so that a
// tile lies within one SNR point), are dealt out to the waves round-robin,
// one sample per lane: every wave gets a share of every SNR point, and the
// high ones cost far more per sample. Each sample is re-formed in the first
// tier's group structure with every term in the FP64 frame 2^(a + K64),
// K64 = 1022 - m, built exactly from one FP32 exp2 of the fractional part and
// an ldexp by the integer part (the arguments are the first tier's FP32
// values); entries still below the frame's starvation bound take the exact
// path. Each wave sums its samples per SNR point (non-decreasing along its
// share), and the block reduces its waves in a fixed order.
template <int D, int G>
__global__ __launch_bounds__(kBlock) void demap_vec_t2(const DemapArgs a, const float* __restrict__ xl) {
  constexpr int LG = Log2G<G>::v;
  constexpr int NL = kMaxBits - LG;
  extern __shared__ double acc_lds[];  // [waves][S][4]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int waves = blockDim.x >> 6;
  const int S = a.S;
  // the SNR runs in the tile sequence: lane s holds run s's padded start and
  // its sample count
  const unsigned int tot_l = lane < S ? a.t2_tot[lane] : 0u;
  uint64_t pstart_l = 0, run = 0;
  for (int s = 0; s < S; ++s) {
    if (lane == s) pstart_l = run;
    run += (__builtin_amdgcn_readlane(tot_l, s) + 63u) & ~63u;
  }
  const int64_t T = (int64_t)(run >> 6);
  if ((int64_t)blockIdx.x * waves >= T) {
    // no tile reaches this block
    for (int i = threadIdx.x; i < S * 4; i += blockDim.x) a.t2_partials[(int64_t)i * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const int M = a.M, m = a.m;
  const int NG = M / G;
  const int ngb = m - LG;
  const float K = Real<float>::shift(m);
  const int K64 = 1022 - m;
  const int dK = K64 - (int)K;
  const double thr64 = __builtin_ldexp(1.0, m - 1022 + 60);
  // 2^(x - K + K64) for a first-tier argument x = a_j + K (log2 units); K is
  // an integer, so the fraction and the floor of x serve for those of a_j
  auto val64 = [&](float x) -> double {
    const float fr = __builtin_amdgcn_fractf(x);    // x - floor(x), in [0, 1)
    const int ni = (int)__builtin_floorf(x);
    return __builtin_ldexp((double)Real<float>::exp2(fr), ni + dK);
  };
  float* __restrict__ llr = static_cast<float*>(a.llr);
  const int64_t wstride = (int64_t)gridDim.x * waves;
  const int64_t wgid = (int64_t)blockIdx.x * waves + wave;
  const int64_t nmine = T > wgid ? (T - wgid + wstride - 1) / wstride : 0;
  double* wacc = acc_lds + (int64_t)wave * S * 4;
  for (int i = lane; i < S * 4; i += 64) wacc[i] = 0.0;
  int s_cur = -1;
  double au = 0.0, av = 0.0, auu = 0.0, avv = 0.0;
  auto flush = [&]() {
    const double w0 = wave_sum(au), w1 = wave_sum(av);
    const double w2 = wave_sum(auu), w3 = wave_sum(avv);
    if (lane == 0) {
      wacc[s_cur * 4 + 0] = w0;
      wacc[s_cur * 4 + 1] = w1;
      wacc[s_cur * 4 + 2] = w2;
      wacc[s_cur * 4 + 3] = w3;
    }
    au = av = auu = avv = 0.0;
  };
  unsigned long long items = 0;         // flagged samples this wave finishes
  unsigned long long exact = 0;         // of those, the ones that needed the exact path
  const unsigned long long smask = S < 64 ? ((1ull << S) - 1ull) : ~0ull;
  for (int64_t r = 0; r < nmine; ++r) {
    const int64_t q = wgid + r * wstride;
    const uint64_t p0 = (uint64_t)q * 64u;
    // the run holding this tile: the last non-empty s whose padded start is <= p0
    const unsigned long long in_run = __ballot(lane < S && pstart_l <= p0 && tot_l > 0u) & smask;
    const int s = 63 - __builtin_clzll(in_run);
    if (s != s_cur) {
      if (s_cur >= 0) flush();
      s_cur = s;
    }
    const uint64_t start = ((uint64_t)__builtin_amdgcn_readlane((unsigned)(pstart_l >> 32), s) << 32) |
                           (uint64_t)__builtin_amdgcn_readlane((unsigned)pstart_l, s);
    const unsigned int cnt = __builtin_amdgcn_readlane(tot_l, s);
    const uint64_t pos = p0 + (uint64_t)lane;
    const bool has = pos - start < (uint64_t)cnt;
    items += (unsigned long long)__builtin_popcountll(__ballot(has));
    bool ex_lane = false;
    if (has) {
      const int64_t n = (int64_t)a.t2_items[(int64_t)s * a.t2_cap + (int64_t)(pos - start)];
      // flagged samples are live: a transmitted index, if any, is in range
      const int tl = a.tx ? (int)a.lab[a.tx[n]] : -1;
      const float c = a.snr.cf[s];
      float y[D];
      load_point<float, D>(a, n, tl, a.snr.sigmaf[s], y);

      double R[G];
      double hi0[NL], hi1[NL], node[NL];
#pragma unroll
      for (int l = 0; l < NL; ++l) { hi0[l] = 0.0; hi1[l] = 0.0; node[l] = 0.0; }
      double total = 0.0;
      for (int g = 0; g < NG; ++g) {
        const float* __restrict__ xg = xl + (int64_t)g * (G * D);
        double e[G];
#pragma unroll
        for (int i = 0; i < G; ++i) e[i] = val64(__builtin_fmaf(-c, sqdist<float, D>(y, xg + i * D), K));
        if (g == 0) {
#pragma unroll
          for (int i = 0; i < G; ++i) R[i] = e[i];
        } else {
#pragma unroll
          for (int i = 0; i < G; ++i) R[i] += e[i];
        }
        double carry = tree_sum<double, G>(e);
        bool placed = false;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          if (!placed && l < ngb) {
            if ((g >> l) & 1) {
              hi0[l] += node[l];
              hi1[l] += carry;
              carry = node[l] + carry;
            } else {
              node[l] = carry;
              placed = true;
            }
          }
        }
        if (!placed) total = carry;
      }
      double side[2 * kMaxBits];
#pragma unroll
      for (int i = 0; i < 2 * kMaxBits; ++i) side[i] = 0.0;
#pragma unroll
      for (int k = 0; k < LG; ++k) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 0; i < G; ++i) {
          if ((i >> k) & 1) s1 += R[i];
          else s0 += R[i];
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
      // log2 of the transmitted point's own term as it entered the sums
      const double lt_t =
          tl >= 0 ? log2_wide(val64(__builtin_fmaf(-c, sqdist<float, D>(y, xl + (int64_t)tl * D), K))) : 0.0;
      double smin = total;
#pragma unroll
      for (int i = 0; i < 2 * kMaxBits; ++i)
        if (i < 2 * m) smin = __builtin_fmin(smin, side[i]);
      float* lout = llr ? llr + (int64_t)s * a.llr_stride_s + n * m : nullptr;
      float u = 0.f, v = 0.f;
      if (smin >= thr64) {
        const double lt = log2_wide(total);
        double vacc = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxBits; ++k) {
          if (k < m) {
            const double l0 = log2_wide(side[2 * k]), l1 = log2_wide(side[2 * k + 1]);
            if (lout) lout[k] = (float)(0.6931471805599453094 * (l0 - l1));
            vacc += lt - (((tl >> k) & 1) ? l1 : l0);
          }
        }
        u = (float)(lt - lt_t);
        v = (float)vacc;
      } else {
        ExactArgs<float> ex = exact_args<float>(a, s);
        finish_item_frame64<D>(ex, n, tl, total, side, thr64, K64, lt_t, lout, u, v);
        ex_lane = true;
      }
      if (tl >= 0) {
        const double du = (double)u, dv = (double)v;
        au += du;
        av += dv;
        auu = __builtin_fma(du, du, auu);
        avv = __builtin_fma(dv, dv, avv);
      }
    }
    exact += (unsigned long long)__builtin_popcountll(__ballot(ex_lane));
  }
  if (s_cur >= 0) flush();
  // one count per wave: same-address atomics from every item would serialise
  if (lane == 0 && items) atomicAdd(a.recomputed, items);
  if (lane == 0 && exact) atomicAdd(a.exact, exact);
  __syncthreads();
  for (int i = threadIdx.x; i < S * 4; i += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < waves; ++w) t += acc_lds[w * S * 4 + i];
    a.t2_partials[(int64_t)i * gridDim.x + blockIdx.x] = t;
  }
}

// part 0: the first tier (exact or, with ml, max-log); part 1 (FP32 exact
// form only): the gather of the first tier's lists and the second tier. The
// events of `l` time part 0's kernel only.
template <typename T, int D, int G>
hipError_t launch_vec_one(const DemapArgs& a, int grid, const Launch& l, bool ml, int part) {
  const uint32_t acc = (uint32_t)(sizeof(double) * (kBlock / 64) * a.S * 4);
  if (part == 1) {
    if (!a.t2_items || !a.t2_tot || !a.t2_partials) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
      launch_t2_collect(a, grid, l.stream);
      hipLaunchKernelGGL((demap_vec_t2<D, G>), dim3(t2_grid(grid)), dim3(kBlock), acc, l.stream, a,
                         static_cast<const float*>(a.xl));
    }
    return hipGetLastError();
  }
  // the FP32 exact form lists its starved items: no launch without the lists
  if (!ml && sizeof(T) == 4 && (!a.t2_list || !a.t2_nitem || a.t2_tpw < 1)) return hipErrorInvalidValue;
  if (ml)
    launch_kernel(l, demap_vec<T, D, G, true>, dim3(grid), dim3(kBlock), acc, a, static_cast<const T*>(a.xl));
  else
    launch_kernel(l, demap_vec<T, D, G, false>, dim3(grid), dim3(kBlock),
                  acc + (sizeof(T) == 4 ? (uint32_t)(sizeof(unsigned int) * (kBlock / 64) * a.S) : 0u), a,
                  static_cast<const T*>(a.xl));
  return hipGetLastError();
}

// ml: the max-log form.
template <typename T, int D>
hipError_t launch_vec_td(const DemapArgs& a, int grid, const Launch& l, bool ml, int part) {
  switch (a.M >= 16 ? 16 : a.M) {
    case 2: return launch_vec_one<T, D, 2>(a, grid, l, ml, part);
    case 4: return launch_vec_one<T, D, 4>(a, grid, l, ml, part);
    case 8: return launch_vec_one<T, D, 8>(a, grid, l, ml, part);
    default: return launch_vec_one<T, D, 16>(a, grid, l, ml, part);
  }
}

}  // namespace air
