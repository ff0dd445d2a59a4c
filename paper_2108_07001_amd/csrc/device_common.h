// device_common.h -- launch arguments and device helpers shared by the demapping kernels.
//
// Metric convention on the device: for a received point y, SNR s and
// constellation point x_j (label order), the log2-likelihood up to a
// sample constant is a_j = -c_s |y - x_j|^2 with c_s = 1 / (2 sigma_s^2 ln 2)
// (sigma_s^2 = Es / (D 10^(snr_db/10)) per real dimension). The kernels
// exponentiate arg_j = a_j + K with the fixed shift K = Emax - 1 - m of the
// working type (126 - m for FP32, 1022 - m for FP64): a_j <= 0, so no term
// and no sum of M terms can overflow, and no per-sample maximum pass is
// needed. A bit side (or the total) whose sum falls below
// starve(m) = 2^(m + Emin + guard) is "starved": terms flushed below the
// normal range could then matter, and that entry is recomputed exactly with
// its own maximum as shift (slow_rel). guard = 20 bits for FP32 (the flushed
// mass is then < 2^-20 of the side), 60 for FP64.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exact_rule.h"

namespace air {

constexpr int kMaxSnrPerLaunch = 64;
constexpr int kMaxBits = 12;        // M <= 4096
constexpr int kMaxD = 16;
constexpr int kBlock = 256;         // threads per block of the vector kernels
constexpr int kMaxGrid = 1536;      // upper bound on blocks of one demapping launch

// Where a demapping kernel is launched: the stream and, for a timed launch,
// two events that take the kernel's own start and end times from its
// dispatch (no marker commands between the kernels). Both null: untimed.
struct Launch {
  hipStream_t stream;
  hipEvent_t start;
  hipEvent_t stop;
};

template <typename F, typename... Args>
inline void launch_kernel(const Launch& l, F kernel, dim3 grid, dim3 block, uint32_t shmem, Args... args) {
  if (l.start || l.stop)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, l.stream, l.start, l.stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, l.stream, args...);
}

// Per-call device words: the tx-range error of a call and the number of items
// sent through the exact path; zero when the call starts.
struct CallWords {
  int err;
  int pad;
  unsigned long long recomputed;   // items finished outside the first tier's sums
  unsigned long long exact;        // of those, items that needed the exact path
};

// Zeroes the words of the next call (one thread).
__device__ inline void clear_call_words(CallWords* next) {
  if (next) {
    next->err = 0;
    next->pad = 0;
    next->recomputed = 0ull;
    next->exact = 0ull;
  }
}

// Per-SNR scalars of one launch, passed by value in the kernel arguments.
struct SnrTable {
  double sigma[kMaxSnrPerLaunch];   // noise standard deviation per real dimension
  double c[kMaxSnrPerLaunch];       // 1 / (2 sigma^2 ln 2)
  float sigmaf[kMaxSnrPerLaunch];
  float cf[kMaxSnrPerLaunch];
};

// Arguments of every demapping kernel.
struct DemapArgs {
  const void* in;                   // Y (N x D) or, in sweep mode, unit noise Z (N x D)
  const uint32_t* tx;               // N transmitted indices into X, or nullptr
  void* llr;                        // [S][N][m] LLRs (nats) or nullptr
  double* partials;                 // [S][4][gridDim.x]: sum u, sum v, sum u^2, sum v^2
  int* err;                         // set to 1 when a tx index >= M is seen
  unsigned long long* recomputed;   // (sample, SNR) items finished outside the fast sums
  unsigned long long* exact;        // of those, items that needed the exact path
  const void* xl;                   // M x D coordinates in label order (float or double)
  const uint32_t* lab;              // label of original point index j
  int64_t N;
  int64_t llr_stride_s;             // elements between consecutive SNR planes of llr
  int M, m, D, S;
  int sweep;                        // 1: y = x_t + sigma_s z from `in`
  // second tier (matrix-core forms and the FP32 vector kernel)
  unsigned long long* t2_list;      // [S][waves][tpw]: sample tile (32 bits) | lane mask (32)
  double* t2_partials;              // [S][4][gridDim.x], as partials, from the second tier
  int t2_tpw;                       // list slots per (SNR point, wave)
  unsigned int* t2_nitem;           // [S][waves]: samples flagged in each wave's list
  // the flagged samples gathered per SNR point: point s's samples, in (wave,
  // slot, lane) order, from entry s * t2_cap of t2_items
  uint32_t* t2_items;               // sample indices
  int64_t t2_cap;                   // entries of t2_items per SNR point (waves x tpw x 32)
  unsigned int* t2_tot;             // [S]: samples flagged at each SNR point
  SnrTable snr;
};

template <typename T> struct Real;

template <> struct Real<float> {
  static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ __forceinline__ float log2(float x) { return __builtin_amdgcn_logf(x); }
  static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
  static __device__ __forceinline__ float shift(int m) { return 126.0f - (float)m; }
  static __device__ __forceinline__ float starve(int m) { return __builtin_ldexpf(1.0f, m - 126 + 20); }
  static __device__ __forceinline__ float ln2() { return 0.693147180559945309f; }
  static __device__ __forceinline__ float nan() { return __builtin_nanf(""); }
  static __device__ __forceinline__ float inf() { return __builtin_inff(); }
  static __device__ __forceinline__ float sigma(const SnrTable& t, int s) { return t.sigmaf[s]; }
  static __device__ __forceinline__ float c(const SnrTable& t, int s) { return t.cf[s]; }
};

template <> struct Real<double> {
  static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
  static __device__ __forceinline__ double log2(double x) { return ::log2(x); }
  static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
  static __device__ __forceinline__ double shift(int m) { return 1022.0 - (double)m; }
  static __device__ __forceinline__ double starve(int m) { return __builtin_ldexp(1.0, m - 1022 + 60); }
  static __device__ __forceinline__ double ln2() { return 0.6931471805599453094; }
  static __device__ __forceinline__ double nan() { return __builtin_nan(""); }
  static __device__ __forceinline__ double inf() { return __builtin_inf(); }
  static __device__ __forceinline__ double sigma(const SnrTable& t, int s) { return t.sigma[s]; }
  static __device__ __forceinline__ double c(const SnrTable& t, int s) { return t.c[s]; }
};

// Received point of sample n at SNR s: read from Y, or x_t + sigma z (sweep).
template <typename T, int D>
__device__ __forceinline__ void load_point(const DemapArgs& a, int64_t n, int tl, T sigma, T (&y)[D]) {
  const T* in = static_cast<const T*>(a.in) + n * D;
  if (a.sweep) {
    const T* xt = static_cast<const T*>(a.xl) + (int64_t)tl * D;
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = Real<T>::fma(sigma, in[d], xt[d]);
  } else {
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = in[d];
  }
}

template <typename T, int D>
__device__ __forceinline__ T sqdist(const T (&y)[D], const T* __restrict__ x) {
  T d2 = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    T df = y[d] - x[d];
    d2 = Real<T>::fma(df, df, d2);
  }
  return d2;
}

// ---- exact recomputation (rare path) -------------------------------------
// Used for items whose fast-path sums fall below the starvation bound. All
// metrics are taken relative to a reference point r (the nearest point), and
// the difference a_j - a_r = -c (|y-x_j|^2 - |y-x_r|^2) is formed as
// -c sum_d (x_r - x_j)_d (2 y - x_r - x_j)_d, which keeps its relative
// accuracy even when y is far from every point (|a_j| huge, difference not).
// Out of line and reloading the received point, so that the fast path's
// registers stay untouched.

template <typename T, int D>
__device__ __forceinline__ void reload_point(const T* __restrict__ in, int sweep,
                                             const T* __restrict__ xl, T sigma, int64_t n, int tl,
                                             T (&y)[D]) {
  const T* p = in + n * D;
  if (sweep) {
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = Real<T>::fma(sigma, p[d], xl[(int64_t)tl * D + d]);
  } else {
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = p[d];
  }
}

template <typename T, int D>
__device__ __forceinline__ T rel_metric(const T (&y)[D], const T* __restrict__ xr,
                                        const T* __restrict__ xj, T c) {
  T acc = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) acc = Real<T>::fma(xr[d] - xj[d], (y[d] - xr[d]) + (y[d] - xj[d]), acc);
  return -c * acc;
}

// Index (label order) of the point nearest to the received point; ties to the lowest.
template <typename T, int D>
__device__ __noinline__ int slow_nearest(const T* __restrict__ in, int sweep, const T* __restrict__ xl,
                                         int M, T sigma, int64_t n, int tl) {
  T y[D];
  reload_point<T, D>(in, sweep, xl, sigma, n, tl, y);
  int best = 0;
  T bd = sqdist<T, D>(y, xl);
#pragma unroll 4
  for (int j = 1; j < M; ++j) {
    T d2 = sqdist<T, D>(y, xl + (int64_t)j * D);
    if (d2 < bd) { bd = d2; best = j; }
  }
  return best;
}

// log2 sum_{j in selection} 2^(a_j - a_r): bit side (k, b), all points (k = -1);
// or a_t - a_r itself (k = -2).
template <typename T, int D>
__device__ __noinline__ T slow_rel(const T* __restrict__ in, int sweep, const T* __restrict__ xl,
                                   int M, T sigma, T c, int64_t n, int tl, int r, int k, int b) {
  T y[D];
  reload_point<T, D>(in, sweep, xl, sigma, n, tl, y);
  const T* xr = xl + (int64_t)r * D;
  if (k == -2) return rel_metric<T, D>(y, xr, xl + (int64_t)tl * D, c);
  // the selection's labels: all of them, or those with bit k equal to b
  // (index i with b inserted at bit k)
  const int cnt = k >= 0 ? M >> 1 : M;
  const int lowmask = k >= 0 ? (1 << k) - 1 : 0;
  auto label = [&](int i) { return k >= 0 ? (((i & ~lowmask) << 1) | (b << k) | (i & lowmask)) : i; };
  T dmax = -__builtin_huge_val();
#pragma unroll 4
  for (int i = 0; i < cnt; ++i) {
    T dj = rel_metric<T, D>(y, xr, xl + (int64_t)label(i) * D, c);
    dmax = dj > dmax ? dj : dmax;
  }
  T sum = 0;
#pragma unroll 4
  for (int i = 0; i < cnt; ++i)
    sum += Real<T>::exp2(rel_metric<T, D>(y, xr, xl + (int64_t)label(i) * D, c) - dmax);
  return dmax + Real<T>::log2(sum);
}

// What the exact path needs of one call: where the sample's point comes from
// and the constellation, with the SNR's scalars in the working type.
template <typename T>
struct ExactArgs {
  const T* in;                      // received points, or unit noise in sweep mode
  int sweep;
  const T* xl;                      // label-ordered coordinates
  int M, m;
  T sigma, c;
  unsigned long long* recomputed;   // count of items that took the exact path
};

template <typename T>
__device__ __forceinline__ ExactArgs<T> exact_args(const DemapArgs& a, int s) {
  return ExactArgs<T>{static_cast<const T*>(a.in), a.sweep, static_cast<const T*>(a.xl), a.M, a.m,
                      Real<T>::sigma(a.snr, s), Real<T>::c(a.snr, s), a.recomputed};
}

// Outputs of one (sample, SNR) item whose fast-path sums are all above the
// starvation bound: the m LLRs (if llr_out) and u, v (when tl >= 0).
//  total:   sum_j 2^arg_j;  side[2k+b]: the same over bit side (k, b).
//  arg_t:   arg of the transmitted point.
template <typename T>
__device__ __forceinline__ void finish_fast(int m, int tl, T total, const T (&side)[2 * kMaxBits], T arg_t,
                                            T* llr_out, T& u, T& v) {
  const T lam_tot = Real<T>::log2(total);
  T acc = 0;
#pragma unroll
  for (int k = 0; k < kMaxBits; ++k) {
    if (k < m) {
      const T l0 = Real<T>::log2(side[2 * k]), l1 = Real<T>::log2(side[2 * k + 1]);
      if (llr_out) llr_out[k] = Real<T>::ln2() * (l0 - l1);
      acc += lam_tot - (((tl >> k) & 1) ? l1 : l0);
    }
  }
  if (tl >= 0) {
    // log2 of the very term that entered the sum (not arg_t itself): u >= 0
    // then holds exactly, whatever the rounding of exp2 and log2.
    u = lam_tot - Real<T>::log2(Real<T>::exp2(arg_t));
    v = acc;
  }
}

// Outputs of one (sample, SNR) item from its fast-path sums, as finish_fast,
// with the entries below the starvation bound recomputed exactly; the return
// value says whether that happened (the caller counts such items).
template <typename T, int D>
__device__ __forceinline__ bool finish_item(const ExactArgs<T>& a, int64_t n, int tl,
                                            T total, const T (&side)[2 * kMaxBits], T arg_t,
                                            T* llr_out, T& u, T& v) {
  const int m = a.m;
  const T thr = Real<T>::starve(m);
  T lam[2 * kMaxBits];
  T lam_tot;
  bool slow = !(total >= thr);
  lam_tot = Real<T>::log2(total);
#pragma unroll
  for (int i = 0; i < 2 * kMaxBits; ++i) {
    if (i < 2 * m) {
      slow |= !(side[i] >= thr);
      lam[i] = Real<T>::log2(side[i]);
    }
  }
  bool total_slow = false;
  T delta_t = 0;
  if (slow) {
    // Starved entries are recomputed relative to the nearest point r. If the
    // total itself is starved, every entry is recomputed and all stay
    // relative to a_r (a side need not be below the total bit for bit: the
    // two are summed in different orders); otherwise the recomputed sides are
    // put back in the fast path's units by adding K + a_r, which is then small.
    const T* in = a.in;
    const T* xl = a.xl;
    const T sigma = a.sigma, c = a.c;
    const int r = slow_nearest<T, D>(in, a.sweep, xl, a.M, sigma, n, tl);
    total_slow = !(total >= thr);
    T base = 0;
    if (total_slow) {
      lam_tot = slow_rel<T, D>(in, a.sweep, xl, a.M, sigma, c, n, tl, r, -1, 0);
      if (tl >= 0) delta_t = slow_rel<T, D>(in, a.sweep, xl, a.M, sigma, c, n, tl, r, -2, 0);
    } else {
      T y[D];
      reload_point<T, D>(in, a.sweep, xl, sigma, n, tl, y);
      base = Real<T>::shift(m) - c * sqdist<T, D>(y, xl + (int64_t)r * D);
    }
    const uint32_t redo = exact_entries<T>(total, side, m, thr);
#pragma unroll
    for (int i = 0; i < 2 * kMaxBits; ++i)
      if (i < 2 * m && ((redo >> i) & 1u))
        lam[i] = base + slow_rel<T, D>(in, a.sweep, xl, a.M, sigma, c, n, tl, r, i >> 1, i & 1);
  }
  if (llr_out) {
#pragma unroll
    for (int k = 0; k < kMaxBits; ++k)
      if (k < m) llr_out[k] = Real<T>::ln2() * (lam[2 * k] - lam[2 * k + 1]);
  }
  if (tl >= 0) {
    // log2 of the very term that entered the sum (not arg_t itself): u >= 0
    // then holds exactly, whatever the rounding of exp2 and log2.
    u = total_slow ? lam_tot - delta_t : lam_tot - Real<T>::log2(Real<T>::exp2(arg_t));
    T acc = 0;
#pragma unroll
    for (int k = 0; k < kMaxBits; ++k)
      if (k < m) acc += lam_tot - (((tl >> k) & 1) ? lam[2 * k + 1] : lam[2 * k]);
    v = acc;
  }
  return slow;
}

// floor(x) as an integer in one instruction (v_cvt_flr_i32_f32; the compiler
// forms it from a floor and a conversion). For finite x within the int range.
// `after` is a value the compiler formed from x (the fraction of x): the
// instruction is held behind it, so when x is a matrix-core result the
// compiler's own wait states before that reader cover this one too (it does
// not place them before inline assembly).
__device__ __forceinline__ int floor_i32(float x, float after) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x), "v"(after));
  return r;
}

// log2 of a positive double through its binary exponent and an FP32 log2 of
// the mantissa: absolute error ~2e-7, far inside every tolerance on the
// quantities it feeds (differences of such logs), at a fraction of the cost
// of the FP64 library routine.
__device__ __forceinline__ double log2_wide(double x) {
  int e;
  const double mant = __builtin_frexp(x, &e);   // in [0.5, 1)
  return (double)e + (double)__builtin_amdgcn_logf((float)mant);
}

// Outputs of one FP32-family item from sums in the FP64 frame 2^(a + K64)
// (the matrix-core path's second tier). Entries below thr64 are recomputed
// exactly relative to the nearest point r and put back in the frame by
// adding K64 + a_r; if the total itself is below thr64 every entry is
// recomputed and all stay relative to a_r. lt_t is log2 of the transmitted
// point's own term in the frame (used when tl >= 0 and the total is not
// recomputed). Only the starved entries cost a pass over the constellation.
// The caller counts the item (it is one of the second tier's items).
template <int D>
__device__ __forceinline__ void finish_item_frame64(const ExactArgs<float>& a, int64_t n, int tl,
                                                    double total, const double (&side)[2 * kMaxBits],
                                                    double thr64, int K64, double lt_t,
                                                    float* llr_out, float& u, float& v) {
  const int m = a.m;
  const float* in = a.in;
  const float* xl = a.xl;
  const float sigma = a.sigma, c = a.c;
  const int r = slow_nearest<float, D>(in, a.sweep, xl, a.M, sigma, n, tl);
  const bool total_slow = !(total >= thr64);
  double lam[2 * kMaxBits];
  double lam_tot, base = 0.0, delta_t = 0.0;
  if (total_slow) {
    lam_tot = (double)slow_rel<float, D>(in, a.sweep, xl, a.M, sigma, c, n, tl, r, -1, 0);
    if (tl >= 0) delta_t = (double)slow_rel<float, D>(in, a.sweep, xl, a.M, sigma, c, n, tl, r, -2, 0);
  } else {
    float y[D];
    reload_point<float, D>(in, a.sweep, xl, sigma, n, tl, y);
    base = (double)K64 - (double)c * (double)sqdist<float, D>(y, xl + (int64_t)r * D);
    lam_tot = log2_wide(total);
  }
  const uint32_t redo = exact_entries<double>(total, side, m, thr64);
#pragma unroll
  for (int i = 0; i < 2 * kMaxBits; ++i) {
    if (i < 2 * m) {
      if ((redo >> i) & 1u)
        lam[i] = base + (double)slow_rel<float, D>(in, a.sweep, xl, a.M, sigma, c, n, tl, r, i >> 1, i & 1);
      else
        lam[i] = log2_wide(side[i]);
    }
  }
  if (llr_out) {
#pragma unroll
    for (int k = 0; k < kMaxBits; ++k)
      if (k < m) llr_out[k] = (float)(0.6931471805599453094 * (lam[2 * k] - lam[2 * k + 1]));
  }
  if (tl >= 0) {
    u = (float)(total_slow ? lam_tot - delta_t : lam_tot - lt_t);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxBits; ++k)
      if (k < m) acc += lam_tot - (((tl >> k) & 1) ? lam[2 * k + 1] : lam[2 * k]);
    v = (float)acc;
  }
}

// Sum of a double over the 64 lanes of a wave (every lane gets the result).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

}  // namespace air
