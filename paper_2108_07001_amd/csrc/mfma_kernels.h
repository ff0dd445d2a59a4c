// mfma_kernels.h -- matrix-core demapping (AIR_FP16X3, AIR_BF16X3): the
// exponent-tile arithmetic, the per-tile bodies of both tiers, the second-tier
// kernel and its list gathering. The first-tier kernel of the sweep and
// air_mi_gmi calls is in mfma_wide.h; the serving kernels in serve_kernels.h.
//
// The exponent tile arg[i][j] = a_j(x_i) + shift of 32 constellation points
// (rows i) by 32 received samples (columns j) is one chain of
// v_mfma_f32_32x32x16_{f16,bf16} products in the expanded form
//
//   a = (2c y).x_i - c |x_i|^2 - c |y|^2,
//
// with FP32 accumulation. The factors of the two products are split into
// parts of the operand type (round to nearest even at every step):
//  - half precision (11 significant bits): hi + lo, three of the four cross
//    products kept (hi*hi + hi*lo + lo*hi), a relative error of about 2^-22
//    per term; feature order along K
//      [w_hi.x_hi (D) | w_hi.x_lo (D) | w_lo.x_hi (D) | nc_hi q_hi, nc_hi q_lo, nc_lo q_hi | S.1 | 0...]
//  - bfloat16 (8 significant bits): hi + mid + lo, the six cross products of
//    order up to two kept (hi*hi, hi*mid, hi*lo, mid*hi, mid*mid, lo*hi; the
//    dropped ones are below 2^-26 of the term), feature order
//      [w_hi.x_hi | w_hi.x_mid | w_hi.x_lo | w_mid.x_hi | w_mid.x_mid | w_lo.x_hi (D each) |
//       nc_hi q_hi, nc_hi q_mid, nc_hi q_lo, nc_mid q_hi, nc_mid q_mid, nc_lo q_hi | S.1 | 0...]
// with w = 2 c y, nc = -c, q = |x|^2; the point side of every K slot is a
// precomputed record (16 bytes per lane-half per 16 K slots), the sample side
// is formed in registers once per (sample, SNR). Either form is then limited
// by the FP32 accumulation of the products, about 2^-24 of c (|y|^2 + |x|^2)
// per addition. The per-sample constant
// (K - c|y|^2 here, fed as the accumulator input; a rounded copy S in the
// last slot in the first tier) carries no information: every output is a
// difference of logarithms of the same sample's terms.
//
// Layout of the 32x32 accumulator (measured on gfx950): lane l holds column
// j = l % 32 (one sample) and rows r = 8 (e / 4) + 4 (l / 32) + e % 4 for its
// 16 elements e. A 32-point tile holds the points whose labels are
// 32 t + r, so label bits {0,1,3,4} are the element bits of e, bit 2 is the
// lane half, and bits >= 5 are the tile index t. The bit-side sums are then
// formed as in the vector kernels: R[e] accumulates over tiles, a
// binary-counter tree over t feeds the high bits, and the two lane halves of
// a sample exchange their partial sums once per (sample tile, SNR).
//
// The transmitted point's own term is taken from a second product whose A
// rows are the 32 samples' transmitted points (the diagonal of that tile),
// so u = log2 S - log2 e_t uses bit-for-bit the term that entered S.
//
// Two tiers. The first sums the FP32 terms 2^arg with the fixed shift K
// (window of ~150 nats of |LLR|). An item with a starved entry is left out of
// its sums and its tile is listed in the wave's own slots; the lists are
// gathered into one launch-wide list, and the second-tier kernel re-forms
// those tiles' sums in an FP64 frame, each term split as
// 2^frac(a) * 2^floor(a) (one exp2 in [1, 2), one ldexp), which widens the
// window to ~1300 nats. What is still starved there takes the exact per-item
// path. Both kernels write per-block partial sums in a fixed order, so every
// result is independent of timing.
#pragma once
#include "device_common.h"
#include "tier2_list.h"

namespace air {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));

constexpr int kTileLevels = kMaxBits - 5;   // label bits carried by the point-tile index

// K slots of a point record, padded to whole 16-slot chunks (q = |x|^2).
// Slot for slot (one product per chunk, the sample side pairing each slot):
//  half precision: [x_hi | x_lo | x_hi | q_hi, q_lo, q_hi | 1];
//  bfloat16: [x_hi | x_mid | x_lo | x_hi | x_mid | x_hi |
//    q_hi, q_mid, q_lo, q_hi, q_mid, q_hi | 1].
// Shared chunks (each point part once):
//  half precision: [x_hi | q_hi, q_lo | 1 | x_lo];
//  bfloat16: [x_hi | q_hi, q_mid, q_lo | 1 | x_mid | x_lo];
//  each chunk is taken by up to L + 1 products (L = 1 half, 2 bfloat16), one
//  per split level l of the sample side, which pairs l with the chunk's point
//  parts of level p <= L - l.
// Both keep the same cross products (half: hi·hi, hi·lo, lo·hi; bfloat16:
// hi·hi, hi·mid, mid·hi, hi·lo, lo·hi, mid·mid; the shift's 1 pairs with the
// hi level only). Sharing makes the records smaller, which matters where the
// run-time-M kernels stream them from L2; it is used where it saves a chunk
// without costing a product (half precision, 10 <= D <= 15) or saves several
// (bfloat16, D > 4: at D <= 4 the extra product per chunk costs more than
// the smaller records save).
__host__ __device__ constexpr bool shared_chunks(int D, bool bf) { return bf ? D > 4 : D >= 10 && D <= 15; }
__host__ __device__ constexpr int split_levels(bool bf) { return bf ? 2 : 1; }   // L
__host__ __device__ constexpr int record_slots(int D, bool bf) {
  return shared_chunks(D, bf) ? (bf ? 3 * D + 4 : 2 * D + 3) : (bf ? 6 * D + 7 : 3 * D + 4);
}
__host__ __device__ constexpr int shift_slot(int D, bool bf) {
  return shared_chunks(D, bf) ? D + split_levels(bf) + 1 : record_slots(D, bf) - 1;
}
__host__ __device__ constexpr int mfma_nk(int D, bool bf = false) { return (record_slots(D, bf) + 15) / 16; }

// Split level of the point part in slot s of a shared-chunk record (0 hi,
// then mid, lo; the shift's 1 counts as the lowest level L), L + 1 for
// padding (pairs with nothing).
__host__ __device__ constexpr int shared_slot_level(int D, bool bf, int s) {
  const int L = split_levels(bf);
  return s < D ? 0
       : s < D + L + 1 ? s - D
       : s == D + L + 1 ? L
       : s < record_slots(D, bf) ? (bf && s < 2 * D + 4 ? 1 : L)
       : L + 1;
}

// Products of the K chain: one per chunk, except with shared chunks, where a
// chunk takes as many as the sample levels its highest point part pairs with
// (chunk by chunk, levels in increasing order).
template <int D, bool BF>
struct KPlan {
  static constexpr int NK = mfma_nk(D, BF);      // record chunks
  static constexpr int L = split_levels(BF);
  static constexpr int levels(int c) {
    if (!shared_chunks(D, BF)) return 1;
    int lo = L + 1;
    for (int s = 16 * c; s < 16 * c + 16; ++s)
      lo = shared_slot_level(D, BF, s) < lo ? shared_slot_level(D, BF, s) : lo;
    return L + 1 - lo;
  }
  static constexpr int count() {
    int n = 0;
    for (int c = 0; c < NK; ++c) n += levels(c);
    return n;
  }
  static constexpr int NP = count();             // products
  static constexpr int chunk(int p) {
    for (int c = 0; c < NK; ++c) {
      if (p < levels(c)) return c;
      p -= levels(c);
    }
    return 0;
  }
  static constexpr int level(int p) {
    for (int c = 0; c < NK; ++c) {
      if (p < levels(c)) return p;
      p -= levels(c);
    }
    return 0;
  }
};
static_assert(KPlan<12, false>::NK == 2 && KPlan<12, false>::NP == 3, "half-precision 12-D plan");
static_assert(KPlan<8, true>::NK == 2 && KPlan<8, true>::NP == 5, "bfloat16 8-D plan");
static_assert(KPlan<4, true>::NK == 2 && KPlan<4, true>::NP == 2, "bfloat16 4-D plan");
static_assert(KPlan<8, false>::NK == 2 && KPlan<8, false>::NP == 2, "half-precision 8-D plan");

template <bool BF> struct MfmaOp;
template <> struct MfmaOp<false> {
  typedef half8_t vec;
  typedef _Float16 elem;
  static __device__ __forceinline__ float16_t mma(vec a, vec b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaOp<true> {
  typedef bf16x8_t vec;
  typedef __bf16 elem;
  static __device__ __forceinline__ float16_t mma(vec a, vec b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// hi + lo split of an FP32 value in half precision (round to nearest even).
__device__ __forceinline__ void split2(float v, _Float16& hi, _Float16& lo) {
  hi = (_Float16)v;
  lo = (_Float16)(v - (float)hi);
}

// hi + mid + lo split of two FP32 values in bfloat16 (round to nearest even,
// two values per conversion). Each remainder v - hi, (v - hi) - mid is exact
// in FP32: a value minus its rounding to fewer significant bits.
__device__ __forceinline__ void split3_bf16(float v0, float v1, __bf16 (&hi)[2], __bf16 (&mid)[2],
                                            __bf16 (&lo)[2]) {
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 v = {v0, v1};
  const b2 h = __builtin_convertvector(v, b2);
  const f2 r1 = v - __builtin_convertvector(h, f2);
  const b2 md = __builtin_convertvector(r1, b2);
  const f2 r2 = r1 - __builtin_convertvector(md, f2);
  const b2 l = __builtin_convertvector(r2, b2);
  hi[0] = h.x;
  hi[1] = h.y;
  mid[0] = md.x;
  mid[1] = md.y;
  lo[0] = l.x;
  lo[1] = l.y;
}

// Sample-side operand words of both K halves for the products of the K
// chain, from w = 2 c y, nc = -c and the value S of the shift slot (0 when
// the accumulator carries the shift), in the order of the point records:
// emit(p, q, word of half 0, word of half 1) for product p and packed word q
// (0..3) of the half. Returns false when a value leaves the half-precision
// range (bfloat16 has the FP32 range).
template <int D, bool BF, class Emit>
__device__ __forceinline__ bool sample_words(const float (&w)[D], float nc, float S, Emit&& emit) {
  typedef typename MfmaOp<BF>::elem E;
  typedef KPlan<D, BF> P;
  constexpr int L = P::L;
  auto word = [](E a0, E a1) {
    E pr[2] = {a0, a1};
    uint32_t v;
    __builtin_memcpy(&v, pr, 4);
    return v;
  };
  // the split parts of every w_d and of nc: wl[level][d], nl[level]
  // (half precision: hi, lo, two dimensions at a time with the packed RNE
  // conversion; bfloat16: hi, mid, lo)
  E wl[L + 1][D], nl[L + 1];
  bool ok = true;
  if constexpr (BF) {
#pragma unroll
    for (int d = 0; d < D; d += 2) {
      const int d1 = d + 1 < D ? d + 1 : d;
      __bf16 hi[2], mid[2], lo[2];
      split3_bf16(w[d], d + 1 < D ? w[d1] : 0.0f, hi, mid, lo);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        if (d + i < D) {
          wl[0][d + i] = hi[i];
          wl[1][d + i] = mid[i];
          wl[L][d + i] = lo[i];
        }
    }
    __bf16 hi[2], mid[2], lo[2];
    split3_bf16(nc, 0.0f, hi, mid, lo);
    nl[0] = hi[0];
    nl[1] = mid[0];
    nl[L] = lo[0];
  } else {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    ok = __builtin_fabsf(nc) < 60000.0f;
#pragma unroll
    for (int d = 0; d < D; d += 2) {
      const float w0 = w[d];
      const float w1 = d + 1 < D ? w[d + 1 < D ? d + 1 : d] : 0.0f;
      ok &= __builtin_fmaxf(__builtin_fabsf(w0), __builtin_fabsf(w1)) < 60000.0f;
      const f2 wv = {w0, w1};
      const h2 hi = __builtin_convertvector(wv, h2);
      const h2 lo = __builtin_convertvector(wv - __builtin_convertvector(hi, f2), h2);
      wl[0][d] = hi.x;
      wl[L][d] = lo.x;
      if (d + 1 < D) {
        wl[0][d + 1] = hi.y;
        wl[L][d + 1] = lo.y;
      }
    }
    split2(nc, nl[0], nl[L]);
  }
  const E sb = (E)S;
  if constexpr (shared_chunks(D, BF)) {
    // the sample value that slot s pairs with at level l (0 if none)
    auto val = [&](int s, int l) -> E {
      if (shared_slot_level(D, BF, s) + l > L) return (E)0.0f;
      if (s < D) return wl[l][s];
      if (s < D + L + 1) return nl[l];
      if (s == D + L + 1) return sb;
      if (BF && s < 2 * D + 4) return wl[l][s - D - 4];
      return wl[l][s - (BF ? 2 * D + 4 : D + 3)];
    };
#pragma unroll
    for (int p = 0; p < P::NP; ++p) {
      const int c0 = 16 * P::chunk(p), l = P::level(p);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        emit(p, q, word(val(c0 + 2 * q, l), val(c0 + 2 * q + 1, l)), word(val(c0 + 8 + 2 * q, l), val(c0 + 9 + 2 * q, l)));
    }
  } else {
    // slot for slot: the features in record order, then each lane's half of
    // every chunk
    E F[16 * P::NK];
#pragma unroll
    for (int k = 0; k < 16 * P::NK; ++k) F[k] = (E)0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if constexpr (BF) {
        F[d] = wl[0][d];
        F[D + d] = wl[0][d];
        F[2 * D + d] = wl[0][d];
        F[3 * D + d] = wl[1][d];
        F[4 * D + d] = wl[1][d];
        F[5 * D + d] = wl[2][d];
      } else {
        F[d] = wl[0][d];
        F[D + d] = wl[0][d];
        F[2 * D + d] = wl[1][d];
      }
    }
    if constexpr (BF) {
      F[6 * D] = nl[0];
      F[6 * D + 1] = nl[0];
      F[6 * D + 2] = nl[0];
      F[6 * D + 3] = nl[1];
      F[6 * D + 4] = nl[1];
      F[6 * D + 5] = nl[2];
    } else {
      F[3 * D] = nl[0];
      F[3 * D + 1] = nl[0];
      F[3 * D + 2] = nl[1];
    }
    F[shift_slot(D, BF)] = sb;
#pragma unroll
    for (int kk = 0; kk < P::NK; ++kk)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        emit(kk, q, word(F[16 * kk + 2 * q], F[16 * kk + 2 * q + 1]), word(F[16 * kk + 8 + 2 * q], F[16 * kk + 9 + 2 * q]));
  }
  return ok;
}

// Sample-side operands of this lane's K half (h), selected on packed 32-bit
// words so that the choice never becomes an index.
template <int D, bool BF>
__device__ __forceinline__ bool sample_operands(const float (&w)[D], float nc, float S, int h,
                                                typename MfmaOp<BF>::vec (&B)[KPlan<D, BF>::NP]) {
  const uint32_t hmask = 0u - (uint32_t)h;
  uint32_t wd[KPlan<D, BF>::NP][4];
  const bool ok = sample_words<D, BF>(w, nc, S, [&](int p, int q, uint32_t w0, uint32_t w1) {
    wd[p][q] = (w0 & ~hmask) | (w1 & hmask);
  });
#pragma unroll
  for (int p = 0; p < KPlan<D, BF>::NP; ++p) __builtin_memcpy(&B[p], wd[p], 16);
  return ok;
}

// The two values a lane pair (l, l + 32) holds: lo from lane l, hi from lane
// l + 32, the same in both lanes (v_permlane32_swap, no LDS round trip).
__device__ __forceinline__ void halves(float v, float& lo, float& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  lo = __uint_as_float(r[0]);
  hi = __uint_as_float(r[1]);
}
__device__ __forceinline__ void halves(double v, double& lo, double& hi) {
  const uint64_t b = __double_as_longlong(v);
  const auto r0 = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
  const auto r1 = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
  lo = __longlong_as_double((long long)(((uint64_t)r1[0] << 32) | r0[0]));
  hi = __longlong_as_double((long long)(((uint64_t)r1[1] << 32) | r0[1]));
}
// Sum of the two halves' values, bitwise identical in both lanes of the pair.
template <typename F>
__device__ __forceinline__ F pair_sum(F v) {
  F lo, hi;
  halves(v, lo, hi);
  return lo + hi;
}

// Constellation tables a kernel reads per sample: labels of point indices,
// label-ordered FP32 coordinates and the matrix-core point records. They are
// either the global copies or block-local LDS copies.
template <bool BF>
struct Tables {
  const uint32_t* lab;
  const float* xl;
  const typename MfmaOp<BF>::vec* rec;
};

// One block of samples at one SNR point: where the samples come from, the
// constellation size and the SNR's scalars (a launch of the sweep or a job of
// the serving loop).
struct SampleParams {
  const float* in;          // N x D received points, or unit noise in sweep mode
  const uint32_t* tx;       // N transmitted indices, or nullptr
  int64_t N;
  int M, m, sweep;
  float c, sigma;
  int* err;                 // set when a transmitted index is out of range
};

__device__ __forceinline__ SampleParams sample_params(const DemapArgs& a, int s) {
  return SampleParams{static_cast<const float*>(a.in), a.tx, a.N, a.M, a.m, a.sweep,
                      a.snr.cf[s], a.snr.sigmaf[s], a.err};
}

// Raw inputs of this lane's sample in one tile, loaded ahead of use: the
// transmitted label and point, and the unit noise (or received point).
template <int D>
struct TileInput {
  uint32_t t;          // transmitted index as given (validated in setup)
  int tl;              // its label, or 0 when not available
  float z[D];
  float xt[D];         // coordinates of the transmitted point (sweep mode)
  // global loads only (issued a tile ahead of use) ... They are made
  // unconditional (a clamped row, a stand-in buffer when there is no tx) and
  // their values are not masked here, so that no branch separates the loads
  // from their use and the wait for them can count outstanding loads instead
  // of draining all of them. setup() uses t and z only for valid samples (and
  // t only when there are transmitted indices).
  __device__ __forceinline__ void fetch(const SampleParams& p, int64_t st, int j) {
    fetch_n(p, st * 32 + j);
  }
  // sample n (any n: out-of-range indices read a clamped row)
  __device__ __forceinline__ void fetch_n(const SampleParams& p, int64_t n) {
    const int64_t nc = (n >= 0 && n < p.N) ? n : p.N - 1;
    const uint32_t* __restrict__ txp = p.tx ? p.tx : reinterpret_cast<const uint32_t*>(p.in);
    t = txp[nc];
    const float* __restrict__ in = p.in + nc * D;
#pragma unroll
    for (int d = 0; d < D; ++d) z[d] = in[d];
  }
  // ... and the table lookups that depend on them, at the time of use
  template <bool BF>
  __device__ __forceinline__ void resolve(const SampleParams& p, const Tables<BF>& tb) {
    tl = (t < (uint32_t)p.M) ? (int)tb.lab[t] : 0;
#pragma unroll
    for (int d = 0; d < D; ++d) xt[d] = p.sweep ? tb.xl[tl * D + d] : 0.0f;
  }
  template <bool BF>
  __device__ __forceinline__ void load(const SampleParams& p, const Tables<BF>& tb, int64_t st, int j) {
    fetch(p, st, j);
    resolve(p, tb);
  }
};

// One 32-sample tile at one SNR point: the received points, the sample-side
// operands and the accumulator input of this lane's sample.
template <int D, bool BF>
struct SampleTile {
  typedef typename MfmaOp<BF>::vec V;
  typedef typename MfmaOp<BF>::elem E;
  static constexpr int NK = KPlan<D, BF>::NK;    // record chunks
  static constexpr int NP = KPlan<D, BF>::NP;    // products
  int64_t n;
  bool valid, live;
  int tl, tq;          // label of the transmitted point (-1 none, -2 invalid); in-bounds row
  bool ovf;            // sample side outside the f16 range: exact path
  V B[NP];
  float16_t cinit;

  __device__ __forceinline__ void setup(const SampleParams& p, int64_t st, int j, int h,
                                        bool flag_errors, const TileInput<D>& ti) {
    setup_n(p, st * 32 + j, h, flag_errors, ti);
  }
  // sample n of this lane's column (n < 0: no sample)
  __device__ __forceinline__ void setup_n(const SampleParams& p, int64_t sn, int h, bool flag_errors,
                                          const TileInput<D>& ti) {
    const int M = p.M;
    n = sn;
    valid = n >= 0 && n < p.N;
    tl = -1;
    if (valid && p.tx) {
      if (ti.t >= (uint32_t)M) {
        if (flag_errors && h == 0) atomicOr(p.err, 1);
        tl = -2;
      } else {
        tl = ti.tl;
      }
    }
    live = valid && tl != -2;
    tq = tl >= 0 ? tl : 0;
    const float c = p.c;
    const float sigma = p.sigma;
    const float K = Real<float>::shift(p.m);
    float y[D];
    float yy = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const float zi = live ? ti.z[d] : 0.0f;
      y[d] = (p.sweep && live) ? __builtin_fmaf(sigma, zi, ti.xt[d]) : zi;
      yy = __builtin_fmaf(y[d], y[d], yy);
    }
    // sample-side operands of this lane's K half (the shift is in the
    // accumulator input)
    float w[D];
#pragma unroll
    for (int d = 0; d < D; ++d) w[d] = 2.0f * c * y[d];
    ovf = !sample_operands<D, BF>(w, -c, 0.0f, h, B);
    const float c0 = __builtin_fmaf(-c, yy, K);
#pragma unroll
    for (int e = 0; e < 16; ++e) cinit[e] = c0;
  }

  __device__ __forceinline__ float16_t product(const V (&A)[NK]) const {
    float16_t acc = MfmaOp<BF>::mma(A[KPlan<D, BF>::chunk(0)], B[0], cinit);
#pragma unroll
    for (int p = 1; p < NP; ++p) acc = MfmaOp<BF>::mma(A[KPlan<D, BF>::chunk(p)], B[p], acc);
    return acc;
  }

  // arg of the sample's own transmitted point: the diagonal of the product
  // whose A rows are the 32 samples' transmitted points. Row j of column j
  // sits in lane half (j >> 2) & 1, element (j & 3) | ((j >> 3) << 2).
  __device__ __forceinline__ float transmitted_arg(const V* __restrict__ rec, int j, int h) const {
    V At[NK];
    const V* rp = rec + ((int64_t)tq * NK) * 2 + h;
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) At[kk] = rp[2 * kk];
    const float16_t acc = product(At);
    // element (j & 3) | ((j >> 3) << 2), picked by a tree over its four bits;
    // bitwise selects keep the choice from turning into an indexed access
    auto pick = [](float a, float b, uint32_t mask) {
      return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, a) & ~mask) |
                                           (__builtin_bit_cast(uint32_t, b) & mask));
    };
    const uint32_t m0 = 0u - (uint32_t)(j & 1), m1 = 0u - (uint32_t)((j >> 1) & 1);
    const uint32_t m2 = 0u - (uint32_t)((j >> 3) & 1), m3 = 0u - (uint32_t)((j >> 4) & 1);
    float v8[8], v4[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) v8[i] = pick(acc[2 * i], acc[2 * i + 1], m0);
#pragma unroll
    for (int i = 0; i < 4; ++i) v4[i] = pick(v8[2 * i], v8[2 * i + 1], m1);
    const float mine = pick(pick(v4[0], v4[1], m2), pick(v4[2], v4[3], m2), m3);
    float lo, hi;
    halves(mine, lo, hi);
    return ((j >> 2) & 1) ? hi : lo;
  }
};

// Running bit-side sums of one lane over the point tiles (type F: float or double).
template <typename F, int NE>
struct TileSums {
  F R[NE];
  F g0[kTileLevels], g1[kTileLevels], gn[kTileLevels];
  F tot;
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int l = 0; l < kTileLevels; ++l) { g0[l] = 0; g1[l] = 0; gn[l] = 0; }
    tot = 0;
  }
  // add the NE terms of tile t (consumes ev)
  __device__ __forceinline__ void add(F (&ev)[NE], int t, int ntb) {
    if (t == 0) {
#pragma unroll
      for (int e = 0; e < NE; ++e) R[e] = ev[e];
    } else {
#pragma unroll
      for (int e = 0; e < NE; ++e) R[e] += ev[e];
    }
#pragma unroll
    for (int w2 = NE / 2; w2 >= 1; w2 >>= 1)
#pragma unroll
      for (int e = 0; e < w2; ++e) ev[e] = ev[2 * e] + ev[2 * e + 1];
    F carry = ev[0];
    bool placed = false;
#pragma unroll
    for (int l = 0; l < kTileLevels; ++l) {
      if (!placed && l < ntb) {
        if ((t >> l) & 1) {
          g0[l] += gn[l];
          g1[l] += carry;
          carry = gn[l] + carry;
        } else {
          gn[l] = carry;
          placed = true;
        }
      }
    }
    if (!placed) tot = carry;
  }
  // Combine with the other lane half of the sample: side[2k + b] and total,
  // identical in both halves (a + b in one, b + a in the other).
  __device__ __forceinline__ void combine(int ntb, F (&side)[2 * kMaxBits], F& total) const {
    constexpr int NEB = NE == 8 ? 3 : 4;
#pragma unroll
    for (int i = 0; i < 2 * kMaxBits; ++i) side[i] = 0;
    // pairwise fold of R over the element bits; label bits 0, 1, 3, 4 <- element bits 0..3
    F cur[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) cur[e] = R[e];
#pragma unroll
    for (int eb = 0; eb < NEB; ++eb) {
      const int half = NE >> (eb + 1);   // pairs left at this level
      F a0 = cur[0], a1 = cur[1];
#pragma unroll
      for (int i = 1; i < NE / 2; ++i)
        if (i < half) {
          a0 += cur[2 * i];
          a1 += cur[2 * i + 1];
        }
#pragma unroll
      for (int i = 0; i < NE / 2; ++i)
        if (i < half) cur[i] = cur[2 * i] + cur[2 * i + 1];
      const int k = eb < 2 ? eb : eb + 1;
      side[2 * k] = pair_sum(a0);
      side[2 * k + 1] = pair_sum(a1);
    }
    F lo, hi;
    halves(tot, lo, hi);
    side[4] = lo;               // label bit 2 = lane half
    side[5] = hi;
    total = lo + hi;
#pragma unroll
    for (int l = 0; l < kTileLevels; ++l)
      if (l < ntb) {
        side[2 * (5 + l)] = pair_sum(g0[l]);
        side[2 * (5 + l) + 1] = pair_sum(g1[l]);
      }
  }
};

// Record pointer of point row `t * 32 + j` for this lane half. Rows 16..31 of
// a 16-point set land only in elements e >= 8, which are not used; they read
// a valid record (row j - 16) to stay in bounds.
template <bool BF, bool HALF, int NK>
__device__ __forceinline__ const typename MfmaOp<BF>::vec* rec_row(const typename MfmaOp<BF>::vec* rec,
                                                                   int t, int j, int h) {
  const int prow = HALF ? (j & 15) : t * 32 + j;
  return rec + ((int64_t)prow * NK) * 2 + h;
}

// Bytes of the block-local copies of the constellation tables.
__host__ __device__ constexpr int64_t table_bytes(int M, int D, bool bf) {
  return (int64_t)M * 4 + (int64_t)M * D * 4 + 16 + (int64_t)M * mfma_nk(D, bf) * 32;
}

// First tier of one sample tile: all point tiles through the matrix cores,
// FP32 terms 2^(a_j + K), bit-side sums, then this lane half's LLRs (bits
// k = h mod 2) and the sample's MI/GMI terms u, v. need2 is set when an entry
// is below the starvation bound (the item then belongs to the second tier and
// u, v are not final).
template <int D, bool BF, bool HALF>
__device__ __forceinline__ void tier1_tile(const SampleTile<D, BF>& smp, const Tables<BF>& tb,
                                           bool has_tx, int j, int h, int m, int NT, int ntb,
                                           float thr, float* lout, float& u, float& v,
                                           bool& need2, bool all_sides = true) {
  typedef typename MfmaOp<BF>::vec V;
  constexpr int NK = SampleTile<D, BF>::NK;
  constexpr int NE = HALF ? 8 : 16;
  // point tiles: the next tile's records load while this one's exp2 and sums
  // run (other waves on the SIMD cover the product latency)
  TileSums<float, NE> ts;
  ts.init();
  {
    V A[NK];
    const V* rp = rec_row<BF, HALF, NK>(tb.rec, 0, j, h);
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) A[kk] = rp[2 * kk];
    for (int t = 0; t < NT; ++t) {
      const float16_t acc = smp.product(A);
      if (t + 1 < NT) {
        const V* rq = rec_row<BF, HALF, NK>(tb.rec, t + 1, j, h);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) A[kk] = rq[2 * kk];
      }
      float ev[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) ev[e] = Real<float>::exp2(acc[e]);
      ts.add(ev, t, ntb);
    }
  }
  const float arg_t = has_tx ? smp.transmitted_arg(tb.rec, j, h) : 0.f;
  float side[2 * kMaxBits];
  float total;
  ts.combine(ntb, side, total);

  // all_sides false (a job without LLRs, uniform): only the total and the
  // transmitted point's sides count, as in the sweep's first tier
  bool starved = smp.ovf || !(total >= thr);
  if (all_sides) {
#pragma unroll
    for (int i = 0; i < 2 * kMaxBits; ++i)
      if (i < 2 * m) starved |= !(side[i] >= thr);
  } else {
#pragma unroll
    for (int k = 0; k < kMaxBits; ++k)
      if (k < m) starved |= !((((smp.tl >> k) & 1) ? side[2 * k + 1] : side[2 * k]) >= thr);
  }
  u = 0.f;
  v = 0.f;
  if (smp.live && !starved) {
    const float lam_tot = Real<float>::log2(total);
    float vpart = 0.f;
#pragma unroll
    for (int i = 0; i < kMaxBits / 2; ++i) {
      const int k = 2 * i + h;
      if (k < m) {
        const float s0 = h ? side[4 * i + 2] : side[4 * i];
        const float s1 = h ? side[4 * i + 3] : side[4 * i + 1];
        const float l0 = Real<float>::log2(s0), l1 = Real<float>::log2(s1);
        if (lout) lout[k] = Real<float>::ln2() * (l0 - l1);
        if (smp.tl >= 0) vpart += lam_tot - (((smp.tl >> k) & 1) ? l1 : l0);
      }
    }
    v = pair_sum(vpart);
    u = lam_tot - Real<float>::log2(Real<float>::exp2(arg_t));
  }
  need2 = smp.live && starved;
  // an invalid transmitted index leaves the sample's LLRs undefined
  if (smp.valid && !smp.live && lout && h == 0)
    for (int k = 0; k < m; ++k) lout[k] = Real<float>::nan();
}

// Second tier of one listed sample tile: the terms re-formed in an FP64 frame
// 2^(a + K64), K64 = 1022 - m, built exactly from one FP32 exp2 of the
// fractional part and an ldexp by the integer part. Lanes whose sample is
// flagged finish it here, or on the exact path when even this frame starves
// (or the sample side left the f16 range). Returns whether this lane took the
// exact path.
template <int D, bool BF, bool HALF, bool PF2 = false>
__device__ __forceinline__ bool tier2_tile(const SampleTile<D, BF>& smp, const Tables<BF>& tb,
                                           const ExactArgs<float>& ex, bool has_tx, bool flagged,
                                           int j, int h, int m, int NT, int ntb, float* lout,
                                           float& u, float& v) {
  typedef typename MfmaOp<BF>::vec V;
  constexpr int NK = SampleTile<D, BF>::NK;
  constexpr int NE = HALF ? 8 : 16;
  const int K64 = 1022 - m;
  const double thr64 = __builtin_ldexp(1.0, m - 1022 + 60);
  // 2^(x - K + K64) for a product x = a_j + K (log2 units): K is an integer,
  // so the fraction and the floor of x serve for those of a_j = x - K
  const int dK = K64 - (int)Real<float>::shift(m);
  auto val64 = [&](float x) -> double {
    const float fr = __builtin_amdgcn_fractf(x);    // x - floor(x), in [0, 1)
    const int ni = floor_i32(x, fr);
    return __builtin_ldexp((double)Real<float>::exp2(fr), ni + dK);
  };
  TileSums<double, NE> ts;
  ts.init();
  if constexpr (!PF2) {
    V A[NK];
    const V* rp = rec_row<BF, HALF, NK>(tb.rec, 0, j, h);
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) A[kk] = rp[2 * kk];
    for (int t = 0; t < NT; ++t) {
      const float16_t acc = smp.product(A);
      if (t + 1 < NT) {
        const V* rq = rec_row<BF, HALF, NK>(tb.rec, t + 1, j, h);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) A[kk] = rq[2 * kk];
      }
      double ev[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) ev[e] = val64(acc[e]);
      ts.add(ev, t, ntb);
    }
  } else {
    // PF2: point records two tiles ahead (two register sets used in turn):
    // one tile's work does not cover an L2 read when the records are not in
    // LDS (the second tier of a launch; the serving kernels keep one, to stay
    // within their register budget)
    V A0[NK], A1[NK];
    const V* rp = rec_row<BF, HALF, NK>(tb.rec, 0, j, h);
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) A0[kk] = rp[2 * kk];
    if (NT > 1) {
      const V* rq = rec_row<BF, HALF, NK>(tb.rec, 1, j, h);
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) A1[kk] = rq[2 * kk];
    }
    auto tile = [&](V (&A)[NK], int t) {
      const float16_t acc = smp.product(A);
      if (t + 2 < NT) {
        const V* rq = rec_row<BF, HALF, NK>(tb.rec, t + 2, j, h);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) A[kk] = rq[2 * kk];
      }
      double ev[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) ev[e] = val64(acc[e]);
      ts.add(ev, t, ntb);
    };
    for (int t = 0; t < NT; t += 2) {
      tile(A0, t);
      if (t + 1 < NT) tile(A1, t + 1);
    }
  }
  const float arg_t = has_tx ? smp.transmitted_arg(tb.rec, j, h) : 0.f;
  double side[2 * kMaxBits];
  double total;
  ts.combine(ntb, side, total);

  bool st2 = smp.ovf || !(total >= thr64);
#pragma unroll
  for (int i = 0; i < 2 * kMaxBits; ++i)
    if (i < 2 * m) st2 |= !(side[i] >= thr64);
  u = 0.f;
  v = 0.f;
  if (flagged && !st2) {
    const double lt = log2_wide(total);
    double vpart = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxBits / 2; ++i) {
      const int k = 2 * i + h;
      if (k < m) {
        const double l0 = log2_wide(h ? side[4 * i + 2] : side[4 * i]);
        const double l1 = log2_wide(h ? side[4 * i + 3] : side[4 * i + 1]);
        if (lout) lout[k] = (float)(0.6931471805599453094 * (l0 - l1));
        if (smp.tl >= 0) vpart += lt - (((smp.tl >> k) & 1) ? l1 : l0);
      }
    }
    v = (float)pair_sum(vpart);
    u = (float)(lt - log2_wide(val64(arg_t)));
  }
  // beyond the FP64 window: the starved entries take the exact path; a
  // sample side outside the f16 range leaves no usable entry, so all do
  if (flagged && st2 && h == 0) {
    if (smp.ovf) {
      total = 0.0;
#pragma unroll
      for (int i = 0; i < 2 * kMaxBits; ++i) side[i] = 0.0;
    }
    finish_item_frame64<D>(ex, smp.n, smp.tl, total, side, thr64, K64, log2_wide(val64(arg_t)), lout, u,
                           v);
  }
  return flagged && st2 && h == 0;
}

// Second tier: the flagged samples, 32 to a tile (the SNR points' runs, each
// padded to a multiple of 32, numbered as one sequence of tiles), are
// re-formed in the FP64 frame. The tiles are dealt out to the waves
// round-robin, so the work is spread evenly whatever waves of the first tier
// listed it; each wave sums its samples per SNR point, and the block reduces
// its waves in a fixed order.
template <int D, bool BF, bool HALF, bool TBL>
__global__ __launch_bounds__(256, D <= 12 ? 2 : 1) void demap_mfma_t2(const DemapArgs a,
                                                     const typename MfmaOp<BF>::vec* __restrict__ rec,
                                                     const float* __restrict__ xl) {
  typedef typename MfmaOp<BF>::vec V;
  typedef SampleTile<D, BF> ST;
  constexpr int NK = ST::NK;
  extern __shared__ double acc_lds[];      // [waves][S][4], then the tables (TBL)
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int waves = blockDim.x >> 6;
  const int S = a.S;
  // the SNR runs in the tile sequence: lane s holds run s's padded start and its
  // sample count; T tiles in all
  const unsigned int tot_l = lane < S ? a.t2_tot[lane] : 0u;
  uint64_t pstart_l = 0, run = 0;
  for (int s = 0; s < S; ++s) {
    if (lane == s) pstart_l = run;
    run += t2_pad(__builtin_amdgcn_readlane(tot_l, s));
  }
  const int64_t T = (int64_t)(run >> 5);
  if ((int64_t)blockIdx.x * waves >= T) {
    // no tile reaches this block: zero partials, and no tables to stage
    for (int i = threadIdx.x; i < S * 4; i += blockDim.x) a.t2_partials[(int64_t)i * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  Tables<BF> tb{a.lab, xl, rec};
  if (TBL) {
    // small constellations in LDS: the tiles' operands and the exact path's
    // point loops then read no global memory
    const int M = a.M;
    char* lds = reinterpret_cast<char*>(acc_lds);
    const int o_lab = waves * S * 4 * (int)sizeof(double);
    const int o_xl = o_lab + M * 4;
    const int o_rec = (o_xl + M * D * 4 + 15) & ~15;
    uint32_t* l_lab = reinterpret_cast<uint32_t*>(lds + o_lab);
    float* l_xl = reinterpret_cast<float*>(lds + o_xl);
    V* l_rec = reinterpret_cast<V*>(lds + o_rec);
    for (int i = threadIdx.x; i < M; i += blockDim.x) l_lab[i] = a.lab[i];
    for (int i = threadIdx.x; i < M * D; i += blockDim.x) l_xl[i] = xl[i];
    for (int i = threadIdx.x; i < M * NK * 2; i += blockDim.x) l_rec[i] = rec[i];
    __syncthreads();
    tb = Tables<BF>{l_lab, l_xl, l_rec};
  }
  const int m = a.m;
  const int NT = HALF ? 1 : (a.M >> 5);
  const int ntb = HALF ? 0 : m - 5;
  float* __restrict__ llr = static_cast<float*>(a.llr);
  const int64_t wstride = (int64_t)gridDim.x * waves;
  const int64_t wgid = (int64_t)blockIdx.x * waves + wave;

  // wave w takes tiles w, w + waves, ...: every wave gets a share of every
  // SNR point (the high ones cost far more per sample), in increasing order
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
  for (int64_t r = 0; r < nmine; ++r) {
    const int64_t q = wgid + r * wstride;
    const uint64_t p0 = (uint64_t)q * 32u;
    // the run holding this tile: the last non-empty s whose padded start is
    // <= p0 (tiles lie inside the runs, which are multiples of 32 long)
    const unsigned long long in_run =
        __ballot(lane < S && pstart_l <= p0 && tot_l > 0u) & ((S < 64) ? ((1ull << S) - 1ull) : ~0ull);
    const int s = 63 - __builtin_clzll(in_run);
    if (s != s_cur) {
      if (s_cur >= 0) flush();
      s_cur = s;
    }
    const uint64_t start = ((uint64_t)__builtin_amdgcn_readlane((unsigned)(pstart_l >> 32), s) << 32) |
                           (uint64_t)__builtin_amdgcn_readlane((unsigned)pstart_l, s);
    const unsigned int cnt = __builtin_amdgcn_readlane(tot_l, s);
    const uint64_t pos = p0 + (uint64_t)j;
    const bool has = pos - start < (uint64_t)cnt;
    const int64_t sn = has ? (int64_t)a.t2_items[(int64_t)s * a.t2_cap + (int64_t)(pos - start)] : -1;
    items += (unsigned long long)__builtin_popcountll(__ballot(has && h == 0));
    const SampleParams sp = sample_params(a, s);
    TileInput<D> ti;
    ti.fetch_n(sp, sn);
    ti.resolve(sp, tb);
    ST smp;
    smp.setup_n(sp, sn, h, false, ti);

    const bool flagged = smp.valid;
    float* lout = (llr && smp.valid) ? llr + (int64_t)s * a.llr_stride_s + smp.n * m : nullptr;
    float u, v;
    ExactArgs<float> ex = exact_args<float>(a, s);
    ex.xl = tb.xl;
    const bool ex_lane = tier2_tile<D, BF, HALF, true>(smp, tb, ex, a.tx != nullptr, flagged, j, h, m, NT, ntb,
                                                 lout, u, v);
    exact += (unsigned long long)__builtin_popcountll(__ballot(ex_lane));
    if (flagged && h == 0 && smp.tl >= 0) {
      const double du = (double)u, dv = (double)v;
      au += du;
      av += dv;
      auu = __builtin_fma(du, du, auu);
      avv = __builtin_fma(dv, dv, avv);
    }
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

}  // namespace air
