// mfma_wide.h -- first tier of the matrix-core path with one sample per lane
// in the per-sample work.
//
// A wave takes 64 samples per round: two 32-sample column groups A (sample
// tile 2q) and B (tile 2q + 1) that share every point-side operand. Through
// the point loop each lane keeps the partial sums of its half of the rows,
// for both groups, exactly as the 32-sample form does. After the loop one
// v_permlane32_swap per accumulator moves the partial sums so that lane l
// holds both row halves of sample 64 q + l: lanes 0..31 keep group A's low
// rows and receive its high rows, lanes 32..63 receive group B's low rows and
// keep its high rows. Everything per sample -- bit-side folds, starvation
// checks, the 2m + 1 logarithms, LLR stores, the MI/GMI terms -- then runs
// once per lane on 64 distinct samples instead of twice on 32.
//
// The per-sample shift rides in the spare K slot (every point record holds
// 1 there): the sample side puts S = K - c|y|^2 rounded down to the operand
// type, so no accumulator input has to be formed per sample, and every term
// of a sample is in the same frame 2^(a_j + S + c|y|^2) with
// S + c|y|^2 <= K: no overflow, and the frame cancels in every output.
#pragma once
#include <type_traits>

#include "mfma_kernels.h"

namespace air {

// How the per-point values of a sample are combined: sums of the terms
// 2^a_j (exact demapping), or maxima of the exponents a_j (max-log).
template <bool ML>
__device__ __forceinline__ float cmb(float x, float y) {
  if constexpr (ML) return __builtin_fmaxf(x, y);
  else return x + y;
}

// Running sums (maxima for ML) of one lane over the point tiles, with LV
// tile levels. The two forms are written out separately: the sums' form is
// kept exactly as the compiler handles it best (its level arrays stay in
// registers in the run-time-M form).
template <int NE, int LV, bool ML = false>
struct WideSums {
  float R[NE];
  float g0[LV > 0 ? LV : 1], g1[LV > 0 ? LV : 1], gn[LV > 0 ? LV : 1];
  float tot;
  __device__ __forceinline__ void init() {
    const float z = ML ? -__builtin_inff() : 0.f;
#pragma unroll
    for (int l = 0; l < LV; ++l) { g0[l] = z; g1[l] = z; gn[l] = z; }
    tot = z;
  }
  __device__ __forceinline__ void add(float (&ev)[NE], int t, int ntb) {
    if constexpr (ML) {
      // (in the run-time-M form the compiler keeps g0 / g1 of this form in
      // scratch; an order-free update of every level per tile, which avoids
      // that, measured slower)
      if (t == 0) {
#pragma unroll
        for (int e = 0; e < NE; ++e) R[e] = ev[e];
      } else {
#pragma unroll
        for (int e = 0; e < NE; ++e) R[e] = __builtin_fmaxf(R[e], ev[e]);
      }
#pragma unroll
      for (int w2 = NE / 2; w2 >= 1; w2 >>= 1)
#pragma unroll
        for (int e = 0; e < w2; ++e) ev[e] = __builtin_fmaxf(ev[2 * e], ev[2 * e + 1]);
      float carry = ev[0];
      bool placed = false;
#pragma unroll
      for (int l = 0; l < LV; ++l) {
        if (!placed && l < ntb) {
          if ((t >> l) & 1) {
            g0[l] = __builtin_fmaxf(g0[l], gn[l]);
            g1[l] = __builtin_fmaxf(g1[l], carry);
            carry = __builtin_fmaxf(gn[l], carry);
          } else {
            gn[l] = carry;
            placed = true;
          }
        }
      }
      if (!placed) tot = carry;
    } else {
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
      float carry = ev[0];
      bool placed = false;
#pragma unroll
      for (int l = 0; l < LV; ++l) {
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
  }
};

// Per-lane bit-side sums of the exact-size forms with one or two point tiles
// (M = 32, 64). A tile's 16 terms (element e = 4 x + y: y carries label bits
// 0, 1 and x label bits 3, 4) go into four row sums over y and four column
// sums over x (24 operations), which accumulate over the tiles; at the end,
// pairs of the row and column sums give the two sides of each of the four
// element bits (8 operations). The lane-half bit (label bit 2) and the tile
// bit (label bit 5) come from the tiles' totals after the exchange between
// the lane halves; with two tiles each tile's total is taken from its own
// row sums (3 operations), with one tile from its sides.
template <bool ML, int NT>
struct TileMarg {
  float r[4], c[4];     // row and column sums over the tiles
  float tt[2];          // totals of tiles 0 and 1 (NT = 2)
  float es[8];          // element bit eb, side b: es[2 eb + b] (after finish)
  __device__ __forceinline__ void add(const float (&ev)[16], int t) {
    float rr[4], cc[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) rr[x] = cmb<ML>(cmb<ML>(ev[4 * x], ev[4 * x + 1]), cmb<ML>(ev[4 * x + 2], ev[4 * x + 3]));
#pragma unroll
    for (int y = 0; y < 4; ++y) cc[y] = cmb<ML>(cmb<ML>(ev[y], ev[4 + y]), cmb<ML>(ev[8 + y], ev[12 + y]));
    if (NT == 2) tt[t] = cmb<ML>(cmb<ML>(rr[0], rr[1]), cmb<ML>(rr[2], rr[3]));
    if (t == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        r[i] = rr[i];
        c[i] = cc[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        r[i] = cmb<ML>(r[i], rr[i]);
        c[i] = cmb<ML>(c[i], cc[i]);
      }
    }
  }
  __device__ __forceinline__ void finish() {
    es[0] = cmb<ML>(c[0], c[2]);
    es[1] = cmb<ML>(c[1], c[3]);
    es[2] = cmb<ML>(c[0], c[1]);
    es[3] = cmb<ML>(c[2], c[3]);
    es[4] = cmb<ML>(r[0], r[2]);
    es[5] = cmb<ML>(r[1], r[3]);
    es[6] = cmb<ML>(r[0], r[1]);
    es[7] = cmb<ML>(r[2], r[3]);
    if (NT == 1) tt[0] = cmb<ML>(es[6], es[7]);
  }
};

// Exchange of a pair of per-group values between the lane halves: returns
// (low-row half, high-row half) of the lane's own sample.
__device__ __forceinline__ void own_halves(float a, float b, float& lo, float& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  lo = __uint_as_float(r[0]);
  hi = __uint_as_float(r[1]);
}

// Sample side of one 32-sample group for this lane's K half: features of the
// sample in column j, with the shift S in the spare K slot.
template <int D, bool BF>
struct WideOperand {
  typedef typename MfmaOp<BF>::vec V;
  typedef typename MfmaOp<BF>::elem E;
  static constexpr int NK = KPlan<D, BF>::NK;    // record chunks
  static constexpr int NP = KPlan<D, BF>::NP;    // products
  V B[NP];
  bool ovf;      // a sample-side value outside the operand range: exact path

  __device__ __forceinline__ void build(const float (&y)[D], float c, float yy_lim, int m, int h) {
    const float K = Real<float>::shift(m);
    float yy = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) yy = __builtin_fmaf(y[d], y[d], yy);
    float w[D];
#pragma unroll
    for (int d = 0; d < D; ++d) w[d] = 2.0f * c * y[d];
    // S = K - c|y|^2, rounded to the operand type from below: lowering the
    // argument by more than one unit in the last place before rounding to
    // nearest keeps the rounded value <= S
    const float s0 = __builtin_fmaf(-c, yy, K);
    const float ulp = BF ? 0x1p-7f : 0x1p-10f;
    (void)sample_operands<D, BF>(w, -c, s0 - __builtin_fabsf(s0) * ulp, h, B);
    // half-precision range (bfloat16 has the FP32 range): every sample-side
    // value below 60000 in magnitude. With c < 60000 (the caller's bound,
    // c_lim), c|y|^2 < yy_lim = min(59000, 9e8 / c) / c implies |S| < 60000
    // and |2 c y_d| <= 2 c |y| < 60000; one compare instead of one per value
    // (stricter only for received points with a coordinate near |y| at
    // extreme SNR, which then take the exact path). NaN fails it too.
    ovf = BF ? false : !(yy < yy_lim);
  }

  // Operands of both 32-sample groups from this lane's own sample (group h of
  // the lane's column: group A's samples live in lanes 0..31, group B's in
  // 32..63). The lane forms both K halves of its own sample's operand; one
  // v_permlane32_swap per word then hands every lane its K half of both
  // groups' operands, so no lane forms another lane's sample. ovf is the own
  // sample's.
  static __device__ __forceinline__ void build_pair(const float (&y)[D], float c, float yy_lim, int m,
                                                    WideOperand& opA, WideOperand& opB) {
    const float K = Real<float>::shift(m);
    float yy = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) yy = __builtin_fmaf(y[d], y[d], yy);
    float w[D];
#pragma unroll
    for (int d = 0; d < D; ++d) w[d] = 2.0f * c * y[d];
    const float s0 = __builtin_fmaf(-c, yy, K);
    const float ulp = BF ? 0x1p-7f : 0x1p-10f;
    uint32_t w0[NP][4], w1[NP][4];
    (void)sample_words<D, BF>(w, -c, s0 - __builtin_fabsf(s0) * ulp,
                              [&](int p, int q, uint32_t a, uint32_t b) {
                                w0[p][q] = a;
                                w1[p][q] = b;
                              });
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      uint32_t wa[4], wb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // lanes 0..31 keep their half 0 and take half 0 of lane + 32 (group
        // B); lanes 32..63 keep their half 1 and take half 1 of lane - 32
        const auto r = __builtin_amdgcn_permlane32_swap(w0[p][q], w1[p][q], false, false);
        wa[q] = r[0];
        wb[q] = r[1];
      }
      __builtin_memcpy(&opA.B[p], wa, 16);
      __builtin_memcpy(&opB.B[p], wb, 16);
    }
    const bool o = BF ? false : !(yy < yy_lim);
    opA.ovf = o;
    opB.ovf = o;
  }

  __device__ __forceinline__ float16_t product(const V (&A)[NK]) const {
    const float16_t zero = {};
    float16_t acc = MfmaOp<BF>::mma(A[KPlan<D, BF>::chunk(0)], B[0], zero);
#pragma unroll
    for (int p = 1; p < NP; ++p) acc = MfmaOp<BF>::mma(A[KPlan<D, BF>::chunk(p)], B[p], acc);
    return acc;
  }
};

// Element (j & 3) | ((j >> 3) << 2) of a product tile: the diagonal entry of
// column j in the lane half (j >> 2) & 1 (a tree of bitwise selects).
__device__ __forceinline__ float diag_pick(const float16_t& acc, int j) {
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
  return pick(pick(v4[0], v4[1], m2), pick(v4[2], v4[3], m2), m3);
}

// An LLR of the first tier. NT: streamed past the caches (the exact-size
// forms, whose LLR writes are a large share of the launch; the L2 then keeps
// the inputs that the next SNR point reads again). A sample's LLRs are stored
// back to back, so each line is still written whole.
template <bool NT>
__device__ __forceinline__ void store_llr(float v, float* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Raw global inputs of one sample, loaded a round ahead of use (see
// TileInput::fetch for why the loads are unconditional and unmasked).
template <int D>
struct RawInput {
  uint32_t t;
  float z[D];
  __device__ __forceinline__ void fetch(const SampleParams& p, uint32_t st, int j) {
    // 32-bit sample indices: a call holds fewer than 2^32 - 128 samples
    const uint32_t n = st * 32u + (uint32_t)j;
    const uint32_t nlast = (uint32_t)p.N - 1u;
    const uint32_t nc = n < nlast ? n : nlast;
    const uint32_t* __restrict__ txp = p.tx ? p.tx : reinterpret_cast<const uint32_t*>(p.in);
    t = txp[nc];
    const float* __restrict__ in = p.in + (uint64_t)nc * D;
#pragma unroll
    for (int d = 0; d < D; ++d) z[d] = in[d];
  }
};

// One group's sample for this lane's column j: validity, label and y.
template <int D>
struct WideSample {
  uint32_t n;      // 32-bit sample index (a call holds fewer than 2^32 - 128 samples)
  bool valid, live;
  int tl;          // label of the transmitted point (-1 none, -2 invalid index)
  int tq;          // an in-bounds label for record reads
  float y[D];
  template <bool BF>
  __device__ __forceinline__ void setup(const SampleParams& p, const Tables<BF>& tb, uint32_t st, int j,
                                        bool flag_errors, const RawInput<D>& ri) {
    n = st * 32u + (uint32_t)j;
    valid = n < (uint32_t)p.N;
    // table reads at an in-bounds index, unconditionally (selected afterwards),
    // so that no lane-dependent branch surrounds them
    const bool inb = ri.t < (uint32_t)p.M;
    const int lab = (int)tb.lab[inb ? ri.t : 0u];
    float xv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xv[d] = tb.xl[lab * D + d];
    const bool has_t = valid && p.tx != nullptr;
    const bool bad = has_t && !inb;
    if (flag_errors && bad) atomicOr(p.err, 1);
    tl = has_t ? (inb ? lab : -2) : -1;
    live = valid && !bad;
    tq = tl >= 0 ? tl : 0;
    // sweep: y = fma(sigma, z, x_t); a given block: y = fma(1, y, 0 * x) = y.
    // Lanes that are not live keep finite values (the fetch is clamped to a
    // real sample, the record read to label 0): they only feed their own
    // column of each product, whose outputs are dropped.
    const float ga = p.sweep ? p.sigma : 1.0f;
    const float gx = p.sweep ? 1.0f : 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = __builtin_fmaf(ga, ri.z[d], xv[d] * gx);
  }
};

// Flagged samples in one 64-sample round from which a wave of the run-time-M
// first tier hands the rest of its rounds at that SNR point to the second
// tier directly: above a flagged fraction of about 0.55 (12-D, M = 4096) to
// 0.74 (8-D, M = 2048) that is the cheaper route, since the second tier
// costs about 2.5 times the first tier per term and re-forms every flagged
// sample anyway.
constexpr int kDirectRound = 48;

// First tier, 64 samples per wave round. The exact-size forms of small D are
// held to 168 registers (three waves per SIMD); what little the allocator
// then keeps in scratch is reloaded once per SNR point, outside the sample
// loop. The run-time-M forms of D <= 12 are held to 256 registers (two waves
// per SIMD: the products then land in ordinary registers, and a second wave
// covers the point records' L2 reads); their few spills sit outside the
// point loop. MB = log2 M for the small sets
// compiled at their exact size (M = 16, 32, 64: every per-bit loop and the
// point loop are then static), 0 for any M >= 32 taken at run time. The t2
// list and partial-sum layouts are those of demap_mfma, so the second-tier
// kernel is shared.
// Max-log bit sides of one sample computed directly in FP32 (the matrix-core
// operands of a sample out of the operand range): side[2k + b] = the largest
// a_j = -c |y - x_j|^2 over the labels j with bit k equal to b.
template <int D>
__device__ __forceinline__ void maxlog_direct(const float (&y)[D], const float* __restrict__ xl, int M,
                                              int m, float c, float (&side)[2 * kMaxBits]) {
#pragma unroll
  for (int i = 0; i < 2 * kMaxBits; ++i) side[i] = -__builtin_inff();
  for (int j = 0; j < M; ++j) {
    float d2 = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const float df = y[d] - xl[j * D + d];
      d2 = __builtin_fmaf(df, df, d2);
    }
    const float aj = -c * d2;
#pragma unroll
    for (int k = 0; k < kMaxBits; ++k)
      if (k < m) {
        const bool b = (j >> k) & 1;
        side[2 * k] = b ? side[2 * k] : __builtin_fmaxf(side[2 * k], aj);
        side[2 * k + 1] = b ? __builtin_fmaxf(side[2 * k + 1], aj) : side[2 * k + 1];
      }
  }
}

// b if bit k of `word` is set, else a: v_bfi_b32 on the sign-extended bit,
// two instructions (the compiler turns the same select written in C into a
// shift, a compare and a conditional move).
__device__ __forceinline__ float bit_select(float a, float b, int word, int k) {
  const uint32_t msk = (uint32_t)__builtin_amdgcn_sbfe(word, k, 1);
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(msk), "v"(__float_as_uint(b)), "v"(__float_as_uint(a)));
  return __uint_as_float(r);
}

// log2(1 + 2^x) in FP32 without overflow.
__device__ __forceinline__ float softplus2(float x) {
  const float ax = __builtin_fabsf(x);
  return __builtin_fmaxf(x, 0.0f) + Real<float>::log2(1.0f + Real<float>::exp2(-ax));
}

// ML: the max-log form. Each bit side keeps the largest exponent instead of
// the sum of the terms; the LLR is ln 2 times the difference of the two
// sides' maxima, the GMI term is the BMD rate of those LLRs taken as exact,
// sum_k log2(1 + 2^(-(1 - 2 b_k) L_k / ln 2)); the transmitted point's own
// term, the logarithms of the sums and the second tier are not needed (no
// sum can starve). Samples whose operands leave the operand range are done
// by maxlog_direct.
template <int D, bool BF, bool TBL, int MB, bool ML = false>
__global__ __launch_bounds__(256, (MB && D <= 4) ? 3 : (D <= 12 ? 2 : 1)) void demap_mfma_w(const DemapArgs a,
                                                    const typename MfmaOp<BF>::vec* __restrict__ rec,
                                                    const float* __restrict__ xl) {
  typedef typename MfmaOp<BF>::vec V;
  typedef WideOperand<D, BF> OP;
  constexpr bool HALF = MB == 4;                                   // 16-point tiles
  constexpr int LV = MB == 0 ? kTileLevels : (MB > 5 ? MB - 5 : 0);  // tile levels carried
  constexpr int NK = OP::NK;
  constexpr int NE = HALF ? 8 : 16;
  constexpr int NEB = HALF ? 3 : 4;       // element bits carrying label bits
  constexpr bool MARG = MB == 5 || MB == 6;  // one or two point tiles: TileMarg
  // each lane forms only its own sample's operand (build_pair): fewer
  // instructions per round, which the small sets feel; the half-precision
  // run-time-M forms of D > 8 measured 2 % slower with it (12-D/4096) and keep
  // the per-group form (in bfloat16 it is 1 % faster there and ends the
  // spills of the 12-D form)
  constexpr bool OWN = MB != 0 || D <= 8 || BF;
  // run-time-M forms: once a round of a wave has had at least kDirectRound of
  // its 64 samples flagged for the second tier, the wave's later rounds at
  // that SNR point list every live sample for the second tier without
  // forming them here (at high SNR nearly every sample of a large set has a
  // bit side below the FP32 frame, and the first tier's work on it is lost)
  constexpr bool DIRECT = MB == 0 && !ML;
  extern __shared__ double acc_lds[];      // [waves][S][4], then the tables (TBL)
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int waves = blockDim.x >> 6;
  const int S = a.S;
  Tables<BF> tb{a.lab, xl, rec};
  if (TBL) {
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
  const int m = MB ? MB : a.m;
  const int NT = MB ? (HALF ? 1 : 1 << (MB - 5)) : (a.M >> 5);
  const int ntb = MB ? LV : m - 5;
  const float thr = Real<float>::starve(m);
  float* __restrict__ llr = static_cast<float*>(a.llr);
  // exact-size forms: 32-bit pair and wave indices (fewer than 2^26 pairs,
  // 2^16 waves), so that the round loop's counters and compares stay on the
  // scalar unit (-1.9 % per 8-PSK^2 launch); the run-time-M forms, whose
  // rounds are long, measured 2.6 % slower with them and keep 64-bit ones
  typedef typename std::conditional<MB != 0, int, int64_t>::type QI;
  const QI npairs = (QI)((((a.N + 31) >> 5) + 1) >> 1);
  const QI wstride = (QI)gridDim.x * waves;
  const QI wgid = (QI)blockIdx.x * waves + wave;
  const bool hj = (j >> 2) & 1;           // lane half holding row j of a tile

  // Per SNR point the waves take the pairs q0, q0 + wstride, ... with q0 =
  // (wgid + sh) mod wstride, sh = (s * rem mod wstride) rounded down to a
  // multiple of 32, rem = npairs mod wstride: the waves that get one round
  // more than the others change from one SNR point to the next, so over a
  // sweep every wave does nearly the same number of rounds. Shifting by
  // multiples of 32 waves (8 blocks) keeps each pair on the same XCD
  // (blocks are dealt to the 8 XCDs in turn), whose L2 still holds its
  // inputs from the previous SNR point.
  const QI rem = npairs % wstride;
  for (int s = 0; s < S; ++s) {
    double au = 0.0, av = 0.0, auu = 0.0, avv = 0.0;
    unsigned long long* slots = a.t2_list + ((int64_t)s * wstride + wgid) * a.t2_tpw;
    int nlisted = 0;
    unsigned int nflag = 0;                // samples flagged in those entries
    const SampleParams sp = sample_params(a, s);
    // |y|^2 below which the half-precision operands are in range (see
    // WideOperand::build); none at all if c itself is out of range
    const float yy_lim = sp.c < 60000.0f ? __builtin_fminf(59000.0f, 9.0e8f / sp.c) / sp.c : -1.0f;
    const QI q0 = (wgid + ((((QI)s * rem) % wstride) & ~(QI)31)) % wstride;
    // OWN: each lane sets up its own sample only (group A, tile 2 q, in
    // lanes 0..31; group B, tile 2 q + 1, in lanes 32..63) and forms both K
    // halves of its operand (build_pair); otherwise every lane sets up both
    // groups' samples of its column and forms its K half of each
    RawInput<D> inA, inB;
    if (q0 < npairs) {
      if constexpr (OWN) {
        inA.fetch(sp, 2 * q0 + h, j);
      } else {
        inA.fetch(sp, 2 * q0, j);
        inB.fetch(sp, 2 * q0 + 1, j);
      }
    }
    QI q = q0;
    for (; q < npairs; q += wstride) {
      WideSample<D> smA, smB;
      const QI qn = q + wstride < npairs ? q + wstride : npairs - 1;
      OP opA, opB;
      if constexpr (OWN) {
        smA.setup(sp, tb, 2 * q + h, j, s == 0, inA);
        // the next round's inputs, loaded into the registers just consumed
        // (no copy between buffers) a round ahead of use
        inA.fetch(sp, 2 * qn + h, j);
        OP::build_pair(smA.y, sp.c, yy_lim, m, opA, opB);
      } else {
        smA.setup(sp, tb, 2 * q, j, s == 0 && h == 0, inA);
        smB.setup(sp, tb, 2 * q + 1, j, s == 0 && h == 0, inB);
        inA.fetch(sp, 2 * qn, j);
        inB.fetch(sp, 2 * qn + 1, j);
        opA.build(smA.y, sp.c, yy_lim, m, h);
        opB.build(smB.y, sp.c, yy_lim, m, h);
      }
      // the lane's own sample
      const WideSample<D>& sm = (OWN || !h) ? smA : smB;

      // the transmitted points' own terms: diagonals of the products whose A
      // rows are the groups' transmitted points (OWN: both groups' labels of
      // this column in every lane by one exchange between the lane halves)
      float arg_t = 0.f;
      if (!ML && a.tx) {
        int tqA, tqB;
        if constexpr (OWN) {
          const auto tqs = __builtin_amdgcn_permlane32_swap((uint32_t)smA.tq, (uint32_t)smA.tq, false, false);
          tqA = (int)tqs[0];
          tqB = (int)tqs[1];
        } else {
          tqA = smA.tq;
          tqB = smB.tq;
        }
        V At[NK];
        const V* ra = tb.rec + ((int64_t)tqA * NK) * 2 + h;
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) At[kk] = ra[2 * kk];
        const float pa = diag_pick(opA.product(At), j);
        const V* rb = tb.rec + ((int64_t)tqB * NK) * 2 + h;
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) At[kk] = rb[2 * kk];
        const float pb = diag_pick(opB.product(At), j);
        float lo, hi;
        own_halves(pa, pb, lo, hi);
        arg_t = hj ? hi : lo;
      }

      WideSums<NE, LV, ML> sA, sB;
      TileMarg<ML, (MB == 6 ? 2 : 1)> mA, mB;
      if constexpr (!MARG) {
        sA.init();
        sB.init();
      }
      {
        V A[NK];
        const V* rp = rec_row<BF, HALF, NK>(tb.rec, 0, j, h);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) A[kk] = rp[2 * kk];
        for (int t = 0; t < NT; ++t) {
          const float16_t accA = opA.product(A);
          const float16_t accB = opB.product(A);
          if (t + 1 < NT) {
            const V* rq = rec_row<BF, HALF, NK>(tb.rec, t + 1, j, h);
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) A[kk] = rq[2 * kk];
          }
          float ev[NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) ev[e] = ML ? accA[e] : Real<float>::exp2(accA[e]);
          if constexpr (MARG) mA.add(ev, t);
          else sA.add(ev, t, ntb);
#pragma unroll
          for (int e = 0; e < NE; ++e) ev[e] = ML ? accB[e] : Real<float>::exp2(accB[e]);
          if constexpr (MARG) mB.add(ev, t);
          else sB.add(ev, t, ntb);
        }
      }
      // own sample of this lane: group A in lanes 0..31, group B in 32..63
      const uint32_t n = sm.n;
      const bool valid = sm.valid;
      const bool live = sm.live;
      const int tl = sm.tl;
      const bool ovf = (OWN || !h) ? opA.ovf : opB.ovf;

      float side[2 * kMaxBits];
#pragma unroll
      for (int i = 0; i < 2 * kMaxBits; ++i) side[i] = 0.f;
      float total;
      if constexpr (MARG) {
        mA.finish();
        mB.finish();
        // the sample's element-bit sides and tile totals from both lane halves
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          float lo, hi;
          own_halves(mA.es[i], mB.es[i], lo, hi);
          const int eb = i >> 1;
          side[2 * (eb < 2 ? eb : eb + 1) + (i & 1)] = cmb<ML>(lo, hi);
        }
        float t0lo, t0hi;
        own_halves(mA.tt[0], mB.tt[0], t0lo, t0hi);
        if constexpr (MB == 6) {
          float t1lo, t1hi;
          own_halves(mA.tt[1], mB.tt[1], t1lo, t1hi);
          side[10] = cmb<ML>(t0lo, t0hi);      // label bit 5: the tile
          side[11] = cmb<ML>(t1lo, t1hi);
          side[4] = cmb<ML>(t0lo, t1lo);       // label bit 2: the lane half
          side[5] = cmb<ML>(t0hi, t1hi);
          total = cmb<ML>(side[10], side[11]);
        } else {
          side[4] = t0lo;
          side[5] = t0hi;
          total = cmb<ML>(t0lo, t0hi);
        }
      } else {
        // both row halves of the own sample
        float r0[NE], r1[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) own_halves(sA.R[e], sB.R[e], r0[e], r1[e]);
        {
          float t0, t1;
          own_halves(sA.tot, sB.tot, t0, t1);
          total = cmb<ML>(t0, t1);
        }
#pragma unroll
        for (int l = 0; l < LV; ++l)
          if (l < ntb) {
            float x0, x1;
            own_halves(sA.g0[l], sB.g0[l], x0, x1);
            side[2 * (5 + l)] = cmb<ML>(x0, x1);
            own_halves(sA.g1[l], sB.g1[l], x0, x1);
            side[2 * (5 + l) + 1] = cmb<ML>(x0, x1);
          }
        {
          // label bit 2 is the row half
          float c0 = r0[0], c1 = r1[0];
#pragma unroll
          for (int e = 1; e < NE; ++e) {
            c0 = cmb<ML>(c0, r0[e]);
            c1 = cmb<ML>(c1, r1[e]);
          }
          side[4] = c0;
          side[5] = c1;
        }
        {
          // label bits 0, 1, 3 (, 4) are the element bits 0, 1, 2 (, 3)
          float cur[NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) cur[e] = cmb<ML>(r0[e], r1[e]);
#pragma unroll
          for (int eb = 0; eb < NEB; ++eb) {
            const int half = NE >> (eb + 1);
            float a0 = cur[0], a1 = cur[1];
#pragma unroll
            for (int i = 1; i < NE / 2; ++i)
              if (i < half) {
                a0 = cmb<ML>(a0, cur[2 * i]);
                a1 = cmb<ML>(a1, cur[2 * i + 1]);
              }
#pragma unroll
            for (int i = 0; i < NE / 2; ++i)
              if (i < half) cur[i] = cmb<ML>(cur[2 * i], cur[2 * i + 1]);
            const int k = eb < 2 ? eb : eb + 1;
            side[2 * k] = a0;
            side[2 * k + 1] = a1;
          }
        }
      }

      float* lout = (llr && valid) ? llr + (int64_t)s * a.llr_stride_s + (uint64_t)n * m : nullptr;
      if constexpr (ML) {
        (void)total;
        (void)thr;
        if (live && ovf) {
          maxlog_direct<D>(sm.y, tb.xl, a.M, m, sp.c, side);
          ++nlisted;                       // counted as recomputed below
        }
        float v = 0.f;
        if (live) {
          float L[kMaxBits];
#pragma unroll
          for (int k = 0; k < kMaxBits; ++k)
            if (k < m) {
              const float lam = side[2 * k] - side[2 * k + 1];
              L[k] = Real<float>::ln2() * lam;
              if (tl >= 0) v += softplus2(((tl >> k) & 1) ? lam : -lam);
            }
          // the sample's LLRs stored together
          if (lout) {
#pragma unroll
            for (int k = 0; k < kMaxBits; ++k)
              if (k < m) store_llr<MB != 0>(L[k], lout + k);
          }
        } else if (valid && lout) {
          for (int k = 0; k < m; ++k) lout[k] = Real<float>::nan();
        }
        if (live && tl >= 0) {
          const double dv = (double)v;
          av += dv;
          avv = __builtin_fma(dv, dv, avv);
        }
        continue;
      }
      // every sum is finite and >= 0 unless the operands left their range
      // (ovf), so the smallest of them decides. Without LLRs (a uniform
      // choice per call) only the sums that u and v use count: the total and
      // the transmitted point's side of each bit. A starved other side enters
      // nothing but the total, which its own bound keeps within 2^-20 of its
      // value (at most M terms below the FP32 range, each under 2^-20 / M of
      // the bound); lanes without a transmitted label are not live then.
      float smin = total;
      if (llr) {
#pragma unroll
        for (int i = 0; i < 2 * kMaxBits; ++i)
          if (i < 2 * m) smin = __builtin_fminf(smin, side[i]);
      } else {
#pragma unroll
        for (int k = 0; k < kMaxBits; ++k)
          if (k < m) smin = __builtin_fminf(smin, bit_select(side[2 * k], side[2 * k + 1], tl, k));
      }
      const bool starved = ovf || !(smin >= thr);
      float u = 0.f, v = -0.f;                 // -0 + x is x: no add for the first term
      if (live && !starved) {
        const float lam_tot = Real<float>::log2(total);
        float L[kMaxBits];
#pragma unroll
        for (int k = 0; k < kMaxBits; ++k) {
          if (k < m) {
            const float l0 = Real<float>::log2(side[2 * k]), l1 = Real<float>::log2(side[2 * k + 1]);
            L[k] = Real<float>::ln2() * (l0 - l1);
            v += lam_tot - bit_select(l0, l1, tl, k);   // v is dropped unless tl >= 0
          }
        }
        if (lout) {
#pragma unroll
          for (int k = 0; k < kMaxBits; ++k)
            if (k < m) store_llr<MB != 0>(L[k], lout + k);
        }
        u = lam_tot - Real<float>::log2(Real<float>::exp2(arg_t));
      }
      // items with a starved entry are finished by the second tier: each of
      // the two sample tiles is listed with the mask of its starved lanes
      const bool need2 = live && starved;
      const unsigned long long bm = __ballot(need2);
      const unsigned long long mlo = bm & 0xffffffffull, mhi = bm >> 32;
      nflag += __builtin_popcountll(bm);
      if (mlo) {
        if (lane == 0) slots[nlisted] = (mlo << 32) | (unsigned long long)(2 * q);
        ++nlisted;
      }
      if (mhi) {
        if (lane == 0) slots[nlisted] = (mhi << 32) | (unsigned long long)(2 * q + 1);
        ++nlisted;
      }
      if (valid && !live && lout)
        for (int k = 0; k < m; ++k) lout[k] = Real<float>::nan();
      if (live && tl >= 0 && !need2) {
        const double du = (double)u, dv = (double)v;
        au += du;
        av += dv;
        auu = __builtin_fma(du, du, auu);
        avv = __builtin_fma(dv, dv, avv);
      }
      if constexpr (DIRECT) {
        if (__builtin_popcountll(bm) >= kDirectRound) {
          q += wstride;
          break;
        }
      }
    }
    if constexpr (DIRECT) {
      // the rest of the wave's rounds at this SNR point: every live sample
      // (the lane's own one, sample tile 2 q + h) listed as it is
      for (; q < npairs; q += wstride) {
        const uint32_t n = (uint32_t)(2 * q + h) * 32u + (uint32_t)j;
        const bool valid = n < (uint32_t)sp.N;
        const uint32_t t = (valid && sp.tx) ? sp.tx[n] : 0u;
        const bool bad = valid && sp.tx && !(t < (uint32_t)sp.M);
        if (s == 0 && bad) atomicOr(sp.err, 1);
        if (bad && llr)
          for (int k = 0; k < m; ++k) llr[(int64_t)s * a.llr_stride_s + (uint64_t)n * m + k] = Real<float>::nan();
        const unsigned long long bm = __ballot(valid && !bad);
        const unsigned long long mlo = bm & 0xffffffffull, mhi = bm >> 32;
        nflag += __builtin_popcountll(bm);
        if (mlo) {
          if (lane == 0) slots[nlisted] = (mlo << 32) | (unsigned long long)(2 * q);
          ++nlisted;
        }
        if (mhi) {
          if (lane == 0) slots[nlisted] = (mhi << 32) | (unsigned long long)(2 * q + 1);
          ++nlisted;
        }
      }
    }
    if constexpr (ML) {
      // nlisted counted this lane's directly computed samples
      const double wd = wave_sum((double)nlisted);
      if (lane == 0 && wd > 0.0) atomicAdd(a.recomputed, (unsigned long long)wd);
    } else {
      if (lane == 0) a.t2_nitem[(int64_t)s * wstride + wgid] = nflag;
    }
    const double w0 = wave_sum(au), w1 = wave_sum(av);
    const double w2 = wave_sum(auu), w3 = wave_sum(avv);
    if (lane == 0) {
      double* acc = acc_lds + ((int64_t)wave * S + s) * 4;
      acc[0] = w0;
      acc[1] = w1;
      acc[2] = w2;
      acc[3] = w3;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S * 4; i += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < waves; ++w) t += acc_lds[w * S * 4 + i];
    a.partials[(int64_t)i * gridDim.x + blockIdx.x] = t;
  }
}

// The wide first tier (exact or max-log) in the variant the constellation
// size calls for.
template <int D, bool BF, bool ML>
void launch_first_tier(const DemapArgs& a, const typename MfmaOp<BF>::vec* r, const float* x, int grid,
                       const Launch& l) {
  const uint32_t acc = (uint32_t)(sizeof(double) * 4 * a.S * 4);
  const int64_t tbytes = table_bytes(a.M, D, BF);
  const bool tbl = tbytes <= 40 * 1024;
  const uint32_t lds = acc + (uint32_t)tbytes;
  // the exact-size forms hold their tables in LDS (at most 12.5 KB for M = 64)
  if (a.M == 16)
    launch_kernel(l, demap_mfma_w<D, BF, true, 4, ML>, dim3(grid), dim3(256), lds, a, r, x);
  else if (a.M == 32)
    launch_kernel(l, demap_mfma_w<D, BF, true, 5, ML>, dim3(grid), dim3(256), lds, a, r, x);
  else if (a.M == 64)
    launch_kernel(l, demap_mfma_w<D, BF, true, 6, ML>, dim3(grid), dim3(256), lds, a, r, x);
  else if (tbl)
    launch_kernel(l, demap_mfma_w<D, BF, true, 0, ML>, dim3(grid), dim3(256), lds, a, r, x);
  else
    launch_kernel(l, demap_mfma_w<D, BF, false, 0, ML>, dim3(grid), dim3(256), acc, a, r, x);
}

// One part of the matrix-core path for one (D, operand type). part 0: the
// exact first tier; 1: the gather of its lists and the shared second tier;
// 2: the max-log form (one kernel, no second tier). The events of `l` time
// the first tier's kernel only.
template <int D, bool BF>
hipError_t launch_mfma_wide_td(const DemapArgs& a, const void* rec, int grid, const Launch& l, int part) {
  const size_t acc = sizeof(double) * 4 * a.S * 4;
  const int64_t tbytes = table_bytes(a.M, D, BF);
  const bool tbl = tbytes <= 40 * 1024;
  typedef typename MfmaOp<BF>::vec V;
  const V* r = static_cast<const V*>(rec);
  const float* x = static_cast<const float*>(a.xl);
  if (part == 0 || part == 2) {
    if (part == 0) launch_first_tier<D, BF, false>(a, r, x, grid, l);
    else launch_first_tier<D, BF, true>(a, r, x, grid, l);
    return hipGetLastError();
  }
  const hipStream_t st = l.stream;
  launch_t2_collect(a, grid, st);
  const dim3 g2(t2_grid(grid));
  if (a.M == 16)
    hipLaunchKernelGGL((demap_mfma_t2<D, BF, true, true>), g2, dim3(256), acc + tbytes, st, a, r, x);
  else if (tbl)
    hipLaunchKernelGGL((demap_mfma_t2<D, BF, false, true>), g2, dim3(256), acc + tbytes, st, a, r, x);
  else
    hipLaunchKernelGGL((demap_mfma_t2<D, BF, false, false>), g2, dim3(256), acc, st, a, r, x);
  return hipGetLastError();
}

}  // namespace air
