// hd_mfma.h -- hard decisions on the matrix cores, with the decisions of
// hd_kernel (the nearest point by FP32 distances, ties to the lower label).
//
// For constellations of M >= 32 points whose coordinates are of moderate
// range, the distances to all points come from the product tiles of the
// first tier, in a metric scaled per sample so that every term is bounded:
// x_j = c (2 y.x_j - |x_j|^2 - |y|^2) = -c |y - x_j|^2 with
// c = 16 / (|y|^2 + R^2), R = max |x_j|, so c (|y| + |x_j|)^2 <= 32 and the
// split operands and the FP32 sums of the products leave an absolute error
// below ~3e-4 in x_j. A first pass takes each sample's largest x_j; a second
// pass recomputes the tiles and evaluates, with the FP32 procedure of
// hd_kernel, every point whose x_j is within kHdTheta = 2^-9 of it. The
// procedure's own rounding is below 1e-4 in these units, so the point it
// would pick, and every point tied with it, is among those evaluated, and
// the smallest (distance, label) among them is hd_kernel's decision.
#pragma once
#include "hd_kernels.h"
#include "mfma_wide.h"

namespace air {

constexpr float kHdTheta = 0x1p-9f;

// The FP32 distance of hd_kernel: acc = fma(y_d - x_d, y_d - x_d, acc) from 0.
template <int D>
__device__ __forceinline__ float hd_dist(const float (&y)[D], const float* __restrict__ x) {
  float acc = 0.0f;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const float df = y[d] - x[d];
    acc = __builtin_fmaf(df, df, acc);
  }
  return acc;
}

// (distance, label) kept in hd_kernel's order: a smaller distance, or the same
// distance at a lower label, replaces the current one (a NaN never does).
__device__ __forceinline__ void hd_take(float d, int l, float& bd, int& bl) {
  const bool better = d < bd || (d == bd && l < bl);
  bd = better ? d : bd;
  bl = better ? l : bl;
}

// Bytes of the block-local copies of the coordinates and point records.
__host__ __device__ constexpr int64_t hd_table_bytes(int M, int D) {
  return (int64_t)M * D * 4 + 16 + (int64_t)M * mfma_nk(D, false) * 32;
}

// One wave takes 64 samples per round (two 32-sample tiles, as the first
// tier); lane (j, h) holds rows 8 (e / 4) + 4 h + e % 4 of column j of both
// tiles' products and finishes sample j of tile h.
template <int D, bool TBL>
__global__ __launch_bounds__(256, 2) void hd_mfma(const HdArgs a, const MfmaOp<false>::vec* __restrict__ rec,
                                                 float R2) {
  typedef MfmaOp<false>::vec V;
  typedef WideOperand<D, false> OP;
  constexpr int NK = OP::NK;
  extern __shared__ char hd_lds[];
  __shared__ unsigned long long part[4][2];
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const int waves = blockDim.x >> 6;
  const int M = a.M;
  const int NT = M >> 5;
  const float* __restrict__ xl = a.xl;
  const V* __restrict__ rp = rec;
  if (TBL) {
    float* l_xl = reinterpret_cast<float*>(hd_lds);
    V* l_rec = reinterpret_cast<V*>(hd_lds + ((M * D * 4 + 15) & ~15));
    for (int i = threadIdx.x; i < M * D; i += blockDim.x) l_xl[i] = a.xl[i];
    for (int i = threadIdx.x; i < M * NK * 2; i += blockDim.x) l_rec[i] = rec[i];
    __syncthreads();
    xl = l_xl;
    rp = l_rec;
  }
  const int64_t ntiles = (a.N + 31) >> 5;
  const int64_t npairs = (ntiles + 1) >> 1;
  const int64_t wstride = (int64_t)gridDim.x * waves;
  const int64_t wgid = (int64_t)blockIdx.x * waves + wave;
  for (int s = 0; s < a.S; ++s) {
    unsigned int se = 0, be = 0;
    for (int64_t q = wgid; q < npairs; q += wstride) {
      // the samples of column j in the two tiles: as hd_kernel forms them
      float y[2][D];
      int tl[2];
      bool valid[2];
      int64_t n[2];
      OP op[2];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        n[g] = (2 * q + g) * 32 + j;
        valid[g] = n[g] < a.N;
        const int64_t nc = valid[g] ? n[g] : a.N - 1;
        tl[g] = -1;
        if (a.tx) {
          const uint32_t t = a.tx[nc];
          if (t >= (uint32_t)M) {
            if (s == 0 && g == h && valid[g]) atomicOr(a.err, 1);
            tl[g] = -2;
          } else {
            tl[g] = (int)a.lab[t];
          }
        }
        const float* __restrict__ in = a.in + nc * D;
        if (a.sweep) {
          const int lt = tl[g] >= 0 ? tl[g] : 0;
#pragma unroll
          for (int d = 0; d < D; ++d) y[g][d] = __builtin_fmaf(a.sigma[s], in[d], xl[lt * D + d]);
        } else {
#pragma unroll
          for (int d = 0; d < D; ++d) y[g][d] = in[d];
        }
        float yy = 0.0f;
#pragma unroll
        for (int d = 0; d < D; ++d) yy = __builtin_fmaf(y[g][d], y[g][d], yy);
        // m = 126 makes the operand's shift 0: x_j = -c |y - x_j|^2. With this
        // c every operand is in range for finite |y|^2 (c |y|^2 < 16, c <= 16 / R2
        // <= 4096), so only an infinite or NaN |y|^2 counts as out of range.
        op[g].build(y[g], 16.0f / (yy + R2), __FLT_MAX__, 126, h);
      }
      // pass 1: the largest metric of each sample over this lane's rows
      float mx[2] = {-__builtin_inff(), -__builtin_inff()};
      for (int t = 0; t < NT; ++t) {
        V A[NK];
        const V* r = rec_row<false, false, NK>(rp, t, j, h);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) A[kk] = r[2 * kk];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          const float16_t acc = op[g].product(A);
          float m8[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) m8[e] = __builtin_fmaxf(acc[2 * e], acc[2 * e + 1]);
#pragma unroll
          for (int e = 0; e < 4; ++e) m8[e] = __builtin_fmaxf(m8[2 * e], m8[2 * e + 1]);
          mx[g] = __builtin_fmaxf(mx[g], __builtin_fmaxf(__builtin_fmaxf(m8[0], m8[1]),
                                                         __builtin_fmaxf(m8[2], m8[3])));
        }
      }
      // over both row halves: the own sample's (tile h) from the pair of
      // lanes, then the other tile's from the partner lane
      float full[2];
      {
        float lo, hi;
        own_halves(mx[0], mx[1], lo, hi);
        const float own = __builtin_fmaxf(lo, hi);
        float o0, o1;
        own_halves(own, own, o0, o1);
        full[0] = h ? o0 : own;
        full[1] = h ? own : o1;
      }
      // pass 2: the FP32 procedure on every point near the maximum
      float bd[2] = {__builtin_inff(), __builtin_inff()};
      int bl[2] = {0, 0};
      for (int t = 0; t < NT; ++t) {
        V A[NK];
        const V* r = rec_row<false, false, NK>(rp, t, j, h);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) A[kk] = r[2 * kk];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          const float16_t acc = op[g].product(A);
          const float floor_g = full[g] - kHdTheta;
          // the tile's candidates as a bit mask (no branch per element), then
          // the FP32 procedure on each (rarely more than one per sample)
          uint32_t bits = 0u;
#pragma unroll
          for (int e = 0; e < 16; ++e) bits |= acc[e] >= floor_g ? (1u << e) : 0u;
          while (bits) {
            const int e = __builtin_ctz(bits);
            bits &= bits - 1u;
            const int l = t * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
            hd_take(hd_dist<D>(y[g], xl + l * D), l, bd[g], bl[g]);
          }
        }
      }
      // combine the two lanes of each sample; lane (j, h) keeps sample j of tile h
      float d_own;
      int l_own;
      {
        float dlo, dhi;
        own_halves(bd[0], bd[1], dlo, dhi);
        const auto li = __builtin_amdgcn_permlane32_swap((uint32_t)bl[0], (uint32_t)bl[1], false, false);
        d_own = dlo;
        l_own = (int)li[0];
        hd_take(dhi, (int)li[1], d_own, l_own);
      }
      const bool vo = h ? valid[1] : valid[0];
      const int to = h ? tl[1] : tl[0];
      // operands out of their range (extreme inputs): the full FP32 scan
      if (vo && (h ? op[1].ovf : op[0].ovf)) {
        d_own = __builtin_inff();
        l_own = 0;
        for (int l = 0; l < M; ++l) {
          const float dl = hd_dist<D>(h ? y[1] : y[0], xl + l * D);
          if (dl < d_own) {
            d_own = dl;
            l_own = l;
          }
        }
      }
      if (vo) {
        const int64_t no = h ? n[1] : n[0];
        if (a.decided) a.decided[(int64_t)s * a.N + no] = a.pos[l_own];
        if (to >= 0 && l_own != to) {
          se += 1;
          be += (unsigned int)__builtin_popcount((unsigned)(l_own ^ to));
        }
      }
    }
    const double ws = wave_sum((double)se), wb = wave_sum((double)be);
    if (lane == 0) {
      part[wave][0] = (unsigned long long)ws;
      part[wave][1] = (unsigned long long)wb;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      unsigned long long tt = 0;
      for (int w = 0; w < waves; ++w) tt += part[w][threadIdx.x];
      if (a.counts && tt) atomicAdd(a.counts + 2 * s + threadIdx.x, tt);
    }
    __syncthreads();
  }
}

template <int D>
hipError_t launch_hd_mfma_d(const HdArgs& a, const void* rec, float R2, int grid, hipStream_t st) {
  typedef MfmaOp<false>::vec V;
  const V* r = static_cast<const V*>(rec);
  const int64_t tb = hd_table_bytes(a.M, D);
  if (tb <= 40 * 1024)
    hipLaunchKernelGGL((hd_mfma<D, true>), dim3(grid), dim3(256), (size_t)tb, st, a, r, R2);
  else
    hipLaunchKernelGGL((hd_mfma<D, false>), dim3(grid), dim3(256), 0, st, a, r, R2);
  return hipGetLastError();
}

}  // namespace air
