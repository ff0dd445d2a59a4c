// tier2_list.h -- the lists of a first tier's flagged (sample, SNR) items
// and their gathering into one launch-wide list per SNR point, shared by the
// matrix-core and the FP32 vector paths.
//
// A first-tier wave lists, per SNR point, entries (sample tile of 32 | mask of
// the flagged lanes << 32) in its own run of t2_tpw slots and stores the number
// of samples it flagged in t2_nitem[s][wave]; zero masks are allowed and
// skipped. t2_collect then writes every SNR point's flagged sample indices,
// in (wave, slot, lane) order, to that point's region of t2_items, and the
// point's total to t2_tot[s].
#pragma once
#include "device_common.h"

namespace air {

__host__ __device__ inline unsigned int t2_pad(unsigned int n) { return (n + 31u) & ~31u; }

// The flagged samples of the first tier gathered per SNR point: point s's
// samples go to entries s * cap, s * cap + 1, ... of `items` in (wave, slot,
// lane) order. Block (b, s) places waves 256 b ... 256 b + 255 of point s:
// the flagged counts of the point's earlier waves are summed, its own are
// scanned, and each thread then expands its wave's list entries (a sample
// tile and the mask of its flagged lanes; empty masks are skipped)
// into sample indices. The point's last block writes the point's total.
constexpr int kCollectPre = 24;            // earlier 256-wave groups one block sums
static_assert(kMaxGrid * 4 <= 256 * kCollectPre, "a demapping launch has too many waves to collect");

static __global__ __launch_bounds__(256) void t2_collect(const unsigned int* __restrict__ nitem,
                                                  const unsigned long long* __restrict__ list, int W,
                                                  int tpw, int64_t cap, unsigned int* __restrict__ tot,
                                                  uint32_t* __restrict__ items) {
  __shared__ unsigned int wpart[2][4];
  const int b = blockIdx.x;
  const int s = blockIdx.y;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const unsigned int* c = nitem + (int64_t)s * W;
  // every count this thread needs in flight at once
  unsigned int pv[kCollectPre];
#pragma unroll
  for (int i = 0; i < kCollectPre; ++i) pv[i] = i < b ? c[t + 256 * i] : 0u;
  const int w = b * 256 + t;
  const unsigned int own = w < W ? c[w] : 0u;
  unsigned int pre = 0;
#pragma unroll
  for (int i = 0; i < kCollectPre; ++i) pre += pv[i];
  unsigned int inc = own;                  // inclusive scan over the wave's lanes
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    pre += __shfl_xor(pre, off);
    const unsigned int v = __shfl_up(inc, off);
    if (lane >= off) inc += v;
  }
  if (lane == 63) {
    wpart[0][wave] = pre;
    wpart[1][wave] = inc;
  }
  __syncthreads();
  unsigned int base = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) base += wpart[0][k] + (k < wave ? wpart[1][k] : 0u);
  if (b == (int)gridDim.x - 1 && t == 255) tot[s] = base + inc;
  if (own == 0) return;
  uint32_t* out = items + (int64_t)s * cap + (base + inc - own);
  const unsigned long long* src = list + ((int64_t)s * W + w) * tpw;
  unsigned int got = 0;
  for (int q = 0; q < tpw && got < own; ++q) {
    const unsigned long long ent = src[q];
    const uint32_t tile = (uint32_t)(ent & 0xffffffffull);
    uint32_t mask = (uint32_t)(ent >> 32);
    while (mask && got < own) {
      out[got++] = tile * 32u + (uint32_t)__builtin_ctz(mask);
      mask &= mask - 1u;
    }
  }
}

// Blocks of a second-tier launch: at most 512 (2048 waves, one round of the
// chip at two waves per SIMD); the gathered list is spread over them evenly.
__host__ __device__ inline int t2_grid(int grid) { return grid < 512 ? grid : 512; }

// The first tier's flagged samples gathered per SNR point, with their counts.
inline void launch_t2_collect(const DemapArgs& a, int grid, hipStream_t st) {
  const int W = grid * 4;
  hipLaunchKernelGGL(t2_collect, dim3((unsigned)((W + 255) / 256), (unsigned)a.S), dim3(256), 0, st, a.t2_nitem,
                     a.t2_list, W, a.t2_tpw, a.t2_cap, a.t2_tot, a.t2_items);
}

}  // namespace air
