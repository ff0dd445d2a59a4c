// serve_kernels.h -- batched matrix-core kernels of the serving loop.
//
// A batch holds jobs of uneven M, D and N. Jobs that share a kernel class
// (D, operand type, 16-point form) are contiguous in the batch's descriptor
// array, and one launch per class walks the flattened (job, chunk) work items
// of all of them: wave w of the grid takes items w, w + waves, ... Each item
// is a fixed run of sample tiles of one job, so every sum the kernels form
// depends on the job alone -- never on which jobs share the batch or which
// wave ran the item -- and a job's result is bitwise the same alone and in
// any mix. The per-tile arithmetic is the one of the sweep kernels
// (tier1_tile / tier2_tile).
#pragma once

#include "mfma_kernels.h"

namespace air {

// Result record of one job, written by the kernels (cleared by the host).
struct JobOut {
  double stats[4];                  // MI, GMI, SE_MI, SE_GMI (bits per symbol)
  unsigned long long recomputed;    // items finished by the second tier or the exact path
  int err;                          // a transmitted index >= M was seen
  int pad;
};

// One job of a batch, as the kernels see it.
struct JobDesc {
  const float* in;                  // N x D received points, or unit noise (sweep)
  const uint32_t* tx;               // N transmitted indices, or nullptr (LLRs only)
  float* llr;                       // N x m LLRs (nats), or nullptr
  const uint32_t* lab;              // label of point index j
  const float* xl;                  // M x D coordinates in label order
  const void* rec;                  // matrix-core point records, label order
  double* partials;                 // [nitems][8]: sums u, v, u^2, v^2 of tier 1, then tier 2
  unsigned long long* list;         // [nitems][chunk]: tiles left to tier 2 (tile | lane mask << 32)
  unsigned int* count;              // [nitems]: entries of each item's list
  JobOut* out;
  int64_t N;
  int64_t item0;                    // first item of this job in its class launch
  int nitems;
  int chunk;                        // sample tiles per item
  int M, m, sweep;
  float c, sigma;                   // metric scale 1/(2 sigma^2 ln 2) and noise deviation
};

// Sample tiles per work item of a job with N samples: a function of N alone
// (at most 4096 items per job).
__host__ __device__ inline int serve_chunk(int64_t N) {
  const int64_t tiles = (N + 31) / 32;
  const int64_t c = (tiles + 4095) / 4096;
  return (int)(c < 1 ? 1 : c);
}

// The job of work item `it`: the last job whose first item is <= it.
__device__ __forceinline__ int serve_job_of(const JobDesc* __restrict__ jobs, int njobs, int64_t it) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].item0 <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ SampleParams job_params(const JobDesc& jd) {
  return SampleParams{jd.in, jd.tx, jd.N, jd.M, jd.m, jd.sweep, jd.c, jd.sigma, &jd.out->err};
}

// Flagged samples of a 32-sample tile from which a serving work item hands
// its remaining tiles to the second tier directly (three quarters, as in the
// sweep's first tier).
constexpr int kDirectTile = 24;

template <int D, bool BF, bool HALF>
__global__ __launch_bounds__(256) void serve_tier1(const JobDesc* __restrict__ jobs, int njobs,
                                                   int64_t nitems) {
  typedef typename MfmaOp<BF>::vec V;
  typedef SampleTile<D, BF> ST;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int64_t waves = blockDim.x >> 6;
  const int64_t wstride = (int64_t)gridDim.x * waves;
  for (int64_t it = (int64_t)blockIdx.x * waves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); it < nitems;
       it += wstride) {
    const JobDesc& jd = jobs[serve_job_of(jobs, njobs, it)];
    const int64_t li = it - jd.item0;
    const int m = jd.m;
    const int NT = HALF ? 1 : (jd.M >> 5);
    const int ntb = HALF ? 0 : m - 5;
    const float thr = Real<float>::starve(m);
    const SampleParams sp = job_params(jd);
    const Tables<BF> tb{jd.lab, jd.xl, static_cast<const V*>(jd.rec)};
    const int64_t ntiles = (jd.N + 31) >> 5;
    const int64_t st0 = li * jd.chunk;
    const int64_t st1 = st0 + jd.chunk < ntiles ? st0 + jd.chunk : ntiles;
    unsigned long long* slots = jd.list + li * jd.chunk;
    double au = 0.0, av = 0.0, auu = 0.0, avv = 0.0;
    int nlisted = 0;
    // once a tile of the item has had at least kDirectTile of its 32 samples
    // flagged, the item's later tiles go to the second tier as they are (as
    // in the sweep's first tier; the item's tiles are a function of the job
    // alone, so the choice is too)
    bool direct = false;
    for (int64_t st = st0; st < st1; ++st) {
      TileInput<D> ti;
      ti.load(sp, tb, st, j);
      ST smp;
      smp.setup(sp, st, j, h, true, ti);
      float* lout = (jd.llr && smp.valid) ? jd.llr + smp.n * m : nullptr;
      float u = 0.f, v = 0.f;
      bool need2;
      if (!direct) {
        tier1_tile<D, BF, HALF>(smp, tb, jd.tx != nullptr, j, h, m, NT, ntb, thr, lout, u, v, need2,
                                jd.llr != nullptr || jd.tx == nullptr);
      } else {
        need2 = smp.live;
        if (smp.valid && !smp.live && lout && h == 0)
          for (int k = 0; k < m; ++k) lout[k] = Real<float>::nan();
      }
      const unsigned long long fm = __ballot(need2 && h == 0) & 0xffffffffull;
      if (!HALF && __builtin_popcountll(fm) >= kDirectTile) direct = true;
      if (fm != 0) {
        if (lane == 0) slots[nlisted] = (fm << 32) | (unsigned long long)st;
        ++nlisted;
      }
      if (h == 0 && smp.live && smp.tl >= 0 && !need2) {
        const double du = (double)u, dv = (double)v;
        au += du;
        av += dv;
        auu = __builtin_fma(du, du, auu);
        avv = __builtin_fma(dv, dv, avv);
      }
    }
    const double w0 = wave_sum(au), w1 = wave_sum(av);
    const double w2 = wave_sum(auu), w3 = wave_sum(avv);
    if (lane == 0) {
      double* p = jd.partials + li * 8;
      p[0] = w0;
      p[1] = w1;
      p[2] = w2;
      p[3] = w3;
      jd.count[li] = (unsigned int)nlisted;
    }
  }
}

template <int D, bool BF, bool HALF>
__global__ __launch_bounds__(256, D <= 12 ? 2 : 1) void serve_tier2(const JobDesc* __restrict__ jobs, int njobs,
                                                   int64_t nitems) {
  typedef typename MfmaOp<BF>::vec V;
  typedef SampleTile<D, BF> ST;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int64_t waves = blockDim.x >> 6;
  const int64_t wstride = (int64_t)gridDim.x * waves;
  for (int64_t it = (int64_t)blockIdx.x * waves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); it < nitems;
       it += wstride) {
    const JobDesc& jd = jobs[serve_job_of(jobs, njobs, it)];
    const int64_t li = it - jd.item0;
    const int nlisted = (int)jd.count[li];
    double au = 0.0, av = 0.0, auu = 0.0, avv = 0.0;
    if (nlisted > 0) {
      const int m = jd.m;
      const int NT = HALF ? 1 : (jd.M >> 5);
      const int ntb = HALF ? 0 : m - 5;
      const SampleParams sp = job_params(jd);
      const Tables<BF> tb{jd.lab, jd.xl, static_cast<const V*>(jd.rec)};
      const ExactArgs<float> ex{jd.in, jd.sweep, jd.xl, jd.M, m, jd.sigma, jd.c, &jd.out->recomputed};
      const unsigned long long* slots = jd.list + li * jd.chunk;
      unsigned long long items = 0;
      for (int q = 0; q < nlisted; ++q) {
        const unsigned long long ent = slots[q];
        const int64_t st = (int64_t)(ent & 0xffffffffull);
        const uint32_t mask = (uint32_t)(ent >> 32);
        items += (unsigned long long)__builtin_popcount(mask);
        TileInput<D> ti;
        ti.load(sp, tb, st, j);
        ST smp;
        smp.setup(sp, st, j, h, false, ti);
        const bool flagged = (mask >> j) & 1u;
        float* lout = (jd.llr && smp.valid) ? jd.llr + smp.n * m : nullptr;
        float u, v;
        tier2_tile<D, BF, HALF>(smp, tb, ex, jd.tx != nullptr, flagged, j, h, m, NT, ntb, lout, u, v);
        if (flagged && h == 0 && smp.tl >= 0) {
          const double du = (double)u, dv = (double)v;
          au += du;
          av += dv;
          auu = __builtin_fma(du, du, auu);
          avv = __builtin_fma(dv, dv, avv);
        }
      }
      if (lane == 0) atomicAdd(&jd.out->recomputed, items);
    }
    const double w0 = wave_sum(au), w1 = wave_sum(av);
    const double w2 = wave_sum(auu), w3 = wave_sum(avv);
    if (lane == 0) {
      double* p = jd.partials + li * 8 + 4;
      p[0] = w0;
      p[1] = w1;
      p[2] = w2;
      p[3] = w3;
    }
  }
}

// Both tiers of one kernel class: `jobs` is the class's contiguous run of
// descriptors, `nitems` the sum of their items.
template <int D, bool BF>
hipError_t launch_serve_td(const JobDesc* jobs, int njobs, int64_t nitems, bool half, int grid,
                           hipStream_t st) {
  if (half) {
    hipLaunchKernelGGL((serve_tier1<D, BF, true>), dim3(grid), dim3(256), 0, st, jobs, njobs, nitems);
    hipLaunchKernelGGL((serve_tier2<D, BF, true>), dim3(grid), dim3(256), 0, st, jobs, njobs, nitems);
  } else {
    hipLaunchKernelGGL((serve_tier1<D, BF, false>), dim3(grid), dim3(256), 0, st, jobs, njobs, nitems);
    hipLaunchKernelGGL((serve_tier2<D, BF, false>), dim3(grid), dim3(256), 0, st, jobs, njobs, nitems);
  }
  return hipGetLastError();
}

}  // namespace air
