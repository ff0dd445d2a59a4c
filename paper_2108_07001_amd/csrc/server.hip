// server.hip -- the serving loop of libair (air_server_* in include/air.h).
//
// Jobs of uneven M, D and N arrive at any time. A host worker thread admits
// them in arrival order while their device footprint (staged inputs, staged
// LLRs, per-item partial sums and tile lists) fits in a fixed device arena
// allocated once at creation, groups the admitted jobs into batches
// (continuous batching: whatever is admitted when a launch slot frees up goes
// into the next launch), and runs each batch on one of a few streams, so that
// the input copies of one batch overlap the kernels of another and small jobs
// are not held behind a large one. A batch is: one host-to-device copy of its
// job descriptors, the staged input copies, one launch per kernel class of
// each tier, one fixed-order reduction per job, and one device-to-host copy of
// the result records. Completion is observed by polling the batch's event;
// the worker then stamps the jobs, releases their arena blocks and queues the
// results for air_server_poll.
#include "../../include/air.h"
#include "host_state.h"
#include "serve_kernels.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

namespace air {

// Batched launchers, one per (operand type, D), defined in serve_inst_*.hip.
using ServeFn = hipError_t (*)(const JobDesc*, int, int64_t, bool, int, hipStream_t);
#define AIR_DECL(tag, D) \
  hipError_t launch_serve_##tag##_d##D(const JobDesc*, int, int64_t, bool, int, hipStream_t);
#define AIR_DECL_ALL(tag)                                                                        \
  AIR_DECL(tag, 1) AIR_DECL(tag, 2) AIR_DECL(tag, 3) AIR_DECL(tag, 4) AIR_DECL(tag, 5)          \
  AIR_DECL(tag, 6) AIR_DECL(tag, 7) AIR_DECL(tag, 8) AIR_DECL(tag, 9) AIR_DECL(tag, 10)         \
  AIR_DECL(tag, 11) AIR_DECL(tag, 12) AIR_DECL(tag, 13) AIR_DECL(tag, 14) AIR_DECL(tag, 15)     \
  AIR_DECL(tag, 16)
AIR_DECL_ALL(f16)
AIR_DECL_ALL(bf16)
#undef AIR_DECL_ALL
#undef AIR_DECL
#define AIR_FN(tag, D) launch_serve_##tag##_d##D
static const ServeFn kServeF16[kMaxD + 1] = {
    nullptr, AIR_FN(f16, 1), AIR_FN(f16, 2), AIR_FN(f16, 3), AIR_FN(f16, 4), AIR_FN(f16, 5),
    AIR_FN(f16, 6), AIR_FN(f16, 7), AIR_FN(f16, 8), AIR_FN(f16, 9), AIR_FN(f16, 10),
    AIR_FN(f16, 11), AIR_FN(f16, 12), AIR_FN(f16, 13), AIR_FN(f16, 14), AIR_FN(f16, 15),
    AIR_FN(f16, 16)};
static const ServeFn kServeBF16[kMaxD + 1] = {
    nullptr, AIR_FN(bf16, 1), AIR_FN(bf16, 2), AIR_FN(bf16, 3), AIR_FN(bf16, 4), AIR_FN(bf16, 5),
    AIR_FN(bf16, 6), AIR_FN(bf16, 7), AIR_FN(bf16, 8), AIR_FN(bf16, 9), AIR_FN(bf16, 10),
    AIR_FN(bf16, 11), AIR_FN(bf16, 12), AIR_FN(bf16, 13), AIR_FN(bf16, 14), AIR_FN(bf16, 15),
    AIR_FN(bf16, 16)};
#undef AIR_FN

// Fixed-order reduction of one job per block: wave q sums quantity q over
// the job's items (lane l takes items l, l + 64, ..., tier 1 then tier 2 of
// each), then a fixed butterfly. MI = log2 M - mean u, GMI = m - mean v, with
// standard errors from the sample variances; NaN when a transmitted index
// was out of range or the job has no transmitted indices.
__global__ __launch_bounds__(256) void serve_finish(const JobDesc* __restrict__ jobs) {
  __shared__ double sums[4];
  const JobDesc& jd = jobs[blockIdx.x];
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double t = 0.0;
  for (int i = lane; i < jd.nitems; i += 64) {
    t += jd.partials[(int64_t)i * 8 + q];
    t += jd.partials[(int64_t)i * 8 + 4 + q];
  }
  t = wave_sum(t);
  if (lane == 0) sums[q] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double n = (double)jd.N;
    const double su = sums[0], sv = sums[1], suu = sums[2], svv = sums[3];
    double mi = log2((double)jd.M) - su / n;
    double gmi = (double)jd.m - sv / n;
    double se_mi = __builtin_nan(""), se_gmi = __builtin_nan("");
    if (jd.N > 1) {
      const double vu = (suu - su * su / n) / (n - 1.0);
      const double vv = (svv - sv * sv / n) / (n - 1.0);
      se_mi = sqrt((vu > 0.0 ? vu : 0.0) / n);
      se_gmi = sqrt((vv > 0.0 ? vv : 0.0) / n);
    }
    if (jd.out->err || !jd.tx) mi = gmi = se_mi = se_gmi = __builtin_nan("");
    jd.out->stats[0] = mi;
    jd.out->stats[1] = gmi;
    jd.out->stats[2] = se_mi;
    jd.out->stats[3] = se_gmi;
  }
}

namespace {

constexpr int kSlots = 3;          // launch slots, one stream each
constexpr int kMaxBatch = 64;      // jobs per launch
constexpr int kMaxClassGrid = 2048;
constexpr size_t kAlign = 256;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator of byte ranges of the device arena; free ranges are
// kept sorted by offset and merged with their neighbours on release.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, o = it->first + n;
      free_.erase(it);
      if (rest) free_[o] = rest;
      used_ += n;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    size_t o = off, len = n;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        o = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + n == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[o] = len;
    used_ -= n;
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

enum class Mem { Device, Host, Foreign };

// Where a caller pointer lives: device memory of `device`, host memory
// (pinned or pageable), or device memory of another device.
Mem classify(const void* p, int device) {
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return Mem::Host;
  }
  if (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged)
    return at.device == device ? Mem::Device : Mem::Foreign;
  return Mem::Host;
}

struct Job {
  air_job j;
  const air_const* c = nullptr;
  int cls = 0;                   // kernel class: D, operand type, 16-point form
  bool in_host = false, tx_host = false, llr_host = false;
  int chunk = 1, nitems = 0;
  size_t foot = 0, off = 0;      // arena block
  size_t o_in = 0, o_tx = 0, o_llr = 0, o_part = 0, o_list = 0, o_count = 0;
  double sigma = 0.0, c_scale = 0.0;
  air_result res;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* d_block = nullptr;       // device: descriptors, then result records
  char* h_block = nullptr;       // pinned host twin of d_block
  std::vector<Job*> jobs;
  bool busy = false;
};

constexpr size_t kDescBytes = sizeof(JobDesc) * kMaxBatch;
constexpr size_t kBlockBytes = kDescBytes + sizeof(JobOut) * kMaxBatch;

}  // namespace
}  // namespace air

using namespace air;

struct air_server {
  air_ctx* ctx = nullptr;
  int device = 0;
  size_t budget = 0;
  int max_inflight = 0;
  char* arena_base = nullptr;
  Arena arena;
  Slot slots[kSlots];
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;        // submitted, waiting for admission
  std::deque<Job*> admitted;     // holding arena space, waiting for a launch slot
  std::deque<air_result> results;
  uint64_t next_id = 1;
  uint64_t submitted = 0, completed = 0, batches = 0;
  int inflight = 0;              // admitted or running
  int max_batch = 0;
  bool stopping = false;
  air_status fatal = AIR_OK;
  std::string fatal_msg;
  std::string err;               // last submit/create error (caller thread)
};

namespace {

air_status srv_fail(air_server* s, air_status st, const std::string& msg) {
  if (s) s->err = msg;
  return st;
}

// Device bytes of one job and the offsets of its pieces in its arena block.
void layout(Job* jb) {
  const int64_t N = jb->j.N;
  const int D = jb->c->D, m = jb->c->m;
  const int64_t tiles = (N + 31) / 32;
  jb->chunk = serve_chunk(N);
  jb->nitems = (int)((tiles + jb->chunk - 1) / jb->chunk);
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  if (jb->in_host) jb->o_in = take(sizeof(float) * (size_t)N * D);
  if (jb->tx_host) jb->o_tx = take(sizeof(uint32_t) * (size_t)N);
  if (jb->llr_host) jb->o_llr = take(sizeof(float) * (size_t)N * m);
  jb->o_part = take(sizeof(double) * 8 * (size_t)jb->nitems);
  jb->o_list = take(sizeof(unsigned long long) * (size_t)jb->nitems * jb->chunk);
  jb->o_count = take(sizeof(unsigned int) * (size_t)jb->nitems);
  jb->foot = o;
}

// Completes every job the server still holds with `st` (after a device error).
void fail_all(air_server* s, std::unique_lock<std::mutex>& lk, air_status st) {
  auto finish = [&](Job* jb) {
    jb->res.status = st;
    jb->res.t_done_ns = now_ns();
    s->results.push_back(jb->res);
    ++s->completed;
    delete jb;
  };
  for (Job* jb : s->queue) finish(jb);
  for (Job* jb : s->admitted) finish(jb);
  s->queue.clear();
  s->admitted.clear();
  for (Slot& sl : s->slots) {
    for (Job* jb : sl.jobs) finish(jb);
    sl.jobs.clear();
    sl.busy = false;
  }
  s->inflight = 0;
  (void)lk;
  s->cv_done.notify_all();
}

// Enqueue one batch on a slot's stream. Called by the worker without the lock.
hipError_t launch_batch(air_server* s, Slot& sl) {
  std::vector<Job*>& jobs = sl.jobs;
  std::stable_sort(jobs.begin(), jobs.end(), [](const Job* a, const Job* b) { return a->cls < b->cls; });
  const int n = (int)jobs.size();
  JobDesc* hd = reinterpret_cast<JobDesc*>(sl.h_block);
  JobOut* ho = reinterpret_cast<JobOut*>(sl.h_block + kDescBytes);
  const JobDesc* dd = reinterpret_cast<const JobDesc*>(sl.d_block);
  JobOut* dout = reinterpret_cast<JobOut*>(sl.d_block + kDescBytes);
  int64_t item0 = 0;
  for (int k = 0; k < n; ++k) {
    Job* jb = jobs[k];
    if (k > 0 && jobs[k - 1]->cls != jb->cls) item0 = 0;
    char* base = s->arena_base + jb->off;
    const air_const* c = jb->c;
    const bool bf = jb->j.prec == AIR_BF16X3;
    JobDesc& d = hd[k];
    std::memset(&d, 0, sizeof(d));
    d.in = jb->in_host ? reinterpret_cast<const float*>(base + jb->o_in) : jb->j.in;
    d.tx = jb->j.tx ? (jb->tx_host ? reinterpret_cast<const uint32_t*>(base + jb->o_tx) : jb->j.tx) : nullptr;
    d.llr = jb->j.llr ? (jb->llr_host ? reinterpret_cast<float*>(base + jb->o_llr) : jb->j.llr) : nullptr;
    d.lab = c->lab;
    d.xl = c->x32;
    d.rec = bf ? (const void*)c->rec_bf16 : (const void*)c->rec_f16;
    d.partials = reinterpret_cast<double*>(base + jb->o_part);
    d.list = reinterpret_cast<unsigned long long*>(base + jb->o_list);
    d.count = reinterpret_cast<unsigned int*>(base + jb->o_count);
    d.out = dout + k;
    d.N = jb->j.N;
    d.item0 = item0;
    d.nitems = jb->nitems;
    d.chunk = jb->chunk;
    d.M = c->M;
    d.m = c->m;
    d.sweep = jb->j.noise_in ? 1 : 0;
    d.c = (float)jb->c_scale;
    d.sigma = (float)jb->sigma;
    std::memset(&ho[k], 0, sizeof(JobOut));
    item0 += jb->nitems;
  }
  const hipStream_t st = sl.stream;
  const uint64_t t_launch = now_ns();
  for (Job* jb : jobs) jb->res.t_launch_ns = t_launch;
  hipError_t e = hipMemcpyAsync(sl.d_block, sl.h_block, kBlockBytes, hipMemcpyHostToDevice, st);
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    Job* jb = jobs[k];
    const size_t N = (size_t)jb->j.N;
    if (jb->in_host)
      e = hipMemcpyAsync((void*)hd[k].in, jb->j.in, sizeof(float) * N * jb->c->D, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && jb->tx_host && jb->j.tx)
      e = hipMemcpyAsync((void*)hd[k].tx, jb->j.tx, sizeof(uint32_t) * N, hipMemcpyHostToDevice, st);
  }
  // one launch per kernel class and tier
  for (int a = 0; a < n && e == hipSuccess;) {
    int b = a + 1;
    int64_t items = jobs[a]->nitems;
    while (b < n && jobs[b]->cls == jobs[a]->cls) items += jobs[b++]->nitems;
    const Job* ja = jobs[a];
    const ServeFn fn = ja->j.prec == AIR_BF16X3 ? kServeBF16[ja->c->D] : kServeF16[ja->c->D];
    const int64_t g = (items + 3) / 4;
    const int grid = (int)(g < kMaxClassGrid ? g : kMaxClassGrid);
    e = fn(dd + a, b - a, items, ja->c->M == 16, grid, st);
    a = b;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(serve_finish, dim3(n), dim3(256), 0, st, dd);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(ho, dout, sizeof(JobOut) * n, hipMemcpyDeviceToHost, st);
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    Job* jb = jobs[k];
    if (jb->llr_host)
      e = hipMemcpyAsync(jb->j.llr, hd[k].llr, sizeof(float) * (size_t)jb->j.N * jb->c->m,
                         hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipEventRecord(sl.done, st);
  return e;
}

void worker_main(air_server* s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    std::unique_lock<std::mutex> lk(s->mu);
    s->fatal = AIR_E_DEVICE;
    s->fatal_msg = "serving worker cannot select the device";
    fail_all(s, lk, AIR_E_DEVICE);
    return;
  }
  uint64_t last_event = now_ns();
  for (;;) {
    bool progress = false;
    // 1. reap finished batches
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      std::unique_lock<std::mutex> lk(s->mu);
      if (q != hipSuccess) {
        s->fatal = AIR_E_DEVICE;
        s->fatal_msg = std::string("serving batch failed: ") + hipGetErrorString(q);
        fail_all(s, lk, AIR_E_DEVICE);
        return;
      }
      const uint64_t t = now_ns();
      const JobOut* ho = reinterpret_cast<const JobOut*>(sl.h_block + kDescBytes);
      for (size_t k = 0; k < sl.jobs.size(); ++k) {
        Job* jb = sl.jobs[k];
        air_result& r = jb->res;
        r.mi = ho[k].stats[0];
        r.gmi = ho[k].stats[1];
        r.se_mi = ho[k].stats[2];
        r.se_gmi = ho[k].stats[3];
        r.recomputed = ho[k].recomputed;
        r.status = ho[k].err ? AIR_E_RANGE : AIR_OK;
        r.t_done_ns = t;
        s->arena.release(jb->off, jb->foot);
        s->results.push_back(r);
        ++s->completed;
        --s->inflight;
        delete jb;
      }
      sl.jobs.clear();
      sl.busy = false;
      progress = true;
      last_event = t;
      s->cv_done.notify_all();
    }
    // 2. admit in arrival order while the footprint fits; 3. form a batch
    Slot* free_slot = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      while (!s->queue.empty() && s->inflight < s->max_inflight) {
        Job* jb = s->queue.front();
        if (!s->arena.alloc(jb->foot, &jb->off)) break;
        s->queue.pop_front();
        jb->res.t_admit_ns = now_ns();
        s->admitted.push_back(jb);
        ++s->inflight;
        progress = true;
      }
      if (!s->admitted.empty())
        for (Slot& sl : s->slots)
          if (!sl.busy) {
            free_slot = &sl;
            break;
          }
      if (free_slot) {
        while (!s->admitted.empty() && (int)free_slot->jobs.size() < kMaxBatch) {
          free_slot->jobs.push_back(s->admitted.front());
          s->admitted.pop_front();
        }
        free_slot->busy = true;
        ++s->batches;
        s->max_batch = std::max(s->max_batch, (int)free_slot->jobs.size());
      }
      bool any_busy = false;
      for (Slot& sl : s->slots) any_busy |= sl.busy;
      if (!free_slot && !progress && !any_busy) {
        if (s->stopping && s->queue.empty() && s->admitted.empty()) return;
        s->cv_work.wait(lk);
        continue;
      }
    }
    if (free_slot) {
      const hipError_t e = launch_batch(s, *free_slot);
      if (e != hipSuccess) {
        std::unique_lock<std::mutex> lk(s->mu);
        s->fatal = AIR_E_DEVICE;
        s->fatal_msg = std::string("serving launch failed: ") + hipGetErrorString(e);
        fail_all(s, lk, AIR_E_DEVICE);
        return;
      }
      continue;
    }
    if (!progress) {
      // batches in flight: poll their events; back off after a quiet spell
      if (now_ns() - last_event < 200000) std::this_thread::yield();
      else std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

void destroy_server(air_server* s) {
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stopping = true;
    }
    s->cv_work.notify_all();
    s->worker.join();
  }
  {
    DeviceGuard g(s->device);
    for (Slot& sl : s->slots) {
      if (sl.stream) (void)hipStreamSynchronize(sl.stream);
      for (Job* jb : sl.jobs) delete jb;
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      (void)hipFree(sl.d_block);
      (void)hipHostFree(sl.h_block);
    }
    for (Job* jb : s->queue) delete jb;
    for (Job* jb : s->admitted) delete jb;
    (void)hipFree(s->arena_base);
  }
  delete s;
}

}  // namespace

extern "C" {

air_status air_server_create(air_ctx* ctx, size_t hbm_budget_bytes, int max_inflight, air_server** out) {
  if (!ctx) return AIR_E_INVAL;
  if (!out) return fail(ctx, AIR_E_INVAL, "out is null");
  *out = nullptr;
  if (hbm_budget_bytes < 4096) return fail(ctx, AIR_E_INVAL, "budget must be at least 4096 bytes");
  if (max_inflight < 1) return fail(ctx, AIR_E_INVAL, "max_inflight must be >= 1");
  air_server* s = nullptr;
  try {
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, AIR_E_DEVICE, "cannot select the context's device");
    s = new air_server();
    s->ctx = ctx;
    s->device = ctx->device;
    s->budget = align_up(hbm_budget_bytes);
    s->max_inflight = max_inflight;
    hipError_t e = hipMalloc(&s->arena_base, s->budget);
    for (Slot& sl : s->slots) {
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipMalloc(&sl.d_block, kBlockBytes);
      if (e == hipSuccess) e = hipHostMalloc(&sl.h_block, kBlockBytes, hipHostMallocDefault);
    }
    if (e != hipSuccess) {
      destroy_server(s);
      return hip_fail(ctx, e, "server resources");
    }
    s->arena.reset(s->budget);
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    if (s) destroy_server(s);
    return fail(ctx, AIR_E_NOMEM, "host allocation failed");
  }
  *out = s;
  ctx->err.clear();
  return AIR_OK;
}

air_status air_server_submit(air_server* s, const air_job* job, uint64_t* id_out) {
  if (!s) return AIR_E_INVAL;
  if (!job || !id_out) return srv_fail(s, AIR_E_INVAL, "job and id_out must not be null");
  *id_out = 0;
  const air_const* c = job->c;
  if (!c || c->ctx != s->ctx) return srv_fail(s, AIR_E_INVAL, "constellation is null or from another context");
  if (!job->in) return srv_fail(s, AIR_E_INVAL, "job input is null");
  if (job->N < 1) return srv_fail(s, AIR_E_INVAL, "N must be >= 1");
  if ((job->N + 31) / 32 >= ((int64_t)1 << 32)) return srv_fail(s, AIR_E_UNSUPPORTED, "N too large for one job");
  if (!std::isfinite(job->snr_db)) return srv_fail(s, AIR_E_INVAL, "SNR must be finite");
  if (job->noise_in && !job->tx) return srv_fail(s, AIR_E_INVAL, "noise input needs transmitted indices");
  if (job->prec != AIR_FP16X3 && job->prec != AIR_BF16X3)
    return srv_fail(s, AIR_E_UNSUPPORTED, "the serving loop runs the matrix-core forms (AIR_FP16X3, AIR_BF16X3)");
  if (c->M < 16) return srv_fail(s, AIR_E_UNSUPPORTED, "the serving loop needs M >= 16");
  if (job->prec == AIR_FP16X3 && !c->f16_ok)
    return srv_fail(s, AIR_E_UNSUPPORTED, "constellation coordinates exceed the half-precision range");
  Job* jb = nullptr;
  try {
    DeviceGuard g(s->device);
    if (!g.ok) return srv_fail(s, AIR_E_DEVICE, "cannot select the server's device");
    const Mem min = classify(job->in, s->device);
    const Mem mtx = job->tx ? classify(job->tx, s->device) : Mem::Device;
    const Mem mllr = job->llr ? classify(job->llr, s->device) : Mem::Device;
    if (min == Mem::Foreign || mtx == Mem::Foreign || mllr == Mem::Foreign)
      return srv_fail(s, AIR_E_INVAL, "a job buffer is device memory of another device");
    jb = new Job();
    jb->j = *job;
    jb->c = c;
    jb->in_host = min == Mem::Host;
    jb->tx_host = job->tx && mtx == Mem::Host;
    jb->llr_host = job->llr && mllr == Mem::Host;
    jb->cls = ((c->D * 2 + (job->prec == AIR_BF16X3 ? 1 : 0)) * 2) + (c->M == 16 ? 1 : 0);
    snr_scalars(c, job->snr_db, jb->sigma, jb->c_scale);
    layout(jb);
    std::memset(&jb->res, 0, sizeof(jb->res));
    jb->res.tag = job->tag;
    jb->res.footprint = jb->foot;
    jb->res.t_arrival_ns = job->t_arrival_ns ? job->t_arrival_ns : now_ns();
    if (jb->foot > s->budget) {
      delete jb;
      return srv_fail(s, AIR_E_NOMEM, "job footprint exceeds the server's device budget");
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->fatal != AIR_OK) {
        delete jb;
        return srv_fail(s, s->fatal, s->fatal_msg);
      }
      if (s->stopping) {
        delete jb;
        return srv_fail(s, AIR_E_BUSY, "server is shutting down");
      }
      jb->res.id = s->next_id++;
      *id_out = jb->res.id;
      s->queue.push_back(jb);
      ++s->submitted;
    }
    s->cv_work.notify_one();
  } catch (...) {
    delete jb;
    return srv_fail(s, AIR_E_NOMEM, "host allocation failed");
  }
  s->err.clear();
  return AIR_OK;
}

int air_server_poll(air_server* s, air_result* out, int max) {
  if (!s || (!out && max > 0) || max < 0) return AIR_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  int n = 0;
  while (n < max && !s->results.empty()) {
    out[n++] = s->results.front();
    s->results.pop_front();
  }
  return n;
}

air_status air_server_drain(air_server* s, int timeout_ms) {
  if (!s) return AIR_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto all_done = [s] { return s->completed == s->submitted; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, all_done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), all_done)) {
    return AIR_E_BUSY;
  }
  return s->fatal;
}

air_status air_server_query(air_server* s, air_server_info* info) {
  if (!s || !info) return AIR_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  info->submitted = s->submitted;
  info->completed = s->completed;
  info->batches = s->batches;
  info->in_use = s->arena.used();
  info->peak_in_use = s->arena.peak();
  info->budget = s->budget;
  info->max_batch = s->max_batch;
  info->queued = (int32_t)s->queue.size();
  return AIR_OK;
}

const char* air_server_last_error(const air_server* s) { return s ? s->err.c_str() : "null server"; }

air_status air_server_destroy(air_server* s) {
  if (!s) return AIR_E_INVAL;
  const air_status st = air_server_drain(s, -1);
  destroy_server(s);
  return st;
}

}  // extern "C"
