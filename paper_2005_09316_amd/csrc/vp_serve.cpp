// vp_serve.cpp -- continuous batching: vp_submit / vp_poll.
//
// A scheduler thread per context admits queued jobs in FIFO order when their
// HBM footprint fits the budget minus what admitted jobs hold (and a job slot
// and ring space are free).  Admission writes the job's arguments into a
// host-mapped slot and appends its items to a host-mapped ring: first table
// items when the job's (sky, observation) pair has no tables yet, then -- once
// the host sees the tables built -- its visibility tiles.  A persistent kernel
// (k_serve) on its own stream claims items from the ring as they appear, so
// jobs that arrive while others run share the device tile by tile.  The
// kernel exits after a short idle period; the scheduler relaunches it when
// items are waiting.  Completion is signalled per job through host-mapped
// flags.
#include <hip/hip_runtime.h>
#include <time.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vp.h"
#include "vp_internal.h"
#include "vp_objects.h"

namespace vp {

static uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

enum JobState { kQueued = 0, kRunning = 1, kDone = 2 };

struct JobRec {
  uint64_t ticket = 0;
  vp_job job{};
  int state = kQueued;
  int status = VP_OK;
  uint64_t t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  uint64_t dev_start = 0, dev_done = 0;  // device wall clock at its first tile's start, last tile's end
  uint64_t footprint = 0;
  int slot = -1;
  uint64_t seq = 0, seq_table = 0;
  int64_t ntiles = 0, ntable = 0;
  DerivedEntry *d = nullptr;
  bool owner = false;     // this job builds the pair's tables
  bool tiles_out = false; // tiles published
};

struct Scheduler {
  vp_ctx *ctx = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool quit = false;
  std::string init_error;
  int init_rc = VP_OK;
  bool init_done = false;
  std::deque<JobRec *> queue;
  std::vector<JobRec *> running;
  std::unordered_map<uint64_t, JobRec *> jobs;
  uint64_t next_ticket = 1, next_seq = 1;
  uint64_t in_use = 0;
  ServeHost *H = nullptr;      // host pointer
  ServeHost *H_dev = nullptr;  // the same memory as seen by the device
  ServeDev *D = nullptr;
  std::vector<int> free_slots;
  std::vector<uint64_t> slot_target, slot_ttarget;
  uint64_t tail = 0, ring_inflight = 0;
  hipStream_t kstream = nullptr, aux = nullptr;
  hipEvent_t kev0 = nullptr, kev = nullptr;  // around each launch of the persistent kernel
  bool launched = false;
  uint64_t launches = 0;   // completed launches
  double resident_ms = 0;  // their total duration
  uint64_t epoch = 0;  // launch counter; workers of a launch exit together
  int grid = 0;
  uint64_t idle_ticks = 0;
};

uint64_t job_footprint(const vp_sky *sky, const vp_obs *obs, int dtype) {
  const uint64_t nvis = (uint64_t)obs->T * obs->B * obs->K;
  const uint64_t J = (uint64_t)sky->P + sky->G + sky->S;
  const uint64_t tables = 32 * (J ? J : 1) + 32 * (sky->G ? sky->G : 1) + 96 * (sky->S ? sky->S : 1) +
                          12 * (J ? J : 1) * (uint64_t)obs->Kpad;
  return nvis * (dtype == VP_C64 ? 8 : 16) + tables;
}

static int check_job(vp_ctx *ctx, const vp_job *job) {
  if (!ctx || !job) return set_error(VP_EINVAL, "NULL context or job");
  if (job->kind != VP_JOB_PREDICT && job->kind != VP_JOB_SUBTRACT)
    return set_error(VP_EINVAL, "unknown job kind %d", job->kind);
  int rc = check_call(ctx, job->sky, job->obs, job->precision, job->dtype, job->vis_dev);
  if (rc != VP_OK) return rc;
  if (job->precision != VP_PREC_MIXED)
    return set_error(VP_EINVAL, "serving runs the mixed-precision path (VP_PREC_MIXED)");
  if (job->sky->max_nmax > kNmaxLimit) return set_error(VP_EINVAL, "shapelet order too large");
  return VP_OK;
}

// --- scheduler thread -------------------------------------------------------

static void finish(Scheduler *s, JobRec *j, int status) {
  j->status = status;
  j->state = kDone;
  j->t_done = now_ns();
  if (j->t_start == 0) j->t_start = j->t_done;
  std::lock_guard<std::mutex> lk(s->ctx->mu);
  const_cast<vp_sky *>(j->job.sky)->jobs -= 1;
  const_cast<vp_obs *>(j->job.obs)->jobs -= 1;
}

static void publish(Scheduler *s, int slot, int64_t n, bool table) {
  const uint64_t flag = table ? (1ull << 47) : 0ull;
  for (int64_t t = 0; t < n; ++t)
    s->H->ring[(s->tail + (uint64_t)t) & (kRingSize - 1)] = ((uint64_t)slot << 48) | flag | (uint64_t)t;
  s->tail += (uint64_t)n;
  std::atomic_thread_fence(std::memory_order_release);
  __atomic_store_n(&s->H->tail, s->tail, __ATOMIC_RELEASE);
}

// Tile phase: the job's tables are ready; publish its tiles under a fresh
// sequence number (workers acquire once per newer sequence number, which
// makes the freshly built tables visible to them).
static void publish_tiles(Scheduler *s, JobRec *j) {
  ServeJobDesc &desc = s->H->jobs[j->slot];
  j->seq = s->next_seq++;
  s->slot_target[j->slot] += (uint64_t)j->ntiles;
  desc.seq = j->seq;
  desc.done_target = s->slot_target[j->slot];
  std::atomic_thread_fence(std::memory_order_release);
  publish(s, j->slot, j->ntiles, false);
  j->tiles_out = true;
}

static int admit(Scheduler *s, JobRec *j) {
  vp_ctx *ctx = s->ctx;
  const vp_sky *sky = j->job.sky;
  const vp_obs *obs = j->job.obs;
  DerivedEntry *d = nullptr;
  bool build = false;
  int rc = serve_derived(ctx, sky, obs, &d, &build);
  if (rc != VP_OK) return rc;
  TileArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nrows = (int64_t)obs->T * obs->B;
  a.K = obs->K;
  a.Kpad = obs->Kpad;
  a.uvw = obs->uvw;
  a.fk = obs->fk;
  a.P = sky->P;
  a.G = sky->G;
  a.S = sky->S;
  a.d = d->d;
  a.t = sky->tiles;
  a.vis = j->job.vis_dev;
  a.subtract = j->job.kind == VP_JOB_SUBTRACT;
  a.c64 = j->job.dtype == VP_C64;
  a.conj = obs->sign < 0;
  a.n_rb = (int)((a.nrows + kTileRows - 1) / kTileRows);
  a.n_cb = obs->Kpad / kPgChan;
  a.dfk = obs->dfk;
  a.uniform = obs->uniform;
  a.fresh = 0;
  const int slot = s->free_slots.back();
  s->free_slots.pop_back();
  j->slot = slot;
  j->d = d;
  ServeJobDesc &desc = s->H->jobs[slot];
  desc.a = a;
  desc.ntiles = j->ntiles;
  desc.ntable = 0;
  s->ring_inflight += (uint64_t)j->ntiles;
  s->in_use += j->footprint;
  j->t_admit = now_ns();
  j->state = kRunning;
  const int J = sky->P + sky->G + sky->S;
  if (build && J == 0) {
    derived_built(ctx, d);
    build = false;
  }
  if (build) {
    // table phase: the persistent kernel builds the pair's tables
    j->owner = true;
    j->ntable = (int64_t)(J + kTileRows - 1) / kTileRows + ((int64_t)J * obs->Kpad + kTileRows - 1) / kTileRows;
    j->seq_table = s->next_seq++;
    s->slot_ttarget[slot] += (uint64_t)j->ntable;
    desc.da = make_derive_args(sky, obs, d->d);
    desc.fa = make_flux_args(sky, obs, d->d);
    desc.ntable = j->ntable;
    desc.seq_table = j->seq_table;
    desc.table_target = s->slot_ttarget[slot];
    s->ring_inflight += (uint64_t)j->ntable;
    std::atomic_thread_fence(std::memory_order_release);
    publish(s, slot, j->ntable, true);
  } else if (derived_ready(ctx, d)) {
    publish_tiles(s, j);
  }
  return VP_OK;
}

// A finished launch of the persistent kernel is counted (launches, resident
// time) and forgotten; hipErrorNotReady while it runs, its error if it failed.
static hipError_t reap_kernel(Scheduler *s) {
  if (!s->launched) return hipSuccess;
  hipError_t q = hipEventQuery(s->kev);
  if (q == hipErrorNotReady) return q;
  s->launched = false;
  if (q != hipSuccess) return q;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, s->kev0, s->kev) == hipSuccess) s->resident_ms += ms;
  s->launches += 1;
  return hipSuccess;
}

static int ensure_kernel(Scheduler *s) {
  const hipError_t q = reap_kernel(s);
  if (q == hipErrorNotReady) return VP_OK;
  if (q != hipSuccess) return hip_error(q, "serving kernel");
  uint64_t head = 0;
  hipError_t e = hipMemcpyAsync(&head, &s->D->head, sizeof(head), hipMemcpyDeviceToHost, s->aux);
  if (e == hipSuccess) e = hipStreamSynchronize(s->aux);
  if (e != hipSuccess) return hip_error(e, "reading the serving queue head");
  if (head >= s->tail) return VP_OK;
  e = hipEventRecord(s->kev0, s->kstream);
  if (e == hipSuccess) e = launch_serve(s->H_dev, s->D, s->idle_ticks, ++s->epoch, s->grid, s->kstream);
  if (e == hipSuccess) e = hipEventRecord(s->kev, s->kstream);
  if (e != hipSuccess) return hip_error(e, "launching the serving kernel");
  s->launched = true;
  return VP_OK;
}

// The persistent kernel could not be launched, or its launch failed on the
// device: every running job ends with that error (their tiles share the
// kernel).  No kernel runs now.  The items still in the ring are retired
// (head = tail) so that a later launch does not run them into buffers their
// callers may have freed; tables that were to be built are dropped rather than
// marked ready; each slot's completion targets are re-read from the device
// counters, which count only the items that ran, before the slot is reused
// (a slot whose counters cannot be read stays out of use).
static void abandon_running(Scheduler *s, int rc) {
  bool synced = false;
  std::vector<uint64_t> done(kServeSlots), tdone(kServeSlots);
  {
    const uint64_t tail = s->tail;
    hipError_t e = hipMemcpyAsync(&s->D->head, &tail, sizeof(tail), hipMemcpyHostToDevice, s->aux);
    if (e == hipSuccess) e = hipMemcpyAsync(done.data(), s->D->done, sizeof(uint64_t) * kServeSlots,
                                            hipMemcpyDeviceToHost, s->aux);
    if (e == hipSuccess) e = hipMemcpyAsync(tdone.data(), s->D->tdone, sizeof(uint64_t) * kServeSlots,
                                            hipMemcpyDeviceToHost, s->aux);
    if (e == hipSuccess) e = hipStreamSynchronize(s->aux);
    synced = e == hipSuccess;
  }
  // jobs waiting for tables that an abandoned owner was to build let go of
  // them before the owner drops them
  for (JobRec *j : s->running)
    if (!j->owner) serve_release_derived(s->ctx, j->d);
  for (JobRec *j : s->running)
    if (j->owner) serve_abandon_derived(s->ctx, j->d);
  for (JobRec *j : s->running) {
    s->in_use -= j->footprint;
    s->ring_inflight -= (uint64_t)(j->ntiles + j->ntable);
    if (synced) {
      s->slot_target[j->slot] = done[j->slot];
      s->slot_ttarget[j->slot] = tdone[j->slot];
      s->free_slots.push_back(j->slot);
    }
    finish(s, j, rc);
  }
  s->running.clear();
}

static void scheduler_loop(Scheduler *s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // completions
    for (size_t i = 0; i < s->running.size();) {
      JobRec *j = s->running[i];
      if (!j->tiles_out) {
        if (j->owner && __atomic_load_n(&s->H->tabled[j->slot], __ATOMIC_ACQUIRE) == j->seq_table) {
          derived_built(s->ctx, j->d);
          j->owner = false;
        }
        if (!j->owner && derived_ready(s->ctx, j->d)) publish_tiles(s, j);
        ++i;
        continue;
      }
      const uint64_t st = __atomic_load_n(&s->H->started[j->slot], __ATOMIC_ACQUIRE);
      if (j->t_start == 0 && st == j->seq) {
        j->t_start = now_ns();
        j->dev_start = __atomic_load_n(&s->H->started_clk[j->slot], __ATOMIC_RELAXED);
      }
      const uint64_t fin = __atomic_load_n(&s->H->finished[j->slot], __ATOMIC_ACQUIRE);
      if (fin == j->seq) {
        if (j->dev_start == 0) j->dev_start = __atomic_load_n(&s->H->started_clk[j->slot], __ATOMIC_RELAXED);
        j->dev_done = __atomic_load_n(&s->H->finished_clk[j->slot], __ATOMIC_RELAXED);
        s->in_use -= j->footprint;
        s->ring_inflight -= (uint64_t)(j->ntiles + j->ntable);
        s->free_slots.push_back(j->slot);
        serve_release_derived(s->ctx, j->d);
        finish(s, j, VP_OK);
        s->running[i] = s->running.back();
        s->running.pop_back();
      } else {
        ++i;
      }
    }
    // admissions, FIFO
    while (!s->queue.empty()) {
      JobRec *j = s->queue.front();
      const uint64_t J = (uint64_t)j->job.sky->P + j->job.sky->G + j->job.sky->S;
      const uint64_t table_items = (J + kTileRows - 1) / kTileRows + (J * j->job.obs->Kpad + kTileRows - 1) / kTileRows;
      if (s->free_slots.empty() || s->ring_inflight + (uint64_t)j->ntiles + table_items > kRingSize) break;
      // the budget covers admitted jobs and the tables that finished serving
      // jobs built and nothing else uses; those are released when they stand
      // in the way of the next job
      if (s->in_use + j->footprint > s->ctx->budget) break;
      if (s->in_use + serve_evictable_bytes(s->ctx) + j->footprint > s->ctx->budget) {
        serve_evict(s->ctx);
        if (s->in_use + serve_evictable_bytes(s->ctx) + j->footprint > s->ctx->budget) break;
      }
      s->queue.pop_front();
      int rc = admit(s, j);
      if (rc != VP_OK)
        finish(s, j, rc);
      else
        s->running.push_back(j);
    }
    if (!s->running.empty()) {
      int rc = ensure_kernel(s);
      if (rc != VP_OK) abandon_running(s, rc);
    } else if (s->launched && hipEventQuery(s->kev) == hipSuccess) {
      (void)reap_kernel(s);  // idle: count the launch that just exited
    }
    if (s->quit && s->queue.empty() && s->running.empty()) break;
    if (s->queue.empty() && s->running.empty())
      s->cv.wait_for(lk, std::chrono::milliseconds(2));
    else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

static int start_scheduler(vp_ctx *ctx, Scheduler **out) {
  Scheduler *s = new Scheduler();
  s->ctx = ctx;
  DeviceGuard g(ctx->device);
  hipError_t e = hipHostMalloc((void **)&s->H, sizeof(ServeHost), hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    std::memset(s->H, 0, sizeof(ServeHost));
    e = hipHostGetDevicePointer((void **)&s->H_dev, s->H, 0);
  }
  if (e == hipSuccess) e = hipMalloc((void **)&s->D, sizeof(ServeDev));
  if (e == hipSuccess) e = hipMemset(s->D, 0, sizeof(ServeDev));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->kstream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&s->kev0);
  if (e == hipSuccess) e = hipEventCreate(&s->kev);
  if (e == hipSuccess) e = serve_grid(&s->grid);
  int rate_khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    int rc = hip_error(e, "starting the serving scheduler");
    if (s->kev) (void)hipEventDestroy(s->kev);
    if (s->kev0) (void)hipEventDestroy(s->kev0);
    if (s->aux) (void)hipStreamDestroy(s->aux);
    if (s->kstream) (void)hipStreamDestroy(s->kstream);
    if (s->D) (void)hipFree(s->D);
    if (s->H) (void)hipHostFree(s->H);
    delete s;
    return rc;
  }
  // the workgroups exit together after 2 ms without work (the device is then
  // free for other kernels); the scheduler relaunches when items wait
  s->idle_ticks = (uint64_t)(rate_khz > 0 ? rate_khz : 100000) * 2;
  s->slot_target.assign(kServeSlots, 0);
  s->slot_ttarget.assign(kServeSlots, 0);
  for (int i = kServeSlots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->th = std::thread(scheduler_loop, s);
  *out = s;
  return VP_OK;
}

bool serve_pending(vp_ctx *ctx) {
  Scheduler *s = ctx->sched;
  if (!s) return false;
  std::lock_guard<std::mutex> lk(s->mu);
  return !s->queue.empty() || !s->running.empty();
}

void serve_shutdown(vp_ctx *ctx) {
  Scheduler *s = ctx->sched;
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->quit = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  DeviceGuard g(ctx->device);
  __atomic_store_n(&s->H->stop, 1ull, __ATOMIC_RELEASE);
  if (s->launched) (void)hipEventSynchronize(s->kev);
  (void)hipStreamSynchronize(s->kstream);
  (void)hipStreamSynchronize(s->aux);
  for (auto &kv : s->jobs) delete kv.second;
  (void)hipEventDestroy(s->kev);
  (void)hipEventDestroy(s->kev0);
  (void)hipStreamDestroy(s->aux);
  (void)hipStreamDestroy(s->kstream);
  (void)hipFree(s->D);
  (void)hipHostFree(s->H);
  delete s;
  ctx->sched = nullptr;
}

}  // namespace vp

using namespace vp;

extern "C" {

int vp_job_footprint(vp_ctx *ctx, const vp_job *job, uint64_t *bytes) {
  if (!bytes) return set_error(VP_EINVAL, "NULL out");
  if (!ctx || !job || !job->sky || !job->obs) return set_error(VP_EINVAL, "NULL context, job, sky or observation");
  if (job->dtype != VP_C128 && job->dtype != VP_C64) return set_error(VP_EINVAL, "unknown dtype %d", job->dtype);
  *bytes = job_footprint(job->sky, job->obs, job->dtype);
  return VP_OK;
}

int vp_submit(vp_ctx *ctx, const vp_job *job, uint64_t *ticket) {
  if (!ticket) return set_error(VP_EINVAL, "NULL ticket");
  int rc = check_job(ctx, job);
  if (rc != VP_OK) return rc;
  const uint64_t fp = job_footprint(job->sky, job->obs, job->dtype);
  if (fp > ctx->budget)
    return set_error(VP_ECAPACITY, "job footprint %llu bytes exceeds the HBM budget %llu", (unsigned long long)fp,
                     (unsigned long long)ctx->budget);
  const int64_t ntiles = (int64_t)(((int64_t)job->obs->T * job->obs->B + kTileRows - 1) / kTileRows) *
                         (job->obs->Kpad / kPgChan);
  if ((uint64_t)ntiles > kRingSize || ntiles >= ((int64_t)1 << 48))
    return set_error(VP_ECAPACITY, "job has %lld tiles, more than the serving ring holds", (long long)ntiles);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->sched) {
      Scheduler *s = nullptr;
      rc = start_scheduler(ctx, &s);
      if (rc != VP_OK) return rc;
      ctx->sched = s;
    }
  }
  Scheduler *s = ctx->sched;
  JobRec *j = new JobRec();
  j->job = *job;
  j->t_submit = now_ns();
  if (j->job.t_arrival_ns == 0) j->job.t_arrival_ns = j->t_submit;
  j->footprint = fp;
  j->ntiles = ntiles;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    {
      std::lock_guard<std::mutex> lk2(ctx->mu);
      const_cast<vp_sky *>(job->sky)->jobs += 1;
      const_cast<vp_obs *>(job->obs)->jobs += 1;
    }
    j->ticket = s->next_ticket++;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
  }
  s->cv.notify_all();
  return VP_OK;
}

int vp_serve_stats(vp_ctx *ctx, uint64_t *launches, double *resident_ms) {
  if (!ctx || !launches || !resident_ms) return set_error(VP_EINVAL, "NULL argument");
  Scheduler *s = ctx->sched;
  if (!s) {
    *launches = 0;
    *resident_ms = 0.0;
    return VP_OK;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  *launches = s->launches;
  *resident_ms = s->resident_ms;
  return VP_OK;
}

int vp_poll(vp_ctx *ctx, uint64_t ticket, vp_job_result *res) {
  if (!ctx || !res) return set_error(VP_EINVAL, "NULL context or result");
  Scheduler *s = ctx->sched;
  if (!s) return set_error(VP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return set_error(VP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  JobRec *j = it->second;
  if (j->state != kDone) return VP_EAGAIN;
  res->status = j->status;
  res->t_submit = j->t_submit;
  res->t_admit = j->t_admit;
  res->t_start = j->t_start;
  res->t_done = j->t_done;
  res->dev_first_tile = j->dev_start;
  res->dev_last_tile = j->dev_done;
  s->jobs.erase(it);
  delete j;
  return VP_OK;
}

}  // extern "C"
