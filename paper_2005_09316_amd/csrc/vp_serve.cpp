// vp_serve.cpp -- continuous batching: vp_submit / vp_poll.
//
// The scheduling policy (FIFO admission by HBM footprint, tickets, the
// scheduler thread) is ServeCore (serve_core.cpp); this file is its device
// side.  Admission writes the job's arguments into a host-mapped slot; the
// job then runs in up to three phases, each published as items on a
// host-mapped ring once the previous phase is seen done: table items when the
// job's (sky, observation) pair has no tables yet, the point/Gaussian tiles
// (both on ring 0), and the shapelet tiles (ring 1), which read what the
// point/Gaussian tiles wrote.  Each ring has a persistent kernel (k_serve_pg,
// k_serve_shp) that claims items as they appear, so jobs that arrive while
// others run share the device tile by tile.  The two kernels are launched on
// one stream, ring 0's first, each only when its ring holds items (or ring 1
// is about to), and exit after a short idle period; the scheduler relaunches
// them while items wait.  Completion is signalled per job through
// host-mapped flags.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/vp.h"
#include "serve_core.h"
#include "vp_internal.h"
#include "vp_objects.h"

namespace vp {

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

// Units behind one ring entry.  Every claim is a device-wide atomic, and the
// claims of a burst are served one after another, so a phase gets as few
// entries as its balance allows.  Tiles: one per entry while the phase has no
// more tiles than the kernel has workgroups; one entry per workgroup up to
// four times that; beyond, four entries per workgroup (their costs vary, and
// the last ones set the phase's end) of at most kMaxRun tiles (so that jobs
// queued behind wait for runs of bounded length).  Table units cost alike and
// little (a few microseconds each): kTableEntries entries per phase.
constexpr int64_t kMaxRun = 64;
static int64_t run_length(int64_t units, int grid) {
  const int64_t g = std::max(grid, 1);
  const int64_t e = units <= g ? std::max<int64_t>(units, 1) : (units <= 4 * g ? g : 4 * g);  // entries
  return std::max<int64_t>(1, std::min<int64_t>(kMaxRun, (units + e - 1) / e));
}
constexpr int64_t kTableEntries = 64;
static int64_t table_run_length(int64_t units) {
  return std::max<int64_t>(1, (units + kTableEntries - 1) / kTableEntries);
}
static int64_t entries(int64_t units, int64_t run) { return (units + run - 1) / run; }

static int64_t table_items(const vp_sky *sky, const vp_obs *obs) {
  const int64_t J = (int64_t)sky->P + sky->G + sky->S;
  return (J + kTileRows - 1) / kTileRows + (J * obs->Kpad + kTileRows - 1) / kTileRows;
}

// What the device side keeps per job.
enum JobPhase { kPhTables = 0, kPhPg = 1, kPhShp = 2 };

struct JobExt {
  vp_job job{};
  int slot = -1;
  uint64_t seq = 0, seq_shp = 0, seq_table = 0;
  int64_t ntiles = 0;                       // tiles of each pass
  int64_t ntable = 0;                       // table units, when the job builds its tables
  int64_t run_pg = 1, run_shp = 1, run_table = 1;  // units per ring entry
  int64_t e_pg = 0, e_shp = 0, e_table = 0;        // ring entries per phase (e_table: once building)
  int64_t e_table_max = 0;                  // table entries, should the job build its tables
  DerivedEntry *d = nullptr;
  bool owner = false;     // this job builds the pair's tables
  bool shp = false;       // the job has a shapelet phase
  int phase = kPhTables;  // the phase published last (kPhTables: tiles not yet published)
  uint64_t ring_items(int r) const { return r == 0 ? (uint64_t)(e_pg + e_table) : (shp ? (uint64_t)e_shp : 0); }
};

static JobExt &ext(CoreJob &j) { return *(JobExt *)j.payload; }

class HipExecutor : public ServeExecutor {
 public:
  vp_ctx *ctx = nullptr;
  ServeHost *H = nullptr;      // host pointer
  ServeHost *H_dev = nullptr;  // the same memory as seen by the device
  ServeDev *D = nullptr;
  std::vector<int> free_slots;
  std::vector<uint64_t> slot_target, slot_ttarget;
  uint64_t tail[kServeRings] = {0, 0}, ring_inflight[kServeRings] = {0, 0}, next_seq = 1;
  int shp_expected = 0;  // running jobs in their point/Gaussian phase with a shapelet phase to come
  hipStream_t kstream = nullptr, aux = nullptr;
  hipEvent_t kev0 = nullptr, kev = nullptr;  // around each launch group
  bool launched = false;
  int group_kernels = 0;  // kernels in the launch group in flight
  uint64_t epoch = 0;     // launch counter; workers of a launch exit together
  int grid[kServeRings] = {0, 0};
  uint64_t idle_ticks = 0;
  std::mutex stats_mu;     // launches and resident_ms, read by vp_serve_stats
  uint64_t launches = 0;   // completed kernel launches
  double resident_ms = 0;  // total duration of their launch groups

  int init(vp_ctx *c);
  void teardown();

  void thread_start() override { (void)hipSetDevice(ctx->device); }
  bool has_room(const CoreJob &j) override;
  uint64_t evictable_bytes() override { return serve_evictable_bytes(ctx); }
  void evict() override { serve_evict(ctx); }
  int admit(CoreJob &j) override;
  bool poll(CoreJob &j) override;
  int kick() override;
  void idle() override;
  void abandon(const std::vector<CoreJob *> &running, int rc) override;
  void finished(CoreJob &j) override;
  void retired(CoreJob &j) override;

 private:
  void publish(int ring, int slot, int64_t n, bool table);
  void publish_tiles(JobExt &x);
  void publish_shp(JobExt &x);
  hipError_t reap_kernel();
};

struct Scheduler {
  HipExecutor ex;
  ServeCore *core = nullptr;
};

bool HipExecutor::has_room(const CoreJob &j) {
  const JobExt &x = *(const JobExt *)j.payload;
  const uint64_t need1 = x.ring_items(1);
  const uint64_t need0 = (uint64_t)(x.e_pg + x.e_table_max);  // at most
  return !free_slots.empty() && ring_inflight[0] + need0 <= kRingSize && ring_inflight[1] + need1 <= kRingSize;
}

void HipExecutor::publish(int ring, int slot, int64_t n, bool table) {
  const uint64_t flag = table ? (1ull << 47) : 0ull;
  for (int64_t t = 0; t < n; ++t)
    H->ring[ring][(tail[ring] + (uint64_t)t) & (kRingSize - 1)] = ((uint64_t)slot << 48) | flag | (uint64_t)t;
  tail[ring] += (uint64_t)n;
  std::atomic_thread_fence(std::memory_order_release);
  __atomic_store_n(&H->tail[ring], tail[ring], __ATOMIC_RELEASE);
}

// Point/Gaussian phase: the job's tables are ready; publish its tiles under a
// fresh sequence number (workers acquire once per newer sequence number,
// which makes the freshly built tables visible to them).
void HipExecutor::publish_tiles(JobExt &x) {
  ServeJobDesc &desc = H->jobs[x.slot];
  x.seq = next_seq++;
  slot_target[x.slot] += (uint64_t)x.e_pg;
  desc.seq = x.seq;
  desc.done_target = slot_target[x.slot];
  std::atomic_thread_fence(std::memory_order_release);
  publish(0, x.slot, x.e_pg, false);
  x.phase = kPhPg;
  if (x.shp) ++shp_expected;
}

// Shapelet phase: every point/Gaussian tile of the job is written back; its
// shapelet tiles add to them.  They run in a launch of ring 1's kernel that
// starts after the ring-0 launch that wrote those tiles has ended (the two
// kernels share one stream), so no worker holds an older copy of them.
void HipExecutor::publish_shp(JobExt &x) {
  ServeJobDesc &desc = H->jobs[x.slot];
  x.seq_shp = next_seq++;
  slot_target[x.slot] += (uint64_t)x.e_shp;
  desc.seq_shp = x.seq_shp;
  desc.shp_target = slot_target[x.slot];
  std::atomic_thread_fence(std::memory_order_release);
  publish(1, x.slot, x.e_shp, false);
  x.phase = kPhShp;
  --shp_expected;
}

int HipExecutor::admit(CoreJob &j) {
  JobExt &x = ext(j);
  const vp_sky *sky = x.job.sky;
  const vp_obs *obs = x.job.obs;
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
  a.vis = x.job.vis_dev;
  a.subtract = x.job.kind == VP_JOB_SUBTRACT;
  a.c64 = x.job.dtype == VP_C64;
  a.conj = obs->sign < 0;
  a.n_rb = (int)((a.nrows + kTileRows - 1) / kTileRows);
  a.n_cb = obs->Kpad / kPgChan;
  a.dfk = obs->dfk;
  a.uniform = obs->uniform;
  a.fresh = 0;
  const int slot = free_slots.back();
  free_slots.pop_back();
  x.slot = slot;
  x.d = d;
  ServeJobDesc &desc = H->jobs[slot];
  desc.a = a;
  desc.ntiles = x.ntiles;
  desc.ntable = 0;
  desc.per_pg = x.run_pg;
  desc.per_shp = x.run_shp;
  desc.per_table = x.run_table;
  const int J = sky->P + sky->G + sky->S;
  if (build && J == 0) {
    derived_built(ctx, d);
    build = false;
  }
  if (build) {
    // table phase: the persistent kernel builds the pair's tables
    x.owner = true;
    x.ntable = table_items(sky, obs);
    x.e_table = x.e_table_max;
    x.seq_table = next_seq++;
    slot_ttarget[slot] += (uint64_t)x.e_table;
    desc.da = make_derive_args(sky, obs, d->d);
    desc.fa = make_flux_args(sky, obs, d->d);
    desc.ntable = x.ntable;
    desc.seq_table = x.seq_table;
    desc.table_target = slot_ttarget[slot];
    std::atomic_thread_fence(std::memory_order_release);
    publish(0, slot, x.e_table, true);
  } else if (derived_ready(ctx, d)) {
    publish_tiles(x);
  }
  ring_inflight[0] += x.ring_items(0);
  ring_inflight[1] += x.ring_items(1);
  return VP_OK;
}

bool HipExecutor::poll(CoreJob &j) {
  JobExt &x = ext(j);
  if (x.phase == kPhTables) {
    if (x.owner && __atomic_load_n(&H->tabled[x.slot], __ATOMIC_ACQUIRE) == x.seq_table) {
      derived_built(ctx, x.d);
      x.owner = false;
    }
    if (!x.owner && derived_ready(ctx, x.d)) publish_tiles(x);
    return false;
  }
  if (j.t_start == 0 && __atomic_load_n(&H->started[x.slot], __ATOMIC_ACQUIRE) == x.seq) {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    j.t_start = (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
    j.dev_start = __atomic_load_n(&H->started_clk[x.slot], __ATOMIC_RELAXED);
  }
  const uint64_t fin = __atomic_load_n(&H->finished[x.slot], __ATOMIC_ACQUIRE);
  if (x.phase == kPhPg) {
    if (fin != x.seq) return false;
    if (x.shp) {
      publish_shp(x);
      return false;
    }
  } else if (fin != x.seq_shp) {
    return false;
  }
  if (j.dev_start == 0) j.dev_start = __atomic_load_n(&H->started_clk[x.slot], __ATOMIC_RELAXED);
  j.dev_done = __atomic_load_n(&H->finished_clk[x.slot], __ATOMIC_RELAXED);
  j.status = VP_OK;
  return true;
}

void HipExecutor::finished(CoreJob &j) {
  JobExt &x = ext(j);
  ring_inflight[0] -= x.ring_items(0);
  ring_inflight[1] -= x.ring_items(1);
  free_slots.push_back(x.slot);
  serve_release_derived(ctx, x.d);
}

void HipExecutor::retired(CoreJob &j) {
  JobExt *x = (JobExt *)j.payload;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const_cast<vp_sky *>(x->job.sky)->jobs -= 1;
    const_cast<vp_obs *>(x->job.obs)->jobs -= 1;
  }
  delete x;
  j.payload = nullptr;
}

// A finished launch group is counted (kernel launches, resident time) and
// forgotten; hipErrorNotReady while it runs, its error if it failed.
hipError_t HipExecutor::reap_kernel() {
  if (!launched) return hipSuccess;
  hipError_t q = hipEventQuery(kev);
  if (q == hipErrorNotReady) return q;
  launched = false;
  if (q != hipSuccess) return q;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, kev0, kev) != hipSuccess) ms = 0.f;
  std::lock_guard<std::mutex> lk(stats_mu);
  resident_ms += ms;
  launches += (uint64_t)group_kernels;
  return hipSuccess;
}

// Launches, one after the other on the kernel stream, ring 0's kernel when its
// ring holds unclaimed items and ring 1's when its ring does or a running
// job's shapelet phase is about to be published (it is then usually published
// while ring 0's kernel finishes).  Nothing is launched while a group runs.
int HipExecutor::kick() {
  const hipError_t q = reap_kernel();
  if (q == hipErrorNotReady) return VP_OK;
  if (q != hipSuccess) return hip_error(q, "serving kernel");
  uint64_t head[kServeRings] = {0, 0};
  hipError_t e = hipMemcpyAsync(head, D->head, sizeof(head), hipMemcpyDeviceToHost, aux);
  if (e == hipSuccess) e = hipStreamSynchronize(aux);
  if (e != hipSuccess) return hip_error(e, "reading the serving queue heads");
  const bool run0 = head[0] < tail[0];
  const bool run1 = head[1] < tail[1] || (run0 && shp_expected > 0);
  if (!run0 && !run1) return VP_OK;
  TraceRange tr(run0 ? (run1 ? "vp_serve launch: rings 0, 1" : "vp_serve launch: ring 0") : "vp_serve launch: ring 1");
  group_kernels = 0;
  e = hipEventRecord(kev0, kstream);
  for (int r = 0; r < kServeRings && e == hipSuccess; ++r) {
    if (!(r == 0 ? run0 : run1)) continue;
    e = launch_serve(r, H_dev, D, idle_ticks, ++epoch, grid[r], kstream);
    if (e == hipSuccess) ++group_kernels;
  }
  if (e == hipSuccess) e = hipEventRecord(kev, kstream);
  // a launch that was enqueued is waited for by the event even when a later
  // call failed; the group counts as launched as soon as one kernel is
  launched = group_kernels > 0 && e == hipSuccess;
  if (e != hipSuccess) return hip_error(e, "launching the serving kernels");
  return VP_OK;
}

void HipExecutor::idle() {
  // count a launch group that exited while nothing ran; an error stays with
  // the event and surfaces at the next kick()
  if (launched && hipEventQuery(kev) == hipSuccess) (void)reap_kernel();
}

// The serving kernels could not be launched, or a launch failed on the
// device: every running job ends with that error (their tiles share the
// kernels).  No kernel runs now.  The items still in the rings are retired
// (head = tail) so that a later launch does not run them into buffers their
// callers may have freed; tables that were to be built are dropped rather than
// marked ready; each slot's completion targets are re-read from the device
// counters, which count only the items that ran, before the slot is reused
// (a slot whose counters cannot be read stays out of use).
void HipExecutor::abandon(const std::vector<CoreJob *> &running, int rc) {
  (void)rc;
  if (launched) (void)hipEventSynchronize(kev);
  (void)hipStreamSynchronize(kstream);
  launched = false;
  bool synced = false;
  std::vector<uint64_t> done(kServeSlots), tdone(kServeSlots);
  {
    hipError_t e = hipMemcpyAsync(D->head, tail, sizeof(tail), hipMemcpyHostToDevice, aux);
    if (e == hipSuccess)
      e = hipMemcpyAsync(done.data(), D->done, sizeof(uint64_t) * kServeSlots, hipMemcpyDeviceToHost, aux);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tdone.data(), D->tdone, sizeof(uint64_t) * kServeSlots, hipMemcpyDeviceToHost, aux);
    if (e == hipSuccess) e = hipStreamSynchronize(aux);
    synced = e == hipSuccess;
  }
  // jobs waiting for tables that an abandoned owner was to build let go of
  // them before the owner drops them
  for (CoreJob *j : running)
    if (!ext(*j).owner) serve_release_derived(ctx, ext(*j).d);
  for (CoreJob *j : running)
    if (ext(*j).owner) serve_abandon_derived(ctx, ext(*j).d);
  for (CoreJob *j : running) {
    JobExt &x = ext(*j);
    ring_inflight[0] -= x.ring_items(0);
    ring_inflight[1] -= x.ring_items(1);
    if (x.phase == kPhPg && x.shp) --shp_expected;
    if (synced) {
      slot_target[x.slot] = done[x.slot];
      slot_ttarget[x.slot] = tdone[x.slot];
      free_slots.push_back(x.slot);
    }
  }
}

int HipExecutor::init(vp_ctx *c) {
  ctx = c;
  DeviceGuard g(ctx->device);
  hipError_t e = hipHostMalloc((void **)&H, sizeof(ServeHost), hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    std::memset(H, 0, sizeof(ServeHost));
    e = hipHostGetDevicePointer((void **)&H_dev, H, 0);
  }
  if (e == hipSuccess) e = hipMalloc((void **)&D, sizeof(ServeDev));
  if (e == hipSuccess) e = hipMemset(D, 0, sizeof(ServeDev));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&kstream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&kev0);
  if (e == hipSuccess) e = hipEventCreate(&kev);
  for (int r = 0; r < kServeRings && e == hipSuccess; ++r) e = serve_grid(r, &grid[r]);
  int rate_khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    int rc = hip_error(e, "starting the serving scheduler");
    teardown();
    return rc;
  }
  // a launch's workgroups exit together after 100 us without work: the
  // other ring's kernel, queued behind it, then runs (and the device is free
  // for other kernels); the scheduler relaunches while items wait
  idle_ticks = (uint64_t)(rate_khz > 0 ? rate_khz : 100000) / 10;
  slot_target.assign(kServeSlots, 0);
  slot_ttarget.assign(kServeSlots, 0);
  for (int i = kServeSlots - 1; i >= 0; --i) free_slots.push_back(i);
  return VP_OK;
}

void HipExecutor::teardown() {
  DeviceGuard g(ctx->device);
  if (H) __atomic_store_n(&H->stop, 1ull, __ATOMIC_RELEASE);
  if (launched) (void)hipEventSynchronize(kev);
  if (kstream) (void)hipStreamSynchronize(kstream);
  if (aux) (void)hipStreamSynchronize(aux);
  if (kev) (void)hipEventDestroy(kev);
  if (kev0) (void)hipEventDestroy(kev0);
  if (aux) (void)hipStreamDestroy(aux);
  if (kstream) (void)hipStreamDestroy(kstream);
  if (D) (void)hipFree(D);
  if (H) (void)hipHostFree(H);
  kev = kev0 = nullptr;
  aux = kstream = nullptr;
  D = nullptr;
  H = H_dev = nullptr;
  launched = false;
}

bool serve_pending(vp_ctx *ctx) {
  Scheduler *s = ctx->sched.load(std::memory_order_acquire);
  return s && s->core->pending();
}

void serve_shutdown(vp_ctx *ctx) {
  Scheduler *s = ctx->sched.exchange(nullptr, std::memory_order_acq_rel);
  if (!s) return;
  // not under ctx->mu: the scheduler thread takes it while retiring jobs
  delete s->core;  // drains (nothing is pending here) and stops the thread
  s->ex.teardown();
  delete s;
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
  TraceRange tr("vp_submit");
  if (!ticket) return set_error(VP_EINVAL, "NULL ticket");
  int rc = check_job(ctx, job);
  if (rc != VP_OK) return rc;
  const uint64_t fp = job_footprint(job->sky, job->obs, job->dtype);
  if (fp > ctx->budget)
    return set_error(VP_ECAPACITY, "job footprint %llu bytes exceeds the HBM budget %llu", (unsigned long long)fp,
                     (unsigned long long)ctx->budget);
  const int64_t ntiles = (int64_t)(((int64_t)job->obs->T * job->obs->B + kTileRows - 1) / kTileRows) *
                         (job->obs->Kpad / kPgChan);
  Scheduler *s = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    s = ctx->sched.load(std::memory_order_relaxed);
    if (!s) {
      Scheduler *n = new Scheduler();
      rc = n->ex.init(ctx);
      if (rc != VP_OK) {
        delete n;
        return rc;
      }
      n->core = new ServeCore(&n->ex, ctx->budget);
      ctx->sched.store(n, std::memory_order_release);
      s = n;
    }
  }
  JobExt *x = new JobExt();
  x->job = *job;
  x->ntiles = ntiles;
  x->shp = job->sky->S > 0;
  x->run_pg = run_length(ntiles, s->ex.grid[0]);
  x->run_shp = run_length(ntiles, s->ex.grid[1]);
  x->e_pg = entries(ntiles, x->run_pg);
  x->e_shp = entries(ntiles, x->run_shp);
  const int64_t tunits = table_items(job->sky, job->obs);
  x->run_table = table_run_length(tunits);
  x->e_table_max = entries(tunits, x->run_table);
  if ((uint64_t)(x->e_pg + x->e_table_max) > kRingSize || (uint64_t)x->e_shp > kRingSize ||
      ntiles >= ((int64_t)1 << 40)) {
    delete x;
    return set_error(VP_ECAPACITY, "job has %lld tiles, more than the serving ring holds", (long long)ntiles);
  }
  {
    // the job holds its sky and observation from here until it retires
    std::lock_guard<std::mutex> lk(ctx->mu);
    const_cast<vp_sky *>(job->sky)->jobs += 1;
    const_cast<vp_obs *>(job->obs)->jobs += 1;
  }
  if (x->job.t_arrival_ns == 0) {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    x->job.t_arrival_ns = (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
  }
  CoreJob *j = new CoreJob();
  j->footprint = fp;
  j->payload = x;
  rc = s->core->submit(j, ticket);
  if (rc != VP_OK) {  // not reached: the footprint was checked above
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      const_cast<vp_sky *>(job->sky)->jobs -= 1;
      const_cast<vp_obs *>(job->obs)->jobs -= 1;
    }
    delete x;
    delete j;
    return set_error(rc, "job refused by the scheduler");
  }
  return VP_OK;
}

int vp_poll(vp_ctx *ctx, uint64_t ticket, vp_job_result *res) {
  if (!ctx || !res) return set_error(VP_EINVAL, "NULL context or result");
  Scheduler *s = ctx->sched.load(std::memory_order_acquire);
  if (!s) return set_error(VP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  CoreJob j;
  const int rc = s->core->poll(ticket, &j);
  if (rc == VP_ENOTFOUND) return set_error(VP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  if (rc != VP_OK) return rc;
  res->status = j.status;
  res->t_submit = j.t_submit;
  res->t_admit = j.t_admit;
  res->t_start = j.t_start;
  res->t_done = j.t_done;
  res->dev_first_tile = j.dev_start;
  res->dev_last_tile = j.dev_done;
  return VP_OK;
}

int vp_serve_stats(vp_ctx *ctx, uint64_t *launches, double *resident_ms) {
  if (!ctx || !launches || !resident_ms) return set_error(VP_EINVAL, "NULL argument");
  Scheduler *s = ctx->sched.load(std::memory_order_acquire);
  if (!s) {
    *launches = 0;
    *resident_ms = 0.0;
    return VP_OK;
  }
  std::lock_guard<std::mutex> lk(s->ex.stats_mu);
  *launches = s->ex.launches;
  *resident_ms = s->ex.resident_ms;
  return VP_OK;
}

}  // extern "C"
