// vp_objects.h -- host-side objects behind the opaque handles of vp.h.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <atomic>
#include <mutex>
#include <set>
#include <utility>
#include <vector>

#include "vp_internal.h"

struct vp_ctx;

namespace vp {

struct Scheduler;

// Device allocations owned by one object; released together.
struct DeviceMem {
  std::vector<void *> ptrs;
  size_t total = 0;
  hipError_t alloc(void **p, size_t bytes);
  void release();
};

// Device workspace of vp_peel: the model visibilities, the baseline tables,
// the per-cell tables of the gain solve and the gains of every cell.  Calls on one context take turns on it (mu, and the event of the
// previous call's last kernel).
struct PeelWork {
  std::mutex mu;
  DeviceMem mem;
  void *model = nullptr;
  size_t model_bytes = 0;
  int32_t *tab = nullptr;  // ant1 [B], ant2 [B], pair_bl [n_pairs], comp [n_ant]
  size_t tab_n = 0;
  void *ws = nullptr;      // per-cell tables of the gain solve
  size_t ws_bytes = 0;
  void *gw = nullptr;      // gains of every cell, [T][n_ant][K] complex128
  size_t gw_bytes = 0;
  hipEvent_t done = nullptr;
};

struct DerivedEntry {
  Derived d{};
  DeviceMem mem;
  hipEvent_t ready = nullptr;  // recorded after kernels built the tables (null when the serving kernel did)
  hipStream_t ready_stream = nullptr;
  bool building = false;       // true while the serving kernel builds the tables (guarded by ctx->mu)
  bool serve_built = false;    // built for serving and not handed to a direct call since (guarded by ctx->mu)
  int serve_users = 0;         // admitted serving jobs that use the tables (guarded by ctx->mu)
};

struct ProfRecord {
  int kind;
  hipEvent_t e0, e1;
};

// Records a pair of events around the kernels launched in its lifetime when
// profiling is enabled on the context.
struct ProfScope {
  vp_ctx *ctx;
  hipStream_t stream;
  int kind;
  bool active = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(vp_ctx *c, hipStream_t s, int k);
  void end();
  ~ProfScope();
};

// A named range on the host timeline (roctx) for the lifetime of the guard;
// rocprofv3 --marker-trace records it, and without a profiler it costs a call.
struct TraceRange {
  explicit TraceRange(const char *name);
  ~TraceRange();
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

// Selects a HIP device for the lifetime of the guard, restoring the previous one.
struct DeviceGuard {
  int prev = 0;
  bool ok = false;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);
int run_tiles(vp_ctx *ctx, const struct ::vp_sky *sky, const struct ::vp_obs *obs, int precision, int dtype,
              void *vis, int subtract, hipStream_t stream);
int check_call(vp_ctx *ctx, const struct ::vp_sky *sky, const struct ::vp_obs *obs, int precision, int dtype,
               void *vis);
// Per-(sky, observation) tables, built on `stream` at first use and cached;
// later callers on other streams wait for the build.
int get_derived(vp_ctx *ctx, const struct ::vp_sky *sky, const struct ::vp_obs *obs, hipStream_t stream,
                DerivedEntry **out);
// Serving: find the pair's tables, or allocate them unbuilt (*build = true:
// the caller builds them and calls derived_built).
int serve_derived(vp_ctx *ctx, const struct ::vp_sky *sky, const struct ::vp_obs *obs, DerivedEntry **out,
                  bool *build);
bool derived_ready(vp_ctx *ctx, DerivedEntry *d);
void derived_built(vp_ctx *ctx, DerivedEntry *d);
// A serving job is done with the pair's tables.
void serve_release_derived(vp_ctx *ctx, DerivedEntry *d);
// The tables a serving job was to build were never built (its work was
// abandoned): drop them, so that no later call finds them ready.
void serve_abandon_derived(vp_ctx *ctx, DerivedEntry *d);
// Bytes of tables that serving jobs built and no admitted job or direct call
// uses, and their release (hipFree: waits for the device).
uint64_t serve_evictable_bytes(vp_ctx *ctx);
void serve_evict(vp_ctx *ctx);
DeriveArgs make_derive_args(const struct ::vp_sky *sky, const struct ::vp_obs *obs, const Derived &d);
FluxArgs make_flux_args(const struct ::vp_sky *sky, const struct ::vp_obs *obs, const Derived &d);
void drop_derived(vp_ctx *ctx, uint64_t sky_id, uint64_t obs_id);
void drop_all_derived(vp_ctx *ctx);

// serving hooks (vp_serve.cpp)
uint64_t job_footprint(const struct ::vp_sky *sky, const struct ::vp_obs *obs, int dtype);
bool serve_pending(vp_ctx *ctx);
void serve_shutdown(vp_ctx *ctx);

}  // namespace vp

struct vp_obs {
  vp_ctx *ctx = nullptr;
  uint64_t id = 0;
  int T = 0, B = 0, K = 0, Kpad = 0;
  double ra0 = 0, dec0 = 0;
  int sign = -1;
  double beam_fwhm = 0, beam_nu_ref = 0;
  double *uvw = nullptr;  // device [T*B][3]
  double *freq = nullptr; // device [K]
  double *fk = nullptr;   // device [Kpad], nu/c
  double dfk = 0;         // channel step of nu/c when uniform
  int uniform = 0;        // channels uniformly spaced (to 1e-12 of nu/c)
  int uniform64 = 0;      // ... to 1e-15 of nu/c (enough for the FP64 path)
  std::vector<double> h_freq;
  int jobs = 0;           // pending serving jobs using it (guarded by ctx->mu)
  vp::DeviceMem mem;
};

struct vp_sky {
  vp_ctx *ctx = nullptr;
  uint64_t id = 0;
  int P = 0, G = 0, S = 0;
  double nu_ref = 0;
  int max_nmax = 0;
  std::vector<int32_t> h_nmax;
  double *ra = nullptr, *dec = nullptr, *sref = nullptr, *alpha = nullptr;  // device [J]
  double *g_maj = nullptr, *g_min = nullptr, *g_pa = nullptr;               // device [G]
  double *s_beta1 = nullptr, *s_beta2 = nullptr, *s_pa = nullptr;          // device [S]
  int32_t *lpow = nullptr;  // device [S]: spectral term of each shapelet component, or null (all 0)
  vp::ShpTiles tiles;
  int jobs = 0;
  vp::DeviceMem mem;
};

struct vp_ctx {
  int device = 0;
  uint64_t budget = 0;
  std::mutex mu;  // guards the object sets, the derived cache and job counts
  uint64_t next_id = 0;
  std::set<vp_obs *> obs;
  std::set<vp_sky *> skies;
  std::map<std::pair<uint64_t, uint64_t>, vp::DerivedEntry *> derived;
  uint64_t lib_bytes = 0;
  bool profile = false;
  std::mutex prof_mu;
  std::vector<vp::ProfRecord> prof_pending;
  // created by the first vp_submit (under mu), read by vp_poll without it
  std::atomic<vp::Scheduler *> sched{nullptr};
  vp::PeelWork *peel = nullptr;
  float *lut = nullptr;    // basis table of VP_PREC_LUT, built at its first use (guarded by mu)
  vp::DeviceMem lut_mem;
};
