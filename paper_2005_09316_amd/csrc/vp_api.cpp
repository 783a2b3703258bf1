// vp_api.cpp -- C ABI of libvp: contexts, observations, sky models, predict
// and subtract.  Serving (vp_submit / vp_poll) lives in vp_serve.cpp.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <chrono>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/vp.h"
#include "vp_internal.h"
#include "vp_objects.h"

namespace vp {

static thread_local std::string g_err;

int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_error(hipError_t e, const char *what) {
  return set_error(e == hipErrorOutOfMemory ? VP_ENOMEM : VP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int dev) {
  ok = hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess;
}
DeviceGuard::~DeviceGuard() {
  if (ok) (void)hipSetDevice(prev);
}

static bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename T>
static hipError_t upload(T **dst, const T *src, int64_t n, DeviceMem &mem) {
  *dst = nullptr;
  if (n <= 0) return hipSuccess;
  hipError_t e = mem.alloc((void **)dst, sizeof(T) * (size_t)n);
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, sizeof(T) * (size_t)n, hipMemcpyHostToDevice);
}

hipError_t DeviceMem::alloc(void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) {
    ptrs.push_back(*p);
    total += bytes;
  }
  return e;
}

void DeviceMem::release() {
  for (void *p : ptrs) (void)hipFree(p);
  ptrs.clear();
  total = 0;
}

// ---------------------------------------------------------------------------
// derived (sky, obs) tables
// ---------------------------------------------------------------------------

static int alloc_derived(const vp_sky *sky, const vp_obs *obs, DerivedEntry **out) {
  DerivedEntry *d = new DerivedEntry();
  const int J = sky->P + sky->G + sky->S;
  const int Jc = std::max(J, 1), Gc = std::max(sky->G, 1), Sc = std::max(sky->S, 1);
  hipError_t e = d->mem.alloc((void **)&d->d.pos, sizeof(double4) * Jc);
  if (e == hipSuccess) e = d->mem.alloc((void **)&d->d.gq, sizeof(double4) * Gc);
  if (e == hipSuccess) e = d->mem.alloc((void **)&d->d.sframe, sizeof(double) * 12 * Sc);
  if (e == hipSuccess) e = d->mem.alloc((void **)&d->d.flux32, sizeof(float) * (size_t)Jc * obs->Kpad);
  if (e == hipSuccess) e = d->mem.alloc((void **)&d->d.flux64, sizeof(double) * (size_t)Jc * obs->Kpad);
  if (e != hipSuccess) {
    d->mem.release();
    delete d;
    return hip_error(e, "allocating per-(sky, observation) tables");
  }
  *out = d;
  return VP_OK;
}

DeriveArgs make_derive_args(const vp_sky *sky, const vp_obs *obs, const Derived &d) {
  DeriveArgs da;
  da.P = sky->P; da.G = sky->G; da.S = sky->S;
  da.ra = sky->ra; da.dec = sky->dec;
  da.g_maj = sky->g_maj; da.g_min = sky->g_min; da.g_pa = sky->g_pa;
  da.s_beta1 = sky->s_beta1; da.s_beta2 = sky->s_beta2; da.s_pa = sky->s_pa;
  da.ra0 = obs->ra0; da.dec0 = obs->dec0;
  da.d = d;
  return da;
}

FluxArgs make_flux_args(const vp_sky *sky, const vp_obs *obs, const Derived &d) {
  FluxArgs fa;
  fa.J = sky->P + sky->G + sky->S; fa.K = obs->K; fa.Kpad = obs->Kpad;
  fa.sref = sky->sref; fa.alpha = sky->alpha; fa.ra = sky->ra; fa.dec = sky->dec; fa.freq = obs->freq;
  fa.nu_ref = sky->nu_ref; fa.ra0 = obs->ra0; fa.dec0 = obs->dec0;
  fa.beam_fwhm = obs->beam_fwhm; fa.beam_nu_ref = obs->beam_nu_ref;
  fa.j0 = sky->P + sky->G;
  fa.lpow = sky->lpow;
  fa.d = d;
  return fa;
}

int get_derived(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, hipStream_t stream, DerivedEntry **out) {
  const auto key = std::make_pair(sky->id, obs->id);
  for (;;) {
    std::unique_lock<std::mutex> lk(ctx->mu);
    auto it = ctx->derived.find(key);
    if (it != ctx->derived.end()) {
      DerivedEntry *d = it->second;
      if (d->building) {  // being built by the serving kernel
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        continue;
      }
      if (d->ready && d->ready_stream != stream) {
        hipError_t e = hipStreamWaitEvent(stream, d->ready, 0);
        if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
      }
      d->serve_built = false;  // a direct call's kernels may read it from now on: never evicted by serving
      *out = d;
      return VP_OK;
    }
    DerivedEntry *d = nullptr;
    int rc = alloc_derived(sky, obs, &d);
    if (rc != VP_OK) return rc;
    hipError_t e = hipEventCreateWithFlags(&d->ready, hipEventDisableTiming);
    if (e == hipSuccess) {
      ProfScope ps(ctx, stream, 0);
      e = launch_derive(make_derive_args(sky, obs, d->d), stream);
      if (e == hipSuccess) e = launch_flux(make_flux_args(sky, obs, d->d), stream);
      ps.end();
    }
    if (e == hipSuccess) e = hipEventRecord(d->ready, stream);
    if (e != hipSuccess) {
      if (d->ready) (void)hipEventDestroy(d->ready);
      d->mem.release();
      delete d;
      return hip_error(e, "building per-(sky, observation) tables");
    }
    d->ready_stream = stream;
    ctx->derived[key] = d;
    ctx->lib_bytes += d->mem.total;
    *out = d;
    return VP_OK;
  }
}

int serve_derived(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, DerivedEntry **out, bool *build) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  const auto key = std::make_pair(sky->id, obs->id);
  auto it = ctx->derived.find(key);
  if (it != ctx->derived.end()) {
    it->second->serve_users += 1;
    *out = it->second;
    *build = false;
    return VP_OK;
  }
  DerivedEntry *d = nullptr;
  int rc = alloc_derived(sky, obs, &d);
  if (rc != VP_OK) return rc;
  d->building = true;
  d->serve_built = true;
  d->serve_users = 1;
  ctx->derived[key] = d;
  ctx->lib_bytes += d->mem.total;
  *out = d;
  *build = true;
  return VP_OK;
}

bool derived_ready(vp_ctx *ctx, DerivedEntry *d) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (d->building) return false;
  return !d->ready || hipEventQuery(d->ready) == hipSuccess;
}

void derived_built(vp_ctx *ctx, DerivedEntry *d) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  d->building = false;
}

static void free_entry(vp_ctx *ctx, DerivedEntry *d) {
  // caller holds ctx->mu and has removed d from ctx->derived
  if (d->ready) {
    (void)hipEventSynchronize(d->ready);
    (void)hipEventDestroy(d->ready);
  }
  ctx->lib_bytes -= d->mem.total;
  d->mem.release();
  delete d;
}

void serve_release_derived(vp_ctx *ctx, DerivedEntry *d) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  d->serve_users -= 1;
}

void serve_abandon_derived(vp_ctx *ctx, DerivedEntry *d) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  d->serve_users -= 1;
  for (auto it = ctx->derived.begin(); it != ctx->derived.end(); ++it)
    if (it->second == d) {
      ctx->derived.erase(it);
      free_entry(ctx, d);
      return;
    }
}

uint64_t serve_evictable_bytes(vp_ctx *ctx) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  uint64_t b = 0;
  for (auto &kv : ctx->derived)
    if (kv.second->serve_built && kv.second->serve_users == 0 && !kv.second->building) b += kv.second->mem.total;
  return b;
}

void serve_evict(vp_ctx *ctx) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (auto it = ctx->derived.begin(); it != ctx->derived.end();) {
    DerivedEntry *d = it->second;
    if (d->serve_built && d->serve_users == 0 && !d->building) {
      it = ctx->derived.erase(it);
      free_entry(ctx, d);
    } else {
      ++it;
    }
  }
}

void drop_derived(vp_ctx *ctx, uint64_t sky_id, uint64_t obs_id) {
  // caller holds ctx->mu; an id of 0 matches nothing
  for (auto it = ctx->derived.begin(); it != ctx->derived.end();) {
    if ((sky_id && it->first.first == sky_id) || (obs_id && it->first.second == obs_id)) {
      if (it->second->ready) {
        (void)hipEventSynchronize(it->second->ready);
        (void)hipEventDestroy(it->second->ready);
      }
      ctx->lib_bytes -= it->second->mem.total;
      it->second->mem.release();
      delete it->second;
      it = ctx->derived.erase(it);
    } else {
      ++it;
    }
  }
}

void drop_all_derived(vp_ctx *ctx) {
  // caller holds ctx->mu
  for (auto &kv : ctx->derived) {
    if (kv.second->ready) {
      (void)hipEventSynchronize(kv.second->ready);
      (void)hipEventDestroy(kv.second->ready);
    }
    ctx->lib_bytes -= kv.second->mem.total;
    kv.second->mem.release();
    delete kv.second;
  }
  ctx->derived.clear();
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------

TraceRange::TraceRange(const char *name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

ProfScope::ProfScope(vp_ctx *c, hipStream_t s, int k) : ctx(c), stream(s), kind(k) {
  if (ctx && ctx->profile) {
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
        hipEventRecord(e0, stream) == hipSuccess)
      active = true;
  }
}

void ProfScope::end() {
  if (!active) return;
  active = false;
  if (hipEventRecord(e1, stream) == hipSuccess) {
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->prof_pending.push_back({kind, e0, e1});
  } else {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
}

ProfScope::~ProfScope() { end(); }

// ---------------------------------------------------------------------------
// predict / subtract
// ---------------------------------------------------------------------------

// The basis table of the lookup-table variant, built once per context (the
// build is synchronous: later calls on any stream find it complete).
static int get_lut(vp_ctx *ctx, hipStream_t stream, const float **out) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->lut) {
    void *p = nullptr;
    hipError_t e = ctx->lut_mem.alloc(&p, kLutBytes);
    if (e == hipSuccess) e = launch_lut_build((float *)p, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      ctx->lut_mem.release();
      return hip_error(e, "building the basis lookup table");
    }
    ctx->lut = (float *)p;
  }
  *out = ctx->lut;
  return VP_OK;
}

// Launch the point/Gaussian and shapelet passes over the visibility tiles
// with the pair's tables `d`.  prof: the context whose profiling records the
// launches, or null.
static int launch_passes(vp_ctx *prof, const vp_sky *sky, const vp_obs *obs, int precision, int dtype, void *vis,
                         int subtract, hipStream_t stream, const Derived &d, const float *lut) {
  TileArgs a;
  a.nrows = (int64_t)obs->T * obs->B;
  a.K = obs->K;
  a.Kpad = obs->Kpad;
  a.uvw = obs->uvw;
  a.fk = obs->fk;
  a.P = sky->P; a.G = sky->G; a.S = sky->S;
  a.d = d;
  a.t = sky->tiles;
  a.vis = vis;
  a.subtract = subtract;
  a.c64 = dtype == VP_C64;
  a.conj = obs->sign < 0;
  a.n_rb = (int)((a.nrows + kTileRows - 1) / kTileRows);
  a.n_cb = obs->Kpad / kPgChan;
  a.lut = lut;
  a.dfk = obs->dfk;
  a.uniform = precision == kFP64 || precision == kLut ? obs->uniform64 : obs->uniform;
  // A sky of shapelets only skips the point/Gaussian pass, which would only
  // write zeros (predict) or rewrite the data unchanged (subtract).
  const bool pg_pass = sky->P + sky->G > 0 || sky->S == 0;
  a.fresh = !pg_pass && !subtract;
  hipError_t e = hipSuccess;
  if (pg_pass) {
    ProfScope ps(prof, stream, 1);
    e = launch_pg(a, precision, stream);
  }
  if (e != hipSuccess) return hip_error(e, "launching the point/Gaussian kernel");
  if (sky->S > 0) {
    a.n_cb = (obs->K + kShpChan - 1) / kShpChan;
    ProfScope ps(prof, stream, 2);
    e = launch_shp(a, precision, sky->max_nmax, stream);
    if (e == hipErrorNotSupported) return set_error(VP_EINVAL, "precision %d has no shapelet kernel", precision);
    if (e != hipSuccess) return hip_error(e, "launching the shapelet kernel");
  }
  return VP_OK;
}

int run_tiles(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype, void *vis,
              int subtract, hipStream_t stream) {
  DerivedEntry *d = nullptr;
  int rc = get_derived(ctx, sky, obs, stream, &d);
  if (rc != VP_OK) return rc;
  const float *lut = nullptr;
  if (precision == kLut && sky->S > 0) {
    rc = get_lut(ctx, stream, &lut);
    if (rc != VP_OK) return rc;
  }
  return launch_passes(ctx, sky, obs, precision, dtype, vis, subtract, stream, d->d, lut);
}

int check_call(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype, void *vis) {
  if (!ctx || !sky || !obs) return set_error(VP_EINVAL, "NULL context, sky or observation");
  if (sky->ctx != ctx || obs->ctx != ctx) return set_error(VP_EINVAL, "sky or observation belongs to another context");
  if (precision < VP_PREC_FP64 || precision > VP_PREC_LUT)
    return set_error(VP_EINVAL, "unknown precision %d", precision);
  if (precision == VP_PREC_MIXED_F32MMA)
    return set_error(VP_EINVAL, "precision %d (FP32 MFMA contraction) is retired", precision);
  if (dtype != VP_C128 && dtype != VP_C64) return set_error(VP_EINVAL, "unknown dtype %d", dtype);
  if (!vis) return set_error(VP_EINVAL, "NULL visibility buffer");
  return VP_OK;
}

}  // namespace vp

using namespace vp;

extern "C" {

const char *vp_last_error(void) { return g_err.c_str(); }

const char *vp_version(void) { return "libvp 0.1 (gfx950)"; }

int vp_create_ctx(int hip_device, uint64_t hbm_budget_bytes, vp_ctx **out) {
  if (!out) return set_error(VP_EINVAL, "NULL out");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= n) return set_error(VP_EINVAL, "device %d out of range (%d devices)", hip_device, n);
  DeviceGuard g(hip_device);
  if (!g.ok) return set_error(VP_EDEVICE, "cannot select device %d", hip_device);
  e = device_init(hip_device);
  if (e != hipSuccess) return hip_error(e, "initialising the device");
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return hip_error(e, "hipMemGetInfo");
  vp_ctx *c = new vp_ctx();
  c->device = hip_device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
  *out = c;
  return VP_OK;
}

int vp_destroy_ctx(vp_ctx *ctx) {
  if (!ctx) return set_error(VP_EINVAL, "NULL context");
  if (serve_pending(ctx)) return set_error(VP_EBUSY, "serving jobs still pending");
  serve_shutdown(ctx);
  DeviceGuard g(ctx->device);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    drop_all_derived(ctx);
    for (vp_obs *o : ctx->obs) {
      o->mem.release();
      delete o;
    }
    for (vp_sky *s : ctx->skies) {
      s->mem.release();
      delete s;
    }
    ctx->obs.clear();
    ctx->skies.clear();
  }
  {
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    for (auto &r : ctx->prof_pending) {
      (void)hipEventDestroy(r.e0);
      (void)hipEventDestroy(r.e1);
    }
  }
  if (ctx->peel) {
    if (ctx->peel->done) {
      (void)hipEventSynchronize(ctx->peel->done);
      (void)hipEventDestroy(ctx->peel->done);
    }
    ctx->peel->mem.release();
    delete ctx->peel;
  }
  ctx->lut_mem.release();
  delete ctx;
  return VP_OK;
}

int vp_create_obs(vp_ctx *ctx, const vp_obs_desc *desc, vp_obs **out) {
  if (!ctx || !desc || !out) return set_error(VP_EINVAL, "NULL argument");
  if (desc->n_time <= 0 || desc->n_bl <= 0 || desc->n_chan <= 0)
    return set_error(VP_EINVAL, "n_time, n_bl, n_chan must be positive");
  const int64_t nrows = (int64_t)desc->n_time * desc->n_bl;
  if (nrows > (int64_t)1 << 30 || desc->n_chan > (1 << 20))
    return set_error(VP_EINVAL, "observation too large");
  if (!desc->uvw_m || !desc->freq_hz) return set_error(VP_EINVAL, "NULL uvw or frequency array");
  if (desc->sign != 1 && desc->sign != -1) return set_error(VP_EINVAL, "sign must be +1 or -1");
  if (!finite_all(desc->uvw_m, 3 * nrows)) return set_error(VP_EINVAL, "non-finite uvw");
  if (!finite_all(desc->freq_hz, desc->n_chan)) return set_error(VP_EINVAL, "non-finite frequency");
  for (int k = 0; k < desc->n_chan; ++k)
    if (desc->freq_hz[k] <= 0) return set_error(VP_EINVAL, "frequency %d not positive", k);
  if (!std::isfinite(desc->ra0) || !std::isfinite(desc->dec0)) return set_error(VP_EINVAL, "non-finite phase centre");
  if (!std::isfinite(desc->beam_fwhm_rad) || desc->beam_fwhm_rad < 0)
    return set_error(VP_EINVAL, "beam FWHM must be finite and >= 0");
  if (desc->beam_fwhm_rad > 0 && !(desc->beam_nu_ref_hz > 0 && std::isfinite(desc->beam_nu_ref_hz)))
    return set_error(VP_EINVAL, "beam reference frequency must be positive");
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(VP_EDEVICE, "cannot select device");
  vp_obs *o = new vp_obs();
  o->ctx = ctx;
  o->T = desc->n_time;
  o->B = desc->n_bl;
  o->K = desc->n_chan;
  o->Kpad = (desc->n_chan + kPgChan - 1) / kPgChan * kPgChan;
  o->ra0 = desc->ra0;
  o->dec0 = desc->dec0;
  o->sign = desc->sign;
  o->beam_fwhm = desc->beam_fwhm_rad;
  o->beam_nu_ref = desc->beam_nu_ref_hz;
  o->h_freq.assign(desc->freq_hz, desc->freq_hz + desc->n_chan);
  std::vector<double> fk(o->Kpad);
  for (int k = 0; k < o->Kpad; ++k) fk[k] = desc->freq_hz[std::min(k, o->K - 1)] / kLightSpeed;
  if (o->K >= 2) {
    // uniformly spaced channels let the kernels rotate phasors between
    // channels: the mixed path while the grid holds to 1e-12 of nu/c (phase
    // error below 1e-8 turns for |t0| up to 1e4 m), the FP64 path while it
    // holds to 1e-15 (1e-11 turns)
    const double d = (fk[o->K - 1] - fk[0]) / (o->K - 1);
    double dev = 0.0;
    for (int k = 0; k < o->K; ++k) dev = std::max(dev, std::fabs(fk[k] - std::fma((double)k, d, fk[0])));
    const bool uni = d != 0.0 && dev <= 1e-12 * std::fabs(fk[0]);
    o->uniform = uni ? 1 : 0;
    o->uniform64 = uni && dev <= 1e-15 * std::fabs(fk[0]) ? 1 : 0;
    o->dfk = uni ? d : 0.0;
  }
  hipError_t e = upload(&o->uvw, desc->uvw_m, 3 * nrows, o->mem);
  if (e == hipSuccess) e = upload(&o->freq, desc->freq_hz, (int64_t)o->K, o->mem);
  if (e == hipSuccess) e = upload(&o->fk, fk.data(), (int64_t)o->Kpad, o->mem);
  if (e != hipSuccess) {
    o->mem.release();
    delete o;
    return hip_error(e, "uploading the observation");
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  o->id = ++ctx->next_id;
  ctx->obs.insert(o);
  ctx->lib_bytes += o->mem.total;
  *out = o;
  return VP_OK;
}

int vp_destroy_obs(vp_obs *obs) {
  if (!obs) return set_error(VP_EINVAL, "NULL observation");
  vp_ctx *ctx = obs->ctx;
  DeviceGuard g(ctx->device);
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (obs->jobs > 0) return set_error(VP_EBUSY, "observation used by pending jobs");
  drop_derived(ctx, 0, obs->id);
  ctx->obs.erase(obs);
  ctx->lib_bytes -= obs->mem.total;
  obs->mem.release();
  delete obs;
  return VP_OK;
}

int vp_create_sky(vp_ctx *ctx, const vp_sky_desc *d, vp_sky **out) {
  if (!ctx || !d || !out) return set_error(VP_EINVAL, "NULL argument");
  if (d->n_point < 0 || d->n_gauss < 0 || d->n_shp < 0) return set_error(VP_EINVAL, "negative component count");
  if (!(d->nu_ref_hz > 0) || !std::isfinite(d->nu_ref_hz)) return set_error(VP_EINVAL, "nu_ref must be positive");
  const int P = d->n_point, G = d->n_gauss, Sd = d->n_shp;
  if ((int64_t)P + G + Sd > (1 << 28)) return set_error(VP_EINVAL, "too many components");
  if (P > 0 && (!d->p_ra || !d->p_dec || !d->p_sref || !d->p_alpha)) return set_error(VP_EINVAL, "NULL point array");
  if (G > 0 && (!d->g_ra || !d->g_dec || !d->g_sref || !d->g_alpha || !d->g_maj || !d->g_min || !d->g_pa))
    return set_error(VP_EINVAL, "NULL Gaussian array");
  if (Sd > 0 && (!d->s_ra || !d->s_dec || !d->s_sref || !d->s_alpha || !d->s_beta1 || !d->s_beta2 || !d->s_pa ||
                 !d->s_nmax || !d->s_coeff_off || !d->coeffs))
    return set_error(VP_EINVAL, "NULL shapelet array");
  const double *pa[] = {d->p_ra, d->p_dec, d->p_sref, d->p_alpha};
  for (auto p : pa)
    if (P > 0 && !finite_all(p, P)) return set_error(VP_EINVAL, "non-finite point parameter");
  const double *ga[] = {d->g_ra, d->g_dec, d->g_sref, d->g_alpha, d->g_maj, d->g_min, d->g_pa};
  for (auto p : ga)
    if (G > 0 && !finite_all(p, G)) return set_error(VP_EINVAL, "non-finite Gaussian parameter");
  for (int g = 0; g < G; ++g)
    if (d->g_maj[g] < 0 || d->g_min[g] < 0) return set_error(VP_EINVAL, "Gaussian %d has a negative FWHM", g);
  const double *sa[] = {d->s_ra, d->s_dec, d->s_sref, d->s_alpha, d->s_beta1, d->s_beta2, d->s_pa};
  for (auto p : sa)
    if (Sd > 0 && !finite_all(p, Sd)) return set_error(VP_EINVAL, "non-finite shapelet parameter");
  // Shapelet components: one per spectral term of each shapelet (same
  // position and frame; term q's flux carries ln(nu / nu_ref)^q).
  std::vector<int> src;            // shapelet of the description
  std::vector<int32_t> lp;         // its spectral term
  std::vector<const double *> cp;  // its coefficients, packed for order d->s_nmax
  for (int s = 0; s < Sd; ++s) {
    const int N = d->s_nmax[s];
    if (N < 0 || N > VP_NMAX_LIMIT) return set_error(VP_EINVAL, "shapelet %d: nmax %d outside 0..%d", s, N, VP_NMAX_LIMIT);
    if (!(d->s_beta1[s] > 0) || !(d->s_beta2[s] > 0)) return set_error(VP_EINVAL, "shapelet %d: beta must be positive", s);
    if (d->s_coeff_off[s] < 0) return set_error(VP_EINVAL, "shapelet %d: negative coefficient offset", s);
    const int Q = d->s_nterm ? d->s_nterm[s] : 1;
    if (Q < 1 || Q > VP_NTERM_LIMIT)
      return set_error(VP_EINVAL, "shapelet %d: %d spectral terms outside 1..%d", s, Q, VP_NTERM_LIMIT);
    const int64_t cnt = (int64_t)(N + 1) * (N + 2) / 2;
    for (int q = 0; q < Q; ++q) {
      const double *c = d->coeffs + d->s_coeff_off[s] + q * cnt;
      if (!finite_all(c, cnt)) return set_error(VP_EINVAL, "shapelet %d: non-finite coefficient", s);
      src.push_back(s);
      lp.push_back(q);
      cp.push_back(c);
    }
  }
  const int S = (int)src.size();
  if ((int64_t)P + G + S > (1 << 28)) return set_error(VP_EINVAL, "too many components");
  int max_nmax = 0;
  std::vector<int32_t> nmax(S);
  std::vector<int64_t> coff(S);
  int64_t ncoef = 0;
  for (int i = 0; i < S; ++i) {
    const int N = d->s_nmax[src[i]];
    const double *c = cp[i];
    // effective order: the highest n1 + n2 with a non-zero coefficient (orders
    // above it contribute nothing, and the kernels' work follows the order)
    int neff = 0;
    for (int n1 = 0, j = 0; n1 <= N; ++n1)
      for (int n2 = 0; n2 <= N - n1; ++n2, ++j)
        if (c[j] != 0.0) neff = std::max(neff, n1 + n2);
    nmax[i] = neff;
    coff[i] = ncoef;
    ncoef += (int64_t)(neff + 1) * (neff + 2) / 2;
    max_nmax = std::max(max_nmax, neff);
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(VP_EDEVICE, "cannot select device");
  vp_sky *k = new vp_sky();
  k->ctx = ctx;
  k->P = P; k->G = G; k->S = S;
  k->nu_ref = d->nu_ref_hz;
  k->max_nmax = max_nmax;
  k->h_nmax = nmax;
  const int J = P + G + S;
  std::vector<double> ra(J), dec(J), sref(J), alpha(J), coeffs(ncoef), b1(S), b2(S), spa(S);
  for (int i = 0; i < P; ++i) { ra[i] = d->p_ra[i]; dec[i] = d->p_dec[i]; sref[i] = d->p_sref[i]; alpha[i] = d->p_alpha[i]; }
  for (int i = 0; i < G; ++i) { ra[P + i] = d->g_ra[i]; dec[P + i] = d->g_dec[i]; sref[P + i] = d->g_sref[i]; alpha[P + i] = d->g_alpha[i]; }
  bool terms = false;
  for (int i = 0; i < S; ++i) {
    const int s = src[i];
    ra[P + G + i] = d->s_ra[s]; dec[P + G + i] = d->s_dec[s]; sref[P + G + i] = d->s_sref[s]; alpha[P + G + i] = d->s_alpha[s];
    b1[i] = d->s_beta1[s]; b2[i] = d->s_beta2[s]; spa[i] = d->s_pa[s];
    terms = terms || lp[i] > 0;
    // packed n1-major over n1 + n2 <= nmax, re-packed for the effective order
    const int N = d->s_nmax[s], M = nmax[i];
    const double *c = cp[i];
    double *o = coeffs.data() + coff[i];
    for (int n1 = 0; n1 <= M; ++n1)
      for (int n2 = 0; n2 <= M - n1; ++n2)
        *o++ = c[(int64_t)n1 * (N + 1) - (int64_t)n1 * (n1 - 1) / 2 + n2];
  }
  std::vector<int64_t> a32_off(S), c64_off(S), abf_off(S);
  std::vector<int32_t> ld(S);
  int64_t n32 = 0, n64 = 0, nbf = 0;
  for (int s = 0; s < S; ++s) {
    a32_off[s] = n32; n32 += a32_floats(nmax[s]);
    ld[s] = c64_ld(nmax[s]);
    c64_off[s] = n64; n64 += c64_doubles(nmax[s]);
    abf_off[s] = nbf; nbf += abf_elems(nmax[s]);
  }
  int32_t *d_nmax = nullptr;
  int64_t *d_coff = nullptr, *d_a32off = nullptr, *d_c64off = nullptr, *d_abfoff = nullptr;
  int32_t *d_ld = nullptr;
  double *d_coeffs = nullptr;
  float *d_a32 = nullptr;
  double *d_c64 = nullptr;
  uint16_t *d_abf = nullptr;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(&k->ra, ra.data(), J, k->mem);
  if (e == hipSuccess) e = upload(&k->dec, dec.data(), J, k->mem);
  if (e == hipSuccess) e = upload(&k->sref, sref.data(), J, k->mem);
  if (e == hipSuccess) e = upload(&k->alpha, alpha.data(), J, k->mem);
  if (e == hipSuccess) e = upload(&k->g_maj, d->g_maj, G, k->mem);
  if (e == hipSuccess) e = upload(&k->g_min, d->g_min, G, k->mem);
  if (e == hipSuccess) e = upload(&k->g_pa, d->g_pa, G, k->mem);
  if (e == hipSuccess) e = upload(&k->s_beta1, b1.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&k->s_beta2, b2.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&k->s_pa, spa.data(), S, k->mem);
  if (e == hipSuccess && terms) e = upload(&k->lpow, lp.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&d_nmax, nmax.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&d_coff, coff.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&d_coeffs, coeffs.data(), ncoef, k->mem);
  if (e == hipSuccess) e = upload(&d_a32off, a32_off.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&d_c64off, c64_off.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&d_abfoff, abf_off.data(), S, k->mem);
  if (e == hipSuccess) e = upload(&d_ld, ld.data(), S, k->mem);
  if (e == hipSuccess && n32 > 0) e = k->mem.alloc((void **)&d_a32, sizeof(float) * n32);
  if (e == hipSuccess && n64 > 0) e = k->mem.alloc((void **)&d_c64, sizeof(double) * n64);
  if (e == hipSuccess && nbf > 0) e = k->mem.alloc((void **)&d_abf, sizeof(uint16_t) * nbf);
  if (e == hipSuccess && S > 0) {
    TileBuildArgs ta;
    ta.S = S; ta.nmax = d_nmax; ta.coeff_off = d_coff; ta.coeffs = d_coeffs;
    ta.a32 = d_a32; ta.a32_off = d_a32off; ta.c64 = d_c64; ta.c64_off = d_c64off; ta.c64_ld = d_ld;
    ta.abf = d_abf; ta.abf_off = d_abfoff;
    e = launch_tiles_build(ta, max_nmax, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  }
  if (e != hipSuccess) {
    k->mem.release();
    delete k;
    return hip_error(e, "uploading the sky model");
  }
  k->tiles.a32 = d_a32; k->tiles.a32_off = d_a32off;
  k->tiles.c64 = d_c64; k->tiles.c64_off = d_c64off; k->tiles.c64_ld = d_ld;
  k->tiles.abf = d_abf; k->tiles.abf_off = d_abfoff;
  k->tiles.nmax = d_nmax;
  std::lock_guard<std::mutex> lk(ctx->mu);
  k->id = ++ctx->next_id;
  ctx->skies.insert(k);
  ctx->lib_bytes += k->mem.total;
  *out = k;
  return VP_OK;
}

int vp_destroy_sky(vp_sky *sky) {
  if (!sky) return set_error(VP_EINVAL, "NULL sky");
  vp_ctx *ctx = sky->ctx;
  DeviceGuard g(ctx->device);
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (sky->jobs > 0) return set_error(VP_EBUSY, "sky used by pending jobs");
  drop_derived(ctx, sky->id, 0);
  ctx->skies.erase(sky);
  ctx->lib_bytes -= sky->mem.total;
  sky->mem.release();
  delete sky;
  return VP_OK;
}

int vp_predict(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype, void *vis_dev,
               void *hip_stream) {
  TraceRange tr("vp_predict");
  int rc = check_call(ctx, sky, obs, precision, dtype, vis_dev);
  if (rc != VP_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(VP_EDEVICE, "cannot select device");
  return run_tiles(ctx, sky, obs, precision, dtype, vis_dev, 0, (hipStream_t)hip_stream);
}

int vp_predict_noalloc(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype, void *vis_dev,
                       void *hip_stream) {
  TraceRange tr("vp_predict_noalloc");
  int rc = check_call(ctx, sky, obs, precision, dtype, vis_dev);
  if (rc != VP_OK) return rc;
  if (precision == VP_PREC_LUT)
    return set_error(VP_EINVAL, "vp_predict_noalloc: the lookup-table variant needs a per-context table");
  // the pair's tables, laid out in the device's scratch array (256-byte aligned parts)
  const int J = sky->P + sky->G + sky->S;
  const uint64_t Jc = (uint64_t)std::max(J, 1), Gc = (uint64_t)std::max(sky->G, 1);
  const uint64_t Sc = (uint64_t)std::max(sky->S, 1), Kp = (uint64_t)obs->Kpad;
  auto up = [](uint64_t b) { return (b + 255) & ~(uint64_t)255; };
  const uint64_t o_gq = up(sizeof(double4) * Jc);
  const uint64_t o_sf = o_gq + up(sizeof(double4) * Gc);
  const uint64_t o_f32 = o_sf + up(sizeof(double) * 12 * Sc);
  const uint64_t o_f64 = o_f32 + up(sizeof(float) * Jc * Kp);
  const uint64_t need = o_f64 + up(sizeof(double) * Jc * Kp);
  if (need > kNoAllocScratchBytes)
    return set_error(VP_EINVAL,
                     "vp_predict_noalloc: %d components x %d padded channels need %llu bytes of tables; "
                     "the scratch holds %llu",
                     J, obs->Kpad, (unsigned long long)need, (unsigned long long)kNoAllocScratchBytes);
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(VP_EDEVICE, "cannot select device %d", ctx->device);
  char *base = (char *)noalloc_scratch(ctx->device);
  if (!base) return set_error(VP_EDEVICE, "no scratch address for device %d", ctx->device);
  Derived d;
  d.pos = (double4 *)base;
  d.gq = (double4 *)(base + o_gq);
  d.sframe = (double *)(base + o_sf);
  d.flux32 = (float *)(base + o_f32);
  d.flux64 = (double *)(base + o_f64);
  const hipStream_t stream = (hipStream_t)hip_stream;
  // every entry the tile kernels read is written here first (the flux table
  // includes its zero padding), so nothing is cleared
  hipError_t e = launch_derive(make_derive_args(sky, obs, d), stream);
  if (e == hipSuccess) e = launch_flux(make_flux_args(sky, obs, d), stream);
  if (e != hipSuccess) return hip_error(e, "building the tables in the scratch array");
  return launch_passes(nullptr, sky, obs, precision, dtype, vis_dev, 0, stream, d, nullptr);
}

int vp_subtract(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype, void *data_dev,
                void *hip_stream) {
  TraceRange tr("vp_subtract");
  int rc = check_call(ctx, sky, obs, precision, dtype, data_dev);
  if (rc != VP_OK) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(VP_EDEVICE, "cannot select device");
  return run_tiles(ctx, sky, obs, precision, dtype, data_dev, 1, (hipStream_t)hip_stream);
}

int vp_profile(vp_ctx *ctx, int enable) {
  if (!ctx) return set_error(VP_EINVAL, "NULL context");
  ctx->profile = enable != 0;
  return VP_OK;
}

int vp_profile_read(vp_ctx *ctx, int64_t *counts, double *total_ms) {
  if (!ctx || !counts || !total_ms) return set_error(VP_EINVAL, "NULL argument");
  DeviceGuard g(ctx->device);
  std::vector<ProfRecord> recs;
  {
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    recs.swap(ctx->prof_pending);
  }
  int64_t c[kProfClasses] = {0, 0, 0, 0};
  double t[kProfClasses] = {0, 0, 0, 0};
  int rc = VP_OK;
  for (auto &r : recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.e0, r.e1);
    if (e != hipSuccess && rc == VP_OK) rc = hip_error(e, "reading kernel timings");
    if (e == hipSuccess && r.kind >= 0 && r.kind < kProfClasses) {
      c[r.kind] += 1;
      t[r.kind] += ms;
    }
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  if (rc != VP_OK) return rc;
  for (int i = 0; i < kProfClasses; ++i) {
    counts[i] = c[i];
    total_ms[i] = t[i];
  }
  return VP_OK;
}

}  // extern "C"
