// vp_peel.cpp -- vp_peel: predict a source's model, calibrate it against the
// data per (time, channel) and subtract the gain-corrupted model (Sec. 5.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/vp.h"
#include "vp_internal.h"
#include "vp_objects.h"

using namespace vp;

extern "C" {

int vp_peel(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, const int32_t *ant1, const int32_t *ant2,
            int32_t n_ant, int32_t n_iter, int precision, int dtype, void *data_dev, void *gains_dev,
            void *hip_stream) {
  TraceRange tr("vp_peel");
  int rc = check_call(ctx, sky, obs, precision, dtype, data_dev);
  if (rc != VP_OK) return rc;
  if (!ant1 || !ant2) return set_error(VP_EINVAL, "NULL tile arrays");
  if (n_ant < 2 || n_ant > VP_PEEL_MAX_ANT)
    return set_error(VP_EINVAL, "n_ant %d outside 2..%d", n_ant, VP_PEEL_MAX_ANT);
  if (n_iter < 0 || n_iter > VP_PEEL_MAX_ITER)
    return set_error(VP_EINVAL, "n_iter %d outside 0..%d", n_iter, VP_PEEL_MAX_ITER);
  const int B = obs->B;
  if ((int64_t)obs->T * obs->K > 0x7fffffff) return set_error(VP_EINVAL, "too many (time, channel) cells");
  const int npairs = n_ant * (n_ant - 1) / 2;
  // tables: ant1 [B], ant2 [B], baseline of each tile pair [npairs], and
  // the connected component of each tile [n_ant] (-1: no baseline)
  std::vector<int32_t> tab((size_t)2 * B + npairs + n_ant, -1);
  for (int b = 0; b < B; ++b) {
    const int i = ant1[b], j = ant2[b];
    if (i < 0 || j < 0 || i >= n_ant || j >= n_ant || i == j)
      return set_error(VP_EINVAL, "baseline %d joins tiles %d and %d", b, i, j);
    const int lo = std::min(i, j), hi = std::max(i, j);
    int32_t &slot = tab[(size_t)2 * B + (size_t)lo * n_ant - (size_t)lo * (lo + 1) / 2 + (hi - lo - 1)];
    if (slot >= 0) return set_error(VP_EINVAL, "baselines %d and %d join the same tiles", slot, b);
    slot = b;
    tab[b] = i;
    tab[(size_t)B + b] = j;
  }
  bool single = true;  // every tile with a baseline in one component
  {
    // union-find over the baselines; a component is named by its root tile
    std::vector<int32_t> up(n_ant);
    for (int k = 0; k < n_ant; ++k) up[k] = k;
    auto root = [&](int k) {
      while (up[k] != k) k = up[k] = up[up[k]];
      return k;
    };
    std::vector<char> used(n_ant, 0);
    for (int b = 0; b < B; ++b) {
      const int ri = root(ant1[b]), rj = root(ant2[b]);
      used[ant1[b]] = used[ant2[b]] = 1;
      if (ri != rj) up[std::max(ri, rj)] = std::min(ri, rj);
    }
    int32_t *comp = tab.data() + 2 * (size_t)B + npairs;
    for (int k = 0; k < n_ant; ++k) comp[k] = used[k] ? root(k) : -1;
    for (int k = 0; k < n_ant; ++k)
      if (comp[k] >= 0 && comp[k] != root(ant1[0])) single = false;
  }
  if (!gain_supported(n_ant)) return set_error(VP_EINVAL, "%d tiles not supported by the gain solve", n_ant);
  DeviceGuard g(ctx->device);
  if (!g.ok) return set_error(VP_EDEVICE, "cannot select device");
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->peel) ctx->peel = new PeelWork();
  }
  PeelWork &w = *ctx->peel;
  std::lock_guard<std::mutex> lk(w.mu);
  hipError_t e = hipSuccess;
  // the previous call's kernels have finished with the workspace
  if (w.done) e = hipEventSynchronize(w.done);
  if (e != hipSuccess) return hip_error(e, "waiting for the previous peel");
  const size_t mbytes = (size_t)obs->T * B * obs->K * (dtype == VP_C64 ? 8 : 16);
  const int64_t cells = (int64_t)obs->T * obs->K;
  // the FP64 path keeps its tables and the operator in FP64 (the latter where it fits)
  const bool w32 = precision != VP_PREC_FP64;
  const size_t cell_bytes = gain_cell_bytes(n_ant, w32);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(cells, (int64_t)(kPeelWsMax / cell_bytes)));
  const size_t wsbytes = (size_t)chunk * cell_bytes;
  const size_t gwbytes = (size_t)cells * n_ant * sizeof(double2);
  if (mbytes > w.model_bytes || tab.size() > w.tab_n || wsbytes > w.ws_bytes || gwbytes > w.gw_bytes) {
    w.mem.release();
    w.model = w.ws = w.gw = nullptr;
    w.tab = nullptr;
    w.model_bytes = std::max(mbytes, w.model_bytes);
    w.tab_n = std::max(tab.size(), w.tab_n);
    w.ws_bytes = std::max(wsbytes, w.ws_bytes);
    w.gw_bytes = std::max(gwbytes, w.gw_bytes);
    e = w.mem.alloc(&w.model, w.model_bytes);
    if (e == hipSuccess) e = w.mem.alloc((void **)&w.tab, sizeof(int32_t) * w.tab_n);
    if (e == hipSuccess) e = w.mem.alloc(&w.ws, w.ws_bytes);
    if (e == hipSuccess) e = w.mem.alloc(&w.gw, w.gw_bytes);
    if (e != hipSuccess) {
      w.mem.release();
      w.model = w.ws = w.gw = nullptr;
      w.tab = nullptr;
      w.model_bytes = w.tab_n = w.ws_bytes = w.gw_bytes = 0;
      return hip_error(e, "allocating the peel workspace");
    }
  }
  e = hipMemcpy(w.tab, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_error(e, "uploading the baseline tables");
  hipStream_t s = (hipStream_t)hip_stream;
  rc = run_tiles(ctx, sky, obs, precision, dtype, w.model, 0, s);
  if (rc != VP_OK) return rc;
  GainArgs a;
  a.T = obs->T;
  a.B = B;
  a.K = obs->K;
  a.n_ant = n_ant;
  a.n_iter = n_iter;
  a.max_cg = VP_PEEL_MAX_CG;
  // relative residual at which a step's conjugate-gradient solve stops: 1e-12
  // with FP64 tables and operator; 1e-6 on the mixed path, whose operator
  // (FP32 W and FP32 products) is itself accurate to ~1e-7 only, so that
  // iterating further refines nothing (the Gauss-Newton fixed point is set by
  // the right-hand side, which keeps its FP64 sums)
  a.cg_tol2 = w32 ? 1e-12 : 1e-24;
  a.model = w.model;
  a.data = data_dev;
  a.c64 = dtype == VP_C64;
  a.ant1 = w.tab;
  a.ant2 = w.tab + B;
  a.pair_bl = w.tab + 2 * (size_t)B;
  a.comp = a.pair_bl + npairs;
  a.gains = (double2 *)gains_dev;
  a.gw = (double2 *)w.gw;
  a.w32 = w32;
  a.single_comp = single ? 1 : 0;
  a.xt = w.ws;
  a.wf = (char *)w.ws + (size_t)chunk * n_ant * n_ant * (w32 ? sizeof(float2) : sizeof(double2));
  {
    ProfScope ps(ctx, s, 3);
    for (int64_t c0 = 0; c0 < cells && e == hipSuccess; c0 += chunk) {
      a.cell0 = (int)c0;
      a.ncell = (int)std::min<int64_t>(chunk, cells - c0);
      e = launch_gain(a, s);
    }
    if (e == hipSuccess) e = launch_gain_subtract(a, s);
  }
  if (e != hipSuccess) return hip_error(e, "launching the gain solve");
  if (!w.done) e = hipEventCreateWithFlags(&w.done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(w.done, s);
  if (e != hipSuccess) return hip_error(e, "recording the peel event");
  return VP_OK;
}

}  // extern "C"
