// vp_serve.cpp -- serving entry points (continuous batching).
#include <hip/hip_runtime.h>

#include "../../include/vp.h"
#include "vp_objects.h"

namespace vp {
bool serve_pending(vp_ctx *) { return false; }
void serve_shutdown(vp_ctx *) {}
}  // namespace vp

using namespace vp;

extern "C" {
int vp_submit(vp_ctx *ctx, const vp_job *job, uint64_t *ticket) {
  (void)ctx; (void)job; (void)ticket;
  return set_error(VP_EINVAL, "serving is not available in this build");
}
int vp_poll(vp_ctx *ctx, uint64_t ticket, vp_job_result *res) {
  (void)ctx; (void)ticket; (void)res;
  return set_error(VP_ENOTFOUND, "unknown ticket");
}
int vp_job_footprint(vp_ctx *ctx, const vp_job *job, uint64_t *bytes) {
  (void)ctx; (void)job; (void)bytes;
  return set_error(VP_EINVAL, "serving is not available in this build");
}
}
