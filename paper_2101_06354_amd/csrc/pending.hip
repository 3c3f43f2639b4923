// Entry points whose kernels are not in this build yet: they validate
// nothing and report SSIMX_ENOTSUP.
#include "host_common.hpp"

using namespace ssimx;

extern "C" {
ssimx_status ssim_map_backward(const ssimx_params*, const ssimx_image*, const ssimx_image*, int, const float*,
                               int64_t, int64_t, float*, int64_t, int64_t, void*, size_t, void*) {
  return SSIMX_ENOTSUP;
}
ssimx_status ssim_pooled_backward(const ssimx_params*, const ssimx_image*, const ssimx_image*, int, const float*,
                                  float*, int64_t, int64_t, void*, size_t, void*) {
  return SSIMX_ENOTSUP;
}
ssimx_status msssim_backward(const ssimx_params*, const float*, int, int, const ssimx_image*, const ssimx_image*,
                             int, const float*, float*, int64_t, int64_t, void*, size_t, void*) {
  return SSIMX_ENOTSUP;
}
ssimx_status ssimx_plan_create(const ssimx_pair*, int, void*, ssimx_plan**) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_run(ssimx_plan*, float*, void*) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_run_unbatched(ssimx_plan*, float*, void*) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_destroy(ssimx_plan*) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_plan_info(const ssimx_plan*, int*, int*) { return SSIMX_ENOTSUP; }
ssimx_status ssimx_workspace_size(const ssimx_params* p, int op, int dtype, int width, int height, int batch,
                                  int n_scales, size_t* bytes) {
  ssimx_status s = check_params(p);
  if (s != SSIMX_OK) return s;
  if (!bytes || width < 1 || height < 1 || batch < 1) return SSIMX_EINVAL;
  if (op == SSIMX_OP_MAP || op == SSIMX_OP_POOLED) {
    *bytes = fwd_ws_bytes(p, dtype, width, height, batch);
    return SSIMX_OK;
  }
  if (op == SSIMX_OP_MSSSIM) {
    if (n_scales < 1 || n_scales > MAX_SCALES) return SSIMX_EINVAL;
    *bytes = ms_layout(p, dtype, width, height, batch, n_scales).total;
    return SSIMX_OK;
  }
  return SSIMX_ENOTSUP;
}
}
