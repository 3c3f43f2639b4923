// Pre-scaled, pooled SSIM: the down-sampling transform of the
// Transforming-across-Scales subsection (an f x f block average, f = max(1,
// ceil(H/256)) unless given), the SSIM map on the down-sampled planes, and a
// spatial pooling method of the aggregation section.  With an 11x11
// rectangular window at stride 5 and CoV pooling this is the paper's
// "Enhanced SSIM" composition.
#include "launch.hpp"
#include "host_common.hpp"
#include "ssimx_internal.hpp"

#include <algorithm>

namespace ssimx {

namespace {

int resolve_factor(int factor, int H) { return factor > 0 ? factor : std::max(1, (H + 255) / 256); }

struct ScaledLayout {
  int f, W, H, Wo, Ho, dtype;
  size_t planes_off, map_off, fwd_off, pool_off, total;
};

ssimx_status scaled_layout(const ssimx_params* p, int factor, const ssimx_pool* pool, int dtype, int W, int H,
                           int batch, ScaledLayout& L) {
  L.f = resolve_factor(factor, H);
  L.W = W / L.f;
  L.H = H / L.f;
  if (L.W < 1 || L.H < 1) return SSIMX_ETOOSMALL;
  L.dtype = L.f > 1 ? SSIMX_F32 : dtype;
  map_dims(p, L.W, L.H, L.Wo, L.Ho);
  if (L.Wo < 1 || L.Ho < 1) return SSIMX_ETOOSMALL;
  Ws ws;
  L.planes_off = ws.take(L.f > 1 ? sizeof(float) * 2 * (size_t)batch * L.W * L.H : 0);
  L.map_off = ws.take(sizeof(float) * (size_t)batch * L.Wo * L.Ho);
  L.fwd_off = ws.take(fwd_ws_bytes(p, L.dtype, L.W, L.H, batch));
  L.pool_off = ws.take(pool_ws_bytes(pool, L.Wo, L.Ho, batch));
  L.total = ws.used;
  return SSIMX_OK;
}

ssimx_status check_scaled(const ssimx_params* p, int factor, const ssimx_pool* pool, int dtype) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if ((s = check_pool(pool)) != SSIMX_OK) return s;
  if (factor < 0) return SSIMX_EINVAL;
  if (dtype < SSIMX_U8 || dtype > SSIMX_BF16) return SSIMX_EDTYPE;
  // down-sampled planes are float32: the integral-image method needs integer planes
  if (factor != 1 && p->algo == SSIMX_ALGO_INTEGRAL_IMAGE) return SSIMX_ENOTSUP;
  return check_path(p, dtype);
}

}  // namespace

}  // namespace ssimx

using namespace ssimx;

extern "C" {

ssimx_status ssimx_scaled_pooled_workspace_size(const ssimx_params* p, int factor, const ssimx_pool* pool, int dtype,
                                                int w, int h, int batch, size_t* bytes) {
  ssimx_status s;
  if ((s = check_scaled(p, factor, pool, dtype)) != SSIMX_OK) return s;
  if (!bytes || batch < 1 || batch > kMaxGridY) return SSIMX_EINVAL;
  ScaledLayout L{};
  if ((s = scaled_layout(p, factor, pool, dtype, w, h, batch, L)) != SSIMX_OK) return s;
  *bytes = L.total;
  return SSIMX_OK;
}

ssimx_status ssimx_scaled_pooled_ssim(const ssimx_params* p, int factor, const ssimx_pool* pool,
                                      const ssimx_image* ref, const ssimx_image* dis, int batch, float* score_out,
                                      void* ws, size_t ws_bytes, void* stream) {
  ssimx_status s;
  if ((s = check_images(ref, dis, batch)) != SSIMX_OK) return s;
  if ((s = check_scaled(p, factor, pool, ref->dtype)) != SSIMX_OK) return s;
  if (!score_out) return SSIMX_EINVAL;
  ScaledLayout L{};
  if ((s = scaled_layout(p, factor, pool, ref->dtype, ref->width, ref->height, batch, L)) != SSIMX_OK) return s;
  if (!ws || ws_bytes < L.total) return SSIMX_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  PlaneArg x{ref->data, ref->pitch, ref->batch_stride}, y{dis->data, dis->pitch, dis->batch_stride};
  if (L.f > 1) {
    float* px = (float*)(base + L.planes_off);
    float* py = px + (size_t)batch * L.W * L.H;
    const int err = launch_downsample_f(ref->dtype, x, y, ref->width, ref->height, L.f, px, py, batch, st);
    if (err) return hip_status(err);
    x = PlaneArg{px, L.W, (int64_t)L.W * L.H};
    y = PlaneArg{py, L.W, (int64_t)L.W * L.H};
  }
  float* map = (float*)(base + L.map_off);
  // the forward workspace as ssim_map lays it out: pooled partials, then the
  // integral images when that method is asked for
  Ws fl;
  float* partial = (float*)(base + L.fwd_off + fl.take(sizeof(float) * (size_t)batch *
                                                       max_partials(p, L.dtype, L.W, L.H)));
  uint32_t* sat = nullptr;
  if (choose_path(p, L.dtype) == Path::kSat)
    sat = (uint32_t*)(base + L.fwd_off + fl.take(sizeof(uint32_t) * 5 * (size_t)batch * (L.W + 1) * (size_t)(L.H + 1)));
  const int tile = pick_tile(p, L.dtype, L.W, L.H, batch);
  s = fwd_pass(p, L.dtype, x, y, L.W, L.H, batch, 0, map, L.Wo, (int64_t)L.Wo * L.Ho, nullptr, 0, partial, sat, tile,
               st);
  if (s != SSIMX_OK) return s;
  return pool_run(pool, map, L.Wo, L.Ho, L.Wo, (int64_t)L.Wo * L.Ho, batch, score_out, 1, base + L.pool_off, st);
}

}  // extern "C"
