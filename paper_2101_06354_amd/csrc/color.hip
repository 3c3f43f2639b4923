// Channel-wise colour SSIM (Channel-wise SSIM subsection): YCbCr by the
// BT.709 transform printed there (Y = 0.213 R + 0.715 G + 0.072 B,
// Cb = 0.539 (B - Y), Cr = 0.635 (R - Y)), the pooled SSIM of each channel,
// and (f(Y) + alpha f(Cb) + beta f(Cr)) / (1 + alpha + beta).
//
// 8-bit RGB on the stride-1 Gaussian band path: the band kernel reads the R,
// G, B planes and forms each channel while staging its tile (staged frame
// 3 b + c is channel c of frame b), so no channel planes are stored.
// Otherwise the three channel planes of a frame are written as three
// consecutive float32 frames and one batched windowed pass over 3 B frames
// serves every channel.  A small kernel forms the weighted average.
#include <math.h>

#include "fast_tile.hpp"
#include "launch.hpp"
#include "host_common.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

namespace {

constexpr float kY709R = 0.213f, kY709G = 0.715f, kY709B = 0.072f, kCb709 = 0.539f, kCr709 = 0.635f;

template <typename T>
__global__ __launch_bounds__(BLOCK) void rgb_to_ycbcr_kernel(const T* rgb, int W, int H, int64_t pitch,
                                                             int64_t cstride, int64_t bstride, float* out) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W * H) return;
  const int b = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const T* p = rgb + (int64_t)b * bstride + (int64_t)r * pitch + c;
  const float R = to_f32<T>(p[0]), G = to_f32<T>(p[cstride]), B = to_f32<T>(p[2 * cstride]);
  const float Y = fmaf(kY709R, R, fmaf(kY709G, G, kY709B * B));
  float* o = out + (int64_t)b * 3 * W * H + idx;
  o[0] = Y;
  o[(int64_t)W * H] = kCb709 * (B - Y);
  o[2 * (int64_t)W * H] = kCr709 * (R - Y);
}

__global__ void color_combine_kernel(const float* ch, int batch, float alpha, float beta, float* out, float* ch_out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const float y = ch[3 * b], cb = ch[3 * b + 1], cr = ch[3 * b + 2];
  out[b] = (float)(((double)y + (double)alpha * cb + (double)beta * cr) / (1.0 + (double)alpha + (double)beta));
  if (ch_out) {
    ch_out[3 * b] = y;
    ch_out[3 * b + 1] = cb;
    ch_out[3 * b + 2] = cr;
  }
}

struct ColorLayout {
  size_t planes_off, scores_off, fwd_off, total;
};

ColorLayout color_layout(const ssimx_params* p, int w, int h, int batch) {
  ColorLayout L{};
  Ws ws;
  L.planes_off = ws.take(sizeof(float) * 2 * 3 * (size_t)batch * w * h);
  L.scores_off = ws.take(sizeof(float) * 3 * (size_t)batch);
  L.fwd_off = ws.take(fwd_ws_bytes(p, SSIMX_F32, w, h, 3 * batch));
  L.total = ws.used;
  return L;
}

ssimx_status check_color(const ssimx_params* p, double alpha, double beta, int dtype) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if (!isfinite(alpha) || !isfinite(beta) || 1.0 + alpha + beta == 0.0) return SSIMX_EINVAL;
  if (dtype != SSIMX_U8 && dtype != SSIMX_U16 && dtype != SSIMX_F32 && dtype != SSIMX_BF16) return SSIMX_EDTYPE;
  if (p->algo == SSIMX_ALGO_INTEGRAL_IMAGE) return SSIMX_ENOTSUP;  // channel planes are float32
  return check_path(p, SSIMX_F32);
}

template <typename T>
void launch_ycbcr(const void* rgb, int w, int h, int64_t pitch, int64_t cs, int64_t bs, int batch, float* out,
                  hipStream_t st) {
  dim3 grid((w * h + BLOCK - 1) / BLOCK, batch);
  hipLaunchKernelGGL(rgb_to_ycbcr_kernel<T>, grid, dim3(BLOCK), 0, st, (const T*)rgb, w, h, pitch, cs, bs, out);
}

}  // namespace

}  // namespace ssimx

using namespace ssimx;

extern "C" {

ssimx_status ssimx_color_workspace_size(const ssimx_params* p, int w, int h, int batch, size_t* bytes) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if (!bytes || batch < 1 || 3 * (int64_t)batch > kMaxGridY) return SSIMX_EINVAL;
  int Wo, Ho;
  map_dims(p, w, h, Wo, Ho);
  if (w < 1 || h < 1 || Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  *bytes = color_layout(p, w, h, batch).total;
  return SSIMX_OK;
}

ssimx_status ssimx_color_ssim(const ssimx_params* p, double alpha, double beta, const void* ref_rgb,
                              const void* dis_rgb, int dtype, int w, int h, int64_t pitch, int64_t channel_stride,
                              int64_t batch_stride, int batch, float* score_out, float* channel_scores, void* ws,
                              size_t ws_bytes, void* stream) {
  ssimx_status s;
  if ((s = check_color(p, alpha, beta, dtype)) != SSIMX_OK) return s;
  if (!ref_rgb || !dis_rgb || !score_out || batch < 1 || 3 * (int64_t)batch > kMaxGridY) return SSIMX_EINVAL;
  if (w < 1 || h < 1) return SSIMX_ETOOSMALL;
  if ((int64_t)w * h > kMaxPlaneElems) return SSIMX_EINVAL;
  if (pitch < w || channel_stride < pitch * (int64_t)h || (batch > 1 && batch_stride < 3 * channel_stride))
    return SSIMX_EINVAL;
  int Wo, Ho;
  map_dims(p, w, h, Wo, Ho);
  if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  const ColorLayout L = color_layout(p, w, h, batch);
  if (!ws || ws_bytes < L.total) return SSIMX_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  float* scores = (float*)(base + L.scores_off);
  if (dtype == SSIMX_U8 && use_fast(p, SSIMX_F32)) {
    const int tile = pick_tile(p, SSIMX_F32, w, h, 3 * batch);
    const Geom g = fast_geom(p, w, h, tile, 3 * batch);
    FastArgs a{};
    fill_fast_common(a, p, SSIMX_U8, PlaneArg{ref_rgb, pitch, batch_stride}, PlaneArg{dis_rgb, pitch, batch_stride},
                     g);
    a.vec_ok = a.vec_ok && channel_stride % 4 == 0;
    a.cstride = channel_stride;
    a.mode = 0;
    a.partial = (float*)(base + L.fwd_off);
    a.batch = 3 * batch;
    int err = launch_fast_stats_rgb(a, batch, st);
    if (!err) err = launch_finalize(a.partial, g.tiles_x * g.tiles_y, 3 * batch, g.Wo * g.Ho, 1.f, scores, 1, st);
    if (err) return hip_status(err);
    hipLaunchKernelGGL(color_combine_kernel, dim3((batch + 63) / 64), dim3(64), 0, st, scores, batch, (float)alpha,
                       (float)beta, score_out, channel_scores);
    return hip_status((int)hipGetLastError());
  }
  float* px = (float*)(base + L.planes_off);
  float* py = px + 3 * (size_t)batch * w * h;
  for (int side = 0; side < 2; ++side) {
    const void* src = side ? dis_rgb : ref_rgb;
    float* dst = side ? py : px;
    switch (dtype) {
      case SSIMX_U8: launch_ycbcr<uint8_t>(src, w, h, pitch, channel_stride, batch_stride, batch, dst, st); break;
      case SSIMX_U16: launch_ycbcr<uint16_t>(src, w, h, pitch, channel_stride, batch_stride, batch, dst, st); break;
      case SSIMX_F32: launch_ycbcr<float>(src, w, h, pitch, channel_stride, batch_stride, batch, dst, st); break;
      default: launch_ycbcr<bf16_t>(src, w, h, pitch, channel_stride, batch_stride, batch, dst, st); break;
    }
  }
  int err = (int)hipGetLastError();
  if (err) return hip_status(err);
  PlaneArg x{px, w, (int64_t)w * h}, y{py, w, (int64_t)w * h};
  const int tile = pick_tile(p, SSIMX_F32, w, h, 3 * batch);
  s = fwd_pass(p, SSIMX_F32, x, y, w, h, 3 * batch, 0, nullptr, 0, 0, scores, 1, (float*)(base + L.fwd_off), nullptr,
               tile, st);
  if (s != SSIMX_OK) return s;
  hipLaunchKernelGGL(color_combine_kernel, dim3((batch + 63) / 64), dim3(64), 0, st, scores, batch, (float)alpha,
                     (float)beta, score_out, channel_scores);
  return hip_status((int)hipGetLastError());
}

}  // extern "C"
