// Pooling finalisation, 2x2 pyramid and the MS-SSIM product.
#include "launch.hpp"
#include "host_common.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

// Mean of each frame's tile partials (mean SSIM of the Background section),
// summed in a fixed order with a compensated (TwoSum) tree so the result is
// deterministic and carries about twice float32 precision.
__global__ __launch_bounds__(BLOCK) void finalize_kernel(const float* partial, int tiles, float inv_count, float* out,
                                                         int64_t out_stride) {
  __shared__ float hs[BLOCK], ls[BLOCK];
  const int frame = blockIdx.x;
  const float m = tile_mean(partial + (int64_t)frame * tiles, tiles, inv_count, hs, ls);
  if (threadIdx.x == 0) out[(int64_t)frame * out_stride] = m;
}

int launch_finalize(const float* partial, int tiles, int batch, int count_per_frame, float /*scale*/, float* out,
                    int64_t out_stride, hipStream_t st) {
  const float inv = (float)(1.0 / (double)count_per_frame);
  hipLaunchKernelGGL(finalize_kernel, dim3(batch), dim3(BLOCK), 0, st, partial, tiles, inv, out, out_stride);
  return (int)hipGetLastError();
}

// 2x2 average of aligned blocks (odd last row / column dropped), written as
// float32 [batch][H/2][W/2].  For integer planes the result is exact.
template <typename T>
__global__ __launch_bounds__(BLOCK) void downsample_kernel(PlaneArg xa, PlaneArg ya, int W2, int H2, float* ox,
                                                           float* oy) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W2 * H2) return;
  const int frame = blockIdx.y;
  const int r = idx / W2, c = idx - r * W2;
  const int64_t o = (int64_t)frame * W2 * H2 + idx;
  {
    const T* X = (const T*)xa.data + (int64_t)frame * xa.bstride + (int64_t)(2 * r) * xa.pitch + 2 * c;
    const float a = to_f32<T>(X[0]), b = to_f32<T>(X[1]), d = to_f32<T>(X[xa.pitch]), e = to_f32<T>(X[xa.pitch + 1]);
    ox[o] = 0.25f * (((a + b) + d) + e);
  }
  {
    const T* Y = (const T*)ya.data + (int64_t)frame * ya.bstride + (int64_t)(2 * r) * ya.pitch + 2 * c;
    const float a = to_f32<T>(Y[0]), b = to_f32<T>(Y[1]), d = to_f32<T>(Y[ya.pitch]), e = to_f32<T>(Y[ya.pitch + 1]);
    oy[o] = 0.25f * (((a + b) + d) + e);
  }
}

int launch_downsample(int dtype, PlaneArg in, int W, int H, float* outx, float* outy, PlaneArg iny, int batch,
                      hipStream_t st) {
  const int W2 = W / 2, H2 = H / 2;
  if (W2 < 1 || H2 < 1) return (int)hipErrorInvalidValue;
  dim3 grid((W2 * H2 + BLOCK - 1) / BLOCK, batch);
  switch (dtype) {
    case SSIMX_U8:
      hipLaunchKernelGGL(downsample_kernel<uint8_t>, grid, dim3(BLOCK), 0, st, in, iny, W2, H2, outx, outy);
      break;
    case SSIMX_U16:
      hipLaunchKernelGGL(downsample_kernel<uint16_t>, grid, dim3(BLOCK), 0, st, in, iny, W2, H2, outx, outy);
      break;
    case SSIMX_F32:
      hipLaunchKernelGGL(downsample_kernel<float>, grid, dim3(BLOCK), 0, st, in, iny, W2, H2, outx, outy);
      break;
    case SSIMX_BF16:
      hipLaunchKernelGGL(downsample_kernel<bf16_t>, grid, dim3(BLOCK), 0, st, in, iny, W2, H2, outx, outy);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// f x f block means (pre-scaling by an integer factor; remainders dropped),
// float32 [batch][H/f][W/f].  The block sum is exact for integer planes and is
// divided once (correctly rounded mean).  One thread per output, its block
// summed row by row.  Factors 2..9 (the pre-scaling factors of frames up to
// 2304 rows) are compile-time constants, so all f * f loads of a block are in
// flight together; other factors take the runtime loop, in the same order.
template <typename T, int F>
__device__ __forceinline__ float block_sum(const T* P, int64_t pitch, int f) {
  float s = 0.f;
  if constexpr (F > 0) {
    float v[F][F];
#pragma unroll
    for (int i = 0; i < F; ++i)
#pragma unroll
      for (int j = 0; j < F; ++j) v[i][j] = to_f32<T>(P[(int64_t)i * pitch + j]);
#pragma unroll
    for (int i = 0; i < F; ++i)
#pragma unroll
      for (int j = 0; j < F; ++j) s += v[i][j];
  } else {
    for (int i = 0; i < f; ++i)
      for (int j = 0; j < f; ++j) s += to_f32<T>(P[(int64_t)i * pitch + j]);
  }
  return s;
}

template <typename T, int F>
__global__ __launch_bounds__(BLOCK) void downsample_f_kernel(PlaneArg xa, PlaneArg ya, int Wf, int Hf, int f,
                                                             float* ox, float* oy) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= Wf * Hf) return;
  const int frame = blockIdx.y;
  const int r = idx / Wf, c = idx - r * Wf;
  const int64_t o = (int64_t)frame * Wf * Hf + idx;
  const float ff = (float)(f * f);
  const T* PX = (const T*)xa.data + (int64_t)frame * xa.bstride + (int64_t)(f * r) * xa.pitch + (int64_t)f * c;
  const T* PY = (const T*)ya.data + (int64_t)frame * ya.bstride + (int64_t)(f * r) * ya.pitch + (int64_t)f * c;
  ox[o] = block_sum<T, F>(PX, xa.pitch, f) / ff;
  oy[o] = block_sum<T, F>(PY, ya.pitch, f) / ff;
}

template <typename T>
int launch_downsample_f_t(PlaneArg x, PlaneArg y, int Wf, int Hf, int f, float* outx, float* outy, int batch,
                          hipStream_t st) {
  const dim3 grid((Wf * Hf + BLOCK - 1) / BLOCK, batch);
#define SSIMX_DSF(FF)                                                                                              \
  case FF:                                                                                                         \
    hipLaunchKernelGGL((downsample_f_kernel<T, FF>), grid, dim3(BLOCK), 0, st, x, y, Wf, Hf, f, outx, outy);       \
    break;
  switch (f) {
    SSIMX_DSF(2)
    SSIMX_DSF(3)
    SSIMX_DSF(4)
    SSIMX_DSF(5)
    SSIMX_DSF(6)
    SSIMX_DSF(7)
    SSIMX_DSF(8)
    SSIMX_DSF(9)
    default:
      hipLaunchKernelGGL((downsample_f_kernel<T, 0>), grid, dim3(BLOCK), 0, st, x, y, Wf, Hf, f, outx, outy);
  }
#undef SSIMX_DSF
  return (int)hipGetLastError();
}

int launch_downsample_f(int dtype, PlaneArg x, PlaneArg y, int W, int H, int f, float* outx, float* outy, int batch,
                        hipStream_t st) {
  const int Wf = W / f, Hf = H / f;
  if (f < 1 || Wf < 1 || Hf < 1) return (int)hipErrorInvalidValue;
  switch (dtype) {
    case SSIMX_U8: return launch_downsample_f_t<uint8_t>(x, y, Wf, Hf, f, outx, outy, batch, st);
    case SSIMX_U16: return launch_downsample_f_t<uint16_t>(x, y, Wf, Hf, f, outx, outy, batch, st);
    case SSIMX_F32: return launch_downsample_f_t<float>(x, y, Wf, Hf, f, outx, outy, batch, st);
    case SSIMX_BF16: return launch_downsample_f_t<bf16_t>(x, y, Wf, Hf, f, outx, outy, batch, st);
    default: return (int)hipErrorInvalidValue;
  }
}

struct MsWeights {
  float w[MAX_SCALES];
};

// score = S_M^{w_M} * prod_{j<M} CS_j^{w_j}; vals[frame][j] holds CS_j for
// j < M-1 and S_M at M-1.  powf of a negative base with a fractional exponent
// is NaN, which propagates unless clamping is asked for.
// Weighted product S_M^{w_M} prod CS_j^{w_j}, or (sum != 0) the weighted
// average sum w_j T_j of the same terms with weights that sum to one.  lvals
// (nullable): the coarsest term is vals * lvals (mean(l) * mean(cs)).
__global__ void ms_combine_kernel(const float* vals, int n_scales, int batch, MsWeights w, int clamp, int sum,
                                  const float* lvals, float* score_out, float* cs_out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= batch) return;
  score_out[f] = ms_combine_frame(vals + (int64_t)f * n_scales, n_scales, w.w, clamp, sum, lvals ? lvals[f] : 1.f,
                                  lvals != nullptr, cs_out ? cs_out + (int64_t)f * n_scales : nullptr);
}

int launch_ms_combine(const float* vals, int n_scales, int batch, const float* w, int flags, float* score_out,
                      float* cs_out, const float* lvals, hipStream_t st) {
  MsWeights mw{};
  for (int j = 0; j < n_scales && j < MAX_SCALES; ++j) mw.w[j] = w[j];
  hipLaunchKernelGGL(ms_combine_kernel, dim3((batch + 63) / 64), dim3(64), 0, st, vals, n_scales, batch, mw,
                     (flags & SSIMX_MS_CS_CLAMP) ? 1 : 0, (flags & SSIMX_MS_SUM) ? 1 : 0, lvals, score_out, cs_out);
  return (int)hipGetLastError();
}

// BT.601 luma of planar RGB and its adjoint.

template <typename T>
__global__ __launch_bounds__(BLOCK) void rgb_to_luma_kernel(const T* rgb, int W, int H, int64_t pitch, int64_t cstride,
                                                            int64_t bstride, float* y) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W * H) return;
  const int b = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const T* p = rgb + (int64_t)b * bstride + (int64_t)r * pitch + c;
  const float R = to_f32<T>(p[0]), G = to_f32<T>(p[cstride]), B = to_f32<T>(p[2 * cstride]);
  y[(int64_t)b * W * H + idx] = fmaf(kBt601R, R, fmaf(kBt601G, G, kBt601B * B));
}

__global__ __launch_bounds__(BLOCK) void luma_grad_to_rgb_kernel(const float* gy, int W, int H, float* g,
                                                                 int64_t pitch, int64_t cstride, int64_t bstride) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W * H) return;
  const int b = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const float v = gy[(int64_t)b * W * H + idx];
  float* p = g + (int64_t)b * bstride + (int64_t)r * pitch + c;
  p[0] = kBt601R * v;
  p[cstride] = kBt601G * v;
  p[2 * cstride] = kBt601B * v;
}

}  // namespace ssimx

using namespace ssimx;

extern "C" {

ssimx_status ssimx_rgb_to_luma(const void* rgb, int dtype, int width, int height, int64_t pitch,
                               int64_t channel_stride, int64_t batch_stride, int batch, float* y_out,
                               void* stream) {
  if (!rgb || !y_out || width < 1 || height < 1 || batch < 1 || batch > kMaxGridY || pitch < width)
    return SSIMX_EINVAL;
  if ((int64_t)width * height > kMaxPlaneElems) return SSIMX_EINVAL;
  if (channel_stride < pitch * (int64_t)height || (batch > 1 && batch_stride < 3 * channel_stride))
    return SSIMX_EINVAL;
  dim3 grid((width * height + BLOCK - 1) / BLOCK, batch);
  hipStream_t st = (hipStream_t)stream;
  if (dtype == SSIMX_F32)
    hipLaunchKernelGGL(rgb_to_luma_kernel<float>, grid, dim3(BLOCK), 0, st, (const float*)rgb, width, height, pitch,
                       channel_stride, batch_stride, y_out);
  else if (dtype == SSIMX_BF16)
    hipLaunchKernelGGL(rgb_to_luma_kernel<bf16_t>, grid, dim3(BLOCK), 0, st, (const bf16_t*)rgb, width, height,
                       pitch, channel_stride, batch_stride, y_out);
  else
    return SSIMX_EDTYPE;
  return hip_status((int)hipGetLastError());
}

ssimx_status ssimx_luma_grad_to_rgb(const float* grad_y, int width, int height, int batch, float* grad_rgb,
                                    int64_t pitch, int64_t channel_stride, int64_t batch_stride, void* stream) {
  if (!grad_y || !grad_rgb || width < 1 || height < 1 || batch < 1 || batch > kMaxGridY || pitch < width)
    return SSIMX_EINVAL;
  if ((int64_t)width * height > kMaxPlaneElems) return SSIMX_EINVAL;
  if (channel_stride < pitch * (int64_t)height || (batch > 1 && batch_stride < 3 * channel_stride))
    return SSIMX_EINVAL;
  dim3 grid((width * height + BLOCK - 1) / BLOCK, batch);
  hipLaunchKernelGGL(luma_grad_to_rgb_kernel, grid, dim3(BLOCK), 0, (hipStream_t)stream, grad_y, width, height,
                     grad_rgb, pitch, channel_stride, batch_stride);
  return hip_status((int)hipGetLastError());
}

}  // extern "C"
