// The differentiable MS-SSIM loss of the training workload in one call: BT.601
// luma of two planar RGB batches, MS-SSIM of the luma planes, the loss
// mean_b(1 - MS-SSIM_b) and, optionally, its gradient with respect to the
// distorted RGB planes (the adjoint of the same pipeline, with the moments
// recomputed by the backward's coefficient kernels).  The Off-the-shelf
// Performance subsection names MS-SSIM as a training objective for deep
// networks; the luma weights and the loss are the workload's.
//
// ssimx_msssim_loss_rgb runs the launches on the caller's stream.  A loss plan
// owns its workspace and replays the same launches as one HIP graph: the
// graph's kernels read the caller's pointers and strides from a small device
// argument block that each run refreshes with one asynchronous copy from a
// pinned ring slot, so new input or output tensors need no new capture.
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "launch.hpp"
#include "host_common.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {
namespace {

// Caller pointers and strides of one loss evaluation.
struct LossIO {
  const void* ref;
  const void* dis;
  int64_t pitch, cstride, bstride;  // elements
  float* loss;                       // [1]
  float* score;                      // nullable [batch]
  void* grad;                        // nullable [batch][3][H][gpitch]
  int64_t gpitch, gcstride, gbstride;
};

// The kernels take the block by value, or (graph replays) from device memory.
__device__ __forceinline__ const LossIO& io_of(const LossIO& v, const LossIO* d) { return d ? *d : v; }

// Luma of the reference (z = 0) and distorted (z = 1) batch into dense planes,
// in the operation order of ssimx_rgb_to_luma.
template <typename T>
__global__ __launch_bounds__(BLOCK) void loss_luma_kernel(LossIO iov, const LossIO* iod, int W, int H, float* yr,
                                                          float* yd) {
  const LossIO& io = io_of(iov, iod);
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W * H) return;
  const int b = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const T* p = (const T*)(blockIdx.z == 0 ? io.ref : io.dis) + (int64_t)b * io.bstride + (int64_t)r * io.pitch + c;
  const float R = to_f32<T>(p[0]), G = to_f32<T>(p[io.cstride]), B = to_f32<T>(p[2 * io.cstride]);
  (blockIdx.z == 0 ? yr : yd)[(int64_t)b * W * H + idx] = fmaf(kBt601R, R, fmaf(kBt601G, G, kBt601B * B));
}

// Per frame (one workgroup each): the pooled value of every scale from the
// forward's tile partials (the finalize arithmetic), the MS-SSIM score (the
// combine arithmetic), 1 - score, and the upstream of every scale's pooled
// term for dL/dscore = gscore (the adjoint's upstream arithmetic).  One launch
// in place of the per-scale finalize, the combine and the upstream launches;
// the score equals msssim's bit for bit.
struct LossReduceArgs {
  const float* part[MAX_SCALES];
  int tiles[MAX_SCALES];
  float inv[MAX_SCALES];  // 1 / map positions
  float w[MAX_SCALES];
  int M, clamp, sum, split;
  const float* lpart;  // split: tile partials of the coarsest mean(l)
  int ltiles;
  float gscore;
  float *score, *om, *up, *up2;
};

__global__ __launch_bounds__(BLOCK) void loss_reduce_kernel(LossReduceArgs a) {
  __shared__ float hs[BLOCK], ls[BLOCK];
  __shared__ float v[MAX_SCALES + 1];
  const int f = blockIdx.x;
  for (int j = 0; j < a.M; ++j) {
    const float m = tile_mean(a.part[j] + (int64_t)f * a.tiles[j], a.tiles[j], a.inv[j], hs, ls);
    if (threadIdx.x == 0) v[j] = m;
    __syncthreads();
  }
  if (a.split) {
    const float m = tile_mean(a.lpart + (int64_t)f * a.ltiles, a.ltiles, a.inv[a.M - 1], hs, ls);
    if (threadIdx.x == 0) v[MAX_SCALES] = m;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float lval = a.split ? v[MAX_SCALES] : 1.f;
    const float s = ms_combine_frame(v, a.M, a.w, a.clamp, a.sum, lval, a.split != 0, nullptr);
    a.score[f] = s;
    a.om[f] = 1.f - s;
    ms_upstream_frame(v, a.M, lval, a.split != 0, s, a.gscore, a.w, a.inv, a.clamp, a.sum, a.up + (int64_t)f * a.M,
                      a.up2 + f);
  }
}

// loss = mean over the batch of (1 - score) in the finalize's compensated
// tree; the scores copied out.
__global__ __launch_bounds__(BLOCK) void loss_total_kernel(LossIO iov, const LossIO* iod, const float* score,
                                                           const float* om, int batch) {
  const LossIO& io = io_of(iov, iod);
  __shared__ float hs[BLOCK], ls[BLOCK];
  const float loss = tile_mean(om, batch, 1.f / (float)batch, hs, ls);
  if (threadIdx.x == 0) io.loss[0] = loss;
  if (io.score)
    for (int b = threadIdx.x; b < batch; b += BLOCK) io.score[b] = score[b];
}

// Gradient of the RGB planes from the luma gradient (the transpose of the
// luma map), written as float32 or bfloat16 (round to nearest even).
template <typename G>
__global__ __launch_bounds__(BLOCK) void loss_grad_kernel(LossIO iov, const LossIO* iod, const float* gy, int W,
                                                          int H) {
  const LossIO& io = io_of(iov, iod);
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W * H) return;
  const int b = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const float v = gy[(int64_t)b * W * H + idx];
  G* p = (G*)io.grad + (int64_t)b * io.gbstride + (int64_t)r * io.gpitch + c;
  const float g[3] = {kBt601R * v, kBt601G * v, kBt601B * v};
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    if constexpr (std::is_same<G, float>::value) {
      p[ch * io.gcstride] = g[ch];
    } else {
      const uint32_t u = __float_as_uint(g[ch]);
      const uint32_t rnd = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // finite values: nearest even
      bf16_t h;
      h.bits = (uint16_t)(((u & 0x7f800000u) == 0x7f800000u) ? ((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u)) : rnd);
      p[ch * io.gcstride] = h;
    }
  }
}

// Shape of a loss evaluation (everything but the caller's pointers).
struct LossShape {
  ssimx_params p;
  float w[MAX_SCALES];
  int n_scales, flags, dtype, grad_dtype, W, H, batch;
};

struct LossLayout {
  size_t yr, yd, ygrad, score, om, lpart, ms, total;
  MsBwdLayout L;
};

LossLayout loss_layout(const LossShape& sh) {
  LossLayout l{};
  Ws ws;
  const size_t plane = sizeof(float) * (size_t)sh.batch * sh.W * sh.H;
  l.yr = ws.take(plane);
  l.yd = ws.take(plane);
  l.ygrad = ws.take(plane);
  l.score = ws.take(sizeof(float) * sh.batch);
  l.om = ws.take(sizeof(float) * sh.batch);
  l.L = ms_bwd_layout(&sh.p, SSIMX_F32, sh.W, sh.H, sh.batch, sh.n_scales);
  const int M = sh.n_scales;
  l.lpart = ws.take(sizeof(float) * (size_t)sh.batch * max_partials(&sh.p, SSIMX_F32, l.L.fwd.W[M - 1], l.L.fwd.H[M - 1]));
  l.ms = ws.take(0);
  l.total = l.ms + l.L.total;
  return l;
}

ssimx_status check_loss_shape(const ssimx_params* p, const float* weights, int n_scales, int flags, int dtype,
                              int W, int H, int batch) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if (dtype != SSIMX_F32 && dtype != SSIMX_BF16) return SSIMX_EDTYPE;
  if (batch < 1 || batch > kMaxGridY) return SSIMX_EINVAL;
  if (W < 1 || H < 1) return SSIMX_ETOOSMALL;
  if ((int64_t)W * H > kMaxPlaneElems) return SSIMX_EINVAL;
  if (p->k > KMAX_GAUSS) return SSIMX_ENOTSUP;
  if ((s = check_ms(p, weights, n_scales, flags, W, H)) != SSIMX_OK) return s;
  if ((s = check_path(p, SSIMX_F32)) != SSIMX_OK) return s;
  return SSIMX_OK;
}

ssimx_status check_loss_io(const LossShape& sh, const LossIO& io, bool with_grad) {
  if (!io.ref || !io.dis || !io.loss) return SSIMX_EINVAL;
  if (io.pitch < sh.W || io.cstride < io.pitch * (int64_t)sh.H || (sh.batch > 1 && io.bstride < 3 * io.cstride))
    return SSIMX_EINVAL;
  if (with_grad) {
    if (sh.grad_dtype != SSIMX_F32 && sh.grad_dtype != SSIMX_BF16) return SSIMX_EDTYPE;
    if (io.gpitch < sh.W || io.gcstride < io.gpitch * (int64_t)sh.H ||
        (sh.batch > 1 && io.gbstride < 3 * io.gcstride))
      return SSIMX_EINVAL;
  }
  return SSIMX_OK;
}

// Every launch of one loss evaluation on `st`.  iod non-null: the kernels that
// touch caller memory read the pointers from that device block (graph
// capture); else from `io`.
ssimx_status loss_launches(const LossShape& sh, const LossIO& io, const LossIO* iod, bool with_grad, char* ws,
                           hipStream_t st) {
  const LossLayout l = loss_layout(sh);
  float* yr = (float*)(ws + l.yr);
  float* yd = (float*)(ws + l.yd);
  const dim3 gl((sh.W * sh.H + BLOCK - 1) / BLOCK, sh.batch, 2);
  if (sh.dtype == SSIMX_F32)
    hipLaunchKernelGGL(loss_luma_kernel<float>, gl, dim3(BLOCK), 0, st, io, iod, sh.W, sh.H, yr, yd);
  else
    hipLaunchKernelGGL(loss_luma_kernel<bf16_t>, gl, dim3(BLOCK), 0, st, io, iod, sh.W, sh.H, yr, yd);
  int err = (int)hipGetLastError();
  if (err) return hip_status(err);
  const ssimx_image ri{yr, SSIMX_F32, sh.W, sh.H, sh.W, (int64_t)sh.W * sh.H};
  const ssimx_image di{yd, SSIMX_F32, sh.W, sh.H, sh.W, (int64_t)sh.W * sh.H};
  char* msb = ws + l.ms;
  const MsLayout& F = l.L.fwd;
  // the windowed pass of every scale (each writing the next scale's 2x2
  // means), without their finalize launches
  const int M = sh.n_scales;
  const bool split = (sh.flags & SSIMX_MS_COARSE_SEPARATE) != 0;
  LossReduceArgs ra{};
  for (int j = 0; j < M; ++j) {
    const PlaneArg x = j == 0 ? PlaneArg{yr, sh.W, (int64_t)sh.W * sh.H}
                              : PlaneArg{msb + F.lvl_x_off[j], F.W[j], (int64_t)F.W[j] * F.H[j]};
    const PlaneArg y = j == 0 ? PlaneArg{yd, sh.W, (int64_t)sh.W * sh.H}
                              : PlaneArg{msb + F.lvl_y_off[j], F.W[j], (int64_t)F.W[j] * F.H[j]};
    const int mode = (j + 1 < M || split) ? 1 : 0;
    const int tile = pick_tile(&sh.p, SSIMX_F32, F.W[j], F.H[j], sh.batch);
    float* nx = j + 1 < M ? (float*)(msb + F.lvl_x_off[j + 1]) : nullptr;
    float* ny = j + 1 < M ? (float*)(msb + F.lvl_y_off[j + 1]) : nullptr;
    ra.part[j] = (const float*)(msb + F.partial_off[j]);
    ssimx_status s = fwd_pass(&sh.p, SSIMX_F32, x, y, F.W[j], F.H[j], sh.batch, mode, nullptr, 0, 0, nullptr, 0,
                              (float*)ra.part[j], nullptr, tile, st, nx, ny, &ra.tiles[j]);
    if (s != SSIMX_OK) return s;
    int Wo, Ho;
    map_dims(&sh.p, F.W[j], F.H[j], Wo, Ho);
    ra.inv[j] = (float)(1.0 / ((double)Wo * Ho));
    ra.w[j] = sh.w[j];
    if (split && j + 1 == M) {  // coarsest term mean(l) * mean(cs): the l partials too
      ra.lpart = (const float*)(ws + l.lpart);
      s = fwd_pass(&sh.p, SSIMX_F32, x, y, F.W[j], F.H[j], sh.batch, 3, nullptr, 0, 0, nullptr, 0,
                   (float*)ra.lpart, nullptr, tile, st, nullptr, nullptr, &ra.ltiles);
      if (s != SSIMX_OK) return s;
    }
  }
  float* score = (float*)(ws + l.score);
  float* om = (float*)(ws + l.om);
  ra.M = M;
  ra.clamp = (sh.flags & SSIMX_MS_CS_CLAMP) ? 1 : 0;
  ra.sum = (sh.flags & SSIMX_MS_SUM) ? 1 : 0;
  ra.split = split ? 1 : 0;
  ra.gscore = -1.f / (float)sh.batch;
  ra.score = score;
  ra.om = om;
  ra.up = (float*)(msb + l.L.up);
  ra.up2 = (float*)(msb + l.L.up2);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(sh.batch), dim3(BLOCK), 0, st, ra);
  if ((err = (int)hipGetLastError())) return hip_status(err);
  hipLaunchKernelGGL(loss_total_kernel, dim3(1), dim3(BLOCK), 0, st, io, iod, score, om, sh.batch);
  if ((err = (int)hipGetLastError())) return hip_status(err);
  if (!with_grad) return SSIMX_OK;
  float* ygrad = (float*)(ws + l.ygrad);
  // the forward's pyramid is still in the workspace and the upstreams are set
  ssimx_status s = ms_bwd_levels(&sh.p, sh.w, M, sh.flags, &ri, &di, sh.batch, nullptr, nullptr, nullptr, ygrad,
                                 sh.W, (int64_t)sh.W * sh.H, msb, l.L, st, true);
  if (s != SSIMX_OK) return s;
  const dim3 gg((sh.W * sh.H + BLOCK - 1) / BLOCK, sh.batch);
  if (sh.grad_dtype == SSIMX_F32)
    hipLaunchKernelGGL(loss_grad_kernel<float>, gg, dim3(BLOCK), 0, st, io, iod, ygrad, sh.W, sh.H);
  else
    hipLaunchKernelGGL(loss_grad_kernel<bf16_t>, gg, dim3(BLOCK), 0, st, io, iod, ygrad, sh.W, sh.H);
  return hip_status((int)hipGetLastError());
}

LossShape make_shape(const ssimx_params* p, const float* weights, int n_scales, int flags, int dtype, int grad_dtype,
                     int W, int H, int batch) {
  LossShape sh{};
  sh.p = *p;
  ms_weights(weights, n_scales, flags, sh.w);
  sh.n_scales = n_scales;
  sh.flags = flags;
  sh.dtype = dtype;
  sh.grad_dtype = grad_dtype;
  sh.W = W;
  sh.H = H;
  sh.batch = batch;
  return sh;
}

constexpr int kRing = 8;  // pinned argument slots of a plan

}  // namespace
}  // namespace ssimx

using namespace ssimx;

struct ssimx_loss_plan {
  LossShape sh;
  void* ws = nullptr;
  LossIO* io_dev = nullptr;        // the block the graph's kernels read
  LossIO* io_host = nullptr;       // pinned ring of kRing slots
  hipEvent_t ev[kRing] = {};
  bool ev_used[kRing] = {};
  int slot = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};  // [without, with] gradient
  hipGraphExec_t exec[2] = {nullptr, nullptr};
};

static void loss_plan_free(ssimx_loss_plan* pl) {
  if (!pl) return;
  for (int i = 0; i < 2; ++i) {
    if (pl->exec[i]) (void)hipGraphExecDestroy(pl->exec[i]);
    if (pl->graph[i]) (void)hipGraphDestroy(pl->graph[i]);
  }
  for (int i = 0; i < kRing; ++i)
    if (pl->ev[i]) (void)hipEventDestroy(pl->ev[i]);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  if (pl->io_host) (void)hipHostFree(pl->io_host);
  if (pl->io_dev) (void)hipFree(pl->io_dev);
  if (pl->ws) (void)hipFree(pl->ws);
  delete pl;
}

extern "C" {

ssimx_status ssimx_msssim_loss_workspace_size(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                              int dtype, int width, int height, int batch, size_t* bytes) {
  ssimx_status s;
  if (!bytes) return SSIMX_EINVAL;
  if ((s = check_loss_shape(p, weights, n_scales, flags, dtype, width, height, batch)) != SSIMX_OK) return s;
  *bytes = loss_layout(make_shape(p, weights, n_scales, flags, dtype, SSIMX_F32, width, height, batch)).total;
  return SSIMX_OK;
}

ssimx_status ssimx_msssim_loss_rgb(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                   const void* ref_rgb, const void* dis_rgb, int dtype, int width, int height,
                                   int64_t pitch, int64_t channel_stride, int64_t batch_stride, int batch,
                                   float* loss_out, float* score_out, void* grad_rgb, int grad_dtype,
                                   int64_t grad_pitch, int64_t grad_channel_stride, int64_t grad_batch_stride,
                                   void* ws, size_t ws_bytes, void* stream) {
  ssimx_status s;
  if ((s = check_loss_shape(p, weights, n_scales, flags, dtype, width, height, batch)) != SSIMX_OK) return s;
  const LossShape sh = make_shape(p, weights, n_scales, flags, dtype, grad_dtype, width, height, batch);
  const LossIO io{ref_rgb, dis_rgb, pitch, channel_stride, batch_stride, loss_out, score_out, grad_rgb,
                  grad_pitch, grad_channel_stride, grad_batch_stride};
  if ((s = check_loss_io(sh, io, grad_rgb != nullptr)) != SSIMX_OK) return s;
  if (!ws || ws_bytes < loss_layout(sh).total) return SSIMX_EWORKSPACE;
  return loss_launches(sh, io, nullptr, grad_rgb != nullptr, (char*)ws, (hipStream_t)stream);
}

ssimx_status ssimx_loss_plan_create(const ssimx_params* p, const float* weights, int n_scales, int flags, int dtype,
                                    int grad_dtype, int width, int height, int batch, ssimx_loss_plan** out) {
  ssimx_status s;
  if (!out) return SSIMX_EINVAL;
  *out = nullptr;
  if ((s = check_loss_shape(p, weights, n_scales, flags, dtype, width, height, batch)) != SSIMX_OK) return s;
  if (grad_dtype != SSIMX_F32 && grad_dtype != SSIMX_BF16) return SSIMX_EDTYPE;
  ssimx_loss_plan* pl = new ssimx_loss_plan();
  pl->sh = make_shape(p, weights, n_scales, flags, dtype, grad_dtype, width, height, batch);
  int err = (int)hipMalloc(&pl->ws, std::max<size_t>(1, loss_layout(pl->sh).total));
  if (!err) err = (int)hipMalloc((void**)&pl->io_dev, sizeof(LossIO));
  if (!err) err = (int)hipHostMalloc((void**)&pl->io_host, sizeof(LossIO) * kRing, hipHostMallocDefault);
  for (int i = 0; i < kRing && !err; ++i) err = (int)hipEventCreateWithFlags(&pl->ev[i], hipEventDisableTiming);
  if (!err) err = (int)hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
  if (err) {
    loss_plan_free(pl);
    g_last_hip = err;
    return SSIMX_ENOMEM;
  }
  *out = pl;
  return SSIMX_OK;
}

ssimx_status ssimx_loss_plan_run(ssimx_loss_plan* pl, const void* ref_rgb, const void* dis_rgb, int64_t pitch,
                                 int64_t channel_stride, int64_t batch_stride, float* loss_out, float* score_out,
                                 void* grad_rgb, int64_t grad_pitch, int64_t grad_channel_stride,
                                 int64_t grad_batch_stride, void* stream) {
  if (!pl) return SSIMX_EINVAL;
  const LossIO io{ref_rgb, dis_rgb, pitch, channel_stride, batch_stride, loss_out, score_out, grad_rgb,
                  grad_pitch, grad_channel_stride, grad_batch_stride};
  const bool with_grad = grad_rgb != nullptr;
  ssimx_status s;
  if ((s = check_loss_io(pl->sh, io, with_grad)) != SSIMX_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int v = with_grad ? 1 : 0;
  int err = 0;
  if (!pl->exec[v]) {  // first run of this variant: capture the launches once
    err = (int)hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
    if (err) return hip_status(err);
    s = loss_launches(pl->sh, io, pl->io_dev, with_grad, (char*)pl->ws, pl->cap);
    hipGraph_t g = nullptr;
    err = (int)hipStreamEndCapture(pl->cap, &g);
    if (s != SSIMX_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (err) return hip_status(err);
    err = (int)hipGraphInstantiate(&pl->exec[v], g, nullptr, nullptr, 0);
    if (err) {
      (void)hipGraphDestroy(g);
      return hip_status(err);
    }
    pl->graph[v] = g;
  }
  // refresh the argument block from a pinned slot whose previous copy is done
  const int i = pl->slot;
  pl->slot = (pl->slot + 1) % kRing;
  if (pl->ev_used[i] && (err = (int)hipEventSynchronize(pl->ev[i]))) return hip_status(err);
  memcpy(&pl->io_host[i], &io, sizeof(LossIO));
  err = (int)hipMemcpyAsync(pl->io_dev, &pl->io_host[i], sizeof(LossIO), hipMemcpyHostToDevice, st);
  if (!err) err = (int)hipEventRecord(pl->ev[i], st);
  if (!err) pl->ev_used[i] = true;
  if (!err) err = (int)hipGraphLaunch(pl->exec[v], st);
  return hip_status(err);
}

ssimx_status ssimx_loss_plan_destroy(ssimx_loss_plan* pl) {
  if (!pl) return SSIMX_EINVAL;
  loss_plan_free(pl);
  return SSIMX_OK;
}

}  // extern "C"
