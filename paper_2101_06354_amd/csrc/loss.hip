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

#include "fast_tile.hpp"
#include "host_common.hpp"
#include "launch.hpp"
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
// A copy, not a reference: selecting between the argument block and global
// memory by address would put the argument block in private memory.
__device__ __forceinline__ LossIO io_of(const LossIO& v, const LossIO* d) {
  if (d) return *d;
  return v;
}

// Luma of the reference (z = 0) and distorted (z = 1) batch into dense planes,
// in the operation order of ssimx_rgb_to_luma.
template <typename T>
__global__ __launch_bounds__(BLOCK) void loss_luma_kernel(LossIO iov, const LossIO* iod, int W, int H, float* yr,
                                                          float* yd) {
  const LossIO io = io_of(iov, iod);
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W * H) return;
  const int b = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const T* p = (const T*)(blockIdx.z == 0 ? io.ref : io.dis) + (int64_t)b * io.bstride + (int64_t)r * io.pitch + c;
  const float R = to_f32<T>(p[0]), G = to_f32<T>(p[io.cstride]), B = to_f32<T>(p[2 * io.cstride]);
  (blockIdx.z == 0 ? yr : yd)[(int64_t)b * W * H + idx] = fmaf(kBt601R, R, fmaf(kBt601G, G, kBt601B * B));
}

// Four consecutive elements from a 16-byte (float) or 8-byte (bfloat16)
// aligned address.
template <typename T>
__device__ __forceinline__ void load4(const T* p, float v[4]) {
  if constexpr (std::is_same<T, float>::value) {
    const float4 q = *(const float4*)p;
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
    const uint2 q = *(const uint2*)p;
    v[0] = __uint_as_float(q.x << 16);
    v[1] = __uint_as_float(q.x & 0xffff0000u);
    v[2] = __uint_as_float(q.y << 16);
    v[3] = __uint_as_float(q.y & 0xffff0000u);
  }
}

// Outputs of the luma + pyramid kernel, [0] reference, [1] distorted.
struct PyrOut {
  float* y[2];   // [batch][H][W]
  float* m1[2];  // [batch][H1][W1], H1 = H / 2, W1 = W / 2; null with one scale
  float* m2[2];  // [batch][H2][W2], H2 = H1 / 2, W2 = W1 / 2; null with fewer than three
  int W1, H1, W2, H2;
};

// Luma of both batches (z = 0 reference, 1 distorted) and the first two
// levels of their 2x2-mean pyramid (Multi-Scale SSIM: low-pass filter and
// down-sample by 2 between scales), one thread per 4x4 luma block: the block's
// four level-1 means and one level-2 mean are formed in registers from the
// float32 luma values, in the addition order of the stand-alone 2x2
// down-sampling, and each plane is read once.  Rows are fetched as 4-element
// vectors when the source layout allows it (a uniform test of the caller's
// pointers and strides, so a graph replay with other tensors stays valid).
template <typename T>
__global__ __launch_bounds__(BLOCK) void loss_luma_pyr_kernel(LossIO iov, const LossIO* iod, int W, int H, int nbx,
                                                              int nby, PyrOut o) {
  const LossIO io = io_of(iov, iod);
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= nbx * nby) return;
  const int by = idx / nbx, bx = idx - by * nbx;
  const int f = blockIdx.y, z = blockIdx.z;
  const T* base = (const T*)(z ? io.dis : io.ref);
  const T* src = base + (int64_t)f * io.bstride;
  const int r0 = 4 * by, c0 = 4 * bx;
  constexpr uintptr_t VA = 4 * sizeof(T);
  const bool vec = (((uintptr_t)base | (uintptr_t)(io.pitch * (int64_t)sizeof(T)) |
                     (uintptr_t)(io.cstride * (int64_t)sizeof(T)) | (uintptr_t)(io.bstride * (int64_t)sizeof(T))) &
                    (VA - 1)) == 0;
  const bool full = c0 + 4 <= W && r0 + 4 <= H;
  float Y[4][4];
  if (vec && full) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T* p = src + (int64_t)(r0 + i) * io.pitch + c0;
      float R[4], G[4], B[4];
      load4<T>(p, R);
      load4<T>(p + io.cstride, G);
      load4<T>(p + 2 * io.cstride, B);
#pragma unroll
      for (int j = 0; j < 4; ++j) Y[i][j] = fmaf(kBt601R, R[j], fmaf(kBt601G, G[j], kBt601B * B[j]));
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        Y[i][j] = 0.f;
        if (r0 + i < H && c0 + j < W) {
          const T* p = src + (int64_t)(r0 + i) * io.pitch + (c0 + j);
          Y[i][j] = fmaf(kBt601R, to_f32<T>(p[0]), fmaf(kBt601G, to_f32<T>(p[io.cstride]),
                                                         kBt601B * to_f32<T>(p[2 * io.cstride])));
        }
      }
  }
  float* yo = o.y[z] + (int64_t)f * W * H;
  if (full && (W & 3) == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *(float4*)(yo + (int64_t)(r0 + i) * W + c0) = make_float4(Y[i][0], Y[i][1], Y[i][2], Y[i][3]);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (r0 + i < H && c0 + j < W) yo[(int64_t)(r0 + i) * W + c0 + j] = Y[i][j];
  }
  if (!o.m1[z]) return;
  float M1[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      M1[i][j] = 0.25f * (((Y[2 * i][2 * j] + Y[2 * i][2 * j + 1]) + Y[2 * i + 1][2 * j]) + Y[2 * i + 1][2 * j + 1]);
  float* m1 = o.m1[z] + (int64_t)f * o.W1 * o.H1;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r1 = 2 * by + i, c1 = 2 * bx;
    if (r1 >= o.H1) continue;
    float* row = m1 + (int64_t)r1 * o.W1;
    if (c1 + 1 < o.W1 && (o.W1 & 1) == 0) {
      *(float2*)(row + c1) = make_float2(M1[i][0], M1[i][1]);
    } else {
      if (c1 < o.W1) row[c1] = M1[i][0];
      if (c1 + 1 < o.W1) row[c1 + 1] = M1[i][1];
    }
  }
  if (!o.m2[z] || by >= o.H2 || bx >= o.W2) return;
  o.m2[z][((int64_t)f * o.H2 + by) * o.W2 + bx] = 0.25f * (((M1[0][0] + M1[0][1]) + M1[1][0]) + M1[1][1]);
}

// float32 -> bfloat16 bits, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_bits_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Per-level adjoint planes of the pyramid, [batch][H_j][W_j] each.
struct GradPyr {
  const float* g[MAX_SCALES];
  int W[MAX_SCALES], H[MAX_SCALES];
  int M;
};

// Gradient of the RGB planes from the per-level luma adjoints: the transpose
// of each 2x2 mean adds a quarter of the coarser level's gradient to each of
// its four sources, composed from the coarsest level a pixel reaches down to
// level 0 (s_j = a_j + s_{j+1} / 4, the order of the level-by-level
// backward), times the upstream d(objective)/d(loss) when given, then the
// transpose of the luma map.  One thread per 4 pixels of a row; float32 or
// bfloat16 (round to nearest even) output.
template <typename G>
__global__ __launch_bounds__(BLOCK) void loss_grad_pyr_kernel(LossIO iov, const LossIO* iod, GradPyr gp, int nqx,
                                                              const float* upstream) {
  const LossIO io = io_of(iov, iod);
  const float us = upstream ? *upstream : 1.f;
  const int W = gp.W[0], H = gp.H[0];
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= nqx * H) return;
  const int r = idx / nqx, c0 = 4 * (idx - r * nqx);
  const int f = blockIdx.y;
  const bool full = c0 + 4 <= W;
  float v[4];
  const float* g0 = gp.g[0] + ((int64_t)f * H + r) * W;
  if (full && (W & 3) == 0) {
    const float4 q = *(const float4*)(g0 + c0);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = c0 + j < W ? g0[c0 + j] : 0.f;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int x = c0 + j;
    float s = 0.f;
    bool have = false;
    for (int l = gp.M - 1; l >= 1; --l) {
      const int xl = x >> l, yl = r >> l;
      if (xl < gp.W[l] && yl < gp.H[l]) {
        const float a = gp.g[l][((int64_t)f * gp.H[l] + yl) * gp.W[l] + xl];
        s = have ? a + 0.25f * s : a;
        have = true;
      }
    }
    if (have) v[j] = v[j] + 0.25f * s;
    v[j] *= us;
  }
  constexpr float wc[3] = {kBt601R, kBt601G, kBt601B};
  G* p = (G*)io.grad + (int64_t)f * io.gbstride + (int64_t)r * io.gpitch + c0;
  constexpr uintptr_t VA = 4 * sizeof(G);
  const bool vec = full && ((((uintptr_t)io.grad | (uintptr_t)(io.gpitch * (int64_t)sizeof(G)) |
                              (uintptr_t)(io.gcstride * (int64_t)sizeof(G)) |
                              (uintptr_t)(io.gbstride * (int64_t)sizeof(G)) | (uintptr_t)(c0 * sizeof(G))) &
                             (VA - 1)) == 0);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    G* q = p + ch * io.gcstride;
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = wc[ch] * v[j];
    if constexpr (std::is_same<G, float>::value) {
      if (vec) {
        *(float4*)q = make_float4(o[0], o[1], o[2], o[3]);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c0 + j < W) q[j] = o[j];
      }
    } else {
      uint16_t h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) h[j] = bf16_bits_rne(o[j]);
      if (vec) {
        *(uint2*)q = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c0 + j < W) q[j].bits = h[j];
      }
    }
  }
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
  const LossIO io = io_of(iov, iod);
  __shared__ float hs[BLOCK], ls[BLOCK];
  const float loss = tile_mean(om, batch, 1.f / (float)batch, hs, ls);
  if (threadIdx.x == 0) io.loss[0] = loss;
  if (io.score)
    for (int b = threadIdx.x; b < batch; b += BLOCK) io.score[b] = score[b];
}

// Gradient of the RGB planes from the luma gradient (times the upstream when
// given; the transpose of the luma map), written as float32 or bfloat16
// (round to nearest even).
template <typename G>
__global__ __launch_bounds__(BLOCK) void loss_grad_kernel(LossIO iov, const LossIO* iod, const float* gy, int W,
                                                          int H, const float* upstream) {
  const LossIO io = io_of(iov, iod);
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W * H) return;
  const int b = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const float v = gy[(int64_t)b * W * H + idx] * (upstream ? *upstream : 1.f);
  G* p = (G*)io.grad + (int64_t)b * io.gbstride + (int64_t)r * io.gpitch + c;
  const float g[3] = {kBt601R * v, kBt601G * v, kBt601B * v};
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    if constexpr (std::is_same<G, float>::value) {
      p[ch * io.gcstride] = g[ch];
    } else {
      bf16_t h;
      h.bits = bf16_bits_rne(g[ch]);
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

// The segmented route: every scale's windowed pass in one launch (forward,
// coefficients, adjoint), the pyramid built by the luma kernel and the
// levels' gradients composed by the output kernel.  It needs the fast
// stride-1 kernels with valid borders at every scale, one argument block per
// pass (the scales, plus the coarsest mean(l) pass when it is split) and
// coefficient rows the adjoint can address.
bool seg_route(const LossShape& sh) {
  ssimx_params pf = sh.p;
  pf.algo = SSIMX_ALGO_SEPARABLE;
  const int passes = sh.n_scales + ((sh.flags & SSIMX_MS_COARSE_SEPARATE) ? 1 : 0);
  if (sh.p.padding != SSIMX_PAD_VALID || passes > kMaxSegs) return false;
  if (!use_fast(&sh.p, SSIMX_F32) || !use_fast(&pf, SSIMX_F32)) return false;
  int Wo, Ho;
  map_dims(&sh.p, sh.W, sh.H, Wo, Ho);
  return ((Wo + 3) & ~3) < kFastMaxPitch && sh.W < kFastMaxPitch;
}

struct LossLayout {
  size_t yr, yd, ygrad, score, om, lpart, ms, total;
  size_t coef_lv[MAX_SCALES];  // segmented route: coefficient planes of levels >= 1
  bool segs;
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
  l.segs = seg_route(sh);
  if (l.segs)
    for (int j = 1; j < M; ++j) {
      int Wo, Ho;
      map_dims(&sh.p, l.L.fwd.W[j], l.L.fwd.H[j], Wo, Ho);
      l.coef_lv[j] = ws.take(sizeof(float) * 3 * (size_t)sh.batch * ((Wo + 3) & ~3) * Ho);
    }
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

ssimx_status check_loss_grad(const LossShape& sh, const LossIO& io) {
  if (sh.grad_dtype != SSIMX_F32 && sh.grad_dtype != SSIMX_BF16) return SSIMX_EDTYPE;
  if (!io.grad || io.gpitch < sh.W || io.gcstride < io.gpitch * (int64_t)sh.H ||
      (sh.batch > 1 && io.gbstride < 3 * io.gcstride))
    return SSIMX_EINVAL;
  return SSIMX_OK;
}

ssimx_status check_loss_io(const LossShape& sh, const LossIO& io, bool with_grad) {
  if (!io.ref || !io.dis || !io.loss) return SSIMX_EINVAL;
  if (io.pitch < sh.W || io.cstride < io.pitch * (int64_t)sh.H || (sh.batch > 1 && io.bstride < 3 * io.cstride))
    return SSIMX_EINVAL;
  return with_grad ? check_loss_grad(sh, io) : SSIMX_OK;
}

// The per-frame reduction and the batch mean after the forward passes; `ra`
// holds the partial buffers, tile counts and (split) the mean(l) partials.
ssimx_status loss_reduce_total(const LossShape& sh, const LossLayout& l, const LossIO& io, const LossIO* iod,
                               char* ws, LossReduceArgs& ra, hipStream_t st) {
  char* msb = ws + l.ms;
  const MsLayout& F = l.L.fwd;
  const int M = sh.n_scales;
  for (int j = 0; j < M; ++j) {
    int Wo, Ho;
    map_dims(&sh.p, F.W[j], F.H[j], Wo, Ho);
    ra.inv[j] = (float)(1.0 / ((double)Wo * Ho));
    ra.w[j] = sh.w[j];
  }
  float* score = (float*)(ws + l.score);
  float* om = (float*)(ws + l.om);
  ra.M = M;
  ra.clamp = (sh.flags & SSIMX_MS_CS_CLAMP) ? 1 : 0;
  ra.sum = (sh.flags & SSIMX_MS_SUM) ? 1 : 0;
  ra.split = (sh.flags & SSIMX_MS_COARSE_SEPARATE) ? 1 : 0;
  ra.gscore = -1.f / (float)sh.batch;
  ra.score = score;
  ra.om = om;
  ra.up = (float*)(msb + l.L.up);
  ra.up2 = (float*)(msb + l.L.up2);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(sh.batch), dim3(BLOCK), 0, st, ra);
  int err = (int)hipGetLastError();
  if (err) return hip_status(err);
  hipLaunchKernelGGL(loss_total_kernel, dim3(1), dim3(BLOCK), 0, st, io, iod, score, om, sh.batch);
  return hip_status((int)hipGetLastError());
}

// Segmented route, forward: luma and pyramid, then every scale's pass (and
// the split mean(l) pass) in one launch writing the tile partials `ra`
// points at.
ssimx_status seg_forward(const LossShape& sh, const LossLayout& l, const LossIO& io, const LossIO* iod, char* ws,
                         LossReduceArgs& ra, hipStream_t st) {
  const MsLayout& F = l.L.fwd;
  char* msb = ws + l.ms;
  const int M = sh.n_scales, B = sh.batch;
  const bool split = (sh.flags & SSIMX_MS_COARSE_SEPARATE) != 0;
  float* lx[MAX_SCALES];
  float* ly[MAX_SCALES];
  lx[0] = (float*)(ws + l.yr);
  ly[0] = (float*)(ws + l.yd);
  for (int j = 1; j < M; ++j) {
    lx[j] = (float*)(msb + F.lvl_x_off[j]);
    ly[j] = (float*)(msb + F.lvl_y_off[j]);
  }
  PyrOut po{};
  po.y[0] = lx[0];
  po.y[1] = ly[0];
  if (M > 1) {
    po.m1[0] = lx[1];
    po.m1[1] = ly[1];
    po.W1 = F.W[1];
    po.H1 = F.H[1];
  }
  if (M > 2) {
    po.m2[0] = lx[2];
    po.m2[1] = ly[2];
    po.W2 = F.W[2];
    po.H2 = F.H[2];
  }
  const int nbx = (sh.W + 3) / 4, nby = (sh.H + 3) / 4;
  const dim3 gl((unsigned)(((int64_t)nbx * nby + BLOCK - 1) / BLOCK), B, 2);
  if (sh.dtype == SSIMX_F32)
    hipLaunchKernelGGL(loss_luma_pyr_kernel<float>, gl, dim3(BLOCK), 0, st, io, iod, sh.W, sh.H, nbx, nby, po);
  else
    hipLaunchKernelGGL(loss_luma_pyr_kernel<bf16_t>, gl, dim3(BLOCK), 0, st, io, iod, sh.W, sh.H, nbx, nby, po);
  int err = (int)hipGetLastError();
  if (err) return hip_status(err);
  for (int j = 3; j < M; ++j) {
    const int64_t pl = (int64_t)F.W[j - 1] * F.H[j - 1];
    err = launch_downsample(SSIMX_F32, PlaneArg{lx[j - 1], F.W[j - 1], pl}, F.W[j - 1], F.H[j - 1], lx[j], ly[j],
                            PlaneArg{ly[j - 1], F.W[j - 1], pl}, B, st);
    if (err) return hip_status(err);
  }
  FastSegs fs{};
  int64_t nb = 0;
  for (int j = 0; j <= M - (split ? 0 : 1); ++j) {
    const int lv = j < M ? j : M - 1;  // pass M: the split mean(l) of the coarsest scale
    const int tile = pick_tile(&sh.p, SSIMX_F32, F.W[lv], F.H[lv], B);
    const Geom g = fast_geom(&sh.p, F.W[lv], F.H[lv], tile, B);
    const int64_t pl = (int64_t)F.W[lv] * F.H[lv];
    FastArgs& a = fs.seg[j];
    fill_fast_common(a, &sh.p, SSIMX_F32, PlaneArg{lx[lv], F.W[lv], pl}, PlaneArg{ly[lv], F.W[lv], pl}, g);
    a.mode = j == M ? 3 : (j + 1 < M || split) ? 1 : 0;
    a.batch = B;
    const int tiles = g.tiles_x * g.tiles_y;
    if (j < M) {
      ra.part[j] = (const float*)(msb + F.partial_off[j]);
      ra.tiles[j] = tiles;
      a.partial = (float*)ra.part[j];
    } else {
      ra.lpart = (const float*)(ws + l.lpart);
      ra.ltiles = tiles;
      a.partial = (float*)ra.lpart;
    }
    fs.start[j] = (int)nb;
    nb += (int64_t)tiles * B;
    if (nb > INT32_MAX) return SSIMX_EINVAL;
    fs.n = j + 1;
  }
  fs.start[fs.n] = (int)nb;
  return hip_status(launch_fast_stats_segs(0, fs, st));
}

// Segmented route, backward: every scale's coefficient planes in one launch,
// every scale's adjoint in one launch (level j's gradient into its own
// plane; the output kernel composes them).
ssimx_status seg_backward(const LossShape& sh, const LossLayout& l, char* ws, hipStream_t st) {
  const MsLayout& F = l.L.fwd;
  char* msb = ws + l.ms;
  const int M = sh.n_scales, B = sh.batch;
  const bool split = (sh.flags & SSIMX_MS_COARSE_SEPARATE) != 0;
  ssimx_params pf = sh.p;
  pf.algo = SSIMX_ALGO_SEPARABLE;
  const float tu = shift_guess(&sh.p);
  float* up = (float*)(msb + l.L.up);
  float* up2 = (float*)(msb + l.L.up2);
  FastSegs fs{};
  int64_t nb = 0;
  for (int j = 0; j < M; ++j) {
    const int64_t pl = (int64_t)F.W[j] * F.H[j];
    const float* x = j ? (const float*)(msb + F.lvl_x_off[j]) : (const float*)(ws + l.yr);
    const float* y = j ? (const float*)(msb + F.lvl_y_off[j]) : (const float*)(ws + l.yd);
    const Geom g = coef_geom(&pf, F.W[j], F.H[j], B);
    FastArgs& a = fs.seg[j];
    fill_fast_common(a, &pf, SSIMX_F32, PlaneArg{x, F.W[j], pl}, PlaneArg{y, F.W[j], pl}, g);
    a.mode = j == M - 1 ? (split ? 3 : 0) : 1;
    a.gscale = up + j;
    a.gscale_stride = M;
    a.gscale2 = a.mode == 3 ? up2 : nullptr;
    a.gscale2_stride = 1;
    a.gmul = 1.f;
    a.tu = tu;
    a.tv = 0.f;
    a.coef = j ? (float*)(ws + l.coef_lv[j]) : (float*)(msb + l.L.coef);
    a.cpitch = (g.Wo + 3) & ~3;
    a.batch = B;
    adjoint_tiles(a, F.W[j], F.H[j], B);
    a.out = j ? (float*)(msb + l.L.glev[j]) : (float*)(ws + l.ygrad);
    a.out_pitch = F.W[j];
    a.out_bstride = pl;
    a.coarse = nullptr;
    fs.start[j] = (int)nb;
    nb += (int64_t)g.tiles_x * g.tiles_y * B;
    if (nb > INT32_MAX) return SSIMX_EINVAL;
  }
  fs.n = M;
  fs.start[M] = (int)nb;
  int err = launch_fast_stats_segs(1, fs, st);
  if (err) return hip_status(err);
  nb = 0;
  for (int j = 0; j < M; ++j) {
    fs.start[j] = (int)nb;
    nb += (int64_t)fs.seg[j].qtiles_x * fs.seg[j].qtiles_y * B;
    if (nb > INT32_MAX) return SSIMX_EINVAL;
  }
  fs.start[M] = (int)nb;
  return hip_status(launch_fast_adjoint_segs(fs, st));
}

// The RGB gradient from the luma-level gradients a backward left in the
// workspace, times *upstream when given.
ssimx_status loss_output(const LossShape& sh, const LossLayout& l, const LossIO& io, const LossIO* iod,
                         const float* upstream, char* ws, hipStream_t st) {
  if (l.segs) {
    const MsLayout& F = l.L.fwd;
    GradPyr gp{};
    gp.M = sh.n_scales;
    for (int j = 0; j < sh.n_scales; ++j) {
      gp.g[j] = j ? (const float*)(ws + l.ms + l.L.glev[j]) : (const float*)(ws + l.ygrad);
      gp.W[j] = F.W[j];
      gp.H[j] = F.H[j];
    }
    const int nqx = (sh.W + 3) / 4;
    const dim3 gg((unsigned)(((int64_t)nqx * sh.H + BLOCK - 1) / BLOCK), sh.batch);
    if (sh.grad_dtype == SSIMX_F32)
      hipLaunchKernelGGL(loss_grad_pyr_kernel<float>, gg, dim3(BLOCK), 0, st, io, iod, gp, nqx, upstream);
    else
      hipLaunchKernelGGL(loss_grad_pyr_kernel<bf16_t>, gg, dim3(BLOCK), 0, st, io, iod, gp, nqx, upstream);
  } else {
    const float* ygrad = (const float*)(ws + l.ygrad);
    const dim3 gg((sh.W * sh.H + BLOCK - 1) / BLOCK, sh.batch);
    if (sh.grad_dtype == SSIMX_F32)
      hipLaunchKernelGGL(loss_grad_kernel<float>, gg, dim3(BLOCK), 0, st, io, iod, ygrad, sh.W, sh.H, upstream);
    else
      hipLaunchKernelGGL(loss_grad_kernel<bf16_t>, gg, dim3(BLOCK), 0, st, io, iod, ygrad, sh.W, sh.H, upstream);
  }
  return hip_status((int)hipGetLastError());
}

// How far a loss evaluation goes: the loss alone, the loss and the luma-level
// gradients left in the workspace, or both and the RGB gradient.
enum LossPhase { kLossOnly, kLossLevels, kLossGrad };

// Every launch of one loss evaluation on `st`.  iod non-null: the kernels that
// touch caller memory read the pointers from that device block (graph
// capture); else from `io`.
ssimx_status loss_launches(const LossShape& sh, const LossIO& io, const LossIO* iod, LossPhase phase, char* ws,
                           hipStream_t st) {
  const LossLayout l = loss_layout(sh);
  if (l.segs) {
    LossReduceArgs ra{};
    ssimx_status s = seg_forward(sh, l, io, iod, ws, ra, st);
    if (s != SSIMX_OK) return s;
    if ((s = loss_reduce_total(sh, l, io, iod, ws, ra, st)) != SSIMX_OK || phase == kLossOnly) return s;
    if ((s = seg_backward(sh, l, ws, st)) != SSIMX_OK || phase == kLossLevels) return s;
    return loss_output(sh, l, io, iod, nullptr, ws, st);
  }
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
    if (split && j + 1 == M) {  // coarsest term mean(l) * mean(cs): the l partials too
      ra.lpart = (const float*)(ws + l.lpart);
      s = fwd_pass(&sh.p, SSIMX_F32, x, y, F.W[j], F.H[j], sh.batch, 3, nullptr, 0, 0, nullptr, 0,
                   (float*)ra.lpart, nullptr, tile, st, nullptr, nullptr, &ra.ltiles);
      if (s != SSIMX_OK) return s;
    }
  }
  ssimx_status s = loss_reduce_total(sh, l, io, iod, ws, ra, st);
  if (s != SSIMX_OK || phase == kLossOnly) return s;
  float* ygrad = (float*)(ws + l.ygrad);
  // the forward's pyramid is still in the workspace and the upstreams are set
  s = ms_bwd_levels(&sh.p, sh.w, M, sh.flags, &ri, &di, sh.batch, nullptr, nullptr, nullptr, ygrad, sh.W,
                    (int64_t)sh.W * sh.H, msb, l.L, st, true);
  if (s != SSIMX_OK || phase == kLossLevels) return s;
  return loss_output(sh, l, io, iod, nullptr, ws, st);
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
  return loss_launches(sh, io, nullptr, grad_rgb ? kLossGrad : kLossOnly, (char*)ws, (hipStream_t)stream);
}

ssimx_status ssimx_msssim_loss_rgb_deferred(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                            const void* ref_rgb, const void* dis_rgb, int dtype, int width,
                                            int height, int64_t pitch, int64_t channel_stride, int64_t batch_stride,
                                            int batch, float* loss_out, float* score_out, void* ws, size_t ws_bytes,
                                            void* stream) {
  ssimx_status s;
  if ((s = check_loss_shape(p, weights, n_scales, flags, dtype, width, height, batch)) != SSIMX_OK) return s;
  const LossShape sh = make_shape(p, weights, n_scales, flags, dtype, SSIMX_F32, width, height, batch);
  const LossIO io{ref_rgb, dis_rgb, pitch, channel_stride, batch_stride, loss_out, score_out, nullptr, 0, 0, 0};
  if ((s = check_loss_io(sh, io, false)) != SSIMX_OK) return s;
  if (!ws || ws_bytes < loss_layout(sh).total) return SSIMX_EWORKSPACE;
  return loss_launches(sh, io, nullptr, kLossLevels, (char*)ws, (hipStream_t)stream);
}

ssimx_status ssimx_msssim_loss_rgb_grad(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                        int dtype, int width, int height, int batch, const float* upstream,
                                        void* grad_rgb, int grad_dtype, int64_t grad_pitch,
                                        int64_t grad_channel_stride, int64_t grad_batch_stride, const void* ws,
                                        size_t ws_bytes, void* stream) {
  ssimx_status s;
  if ((s = check_loss_shape(p, weights, n_scales, flags, dtype, width, height, batch)) != SSIMX_OK) return s;
  const LossShape sh = make_shape(p, weights, n_scales, flags, dtype, grad_dtype, width, height, batch);
  const LossIO io{nullptr, nullptr, 0, 0, 0, nullptr, nullptr, grad_rgb, grad_pitch, grad_channel_stride,
                  grad_batch_stride};
  if ((s = check_loss_grad(sh, io)) != SSIMX_OK) return s;
  const LossLayout l = loss_layout(sh);
  if (!ws || ws_bytes < l.total) return SSIMX_EWORKSPACE;
  return loss_output(sh, l, io, nullptr, upstream, (char*)ws, (hipStream_t)stream);
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
    s = loss_launches(pl->sh, io, pl->io_dev, with_grad ? kLossGrad : kLossOnly, (char*)pl->ws, pl->cap);
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
