// Ragged batches: many independent pairs (each with its own size, window,
// stride and borders) in one persistent launch, captured in a hipGraph.
//
// ssimx_plan_create builds, on the host,
//   * one descriptor per pair holding the argument block of the tile body
//     that serves it, with the tile shape of the autotune cache: the stride-1
//     band body for 11x11 windows with usable taps, the strided band body
//     for 11x11 windows at stride 4, the byte-dot band body for 8x8
//     rectangular windows on 8-bit planes at strides 1 and 4, and the
//     generic separable / integer tile-sum bodies for everything else;
//   * a flat work list of (pair, tile) items, costliest pairs first;
// and captures persistent kernel -> per-pair finalise into a graph.  The
// persistent blocks take the items round-robin, so the list is balanced
// longest-first and each block exits after a fixed number of items.  Each
// tile writes its pooled partial to a fixed slot and the
// finalise sums a pair's slots in a fixed order, so scores do not depend on
// the schedule and equal those of the per-pair launches bit for bit.
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "launch.hpp"
#include "box_band.hpp"
#include "box_tile.hpp"
#include "fast_tile_body.hpp"
#include "strided_tile.hpp"
#include "host_common.hpp"
#include "sep_tile.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

enum PairKind { kKindFast = 0, kKindSep = 1, kKindBox = 2, kKindStrided4 = 3, kKindBand8s1 = 4, kKindBand8s4 = 5 };

struct PairDesc {
  int kind;
  int tiles;
  int part_off;
  int count;  // map positions of the pair
  FastArgs fa;   // stride-1 and strided band bodies
  SepArgs sa;
  BoxArgs ba;
  BandArgs bb;
};

constexpr int kPlanSmemBytes = 48 * 1024;
constexpr int kPlanSmemFloats = kPlanSmemBytes / 4;
static_assert(fast::fast_smem_floats<11>() <= kPlanSmemFloats, "band tile does not fit the plan buffer");
static_assert(strided::strided_smem_floats<11, 4>() <= kPlanSmemFloats, "strided tile does not fit the plan buffer");
static_assert(bband::band_lds_dwords<8, 4>() <= kPlanSmemFloats, "box band tile does not fit the plan buffer");
static_assert(bband::band_lds_dwords<8, 1>() <= kPlanSmemFloats, "box band tile does not fit the plan buffer");

// Items are dealt round-robin to the persistent blocks from a list sorted
// costliest first.  The loop bounds depend only on blockIdx / gridDim /
// n_items, so every wave of a block takes the same trip count and meets the
// same barriers, and every block exits after ceil(n_items / gridDim) items.
template <typename T>
__global__ __launch_bounds__(BLOCK, 3) void ragged_kernel(const PairDesc* __restrict__ descs,
                                                          const int2* __restrict__ items, int n_items,
                                                          float* partial) {
  __shared__ __align__(16) float smem[kPlanSmemFloats];
  __shared__ float red[BLOCK / 64];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int2 w = items[it];
    const PairDesc& d = descs[w.x];
    float acc;
    if (d.kind == kKindFast) {
      acc = fast::fast_stats_tile<11, T, 0>(d.fa, 0, w.y, smem);
    } else if (d.kind == kKindStrided4) {
      acc = strided::strided_tile<11, 4, T>(d.fa, 0, w.y, smem);
    } else if (d.kind == kKindSep) {
      acc = sep_fwd_tile<T>(d.sa, 0, w.y, smem);
    } else if constexpr (std::is_same<T, uint8_t>::value) {
      if (d.kind == kKindBand8s1)
        acc = bband::box_band_tile<8, 1>(d.bb, 0, w.y, (uint32_t*)smem);
      else if (d.kind == kKindBand8s4)
        acc = bband::box_band_tile<8, 4, false>(d.bb, 0, w.y, (uint32_t*)smem);
      else
        acc = box_fwd_tile<T>(d.ba, 0, w.y, (unsigned char*)smem);
    } else if constexpr (std::is_integral<T>::value) {
      acc = box_fwd_tile<T>(d.ba, 0, w.y, (unsigned char*)smem);
    } else {
      acc = 0.f;  // integer-box pairs only exist in integer plans
    }
    const float tot = block_sum<BLOCK>(acc, red);
    if (threadIdx.x == 0) partial[d.part_off + w.y] = tot;
  }
}

// Same arithmetic and order as finalize_kernel, per pair segment.
__global__ __launch_bounds__(BLOCK) void seg_finalize_kernel(const float* partial, const PairDesc* descs,
                                                             float* out) {
  __shared__ float hs[BLOCK], ls[BLOCK];
  const PairDesc& d = descs[blockIdx.x];
  const float* p = partial + d.part_off;
  float s = 0.f, c = 0.f;
  for (int i = threadIdx.x; i < d.tiles; i += BLOCK) {
    float e;
    two_sum(s, p[i], s, e);
    c += e;
  }
  hs[threadIdx.x] = s;
  ls[threadIdx.x] = c;
  __syncthreads();
  for (int w = BLOCK / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      float e, t;
      two_sum(hs[threadIdx.x], hs[threadIdx.x + w], t, e);
      hs[threadIdx.x] = t;
      ls[threadIdx.x] += ls[threadIdx.x + w] + e;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float inv = (float)(1.0 / (double)d.count);
    const float hi = hs[0], lo = ls[0];
    const float ph = hi * inv;
    const float pe = fmaf(hi, inv, -ph);
    out[blockIdx.x] = ph + (pe + lo * inv);
  }
}

}  // namespace ssimx

using namespace ssimx;

struct ssimx_plan {
  int n = 0, n_items = 0, n_blocks = 0, dtype = 0;
  std::vector<PairDesc> host_descs;
  PairDesc* descs = nullptr;
  int2* items = nullptr;
  float* partial = nullptr;
  float* scores = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace ssimx {

static Geom plan_generic_geom(const ssimx_params* p, int dtype, Path path, int W, int H, int tile_idx) {
  Geom g = make_geom_path(p, dtype, W, H, tile_idx);
  int tw = g.TW, th = g.TH;
  auto bytes = [&](const Geom& gg) {
    return path == Path::kBox ? box_tile_lds_bytes(gg, dtype == SSIMX_U8 ? 4 : 8)
                              : sizeof(float) * sep_tile_lds_floats(gg.IH, gg.IW, gg.TW);
  };
  while (bytes(g) > (size_t)kPlanSmemBytes && (tw > 1 || th > 1)) {
    if (th >= tw && th > 1)
      th = std::max(1, th / 2);
    else
      tw = std::max(1, tw / 2);
    g.TW = std::max(1, std::min(tw, g.Wo));
    g.TH = std::max(1, std::min(th, g.Ho));
    g.IW = (g.TW - 1) * g.s + g.k;
    g.IH = (g.TH - 1) * g.s + g.k;
    g.tiles_x = (g.Wo + g.TW - 1) / g.TW;
    g.tiles_y = (g.Ho + g.TH - 1) / g.TH;
  }
  return g;
}

static ssimx_status build_desc(const ssimx_pair& pr, PairDesc& d, double& cost) {
  ssimx_params p = pr.p;
  if (p.window == SSIMX_WIN_BOX) p.algo = SSIMX_ALGO_SEPARABLE;  // tile-local sums in both runs
  const int dtype = pr.ref.dtype;
  const int W = pr.ref.width, H = pr.ref.height;
  int Wo, Ho;
  map_dims(&p, W, H, Wo, Ho);
  PlaneArg x{pr.ref.data, pr.ref.pitch, pr.ref.batch_stride}, y{pr.dis.data, pr.dis.pitch, pr.dis.batch_stride};
  const int tile_idx = pick_tile(&p, dtype, W, H, 1);
  memset(&d, 0, sizeof(d));
  d.count = Wo * Ho;
  // tile cost: map positions per tile times the measured time per position
  // of each body on 1080p frames (picoseconds)
  if (use_fast(&p, dtype) && p.k == 11) {
    d.kind = kKindFast;
    const Geom g = fast_geom(&p, W, H, tile_idx);
    fill_fast_common(d.fa, &p, dtype, x, y, g);
    d.fa.mode = 0;
    d.fa.map = pr.map_out;
    d.fa.map_pitch = pr.map_pitch;
    d.fa.batch = 1;
    d.tiles = g.tiles_x * g.tiles_y;
    cost = 64.0 * g.TH * 4.7;
  } else if (use_strided(&p, dtype) && p.k == 11 && p.stride == 4) {
    d.kind = kKindStrided4;
    const Geom g = strided_geom(&p, W, H, tile_idx);
    fill_fast_common(d.fa, &p, dtype, x, y, g);
    d.fa.mode = 0;
    d.fa.map = pr.map_out;
    d.fa.map_pitch = pr.map_pitch;
    d.fa.batch = 1;
    d.tiles = g.tiles_x * g.tiles_y;
    cost = 64.0 * g.TH * 38.0;
  } else if (band_eligible(&p, dtype) && p.k == 8 && (p.stride == 1 || p.stride == 4) &&
             aligned_vec(x.data, x.pitch, x.bstride, 1) && aligned_vec(y.data, y.pitch, y.bstride, 1)) {
    d.kind = p.stride == 1 ? kKindBand8s1 : kKindBand8s4;
    const Geom g = band_geom(&p, W, H, tile_idx);
    BandArgs& a = d.bb;
    a.x = x;
    a.y = y;
    a.g = g;
    a.C1 = (float)p.C1;
    a.C2 = (float)p.C2;
    a.inv_k4 = (float)(1.0 / 4096.0);
    a.mode = 0;
    a.map = pr.map_out;
    a.map_pitch = pr.map_pitch;
    d.tiles = g.tiles_x * g.tiles_y;
    cost = 256.0 * g.TH * (p.stride == 1 ? 2.5 : 13.4);
  } else if (choose_path(&p, dtype) == Path::kSep) {
    d.kind = kKindSep;
    const Geom g = plan_generic_geom(&p, dtype, Path::kSep, W, H, tile_idx);
    SepArgs& a = d.sa;
    a.x = x;
    a.y = y;
    a.g = g;
    a.C1 = (float)p.C1;
    a.C2 = (float)p.C2;
    a.mode = 0;
    a.map = pr.map_out;
    a.map_pitch = pr.map_pitch;
    gaussian_taps_f32(p.window, p.k, p.sigma, a.taps);
    d.tiles = g.tiles_x * g.tiles_y;
    cost = (double)g.TH * g.TW * (10.0 * p.stride * p.stride);
  } else {
    d.kind = kKindBox;
    const Geom g = plan_generic_geom(&p, dtype, Path::kBox, W, H, tile_idx);
    BoxArgs& a = d.ba;
    a.x = x;
    a.y = y;
    a.g = g;
    a.C1 = (float)p.C1;
    a.C2 = (float)p.C2;
    a.mode = 0;
    a.map = pr.map_out;
    a.map_pitch = pr.map_pitch;
    a.batch = 1;
    d.tiles = g.tiles_x * g.tiles_y;
    cost = (double)g.TH * g.TW * (13.0 * p.stride * p.stride);
  }
  return SSIMX_OK;
}

static void plan_free(ssimx_plan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  if (pl->descs) (void)hipFree(pl->descs);
  if (pl->items) (void)hipFree(pl->items);
  if (pl->partial) (void)hipFree(pl->partial);
  if (pl->scores) (void)hipFree(pl->scores);
  delete pl;
}

static int launch_ragged(const ssimx_plan* pl, hipStream_t st) {
  switch (pl->dtype) {
    case SSIMX_U8:
      hipLaunchKernelGGL(ragged_kernel<uint8_t>, dim3(pl->n_blocks), dim3(BLOCK), 0, st, pl->descs, pl->items,
                         pl->n_items, pl->partial);
      break;
    case SSIMX_U16:
      hipLaunchKernelGGL(ragged_kernel<uint16_t>, dim3(pl->n_blocks), dim3(BLOCK), 0, st, pl->descs, pl->items,
                         pl->n_items, pl->partial);
      break;
    case SSIMX_F32:
      hipLaunchKernelGGL(ragged_kernel<float>, dim3(pl->n_blocks), dim3(BLOCK), 0, st, pl->descs, pl->items,
                         pl->n_items, pl->partial);
      break;
    case SSIMX_BF16:
      hipLaunchKernelGGL(ragged_kernel<bf16_t>, dim3(pl->n_blocks), dim3(BLOCK), 0, st, pl->descs, pl->items,
                         pl->n_items, pl->partial);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(seg_finalize_kernel, dim3(pl->n), dim3(BLOCK), 0, st, pl->partial, pl->descs, pl->scores);
  return (int)hipGetLastError();
}

}  // namespace ssimx

extern "C" {

ssimx_status ssimx_plan_create(const ssimx_pair* pairs, int n, void* stream, ssimx_plan** out) {
  if (!pairs || n < 1 || !out) return SSIMX_EINVAL;
  *out = nullptr;
  const int dtype = pairs[0].ref.dtype;
  for (int i = 0; i < n; ++i) {
    const ssimx_pair& pr = pairs[i];
    ssimx_status s;
    if ((s = check_params(&pr.p)) != SSIMX_OK) return s;
    if ((s = check_images(&pr.ref, &pr.dis, 1)) != SSIMX_OK) return s;
    if (pr.ref.dtype != dtype) return SSIMX_ENOTSUP;
    ssimx_params p = pr.p;
    if (p.window == SSIMX_WIN_BOX) p.algo = SSIMX_ALGO_SEPARABLE;
    if ((s = check_path(&p, dtype)) != SSIMX_OK) return s;
    int Wo, Ho;
    map_dims(&p, pr.ref.width, pr.ref.height, Wo, Ho);
    if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
    if (pr.map_out && pr.map_pitch < Wo) return SSIMX_EINVAL;
  }
  ssimx_plan* pl = new (std::nothrow) ssimx_plan();
  if (!pl) return SSIMX_ENOMEM;
  pl->n = n;
  pl->dtype = dtype;
  pl->host_descs.resize(n);
  std::vector<double> cost(n);
  int total = 0;
  for (int i = 0; i < n; ++i) {
    build_desc(pairs[i], pl->host_descs[i], cost[i]);
    pl->host_descs[i].part_off = total;
    total += pl->host_descs[i].tiles;
  }
  // work list: costliest tiles first (longest-processing-time order)
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<int2> items;
  items.reserve(total);
  for (int i : order)
    for (int t = 0; t < pl->host_descs[i].tiles; ++t) items.push_back(make_int2(i, t));
  pl->n_items = (int)items.size();
  int dev = 0, cus = 0, per_cu = 0;
  int err = (int)hipGetDevice(&dev);
  if (!err) err = (int)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (!err) {
    const void* fn = dtype == SSIMX_U8    ? (const void*)ragged_kernel<uint8_t>
                     : dtype == SSIMX_U16 ? (const void*)ragged_kernel<uint16_t>
                     : dtype == SSIMX_F32 ? (const void*)ragged_kernel<float>
                                          : (const void*)ragged_kernel<bf16_t>;
    err = (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLOCK, 0);
  }
  pl->n_blocks = std::max(1, std::min(pl->n_items, std::max(1, cus) * std::max(1, per_cu)));
  if (!err) err = (int)hipMalloc(&pl->descs, sizeof(PairDesc) * n);
  if (!err) err = (int)hipMalloc(&pl->items, sizeof(int2) * items.size());
  if (!err) err = (int)hipMalloc(&pl->partial, sizeof(float) * std::max(1, total));
  if (!err) err = (int)hipMalloc(&pl->scores, sizeof(float) * n);
  if (!err) err = (int)hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
  // descriptors point the tile bodies at the plan's partial slots
  for (int i = 0; i < n && !err; ++i) {
    PairDesc& d = pl->host_descs[i];
    d.fa.partial = pl->partial + d.part_off;
    d.sa.partial = pl->partial + d.part_off;
    d.ba.partial = pl->partial + d.part_off;
    d.bb.partial = pl->partial + d.part_off;
  }
  if (!err) err = (int)hipMemcpy(pl->descs, pl->host_descs.data(), sizeof(PairDesc) * n, hipMemcpyHostToDevice);
  if (!err) err = (int)hipMemcpy(pl->items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
  if (!err) err = (int)hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
  if (!err) {
    const int lerr = launch_ragged(pl, pl->cap);
    const int cerr = (int)hipStreamEndCapture(pl->cap, &pl->graph);
    err = lerr ? lerr : cerr;
  }
  if (!err) err = (int)hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
  if (err) {
    plan_free(pl);
    return hip_status(err);
  }
  (void)stream;
  *out = pl;
  return SSIMX_OK;
}

ssimx_status ssimx_plan_run(ssimx_plan* pl, float* scores_out, void* stream) {
  if (!pl || !scores_out) return SSIMX_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int err = (int)hipGraphLaunch(pl->exec, st);
  if (!err)
    err = (int)hipMemcpyAsync(scores_out, pl->scores, sizeof(float) * pl->n, hipMemcpyDeviceToDevice, st);
  return hip_status(err);
}

ssimx_status ssimx_plan_run_unbatched(ssimx_plan* pl, float* scores_out, void* stream) {
  if (!pl || !scores_out) return SSIMX_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < pl->n; ++i) {
    const PairDesc& d = pl->host_descs[i];
    int err;
    if (d.kind == kKindFast)
      err = launch_fast_stats(pl->dtype, 0, d.fa, 1, st);
    else if (d.kind == kKindStrided4)
      err = launch_strided(pl->dtype, d.fa, 1, st);
    else if (d.kind == kKindBand8s1 || d.kind == kKindBand8s4)
      err = launch_box_band(d.bb, 1, st);
    else if (d.kind == kKindSep)
      err = launch_sep_fwd(pl->dtype, d.sa, 1, sep_lds_bytes(d.sa.g), st);
    else
      err = launch_box_fwd(pl->dtype, d.ba, 1, st);
    if (!err) err = launch_finalize(pl->partial + d.part_off, d.tiles, 1, d.count, 1.f, scores_out + i, 1, st);
    if (err) return hip_status(err);
  }
  return SSIMX_OK;
}

ssimx_status ssimx_plan_destroy(ssimx_plan* pl) {
  if (!pl) return SSIMX_EINVAL;
  plan_free(pl);
  return SSIMX_OK;
}

ssimx_status ssimx_plan_info(const ssimx_plan* pl, int* n_items, int* n_blocks) {
  if (!pl) return SSIMX_EINVAL;
  if (n_items) *n_items = pl->n_items;
  if (n_blocks) *n_blocks = pl->n_blocks;
  return SSIMX_OK;
}

}  // extern "C"
