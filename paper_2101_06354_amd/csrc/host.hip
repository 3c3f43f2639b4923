// Host side of the C-ABI: argument validation, geometry, workspace layout and
// dispatch of the forward calls (ssim_map, ssim_pooled, msssim, box sums,
// integral images).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "launch.hpp"
#include "box_band.hpp"
#include "fast_tile.hpp"
#include "strided_tile.hpp"
#include "host_common.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

thread_local int g_last_hip = 0;

ssimx_status hip_status(int err) {
  if (err != (int)hipSuccess) {
    g_last_hip = err;
    return SSIMX_EHIP;
  }
  return SSIMX_OK;
}

// ---------------------------------------------------------------- validation
ssimx_status check_params(const ssimx_params* p) {
  if (!p) return SSIMX_EINVAL;
  if (p->window != SSIMX_WIN_GAUSSIAN && p->window != SSIMX_WIN_BOX) return SSIMX_EINVAL;
  if (p->k < 1) return SSIMX_EINVAL;
  if (p->window == SSIMX_WIN_GAUSSIAN) {
    if ((p->k & 1) == 0 || p->k > KMAX_GAUSS) return SSIMX_EINVAL;
    if (!(p->sigma > 0.f) || !isfinite(p->sigma)) return SSIMX_EINVAL;
  } else if (p->k > KMAX_BOX) {
    return SSIMX_EINVAL;
  }
  if (!(p->C1 >= 0.0) || !(p->C2 >= 0.0) || !isfinite(p->C1) || !isfinite(p->C2)) return SSIMX_EINVAL;
  if (p->stride < 1) return SSIMX_EINVAL;
  if (p->padding < SSIMX_PAD_VALID || p->padding > SSIMX_PAD_REFLECT) return SSIMX_EINVAL;
  if (p->algo < SSIMX_ALGO_AUTO || p->algo > SSIMX_ALGO_INTEGRAL_IMAGE) return SSIMX_EINVAL;
  return SSIMX_OK;
}

ssimx_status check_images(const ssimx_image* a, const ssimx_image* b, int batch) {
  if (!a || !b || batch < 1 || batch > kMaxGridY) return SSIMX_EINVAL;
  for (const ssimx_image* im : {a, b}) {
    if (!im->data) return SSIMX_EINVAL;
    if (im->dtype < SSIMX_U8 || im->dtype > SSIMX_BF16) return SSIMX_EDTYPE;
    if (im->width < 1 || im->height < 1) return SSIMX_ETOOSMALL;
    if ((int64_t)im->width * im->height > kMaxPlaneElems) return SSIMX_EINVAL;
    if (im->pitch < im->width) return SSIMX_EINVAL;
    if (batch > 1 && im->batch_stride < im->pitch * (int64_t)im->height) return SSIMX_EINVAL;
  }
  if (a->width != b->width || a->height != b->height || a->dtype != b->dtype) return SSIMX_EINVAL;
  return SSIMX_OK;
}

bool is_integer(int dtype) { return dtype == SSIMX_U8 || dtype == SSIMX_U16; }

// Which kernel family computes the statistics.
Path choose_path(const ssimx_params* p, int dtype) {
  if (p->window == SSIMX_WIN_BOX && is_integer(dtype))
    return p->algo == SSIMX_ALGO_INTEGRAL_IMAGE ? Path::kSat : Path::kBox;
  return Path::kSep;
}

ssimx_status check_path(const ssimx_params* p, int dtype) {
  const Path path = choose_path(p, dtype);
  if (path == Path::kSep && p->k > KMAX_GAUSS) return SSIMX_ENOTSUP;  // float box wider than the tap table
  if (path == Path::kSat && p->padding != SSIMX_PAD_VALID) return SSIMX_ENOTSUP;
  if (p->algo == SSIMX_ALGO_INTEGRAL_IMAGE && p->window == SSIMX_WIN_BOX && !is_integer(dtype)) return SSIMX_EDTYPE;
  // uint32 tables hold a window sum only below 2^32: k^2 * 65535^2 reaches it
  // from k = 2, so 16-bit planes take the exact tile sums instead
  if (path == Path::kSat && dtype == SSIMX_U16 && p->k > 1) return SSIMX_ENOTSUP;
  return SSIMX_OK;
}

// ---------------------------------------------------------------- geometry
static const TileCfg kTiles[] = {{32, 32}, {64, 16}, {64, 32}, {32, 16}, {128, 8}, {16, 32}};

// 16-row chunks per tile of the stride-1 fast kernels, for the same index.
// Each tile recomputes K - 1 rows of statistics above its first output row:
// 512 rows spend 1.9% of the row passes there, 128 rows 7.8%.  The kernels
// take each frame's (shorter) last tile row after the full ones, so tall
// tiles no longer leave the end of a launch to a few long tiles (64 x 1080p
// Gaussian forward: 128 rows 0.566 ms, 256 rows 0.525 ms, 512 rows 0.519 ms).
// Small launches shorten the tile by the fill rule below.
static const int kFastChunks[] = {32, 4, 16, 2, 8, 68};

int num_tile_cfgs() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
int fast_chunks(int idx) { return kFastChunks[(idx >= 0 && idx < num_tile_cfgs()) ? idx : 0]; }
TileCfg tile_cfg(int idx) { return kTiles[(idx >= 0 && idx < num_tile_cfgs()) ? idx : 0]; }

void map_dims(const ssimx_params* p, int W, int H, int& Wo, int& Ho) {
  const int Wp = p->padding == SSIMX_PAD_VALID ? W : W + p->k - 1;
  const int Hp = p->padding == SSIMX_PAD_VALID ? H : H + p->k - 1;
  Wo = Wp >= p->k ? (Wp - p->k) / p->stride + 1 : 0;
  Ho = Hp >= p->k ? (Hp - p->k) / p->stride + 1 : 0;
}

static Geom geom_with(const ssimx_params* p, int W, int H, int tw, int th) {
  Geom g{};
  g.W = W;
  g.H = H;
  g.k = p->k;
  g.s = p->stride;
  g.pad = p->padding;
  g.before = p->padding == SSIMX_PAD_VALID ? 0 : (p->k - 1) / 2;
  g.Wp = p->padding == SSIMX_PAD_VALID ? W : W + p->k - 1;
  g.Hp = p->padding == SSIMX_PAD_VALID ? H : H + p->k - 1;
  map_dims(p, W, H, g.Wo, g.Ho);
  g.TW = std::max(1, std::min(tw, g.Wo));
  g.TH = std::max(1, std::min(th, g.Ho));
  g.IW = (g.TW - 1) * g.s + g.k;
  g.IH = (g.TH - 1) * g.s + g.k;
  g.tiles_x = (g.Wo + g.TW - 1) / g.TW;
  g.tiles_y = (g.Ho + g.TH - 1) / g.TH;
  return g;
}

bool aligned_vec(const void* p, int64_t pitch, int64_t bstride, int esize) {
  return ((uintptr_t)p % (4 * esize)) == 0 && pitch % 4 == 0 && bstride % 4 == 0;
}

int dtype_size(int dtype) { return dtype == SSIMX_U8 ? 1 : dtype == SSIMX_F32 ? 4 : 2; }

// Rows per tile of the default tile index for a launch of `batch` frames:
// halved, down to `min_rows` (a height of the tile tables, which the partial
// buffers are sized for), while the launch would hold fewer than kFillBlocks
// workgroups, so that single frames and small batches spread over all CUs.
// For the box band and strided kernels, launches under kFillMinWork map
// positions gain nothing from shorter tiles (measured on per-pair launches of
// ladder frames) and keep their rows; a tuned tile index always keeps them.
constexpr int64_t kFillBlocks = 1024;       // 4 workgroups per CU
constexpr int64_t kFillMinWork = 1 << 20;  // map positions

static int fill_rows(int rows, int min_rows, int64_t tiles_x, int Ho, int batch, int tile_idx, int unit,
                     int64_t positions) {
  if (tile_idx != 0 || batch < 1 || positions * batch < kFillMinWork) return rows;
  while (rows / 2 >= min_rows && (rows / 2) % unit == 0 &&
         tiles_x * ((Ho + rows - 1) / rows) * (int64_t)batch < kFillBlocks)
    rows /= 2;
  return rows;
}

Geom fast_geom(const ssimx_params* p, int W, int H, int tile_idx, int batch, int rows0) {
  int Wo, Ho;
  map_dims(p, W, H, Wo, Ho);
  int rows = (tile_idx == 0 && rows0 > 0) ? rows0 : 16 * fast_chunks(tile_idx);
  // the default's 512 rows only while the launch keeps >= 4096 workgroups
  // (fewer, longer tiles end a launch less evenly), else 256
  if (tile_idx == 0 && rows0 == 0 && batch > 0 && rows > 256 &&
      (int64_t)((Wo + 63) / 64) * ((Ho + rows - 1) / rows) * batch < 4096)
    rows = 256;
  const int th = fill_rows(rows, 32, (Wo + 63) / 64, Ho, batch, tile_idx, 16, kFillMinWork);
  Geom g = geom_with(p, W, H, 64, th);
  g.TW = 64;
  g.TH = th;
  g.tiles_x = (g.Wo + 63) / 64;
  g.tiles_y = (g.Ho + g.TH - 1) / g.TH;
  return g;
}

Geom coef_geom(const ssimx_params* p, int W, int H, int batch) {
  const Geom g = fast_geom(p, W, H, 0, batch, 256);
  return (int64_t)g.tiles_x * g.tiles_y * batch >= 8192 ? g : fast_geom(p, W, H, 0, batch, 128);
}

// Input rows per tile of the 8-bit box band kernel, for the same index.
static const int kBandRows[] = {128, 256, 64, 512, 32, 1024};

Geom band_geom(const ssimx_params* p, int W, int H, int tile_idx, int batch) {
  Geom g = geom_with(p, W, H, 256, 1);
  int rows = kBandRows[(tile_idx >= 0 && tile_idx < num_tile_cfgs()) ? tile_idx : 0];
  rows = fill_rows(rows, 32, (g.Wo + 255) / 256, g.Ho * p->stride, batch, tile_idx, p->stride, (int64_t)g.Wo * g.Ho);
  g.TW = 256;
  g.TH = std::max(1, rows / p->stride);
  g.tiles_x = (g.Wo + 255) / 256;
  g.tiles_y = (g.Ho + g.TH - 1) / g.TH;
  return g;
}

// Map rows per tile of the strided Gaussian kernels, for the same index
// (rounded to whole chunks).
static const int kStridedRows[] = {32, 64, 16, 128, 8, 256};

Geom strided_geom(const ssimx_params* p, int W, int H, int tile_idx, int batch) {
  Geom g = geom_with(p, W, H, strided::kTWo, 1);
  const int cho = p->stride == 2 ? strided::Shape<7, 2>::CHo : p->stride == 3 ? strided::Shape<7, 3>::CHo
                                                                              : strided::Shape<7, 4>::CHo;
  int rows = kStridedRows[(tile_idx >= 0 && tile_idx < num_tile_cfgs()) ? tile_idx : 0];
  rows = fill_rows(rows, 16, (g.Wo + strided::kTWo - 1) / strided::kTWo, g.Ho, batch, tile_idx, 1,
                   (int64_t)g.Wo * g.Ho);
  g.TW = strided::kTWo;
  g.TH = std::max(1, rows / cho) * cho;
  g.tiles_x = (g.Wo + strided::kTWo - 1) / strided::kTWo;
  g.tiles_y = (g.Ho + g.TH - 1) / g.TH;
  return g;
}

// Windows on the float path with stride 2..4 and K in {7, 9, 11, 13}: each
// window centres on its own middle element, so any tap profile is accurate.
bool use_strided(const ssimx_params* p, int dtype) {
  return choose_path(p, dtype) == Path::kSep && strided_supported(p->k, p->stride) && p->k > p->stride;
}

// 8-bit rectangular windows with valid borders go to the band kernel when its
// compile-time window/stride set covers them and the planes allow dword loads.
bool band_eligible(const ssimx_params* p, int dtype) {
  return choose_path(p, dtype) == Path::kBox && dtype == SSIMX_U8 && p->padding == SSIMX_PAD_VALID &&
         box_band_supported(p->k, p->stride);
}

// The fast kernels share one centring value among 4 adjacent windows; it sits
// at window offsets k/2-2 .. k/2+1.  Their weights bound the rounding error
// (sum g (z - t)^2 <= V (1 + 1/g_t)), so windows whose taps there are small
// go to the generic kernel, which centres every window on its middle tap.
bool use_fast(const ssimx_params* p, int dtype) {
  if (choose_path(p, dtype) != Path::kSep || !fast_supported(p->k, p->stride)) return false;
  float taps[KMAX_GAUSS];
  gaussian_taps_f32(p->window, p->k, p->sigma, taps);
  for (int t = p->k / 2 - 2; t <= p->k / 2 + 1; ++t)
    if (taps[t] < 0.04f) return false;
  return true;
}

void fill_fast_common(FastArgs& a, const ssimx_params* p, int dtype, PlaneArg x, PlaneArg y, const Geom& g) {
  a.x = x;
  a.y = y;
  a.g = g;
  a.C1 = (float)p->C1;
  a.C2 = (float)p->C2;
  // vector loads of interior quads form their in-chunk offsets with 24-bit
  // multiplies of the row pitch; wider pitches take the element-wise loads
  a.vec_ok = aligned_vec(x.data, x.pitch, x.bstride, dtype_size(dtype)) &&
             aligned_vec(y.data, y.pitch, y.bstride, dtype_size(dtype)) && x.pitch < kFastMaxPitch &&
             y.pitch < kFastMaxPitch;
  gaussian_taps_f32(p->window, p->k, p->sigma, a.taps);
}

size_t path_lds_bytes(Path path, int dtype, const Geom& g) {
  if (path == Path::kSep) return sep_lds_bytes(g);
  if (path == Path::kBox) {
    const size_t acc = dtype == SSIMX_U8 ? 4 : 8;
    return acc * 5 * (size_t)g.IH * g.TW + 8 * (size_t)g.IH * g.IW + 4 * (BLOCK / 64);
  }
  return 0;
}

Geom make_geom_path(const ssimx_params* p, int dtype, int W, int H, int tile_idx) {
  const TileCfg t = tile_cfg(tile_idx);
  int tw = std::max(1, t.tw / p->stride), th = std::max(1, t.th / p->stride);
  const Path path = choose_path(p, dtype);
  Geom g = geom_with(p, W, H, tw, th);
  while (path_lds_bytes(path, dtype, g) > kLdsLimit && (th > 1 || tw > 1)) {
    if (th >= tw && th > 1)
      th = std::max(1, th / 2);
    else
      tw = std::max(1, tw / 2);
    g = geom_with(p, W, H, tw, th);
  }
  return g;
}

Geom make_geom(const ssimx_params* p, int W, int H, int tile_idx) {
  return make_geom_path(p, SSIMX_U8, W, H, tile_idx);
}

// Worst-case number of pooling partials per frame over every tile config.
int max_partials(const ssimx_params* p, int dtype, int W, int H) {
  const Path path = choose_path(p, dtype);
  int Wo, Ho;
  map_dims(p, W, H, Wo, Ho);
  if (path == Path::kSat) {
    int m = (Wo * Ho + BLOCK - 1) / BLOCK;
    const Geom g = make_geom_path(p, dtype, W, H, 0);
    for (int i = 0; i < num_tile_cfgs(); ++i) m = std::max(m, sat_ssim_tiles(g, dtype, 0, i));
    return m;
  }
  int m = 1;
  for (int i = 0; i < num_tile_cfgs(); ++i) {
    const Geom g = make_geom_path(p, dtype, W, H, i);
    m = std::max(m, g.tiles_x * g.tiles_y);
    if (use_fast(p, dtype)) {
      const Geom f = fast_geom(p, W, H, i);
      m = std::max(m, f.tiles_x * f.tiles_y);
    }
    if (band_eligible(p, dtype)) {
      const Geom b = band_geom(p, W, H, i);
      m = std::max(m, b.tiles_x * b.tiles_y);
    }
    if (use_strided(p, dtype)) {
      const Geom b = strided_geom(p, W, H, i);
      m = std::max(m, b.tiles_x * b.tiles_y);
    }
  }
  return m;
}

void gaussian_taps_f32(int window, int k, float sigma, float* out) {
  if (window == SSIMX_WIN_BOX) {
    for (int t = 0; t < k; ++t) out[t] = (float)(1.0 / k);
    return;
  }
  double g[KMAX_GAUSS], sum = 0.0;
  const double c = (k - 1) / 2.0;
  for (int t = 0; t < k; ++t) {
    const double d = t - c;
    g[t] = exp(-(d * d) / (2.0 * (double)sigma * (double)sigma));
  }
  // sum the small tails first
  for (int t = 0; t < k / 2; ++t) sum += g[t] + g[k - 1 - t];
  if (k & 1) sum += g[k / 2];
  for (int t = 0; t < k; ++t) out[t] = (float)(g[t] / sum);
}

// ---------------------------------------------------------------- workspace
size_t Ws::take(size_t bytes) {
  const size_t off = used;
  used += (bytes + 255) & ~(size_t)255;
  return off;
}

size_t fwd_ws_bytes(const ssimx_params* p, int dtype, int W, int H, int batch) {
  Ws ws;
  ws.take(sizeof(float) * (size_t)batch * max_partials(p, dtype, W, H));
  if (choose_path(p, dtype) == Path::kSat) ws.take(sizeof(uint32_t) * 5 * (size_t)batch * (W + 1) * (size_t)(H + 1));
  return ws.used;
}

// Per-scale sizes of the MS-SSIM pyramid.
void scale_dims(int W, int H, int n_scales, int* Ws_, int* Hs_) {
  Ws_[0] = W;
  Hs_[0] = H;
  for (int j = 1; j < n_scales; ++j) {
    Ws_[j] = Ws_[j - 1] / 2;
    Hs_[j] = Hs_[j - 1] / 2;
  }
}

MsLayout ms_layout(const ssimx_params* p, int dtype, int W, int H, int batch, int n_scales) {
  MsLayout L{};
  Ws ws;
  scale_dims(W, H, n_scales, L.W, L.H);
  for (int j = 0; j < n_scales; ++j) {
    const int dt = j == 0 ? dtype : SSIMX_F32;
    L.partial_off[j] = ws.take(sizeof(float) * (size_t)batch * max_partials(p, dt, L.W[j], L.H[j]));
    if (j > 0) {
      L.lvl_x_off[j] = ws.take(sizeof(float) * (size_t)batch * L.W[j] * L.H[j]);
      L.lvl_y_off[j] = ws.take(sizeof(float) * (size_t)batch * L.W[j] * L.H[j]);
    }
  }
  L.vals_off = ws.take(sizeof(float) * (size_t)batch * n_scales);
  L.lvals_off = ws.take(sizeof(float) * (size_t)batch);
  L.total = ws.used;
  return L;
}

ssimx_status check_ms(const ssimx_params* p, const float* weights, int n_scales, int flags, int W, int H) {
  if (!weights || n_scales < 1 || n_scales > MAX_SCALES) return SSIMX_EINVAL;
  if (flags & ~(SSIMX_MS_RENORM | SSIMX_MS_CS_CLAMP | SSIMX_MS_SUM | SSIMX_MS_COARSE_SEPARATE)) return SSIMX_EINVAL;
  double sum = 0.0;
  for (int j = 0; j < n_scales; ++j) {
    if (!isfinite(weights[j])) return SSIMX_EINVAL;
    sum += weights[j];
  }
  if ((flags & (SSIMX_MS_RENORM | SSIMX_MS_SUM)) && !(sum != 0.0)) return SSIMX_EINVAL;
  int Wj[MAX_SCALES], Hj[MAX_SCALES];
  scale_dims(W, H, n_scales, Wj, Hj);
  for (int j = 0; j < n_scales; ++j) {
    int Wo, Ho;
    if (Wj[j] < 1 || Hj[j] < 1) return SSIMX_ETOOSMALL;
    map_dims(p, Wj[j], Hj[j], Wo, Ho);
    if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  }
  return SSIMX_OK;
}

void ms_weights(const float* weights, int n_scales, int flags, float* w) {
  double sum = 0.0;
  for (int j = 0; j < n_scales; ++j) sum += weights[j];
  const bool norm = (flags & (SSIMX_MS_RENORM | SSIMX_MS_SUM)) != 0;
  for (int j = 0; j < n_scales; ++j) w[j] = norm ? (float)(weights[j] / sum) : weights[j];
}

// ---------------------------------------------------------------- forward core
// One windowed pass over a batch of plane pairs: map (nullable), and the mean
// of the pooled term written to out[frame * out_stride].
ssimx_status fwd_pass(const ssimx_params* p, int dtype, PlaneArg x, PlaneArg y, int W, int H, int batch, int mode,
                      float* map, int64_t map_pitch, int64_t map_bstride, float* out, int64_t out_stride,
                      float* partial, uint32_t* sat, int tile_idx, hipStream_t st, float* ds_x, float* ds_y,
                      int* tiles_out, const float* lw) {
  const Path path = choose_path(p, dtype);
  const float C1 = (float)p->C1, C2 = (float)p->C2;
  int err = 0, tiles = 0;
  bool ds_done = false;
  Geom g = make_geom_path(p, dtype, W, H, tile_idx);
  if (use_fast(p, dtype)) {
    FastArgs a{};
    g = fast_geom(p, W, H, tile_idx, batch);
    fill_fast_common(a, p, dtype, x, y, g);
    a.mode = mode;
    a.map = map;
    a.map_pitch = map_pitch;
    a.map_bstride = map_bstride;
    a.partial = partial;
    a.batch = batch;
    if (ds_x && p->padding == SSIMX_PAD_VALID && W >= 2 && H >= 2) {
      a.ds_x = ds_x;
      a.ds_y = ds_y;
      ds_done = true;
    }
    int epi = ds_done ? 2 : 0;
    if (lw) {
      a.lw_a = lw[0];
      a.lw_b = lw[1];
      epi = 3;
    }
    err = launch_fast_stats(dtype, epi, a, batch, st);
    tiles = g.tiles_x * g.tiles_y;
  } else if (lw) {
    return SSIMX_ENOTSUP;  // luminance weights: the fast path only
  } else if (use_strided(p, dtype)) {
    FastArgs a{};
    g = strided_geom(p, W, H, tile_idx, batch);
    fill_fast_common(a, p, dtype, x, y, g);
    a.mode = mode;
    a.map = map;
    a.map_pitch = map_pitch;
    a.map_bstride = map_bstride;
    a.partial = partial;
    a.batch = batch;
    err = launch_strided(dtype, a, batch, st);
    tiles = g.tiles_x * g.tiles_y;
  } else if (path == Path::kSep) {
    SepArgs a{};
    a.x = x;
    a.y = y;
    a.g = g;
    a.C1 = C1;
    a.C2 = C2;
    a.mode = mode;
    a.map = map;
    a.map_pitch = map_pitch;
    a.map_bstride = map_bstride;
    a.partial = partial;
    gaussian_taps_f32(p->window, p->k, p->sigma, a.taps);
    err = launch_sep_fwd(dtype, a, batch, sep_lds_bytes(g), st);
    tiles = g.tiles_x * g.tiles_y;
  } else if (path == Path::kBox && mode != 2 && band_eligible(p, dtype) &&
             aligned_vec(x.data, x.pitch, x.bstride, 1) && aligned_vec(y.data, y.pitch, y.bstride, 1)) {
    BandArgs a{};
    g = band_geom(p, W, H, tile_idx, batch);
    a.x = x;
    a.y = y;
    a.g = g;
    a.C1 = C1;
    a.C2 = C2;
    a.inv_k4 = (float)(1.0 / ((double)p->k * p->k * p->k * p->k));
    a.mode = mode;
    a.map = map;
    a.map_pitch = map_pitch;
    a.map_bstride = map_bstride;
    a.partial = partial;
    err = launch_box_band(a, batch, st);
    tiles = g.tiles_x * g.tiles_y;
  } else if (path == Path::kBox) {
    BoxArgs a{};
    a.x = x;
    a.y = y;
    a.g = g;
    a.C1 = C1;
    a.C2 = C2;
    a.mode = mode;
    a.map = map;
    a.map_pitch = map_pitch;
    a.map_bstride = map_bstride;
    a.partial = partial;
    a.batch = batch;
    err = launch_box_fwd(dtype, a, batch, st);
    tiles = g.tiles_x * g.tiles_y;
  } else {
    err = launch_sat(dtype, x, y, W, H, batch, sat, st);
    if (err) return hip_status(err);
    err = launch_sat_ssim(sat, g, dtype, batch, C1, C2, mode, map, map_pitch, map_bstride, partial, nullptr, tile_idx,
                          st);
    tiles = sat_ssim_tiles(g, dtype, mode, tile_idx);
  }
  if (err) return hip_status(err);
  if (tiles_out) *tiles_out = tiles;
  if (out) {
    err = launch_finalize(partial, tiles, batch, g.Wo * g.Ho, 1.f, out, out_stride, st);
    if (err) return hip_status(err);
  }
  if (ds_x && !ds_done) {
    err = launch_downsample(dtype, x, W, H, ds_x, ds_y, y, batch, st);
    if (err) return hip_status(err);
  }
  return SSIMX_OK;
}

static ssimx_status fwd_entry(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                              float* map, int64_t map_pitch, int64_t map_bstride, float* score, void* ws,
                              size_t ws_bytes, void* stream, const float* lw = nullptr) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if ((s = check_images(ref, dis, batch)) != SSIMX_OK) return s;
  if ((s = check_path(p, ref->dtype)) != SSIMX_OK) return s;
  if (lw && !use_fast(p, ref->dtype)) return SSIMX_ENOTSUP;
  int Wo, Ho;
  map_dims(p, ref->width, ref->height, Wo, Ho);
  if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  if (map && (map_pitch < Wo || (batch > 1 && map_bstride < map_pitch * (int64_t)Ho))) return SSIMX_EINVAL;
  const size_t need = fwd_ws_bytes(p, ref->dtype, ref->width, ref->height, batch);
  if (!ws || ws_bytes < need) return SSIMX_EWORKSPACE;
  Ws lay;
  float* partial = (float*)((char*)ws + lay.take(sizeof(float) * (size_t)batch *
                                                 max_partials(p, ref->dtype, ref->width, ref->height)));
  uint32_t* sat = nullptr;
  if (choose_path(p, ref->dtype) == Path::kSat)
    sat = (uint32_t*)((char*)ws + lay.take(sizeof(uint32_t) * 5 * (size_t)batch * (ref->width + 1) *
                                           (size_t)(ref->height + 1)));
  PlaneArg x{ref->data, ref->pitch, ref->batch_stride}, y{dis->data, dis->pitch, dis->batch_stride};
  const int tile = pick_tile(p, ref->dtype, ref->width, ref->height, batch);
  return fwd_pass(p, ref->dtype, x, y, ref->width, ref->height, batch, 0, map, map_pitch, map_bstride, score, 1,
                  partial, sat, tile, (hipStream_t)stream, nullptr, nullptr, nullptr, lw);
}

ssimx_status ms_forward(const ssimx_params* p, const float* w, int n_scales, int flags, const ssimx_image* ref,
                        const ssimx_image* dis, int batch, float* score_out, float* cs_out, void* ws,
                        const MsLayout& L, hipStream_t st) {
  char* base = (char*)ws;
  float* vals = (float*)(base + L.vals_off);
  for (int j = 0; j < n_scales; ++j) {
    PlaneArg x, y;
    int dt;
    if (j == 0) {
      x = PlaneArg{ref->data, ref->pitch, ref->batch_stride};
      y = PlaneArg{dis->data, dis->pitch, dis->batch_stride};
      dt = ref->dtype;
    } else {
      x = PlaneArg{base + L.lvl_x_off[j], L.W[j], (int64_t)L.W[j] * L.H[j]};
      y = PlaneArg{base + L.lvl_y_off[j], L.W[j], (int64_t)L.W[j] * L.H[j]};
      dt = SSIMX_F32;
    }
    const bool sep = j + 1 == n_scales && (flags & SSIMX_MS_COARSE_SEPARATE);
    const int mode = (j + 1 < n_scales || sep) ? 1 : 0;
    const int tile = pick_tile(p, dt, L.W[j], L.H[j], batch);
    // the next scale's planes are written by this scale's windowed pass
    float* nx = j + 1 < n_scales ? (float*)(base + L.lvl_x_off[j + 1]) : nullptr;
    float* ny = j + 1 < n_scales ? (float*)(base + L.lvl_y_off[j + 1]) : nullptr;
    ssimx_status s = fwd_pass(p, dt, x, y, L.W[j], L.H[j], batch, mode, nullptr, 0, 0, vals + j, n_scales,
                              (float*)(base + L.partial_off[j]), nullptr, tile, st, nx, ny);
    if (s != SSIMX_OK) return s;
    if (sep) {  // coarsest term mean(l) * mean(cs): the mean of l as well
      s = fwd_pass(p, dt, x, y, L.W[j], L.H[j], batch, 3, nullptr, 0, 0, (float*)(base + L.lvals_off), 1,
                   (float*)(base + L.partial_off[j]), nullptr, tile, st);
      if (s != SSIMX_OK) return s;
    }
  }
  if (score_out) {
    const int err = launch_ms_combine(vals, n_scales, batch, w, flags, score_out, cs_out,
                                      (flags & SSIMX_MS_COARSE_SEPARATE) ? (const float*)(base + L.lvals_off) : nullptr,
                                      st);
    if (err) return hip_status(err);
  }
  return SSIMX_OK;
}

}  // namespace ssimx

using namespace ssimx;

extern "C" {

ssimx_status ssimx_map_shape(const ssimx_params* p, int width, int height, int* width_out, int* height_out) {
  ssimx_status s = check_params(p);
  if (s != SSIMX_OK) return s;
  if (!width_out || !height_out || width < 1 || height < 1) return SSIMX_EINVAL;
  map_dims(p, width, height, *width_out, *height_out);
  if (*width_out < 1 || *height_out < 1) {
    *width_out = std::max(0, *width_out);
    *height_out = std::max(0, *height_out);
    return SSIMX_ETOOSMALL;
  }
  return SSIMX_OK;
}

ssimx_status ssim_map(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                      float* map_out, int64_t map_pitch, int64_t map_batch_stride, float* score_out, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!map_out) return SSIMX_EINVAL;
  return fwd_entry(p, ref, dis, batch, map_out, map_pitch, map_batch_stride, score_out, ws, ws_bytes, stream);
}

ssimx_status ssim_pooled(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                         float* score_out, void* ws, size_t ws_bytes, void* stream) {
  if (!score_out) return SSIMX_EINVAL;
  return fwd_entry(p, ref, dis, batch, nullptr, 0, 0, score_out, ws, ws_bytes, stream);
}

ssimx_status ssim_pooled_lw(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                            float a_s, float b_s, float* score_out, void* ws, size_t ws_bytes, void* stream) {
  if (!score_out || !std::isfinite(a_s) || !std::isfinite(b_s) || b_s < 0.f) return SSIMX_EINVAL;
  const float lw[2] = {a_s, b_s};
  return fwd_entry(p, ref, dis, batch, nullptr, 0, 0, score_out, ws, ws_bytes, stream, lw);
}

ssimx_status msssim(const ssimx_params* p, const float* weights, int n_scales, int flags, const ssimx_image* ref,
                    const ssimx_image* dis, int batch, float* score_out, float* cs_out, void* ws, size_t ws_bytes,
                    void* stream) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if ((s = check_images(ref, dis, batch)) != SSIMX_OK) return s;
  if (!score_out) return SSIMX_EINVAL;
  if ((s = check_ms(p, weights, n_scales, flags, ref->width, ref->height)) != SSIMX_OK) return s;
  if ((s = check_path(p, ref->dtype)) != SSIMX_OK) return s;
  if ((s = check_path(p, SSIMX_F32)) != SSIMX_OK) return s;
  const MsLayout L = ms_layout(p, ref->dtype, ref->width, ref->height, batch, n_scales);
  if (!ws || ws_bytes < L.total) return SSIMX_EWORKSPACE;
  float w[MAX_SCALES];
  ms_weights(weights, n_scales, flags, w);
  return ms_forward(p, w, n_scales, flags, ref, dis, batch, score_out, cs_out, ws, L, (hipStream_t)stream);
}

ssimx_status ssimx_msssim_pyramid_layout(const ssimx_params* p, int dtype, int width, int height, int batch,
                                         int n_scales, int64_t* x_offsets, int64_t* y_offsets, int* widths,
                                         int* heights) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if (width < 1 || height < 1 || batch < 1 || batch > kMaxGridY || n_scales < 1 || n_scales > MAX_SCALES)
    return SSIMX_EINVAL;
  if ((int64_t)width * height > kMaxPlaneElems) return SSIMX_EINVAL;
  if (dtype < SSIMX_U8 || dtype > SSIMX_BF16) return SSIMX_EDTYPE;
  const MsLayout L = ms_layout(p, dtype, width, height, batch, n_scales);
  for (int j = 0; j < n_scales; ++j) {
    if (x_offsets) x_offsets[j] = j == 0 ? -1 : (int64_t)L.lvl_x_off[j];
    if (y_offsets) y_offsets[j] = j == 0 ? -1 : (int64_t)L.lvl_y_off[j];
    if (widths) widths[j] = L.W[j];
    if (heights) heights[j] = L.H[j];
  }
  return SSIMX_OK;
}

ssimx_status ssimx_box_sums(int k, int stride, int algo, const ssimx_image* ref, const ssimx_image* dis, int batch,
                            int32_t* sums_out, void* ws, size_t ws_bytes, void* stream) {
  ssimx_params p{};
  p.window = SSIMX_WIN_BOX;
  p.k = k;
  p.sigma = 1.f;
  p.stride = stride;
  p.padding = SSIMX_PAD_VALID;
  p.algo = algo;
  ssimx_status s;
  if ((s = check_params(&p)) != SSIMX_OK) return s;
  if ((s = check_images(ref, dis, batch)) != SSIMX_OK) return s;
  if (!is_integer(ref->dtype)) return SSIMX_EDTYPE;
  if (!sums_out) return SSIMX_EINVAL;
  int Wo, Ho;
  map_dims(&p, ref->width, ref->height, Wo, Ho);
  if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  PlaneArg x{ref->data, ref->pitch, ref->batch_stride}, y{dis->data, dis->pitch, dis->batch_stride};
  hipStream_t st = (hipStream_t)stream;
  if (algo == SSIMX_ALGO_INTEGRAL_IMAGE) {
    const size_t need = sizeof(uint32_t) * 5 * (size_t)batch * (ref->width + 1) * (size_t)(ref->height + 1);
    if (!ws || ws_bytes < need) return SSIMX_EWORKSPACE;
    const Geom g = make_geom_path(&p, ref->dtype, ref->width, ref->height, 0);
    int err = launch_sat(ref->dtype, x, y, ref->width, ref->height, batch, (uint32_t*)ws, st);
    if (!err)
      err = launch_sat_ssim((uint32_t*)ws, g, ref->dtype, batch, 0.f, 0.f, 2, nullptr, 0, 0, nullptr, sums_out, 0, st);
    return hip_status(err);
  }
  BoxArgs a{};
  a.x = x;
  a.y = y;
  a.g = make_geom_path(&p, ref->dtype, ref->width, ref->height, 0);
  a.mode = 2;
  a.sums = sums_out;
  a.batch = batch;
  return hip_status(launch_box_fwd(ref->dtype, a, batch, st));
}

ssimx_status ssimx_integral_images(const ssimx_image* ref, const ssimx_image* dis, int batch, uint32_t* sat_out,
                                   void* stream) {
  ssimx_status s;
  if ((s = check_images(ref, dis, batch)) != SSIMX_OK) return s;
  if (!is_integer(ref->dtype)) return SSIMX_EDTYPE;
  if (!sat_out) return SSIMX_EINVAL;
  PlaneArg x{ref->data, ref->pitch, ref->batch_stride}, y{dis->data, dis->pitch, dis->batch_stride};
  return hip_status(launch_sat(ref->dtype, x, y, ref->width, ref->height, batch, sat_out, (hipStream_t)stream));
}

const char* ssimx_strerror(int status) {
  switch (status) {
    case SSIMX_OK: return "ok";
    case SSIMX_EINVAL: return "invalid argument";
    case SSIMX_EDTYPE: return "unsupported dtype";
    case SSIMX_ETOOSMALL: return "input smaller than the window";
    case SSIMX_EWORKSPACE: return "workspace missing or too small";
    case SSIMX_EHIP: return "HIP runtime error";
    case SSIMX_ENOTSUP: return "unsupported parameter combination";
    case SSIMX_ENOMEM: return "out of memory";
    case SSIMX_ESCRATCH: return "call needs more scratch than the static no-allocation buffer holds";
    default: return "unknown status";
  }
}

int ssimx_last_hip_error(void) { return g_last_hip; }
int ssimx_version(void) { return SSIMX_VERSION; }

}  // extern "C"
