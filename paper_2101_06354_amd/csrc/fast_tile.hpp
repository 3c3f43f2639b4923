// Arguments of the stride-1, compile-time-K tiled kernels (fast_tile.hip).
#pragma once

#include "ssimx_internal.hpp"

namespace ssimx {

// 8-bit planar RGB source of the colour path: staged frame 3 b + c of a launch
// is channel c (0 Y, 1 Cb, 2 Cr, BT.709 as printed) of RGB frame b.
struct Rgb8 {
  uint8_t v;
};

// Row pitches (elements) below which interior quads are loaded as vectors at
// 32-bit offsets from a chunk's row base (24-bit multiplies of the pitch).
constexpr int64_t kFastMaxPitch = int64_t(1) << 24;

struct FastArgs {
  PlaneArg x, y;
  Geom g;            // TW fixed at 64; TH = output rows per tile (multiple of 16)
  float C1, C2;
  int mode;          // 0: Q = l*cs, 1: cs, 3: l (forward) / g_l l + g_cs cs (coefficients)
  int vec_ok;        // 4-element vector loads allowed for interior footprint rows (aligned, pitch < kFastMaxPitch)
  int64_t cstride;   // Rgb8 sources: elements between the R, G and B planes
  // forward epilogue
  float* map;
  int64_t map_pitch, map_bstride;
  float* partial;
  // forward, optional (valid borders): the 2x2-average down-sampled x, y of
  // the next MS-SSIM scale, float32 [batch][H/2][W/2]; every tile writes the
  // blocks of the input rows and columns it owns
  float* ds_x;
  float* ds_y;
  // coefficient epilogue
  const float* grad_map;
  int64_t gm_pitch, gm_bstride;
  const float* gscale;   // per-frame upstream, gscale[frame * gscale_stride] * gmul (of cs in mode 3)
  int gscale_stride;
  const float* gscale2;  // mode 3: per-frame upstream of l, gscale2[frame * gscale2_stride] * gmul
  int gscale2_stride;
  float gmul;
  float tu, tv;
  float* coef;       // planes A = A_u - A_v, B_u, B_v, each [batch][Ho][cpitch]
  int cpitch;        // map positions per coefficient row (multiple of 4)
  int batch;
  // adjoint (transposed window) pass
  int QH, qtiles_x, qtiles_y;
  float* out;
  int64_t out_pitch, out_bstride;
  const float* coarse;
  int Wc, Hc;
  // luminance-weighted forward (epi 3): weights of the reference's local mean
  float lw_a, lw_b;
  float taps[KMAX_GAUSS];
};

// Several stride-1 passes over float32 plane pairs with one window in one
// launch (the scales of an MS-SSIM pyramid): segment i owns workgroups
// [start[i], start[i + 1]) and runs seg[i]'s pass over its (tile, frame)
// grid, so the small scales fill the tail of the large one instead of
// running as launches of their own.  Partials are indexed by the segment's
// own tile count.  Seven argument blocks keep the launch under the 4 KiB
// kernel-argument limit.
constexpr int kMaxSegs = 7;
struct FastSegs {
  FastArgs seg[kMaxSegs];
  int start[kMaxSegs + 1];
  int n;
};

bool fast_supported(int k, int stride);
// epi 0: forward, 1: adjoint coefficients, 2: forward + 2x2 means (a.ds_x,
// a.ds_y), 3: forward whose pooled partials weigh each value by the
// luminance weight of the reference's local mean (a.lw_a, a.lw_b)
int launch_fast_stats(int dtype, int epi, const FastArgs& a, int batch, hipStream_t st);
int launch_fast_adjoint(int dtype, const FastArgs& a, int batch, hipStream_t st);
// Segmented forms (float32 planes, window seg[0].g.k): epi 0 or 1 of the
// statistics kernel; the adjoint over each segment's (qtiles, frames) grid.
int launch_fast_stats_segs(int epi, const FastSegs& s, hipStream_t st);
int launch_fast_adjoint_segs(const FastSegs& s, hipStream_t st);
// Colour path: pooled partials of the three YCbCr channels of `batch` 8-bit
// RGB frames, staged frames 3 b + c (EPI 0, mode 0).
int launch_fast_stats_rgb(const FastArgs& a, int batch, hipStream_t st);
int fast_chunks(int tile_idx);   // 16-row chunks per tile of the fast kernels

}  // namespace ssimx
