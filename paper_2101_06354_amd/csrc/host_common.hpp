// Host-only helpers shared by the C-ABI translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "launch.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

constexpr size_t kLdsLimit = 64 * 1024;  // dynamic LDS per block used by the tiled kernels

enum class Path { kSep, kBox, kSat };

extern thread_local int g_last_hip;
ssimx_status hip_status(int err);

ssimx_status check_params(const ssimx_params* p);
ssimx_status check_images(const ssimx_image* a, const ssimx_image* b, int batch);
ssimx_status check_path(const ssimx_params* p, int dtype);
ssimx_status check_ms(const ssimx_params* p, const float* weights, int n_scales, int flags, int W, int H);
bool is_integer(int dtype);
Path choose_path(const ssimx_params* p, int dtype);
void map_dims(const ssimx_params* p, int W, int H, int& Wo, int& Ho);
Geom make_geom_path(const ssimx_params* p, int dtype, int W, int H, int tile_idx);
int max_partials(const ssimx_params* p, int dtype, int W, int H);
size_t path_lds_bytes(Path path, int dtype, const Geom& g);
void scale_dims(int W, int H, int n_scales, int* Ws_, int* Hs_);
void ms_weights(const float* weights, int n_scales, int flags, float* w);
size_t fwd_ws_bytes(const ssimx_params* p, int dtype, int W, int H, int batch);

struct FastArgs;
int dtype_size(int dtype);
// batch > 0: fill small launches; rows0 > 0: the default index's tile height
// instead of the table's (a multiple of 16, at most the table's largest)
Geom fast_geom(const ssimx_params* p, int W, int H, int tile_idx, int batch = 0, int rows0 = 0);
// Tiles of the coefficient passes (pooled backward, training loss): 256 rows
// when the launch still holds >= 8192 workgroups, else 128 (the coefficient
// kernel writes three planes per position and loses less to short launches
// on shorter tiles); small launches shorten them further by the fill rule.
Geom coef_geom(const ssimx_params* p, int W, int H, int batch);
Geom band_geom(const ssimx_params* p, int W, int H, int tile_idx, int batch = 0);
Geom strided_geom(const ssimx_params* p, int W, int H, int tile_idx, int batch = 0);
bool use_strided(const ssimx_params* p, int dtype);
bool band_eligible(const ssimx_params* p, int dtype);
bool aligned_vec(const void* p, int64_t pitch, int64_t bstride, int esize);
bool use_fast(const ssimx_params* p, int dtype);
void fill_fast_common(FastArgs& a, const ssimx_params* p, int dtype, PlaneArg x, PlaneArg y, const Geom& g);
// Backward: the shift t_u of the u basis in the coefficient planes, and the
// pixel tiles (QH, qtiles_x, qtiles_y) of the fast adjoint for a W x H level.
float shift_guess(const ssimx_params* p);
void adjoint_tiles(FastArgs& fa, int W, int H, int batch);

// Bump allocator over a caller workspace (256-byte aligned slices).
struct Ws {
  size_t used = 0;
  size_t take(size_t bytes);
};

struct MsLayout {
  int W[MAX_SCALES], H[MAX_SCALES];
  size_t partial_off[MAX_SCALES];
  size_t lvl_x_off[MAX_SCALES], lvl_y_off[MAX_SCALES];
  size_t vals_off;
  size_t lvals_off;  // mean(l) at the coarsest scale (SSIMX_MS_COARSE_SEPARATE)
  size_t total;
};
MsLayout ms_layout(const ssimx_params* p, int dtype, int W, int H, int batch, int n_scales);

// MS-SSIM adjoint workspace: the forward's layout, then the score, the
// per-scale upstreams, the coefficient planes, the padded gradient and the
// per-scale gradients.
struct MsBwdLayout {
  MsLayout fwd;
  size_t msval, up, up2, coef, gpad, glev[MAX_SCALES], total;
};
MsBwdLayout ms_bwd_layout(const ssimx_params* p, int dtype, int W, int H, int batch, int M);
// up_ready: the caller has already written the per-scale upstreams (L.up,
// L.up2) and vals, msv, grad_score are not read.
ssimx_status ms_bwd_levels(const ssimx_params* p, const float* w, int n_scales, int flags, const ssimx_image* ref,
                           const ssimx_image* dis, int batch, const float* vals, const float* msv,
                           const float* grad_score, float* grad_dis, int64_t grad_pitch, int64_t grad_batch_stride,
                           char* base, const MsBwdLayout& L, hipStream_t st, bool up_ready = false);

// ds_x, ds_y (nullable): also write the 2x2-average down-sampled planes
// float32 [batch][H/2][W/2] (fused into the stride-1 band kernel when it runs
// with valid borders, else a separate down-sampling launch).  lw (nullable,
// fast path only): {a_s, b_s} of luminance-weighted pooling.
ssimx_status fwd_pass(const ssimx_params* p, int dtype, PlaneArg x, PlaneArg y, int W, int H, int batch, int mode,
                      float* map, int64_t map_pitch, int64_t map_bstride, float* out, int64_t out_stride,
                      float* partial, uint32_t* sat, int tile_idx, hipStream_t st, float* ds_x = nullptr,
                      float* ds_y = nullptr, int* tiles_out = nullptr, const float* lw = nullptr);
ssimx_status ms_forward(const ssimx_params* p, const float* w, int n_scales, int flags, const ssimx_image* ref,
                        const ssimx_image* dis, int batch, float* score_out, float* cs_out, void* ws,
                        const MsLayout& L, hipStream_t st);

// Spatial pooling of float32 maps (pool.hip).
ssimx_status check_pool(const ssimx_pool* pl);
size_t pool_ws_bytes(const ssimx_pool* pl, int w, int h, int batch);
ssimx_status pool_run(const ssimx_pool* pl, const float* map, int w, int h, int64_t pitch, int64_t bstride,
                      int batch, float* out, int64_t out_stride, void* ws, hipStream_t st);

// Tile configuration for a call: explicit override, else the autotune cache,
// else the default (index 0).
int pick_tile(const ssimx_params* p, int dtype, int W, int H, int batch);

}  // namespace ssimx
