// Host-side declarations shared by the translation units: tile
// configurations and the kernel launchers (each returns a hipError_t as int).
#pragma once

#include "ssimx_internal.hpp"

namespace ssimx {

// Host helpers (defined in host.hip) --------------------------------------
struct TileCfg {
  int tw, th;  // outputs per tile at stride 1 (scaled for larger strides)
};
int num_tile_cfgs();
TileCfg tile_cfg(int idx);
Geom make_geom(const ssimx_params* p, int W, int H, int tile_idx);
void gaussian_taps_f32(int window, int k, float sigma, float* out);

// Launchers (return hipError_t as int) ------------------------------------
int launch_sep_fwd(int dtype, const SepArgs& a, int batch, size_t lds_bytes, hipStream_t st);
int launch_box_fwd(int dtype, const BoxArgs& a, int batch, hipStream_t st);
int launch_finalize(const float* partial, int tiles, int batch, int count_per_frame, float scale, float* out,
                    int64_t out_stride, hipStream_t st);
int launch_downsample(int dtype, PlaneArg in, int W, int H, float* outx, float* outy, PlaneArg iny,
                      int batch, hipStream_t st);
int launch_downsample_f(int dtype, PlaneArg x, PlaneArg y, int W, int H, int f, float* outx, float* outy, int batch,
                        hipStream_t st);
int launch_ms_combine(const float* vals, int n_scales, int batch, const float* w, int flags, float* score_out,
                      float* cs_out, const float* lvals, hipStream_t st);
int launch_sat(int dtype, PlaneArg x, PlaneArg y, int W, int H, int batch, uint32_t* sat, hipStream_t st);
int launch_sat_ssim(const uint32_t* sat, const Geom& g, int dtype, int batch, float C1, float C2, int mode,
                    float* map, int64_t map_pitch, int64_t map_bstride, float* partial, int32_t* sums, int tile_idx,
                    hipStream_t st);
int launch_sat_rowcol(int dtype, PlaneArg x, PlaneArg y, int W, int H, int batch, uint32_t* sat, hipStream_t st);
int launch_sat_ssim_generic(const uint32_t* sat, const Geom& g, int batch, float C1, float C2, int mode, float* map,
                            int64_t map_pitch, int64_t map_bstride, float* partial, int32_t* sums,
                            hipStream_t st);
// Partials per frame written by launch_sat_ssim for a tile index.
int sat_ssim_tiles(const Geom& g, int dtype, int mode, int tile_idx);

size_t sep_lds_bytes(const Geom& g);

}  // namespace ssimx
