// Tile body of the integer rectangular-window kernel (shared by the per-frame
// kernel and the persistent ragged-batch kernel).  Exact integer window sums
// S1x, S1y, S2x, S2y, S12 from tile-local row sums; statistics per
// eqs. mean_from_sum .. corr_from_sum with exact int64 numerators.
#pragma once

#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

template <typename T>
struct BoxAcc;  // accumulator type of the window sums
template <>
struct BoxAcc<uint8_t> {
  using type = int32_t;  // k <= 64: 4096 * 255^2 < 2^31
};
template <>
struct BoxAcc<uint16_t> {
  using type = int64_t;
};

// One tile of the integer box kernel: map store (or the five sums in mode 2)
// and this thread's share of the tile's pooled sum.
template <typename T>
__device__ __forceinline__ float box_fwd_tile(const BoxArgs& a, int frame, int tile, unsigned char* lds_raw) {
  using Acc = typename BoxAcc<T>::type;
  const int IW = a.g.IW, IH = a.g.IH, TW = a.g.TW, TH = a.g.TH, k = a.g.k, s = a.g.s;
  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = txi * TW, oy0 = tyi * TH;
  const int px0 = ox0 * s, py0 = oy0 * s;

  Acc* H5 = (Acc*)lds_raw;                       // [5][IH][TW]
  int32_t* XI = (int32_t*)(H5 + 5 * IH * TW);    // [IH][IW]
  int32_t* YI = XI + IH * IW;

  const T* X = (const T*)a.x.data + (int64_t)frame * a.x.bstride;
  const T* Y = (const T*)a.y.data + (int64_t)frame * a.y.bstride;
  for (int idx = threadIdx.x; idx < IH * IW; idx += BLOCK) {
    const int r = idx / IW, c = idx - r * IW;
    int sy, sx;
    int32_t xv = 0, yv = 0;
    if (padded_source(py0 + r, px0 + c, a.g.H, a.g.W, a.g.pad, a.g.before, a.g.Hp, a.g.Wp, sy, sx)) {
      xv = (int32_t)X[(int64_t)sy * a.x.pitch + sx];
      yv = (int32_t)Y[(int64_t)sy * a.y.pitch + sx];
    }
    XI[idx] = xv;
    YI[idx] = yv;
  }
  __syncthreads();

  const int plane = IH * TW;
  for (int idx = threadIdx.x; idx < IH * TW; idx += BLOCK) {
    const int r = idx / TW, j = idx - r * TW;
    const int32_t* xr = XI + r * IW + j * s;
    const int32_t* yr = YI + r * IW + j * s;
    Acc sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
    for (int t = 0; t < k; ++t) {
      const Acc xv = xr[t], yv = yr[t];
      sx += xv;
      sy += yv;
      sxx += xv * xv;
      syy += yv * yv;
      sxy += xv * yv;
    }
    H5[idx] = sx;
    H5[plane + idx] = sy;
    H5[2 * plane + idx] = sxx;
    H5[3 * plane + idx] = syy;
    H5[4 * plane + idx] = sxy;
  }
  __syncthreads();

  const int64_t kk = (int64_t)k * k;
  const float k4 = (float)(kk * kk);
  float acc = 0.f;
  for (int idx = threadIdx.x; idx < TH * TW; idx += BLOCK) {
    const int i = idx / TW, j = idx - i * TW;
    const int oi = oy0 + i, oj = ox0 + j;
    if (oi >= a.g.Ho || oj >= a.g.Wo) continue;
    int64_t S[5] = {0, 0, 0, 0, 0};
    for (int m = 0; m < k; ++m) {
      const int o = (i * s + m) * TW + j;
#pragma unroll
      for (int q = 0; q < 5; ++q) S[q] += (int64_t)H5[q * plane + o];
    }
    if (a.mode == 2) {
      const int64_t mstride = (int64_t)a.g.Ho * a.g.Wo;
      const int64_t base = (int64_t)frame * mstride + (int64_t)oi * a.g.Wo + oj;
#pragma unroll
      for (int q = 0; q < 5; ++q) a.sums[(int64_t)q * a.batch * mstride + base] = (int32_t)S[q];
      continue;
    }
    const SsimTerms t = ssim_terms_box(S[0], S[1], S[2], S[3], S[4], kk, k4, a.C1, a.C2);
    const float val = ssim_value(t, a.mode);
    if (a.map) a.map[(int64_t)frame * a.map_bstride + (int64_t)oi * a.map_pitch + oj] = val;
    acc += val;
  }
  __syncthreads();  // the caller may reuse lds for the next tile
  return acc;
}

__host__ __device__ inline size_t box_tile_lds_bytes(const Geom& g, int acc_bytes) {
  return (size_t)acc_bytes * 5 * g.IH * g.TW + 8 * (size_t)g.IH * g.IW;
}


}  // namespace ssimx
