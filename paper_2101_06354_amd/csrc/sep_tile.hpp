// Centred separable local statistics of one output tile, staged through LDS.
//
// For every output (i, j) of the tile this produces mean_u, mean_v, var_u,
// var_v of u = x + y and v = x - y under the window w = g g^T (Background
// section, local_means .. local_corr, in the sum/difference basis).  Both 1-D
// passes are centred on a value inside the window (law of total variance):
//   row pass    : t = u at the window's middle column,
//                 a = sum g (u - t), q = sum g (u - t)^2,
//                 row mean h = t + a, row variance V = q - a^2;
//   column pass : T = h of the middle row,
//                 M = sum g (h - T), S = sum g [V + (h - T)^2],
//                 mean = T + M, var = S - M^2.
// With taps summing to one these are exact identities; rounding errors are
// relative to local deviations, not to the magnitude of u.
#pragma once

#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

struct TileStats {
  float mean_u, mean_v, var_u, var_v;
};

__host__ __device__ inline size_t sep_tile_lds_floats(int IH, int IW, int TW) {
  return 2 * (size_t)IH * IW + 4 * (size_t)IH * TW;
}

// Phases 1 and 2 (footprint load and row pass) into LDS; the caller then calls
// sep_tile_column() for its outputs.  `lds` holds sep_tile_lds_floats() floats.
template <typename T>
__device__ __forceinline__ void sep_tile_rows(const Geom& g, const float* taps, PlaneArg xa, PlaneArg ya, int frame,
                                              int ox0, int oy0, float* lds) {
  const int IW = g.IW, IH = g.IH, TW = g.TW, k = g.k, s = g.s;
  const int px0 = ox0 * s, py0 = oy0 * s;
  float* U = lds;
  float* V = U + IH * IW;
  float* HU = V + IH * IW;
  float* HV = HU + IH * TW;
  float* VU = HV + IH * TW;
  float* VV = VU + IH * TW;
  const T* X = (const T*)xa.data + (int64_t)frame * xa.bstride;
  const T* Y = (const T*)ya.data + (int64_t)frame * ya.bstride;
  for (int idx = threadIdx.x; idx < IH * IW; idx += BLOCK) {
    const int r = idx / IW, c = idx - r * IW;
    int sy, sx;
    float xv = 0.f, yv = 0.f;
    if (padded_source(py0 + r, px0 + c, g.H, g.W, g.pad, g.before, g.Hp, g.Wp, sy, sx)) {
      xv = to_f32<T>(X[(int64_t)sy * xa.pitch + sx]);
      yv = to_f32<T>(Y[(int64_t)sy * ya.pitch + sx]);
    }
    U[idx] = xv + yv;
    V[idx] = xv - yv;
  }
  __syncthreads();
  const int kc = k >> 1;
  for (int idx = threadIdx.x; idx < IH * TW; idx += BLOCK) {
    const int r = idx / TW, j = idx - r * TW;
    const float* ur = U + r * IW + j * s;
    const float* vr = V + r * IW + j * s;
    const float tu = ur[kc], tv = vr[kc];
    float au = 0.f, av = 0.f, qu = 0.f, qv = 0.f;
    for (int t = 0; t < k; ++t) {
      const float w = taps[t];
      const float du = ur[t] - tu, dv = vr[t] - tv;
      const float wdu = w * du, wdv = w * dv;
      au += wdu;
      av += wdv;
      qu = fmaf(wdu, du, qu);
      qv = fmaf(wdv, dv, qv);
    }
    HU[idx] = tu + au;
    HV[idx] = tv + av;
    VU[idx] = qu - au * au;
    VV[idx] = qv - av * av;
  }
  __syncthreads();
}

// Phase 3 for tile output (i, j).
__device__ __forceinline__ TileStats sep_tile_column(const Geom& g, const float* taps, const float* lds, int i,
                                                     int j) {
  const int IW = g.IW, IH = g.IH, TW = g.TW, k = g.k, s = g.s;
  const float* HU = lds + 2 * IH * IW;
  const float* HV = HU + IH * TW;
  const float* VU = HV + IH * TW;
  const float* VV = VU + IH * TW;
  const int kc = k >> 1;
  const int r0 = i * s;
  const float Tu = HU[(r0 + kc) * TW + j], Tv = HV[(r0 + kc) * TW + j];
  float mu = 0.f, mv = 0.f, su = 0.f, sv = 0.f;
  for (int m = 0; m < k; ++m) {
    const float w = taps[m];
    const int o = (r0 + m) * TW + j;
    const float du = HU[o] - Tu, dv = HV[o] - Tv;
    const float wdu = w * du, wdv = w * dv;
    mu += wdu;
    mv += wdv;
    su = fmaf(wdu, du, fmaf(w, VU[o], su));
    sv = fmaf(wdv, dv, fmaf(w, VV[o], sv));
  }
  TileStats st;
  st.mean_u = Tu + mu;
  st.mean_v = Tv + mv;
  st.var_u = su - mu * mu;
  st.var_v = sv - mv * mv;
  return st;
}

// Forward tile of the generic separable kernel: map store and this thread's
// share of the tile's pooled sum.  `lds` holds sep_tile_lds_floats() floats.
template <typename T>
__device__ __forceinline__ float sep_fwd_tile(const SepArgs& a, int frame, int tile, float* lds) {
  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = txi * a.g.TW, oy0 = tyi * a.g.TH;
  sep_tile_rows<T>(a.g, a.taps, a.x, a.y, frame, ox0, oy0, lds);
  float acc = 0.f;
  for (int idx = threadIdx.x; idx < a.g.TH * a.g.TW; idx += BLOCK) {
    const int i = idx / a.g.TW, j = idx - i * a.g.TW;
    const int oi = oy0 + i, oj = ox0 + j;
    if (oi >= a.g.Ho || oj >= a.g.Wo) continue;
    const TileStats st = sep_tile_column(a.g, a.taps, lds, i, j);
    const SsimTerms t = ssim_terms_uv(st.mean_u, st.mean_v, st.var_u, st.var_v, a.C1, a.C2);
    const float val = ssim_value(t, a.mode);
    if (a.map) a.map[(int64_t)frame * a.map_bstride + (int64_t)oi * a.map_pitch + oj] = val;
    acc += val;
  }
  __syncthreads();  // the caller may reuse lds for the next tile
  return acc;
}

}  // namespace ssimx
