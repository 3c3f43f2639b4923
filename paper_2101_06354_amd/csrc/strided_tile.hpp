// Tile body of the strided Gaussian band kernels (window K in {7, 9, 11, 13},
// stride S in {2, 3, 4} with K > S), after the Effect-of-stride subsection:
// only the windows at (S i, S j) are evaluated.
//
// A block owns 64 map columns and marches down its tile in chunks of CHo map
// rows (16 / S, or 3 at stride 4: at most 16 new footprint rows per chunk).
// Per chunk:
//   * the new footprint rows are staged in LDS as u = x + y, v = x - y;
//   * row pass: for every staged row and map column, the row mean and the
//     centred row variance of u and v over the K columns S j .. S j + K - 1,
//     centred on the window's middle element (each window centres on a value
//     of its own, so the rounding error is bounded by the local deviations);
//   * the row statistics go to an LDS band of S (CHo - 1) + K rows; the K - S
//     rows shared with the next chunk stay in the band;
//   * column pass: per map position, the centred combination of the K row
//     statistics (law of total variance), centred on the middle row's mean.
// The next chunk's pixels are fetched into registers during the column pass.
#pragma once

#include "fast_tile.hpp"
#include "fast_tile_body.hpp"
#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {
namespace strided {

constexpr int kNT = 256;   // threads per block
constexpr int kTWo = 64;   // map columns per tile
// Footprint rows per chunk (rounded down to a multiple of S); stride 4 takes
// 12 so that the LDS of three blocks fits a compute unit.
template <int S>
constexpr int chunk_rows() {
  return S == 4 ? 12 : 16;
}

template <int K, int S>
struct Shape {
  static_assert(K > S, "windows of consecutive map rows must overlap");
  static constexpr int CHo = chunk_rows<S>() / S;       // map rows per chunk
  static constexpr int NEW = S * CHo;                   // new footprint rows per chunk
  static constexpr int KEEP = K - S;                    // band rows shared by consecutive chunks
  static constexpr int BAND = NEW + KEEP;               // = S (CHo - 1) + K
  static constexpr int IW = S * (kTWo - 1) + K;         // footprint columns
  static constexpr int NQ = (IW + 3) / 4;               // quads per footprint row
  static constexpr int IWP = 4 * NQ + 4;                // LDS row stride of the footprint
  static constexpr int BWP = kTWo + 4;                  // LDS row stride of the band
  static constexpr int PLB = BAND * BWP;                // floats per band map
  static constexpr int NI = NEW * NQ;                   // staging quads per chunk
  static constexpr int PER = (NI + kNT - 1) / kNT;
  static_assert(KEEP <= NEW, "band copy");
};

template <int K, int S>
__host__ __device__ constexpr int strided_smem_floats() {
  return 2 * Shape<K, S>::NEW * Shape<K, S>::IWP + 4 * Shape<K, S>::PLB;
}

template <int K, int S, typename T>
__device__ __forceinline__ void st_fetch(const FastArgs& a, const T* X, const T* Y, int py0, int px0,
                                         fast::Quad<T>* qx, fast::Quad<T>* qy) {
  using Sh = Shape<K, S>;
#pragma unroll
  for (int i = 0; i < Sh::PER; ++i) {
    const int it = threadIdx.x + i * kNT;
    if (it < Sh::NI) {
      const int r = it / Sh::NQ, q = it - r * Sh::NQ;
      fast::fetch4<T>(X, a.x.pitch, a.g, a.vec_ok, py0 + r, px0 + 4 * q, qx[i]);
      fast::fetch4<T>(Y, a.y.pitch, a.g, a.vec_ok, py0 + r, px0 + 4 * q, qy[i]);
    }
  }
}

template <int K, int S, typename T>
__device__ __forceinline__ void st_store(const fast::Quad<T>* qx, const fast::Quad<T>* qy, float* U, float* V) {
  using Sh = Shape<K, S>;
#pragma unroll
  for (int i = 0; i < Sh::PER; ++i) {
    const int it = threadIdx.x + i * kNT;
    if (it < Sh::NI) {
      const int r = it / Sh::NQ, q = it - r * Sh::NQ;
      float xv[4], yv[4];
      fast::unpack4<T>(qx[i], xv);
      fast::unpack4<T>(qy[i], yv);
      *(float4*)&U[r * Sh::IWP + 4 * q] = make_float4(xv[0] + yv[0], xv[1] + yv[1], xv[2] + yv[2], xv[3] + yv[3]);
      *(float4*)&V[r * Sh::IWP + 4 * q] = make_float4(xv[0] - yv[0], xv[1] - yv[1], xv[2] - yv[2], xv[3] - yv[3]);
    }
  }
}

// Row statistics of `nrows` staged rows into band rows [band0, band0 + nrows).
template <int K, int S>
__device__ __forceinline__ void st_row_pass(const float* taps, const float* U, const float* V, int nrows, float* HM,
                                            int band0) {
  using Sh = Shape<K, S>;
  for (int it = threadIdx.x; it < nrows * kTWo; it += kNT) {
    const int r = it / kTWo, j = it - r * kTWo;
    const float* ur = U + r * Sh::IWP + S * j;
    const float* vr = V + r * Sh::IWP + S * j;
    float u[K], v[K];
    if constexpr (S % 4 == 0) {
#pragma unroll
      for (int n = 0; n < (K + 3) / 4; ++n) {
        const float4 a = *(const float4*)&ur[4 * n];
        const float4 b = *(const float4*)&vr[4 * n];
        const float ua[4] = {a.x, a.y, a.z, a.w}, vb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (4 * n + e < K) {
            u[4 * n + e] = ua[e];
            v[4 * n + e] = vb[e];
          }
      }
    } else if constexpr (S % 2 == 0) {
#pragma unroll
      for (int n = 0; n < (K + 1) / 2; ++n) {
        const float2 a = *(const float2*)&ur[2 * n];
        const float2 b = *(const float2*)&vr[2 * n];
        u[2 * n] = a.x;
        v[2 * n] = b.x;
        if (2 * n + 1 < K) {
          u[2 * n + 1] = a.y;
          v[2 * n + 1] = b.y;
        }
      }
    } else {
#pragma unroll
      for (int n = 0; n < K; ++n) {
        u[n] = ur[n];
        v[n] = vr[n];
      }
    }
    const float tu = u[K / 2], tv = v[K / 2];
    float au = 0.f, av = 0.f, qu = 0.f, qv = 0.f;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      // the middle element's deviations are 0 for finite inputs (a
      // non-finite one already makes the centring value non-finite)
      if (t == K / 2) continue;
      const float du = u[t] - tu, dv = v[t] - tv;
      au = fmaf(taps[t], du, au);
      av = fmaf(taps[t], dv, av);
      qu = fmaf(taps[t] * du, du, qu);
      qv = fmaf(taps[t] * dv, dv, qv);
    }
    const int o = (band0 + r) * Sh::BWP + j;
    HM[o] = tu + au;
    HM[Sh::PLB + o] = tv + av;
    HM[2 * Sh::PLB + o] = fmaf(-au, au, qu);
    HM[3 * Sh::PLB + o] = fmaf(-av, av, qv);
  }
}

// Move band rows [NEW, BAND) to [0, KEEP).
template <int K, int S>
__device__ __forceinline__ void st_band_shift(float* HM) {
  using Sh = Shape<K, S>;
  constexpr int NV = Sh::KEEP * kTWo;
  for (int it = threadIdx.x; it < 4 * NV; it += kNT) {
    const int m = it / NV, e = it - m * NV;
    const int row = e / kTWo, c = e - row * kTWo;
    HM[m * Sh::PLB + row * Sh::BWP + c] = HM[m * Sh::PLB + (Sh::NEW + row) * Sh::BWP + c];
  }
}

// One map tile: returns this thread's share of the tile's pooled sum.
template <int K, int S, typename T>
__device__ __forceinline__ float strided_tile(const FastArgs& a, int frame, int tile, float* smem) {
  using Sh = Shape<K, S>;
  float* U = smem;
  float* V = U + Sh::NEW * Sh::IWP;
  float* HM = V + Sh::NEW * Sh::IWP;

  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = __builtin_amdgcn_readfirstlane(txi * kTWo), oy0 = __builtin_amdgcn_readfirstlane(tyi * a.g.TH);
  const int oy_end = __builtin_amdgcn_readfirstlane(min(a.g.Ho, oy0 + a.g.TH));
  const int px0 = S * ox0, py0 = S * oy0;
  const T* X = (const T*)a.x.data + (int64_t)frame * a.x.bstride;
  const T* Y = (const T*)a.y.data + (int64_t)frame * a.y.bstride;
  float taps[K];
#pragma unroll
  for (int t = 0; t < K; ++t) taps[t] = a.taps[t];

  // prologue: the first K - S footprint rows
  fast::Quad<T> qx[Sh::PER], qy[Sh::PER];
  st_fetch<K, S, T>(a, X, Y, py0, px0, qx, qy);
  st_store<K, S, T>(qx, qy, U, V);
  __syncthreads();
  st_row_pass<K, S>(taps, U, V, Sh::KEEP, HM, 0);
  st_fetch<K, S, T>(a, X, Y, py0 + Sh::KEEP, px0, qx, qy);

  float acc = 0.f;
  for (int cy = oy0; cy < oy_end; cy += Sh::CHo) {
    __syncthreads();  // U, V free; band rows [0, KEEP) ready
    st_store<K, S, T>(qx, qy, U, V);
    __syncthreads();
    st_row_pass<K, S>(taps, U, V, Sh::NEW, HM, Sh::KEEP);
    __syncthreads();
    if (cy + Sh::CHo < oy_end) st_fetch<K, S, T>(a, X, Y, py0 + S * (cy + Sh::CHo - oy0) + Sh::KEEP, px0, qx, qy);
    for (int it = threadIdx.x; it < Sh::CHo * kTWo; it += kNT) {
      const int i = it / kTWo, j = it - i * kTWo;
      const int oi = cy + i, oj = ox0 + j;
      const float* h = HM + (S * i) * Sh::BWP + j;
      const float Tu = h[(K / 2) * Sh::BWP], Tv = h[Sh::PLB + (K / 2) * Sh::BWP];
      float Mu = 0.f, Mv = 0.f, Su = 0.f, Sv = 0.f;
#pragma unroll
      for (int m = 0; m < K; ++m) {
        if (m == K / 2) {  // the centring row adds only its variances
          Su = fmaf(taps[m], h[2 * Sh::PLB + m * Sh::BWP], Su);
          Sv = fmaf(taps[m], h[3 * Sh::PLB + m * Sh::BWP], Sv);
          continue;
        }
        const float du = h[m * Sh::BWP] - Tu, dv = h[Sh::PLB + m * Sh::BWP] - Tv;
        Mu = fmaf(taps[m], du, Mu);
        Mv = fmaf(taps[m], dv, Mv);
        Su = fmaf(taps[m], fmaf(du, du, h[2 * Sh::PLB + m * Sh::BWP]), Su);
        Sv = fmaf(taps[m], fmaf(dv, dv, h[3 * Sh::PLB + m * Sh::BWP]), Sv);
      }
      if (oi >= oy_end || oj >= a.g.Wo) continue;
      const float val = ssim_value_uv(Tu + Mu, Tv + Mv, fmaf(-Mu, Mu, Su), fmaf(-Mv, Mv, Sv), 2.f * a.C1,
                                      2.f * a.C2, a.mode);
      if (a.map) a.map[(int64_t)frame * a.map_bstride + (int64_t)oi * a.map_pitch + oj] = val;
      acc += val;
    }
    __syncthreads();
    st_band_shift<K, S>(HM);
  }
  __syncthreads();  // the caller may reuse smem for the next tile
  return acc;
}

}  // namespace strided

bool strided_supported(int k, int stride);
int launch_strided(int dtype, const FastArgs& a, int batch, hipStream_t st);

}  // namespace ssimx
