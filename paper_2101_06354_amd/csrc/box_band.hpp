// Band kernel for rectangular windows on 8-bit planes (valid borders,
// compile-time window size K <= 16 and stride S in {1, 2, 4} with K % S == 0).
//
// The five window sums S1x, S1y, S2x, S2y, S12 of the Performance-Efficiency
// subsection are formed exactly in uint32, as the integral-image method forms
// them, but without the five tables in HBM:
//   * one thread owns one output column and walks down the tile;
//   * per input row it forms the row sums of its K-byte window with byte-dot
//     instructions on packed pixels (sum x = dot4(q, 1), sum x^2 = dot4(q, q),
//     sum xy = dot4(qx, qy), four pixels per instruction);
//   * the row sums are added to five running column totals P, and the totals
//     are sampled every S rows into a register ring of R = K/S + 1 samples, so
//     a window sum is the difference of two samples K rows apart.
// The totals wrap modulo 2^32; differences are exact because every true
// window sum is non-negative and below 2^32 (K <= 16: K^2 255^2 < 2^24).
// Variance numerators k^2 S2 - S1^2 are formed with 24-bit multiplies, also
// modulo 2^32, where every true value fits (eqs. mean_from_sum ..
// corr_from_sum), and are rounded to float once.
//
// Footprint rows are staged in LDS in chunks of R * S rows (one trip round the
// ring); the next chunk is fetched into registers while the current one is
// consumed.
#pragma once

#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

struct BandArgs {
  PlaneArg x, y;
  Geom g;               // TW = 256 output columns, TH output rows per tile
  float C1, C2;
  float inv_k4;         // 1 / k^4
  int mode;             // 0: Q, 1: cs
  float* map;           // nullable
  int64_t map_pitch, map_bstride;
  float* partial;       // [batch][tiles]
};

namespace bband {

constexpr int kNT = 256;  // threads per block = output columns per tile

template <int K, int S>
struct Shape {
  static_assert(K >= 2 && K <= 16, "window size");
  static_assert(S == 1 || S == 2 || S == 4, "stride");
  static_assert(K % S == 0, "window must be a multiple of the stride");
  static constexpr int R = K / S + 1;                    // samples in the ring
  static constexpr int CH = R * S;                       // input rows per chunk
  static constexpr int NQ = (K + 3) / 4;                 // byte quads per window row
  static constexpr bool ALIGNED = (S % 4) == 0;          // window starts on a dword
  static constexpr int NW = ALIGNED ? NQ : NQ + 1;       // dwords read per window row
  static constexpr int RW = (S * (kNT - 1)) / 4 + NW;    // staged dwords per row
  static constexpr int N = CH * RW;                      // staged dwords per plane
  static constexpr int PER = (N + kNT - 1) / kNT;        // prefetch dwords per thread and plane
};

template <int K, int S>
__host__ __device__ constexpr int band_lds_dwords() {
  return 2 * Shape<K, S>::N;
}

// Four bytes of row `row` starting at byte column `col` (zeros outside the
// plane); interior dwords are one aligned load.
__device__ __forceinline__ uint32_t band_dword(const uint8_t* P, int64_t pitch, int W, int H, int row, int col) {
  if (row >= H) return 0u;
  const uint8_t* s = P + (int64_t)row * pitch + col;
  if (col + 3 < W) return *(const uint32_t*)s;
  uint32_t v = 0u;
#pragma unroll
  for (int b = 0; b < 4; ++b)
    if (col + b < W) v |= (uint32_t)s[b] << (8 * b);
  return v;
}

template <int K, int S>
__device__ __forceinline__ void band_fetch(const BandArgs& a, const uint8_t* X, const uint8_t* Y, int r0, int px0,
                                           uint32_t* rx, uint32_t* ry) {
  using Sh = Shape<K, S>;
#pragma unroll
  for (int i = 0; i < Sh::PER; ++i) {
    const int it = threadIdx.x + i * kNT;
    if (it < Sh::N) {
      const int r = it / Sh::RW, c = it - r * Sh::RW;
      rx[i] = band_dword(X, a.x.pitch, a.g.W, a.g.H, r0 + r, px0 + 4 * c);
      ry[i] = band_dword(Y, a.y.pitch, a.g.W, a.g.H, r0 + r, px0 + 4 * c);
    }
  }
}

template <int K, int S>
__device__ __forceinline__ void band_store(const uint32_t* rx, const uint32_t* ry, uint32_t* Xs, uint32_t* Ys) {
  using Sh = Shape<K, S>;
#pragma unroll
  for (int i = 0; i < Sh::PER; ++i) {
    const int it = threadIdx.x + i * kNT;
    if (it < Sh::N) {
      Xs[it] = rx[i];
      Ys[it] = ry[i];
    }
  }
}

// Row sums of one staged row added into the running totals P.
template <int K, int S>
__device__ __forceinline__ void band_row(const uint32_t* xr, const uint32_t* yr, int sh, uint32_t* P) {
  using Sh = Shape<K, S>;
  uint32_t dx[Sh::NW], dy[Sh::NW];
#pragma unroll
  for (int w = 0; w < Sh::NW; ++w) {
    dx[w] = xr[w];
    dy[w] = yr[w];
  }
#pragma unroll
  for (int q = 0; q < Sh::NQ; ++q) {
    uint32_t qx, qy;
    if constexpr (Sh::ALIGNED) {
      qx = dx[q];
      qy = dy[q];
    } else {
      qx = __builtin_amdgcn_alignbyte(dx[q + 1], dx[q], sh);
      qy = __builtin_amdgcn_alignbyte(dy[q + 1], dy[q], sh);
    }
    if (q == Sh::NQ - 1 && (K & 3)) {
      constexpr uint32_t mask = (1u << (8 * (K & 3))) - 1u;
      qx &= mask;
      qy &= mask;
    }
    P[0] = __builtin_amdgcn_udot4(qx, 0x01010101u, P[0], false);
    P[1] = __builtin_amdgcn_udot4(qy, 0x01010101u, P[1], false);
    P[2] = __builtin_amdgcn_udot4(qx, qx, P[2], false);
    P[3] = __builtin_amdgcn_udot4(qy, qy, P[3], false);
    P[4] = __builtin_amdgcn_udot4(qx, qy, P[4], false);
  }
}

// SSIM terms from the five exact window sums of a K x K window (K <= 16, 8-bit
// data).  All numerators are exact modulo 2^32 and their true values fit.
template <int K>
__device__ __forceinline__ SsimTerms band_terms(uint32_t sx, uint32_t sy, uint32_t sxx, uint32_t syy, uint32_t sxy,
                                                float inv_k4, float C1, float C2) {
  constexpr uint32_t kk = K * K;
  const uint32_t nxx = __umul24(kk, sxx) - __umul24(sx, sx);
  const uint32_t nyy = __umul24(kk, syy) - __umul24(sy, sy);
  const uint32_t nxy = __umul24(kk, sxy) - __umul24(sx, sy);
  // Luminance terms in the sum/difference basis (both exact in float):
  // 2 sx sy = (su^2 - sv^2)/2 and sx^2 + sy^2 = (su^2 + sv^2)/2.  Swapping x
  // and y only negates sv, so every evaluation order, fused or not, gives
  // bitwise symmetric terms, and sv = 0 gives A1 == B1.
  const float su = (float)(sx + sy), sv = (float)sx - (float)sy;
  const float Pu = (0.5f * su) * su, Rv = (0.5f * sv) * sv;
  SsimTerms t;
  t.A1 = fmaf(Pu - Rv, inv_k4, C1);
  t.B1 = fmaf(Pu + Rv, inv_k4, C1);
  t.D1 = (2.f * Rv) * inv_k4;
  t.A2 = fmaf((float)(int32_t)(2u * nxy), inv_k4, C2);
  t.B2 = fmaf((float)(nxx + nyy), inv_k4, C2);
  t.D2 = (float)(nxx + nyy - 2u * nxy) * inv_k4;
  return t;
}

// One 256-column tile: returns this thread's share of the tile's pooled sum.
// `lds` holds band_lds_dwords<K, S>() dwords.  PF = false loads each chunk
// right before it is consumed instead of one chunk ahead (fewer live
// registers, for callers that also host other tile bodies).
template <int K, int S, bool PF = true>
__device__ __forceinline__ float box_band_tile(const BandArgs& a, int frame, int tile, uint32_t* lds) {
  using Sh = Shape<K, S>;
  constexpr int R = Sh::R;
  uint32_t* Xs = lds;
  uint32_t* Ys = lds + Sh::N;

  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = __builtin_amdgcn_readfirstlane(txi * kNT);
  const int oy0 = __builtin_amdgcn_readfirstlane(tyi * a.g.TH);
  const int oy_end = __builtin_amdgcn_readfirstlane(min(a.g.Ho, oy0 + a.g.TH));
  const int m_max = oy_end - oy0 + R - 2;  // last ring sample of the tile
  const int px0 = S * ox0, ry0 = S * oy0;
  const uint8_t* X = (const uint8_t*)a.x.data + (int64_t)frame * a.x.bstride;
  const uint8_t* Y = (const uint8_t*)a.y.data + (int64_t)frame * a.y.bstride;
  const int oj = ox0 + threadIdx.x;
  const int boff = S * threadIdx.x;
  const int w0 = boff >> 2, sh = boff & 3;

  uint32_t hist[R][5];
  uint32_t P[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
  for (int q = 0; q < 5; ++q) hist[0][q] = 0u;  // sample 0: nothing summed yet

  uint32_t rx[Sh::PER], ry[Sh::PER];
  if constexpr (PF) band_fetch<K, S>(a, X, Y, ry0, px0, rx, ry);
  float acc = 0.f;
  // m0 runs over 1, 1 + R, 1 + 2R, ...: sample m = m0 + u lives in ring slot
  // (1 + u) % R, and the sample K rows earlier in slot (2 + u) % R.
  for (int m0 = 1; m0 <= m_max; m0 += R) {
    __syncthreads();  // staging buffer free
    if constexpr (!PF) band_fetch<K, S>(a, X, Y, ry0 + S * (m0 - 1), px0, rx, ry);
    band_store<K, S>(rx, ry, Xs, Ys);
    __syncthreads();
    if constexpr (PF)
      if (m0 + R <= m_max) band_fetch<K, S>(a, X, Y, ry0 + S * (m0 - 1 + R), px0, rx, ry);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int m = m0 + u;
      if (m <= m_max) {
        // the S rows of a sample only add into P: kept rolled to bound the
        // number of live registers
#pragma unroll 1
        for (int rr = 0; rr < S; ++rr) {
          const int lr = u * S + rr;
          band_row<K, S>(Xs + lr * Sh::RW + w0, Ys + lr * Sh::RW + w0, sh, P);
        }
        const int slot = (1 + u) % R, prev = (2 + u) % R;
#pragma unroll
        for (int q = 0; q < 5; ++q) hist[slot][q] = P[q];
        if (m >= R - 1) {
          const int oi = oy0 + m - (R - 1);
          if (oj < a.g.Wo) {
            const SsimTerms t =
                band_terms<K>(hist[slot][0] - hist[prev][0], hist[slot][1] - hist[prev][1],
                              hist[slot][2] - hist[prev][2], hist[slot][3] - hist[prev][3],
                              hist[slot][4] - hist[prev][4], a.inv_k4, a.C1, a.C2);
            const float val = ssim_value(t, a.mode);
            if (a.map) a.map[(int64_t)frame * a.map_bstride + (int64_t)oi * a.map_pitch + oj] = val;
            acc += val;
          }
        }
      }
    }
  }
  __syncthreads();  // the caller may reuse lds for the next tile
  return acc;
}

}  // namespace bband

// Host side (box_band.hip)
bool box_band_supported(int k, int s);
int launch_box_band(const BandArgs& a, int batch, hipStream_t st);

}  // namespace ssimx
