// The paper's integral images (eq. integral_image_start and the four after
// it) in HBM, and the four-corner window sums of eq. integral_image_end.
//
// Layout: sat[q][frame][r][c], q = 0..4 (x, y, x^2, y^2, xy), r in [0, H],
// c in [0, W]; row 0 and column 0 are zero.  Every entry is kept modulo 2^32
// (uint32 wrap-around); four-corner differences are exact because every true
// window sum is non-negative and below 2^32.
//
// Table build in three passes over row groups of G image rows, without a
// separate column-scan pass over the tables:
//   A  per group: row prefix sums (a block-wide scan per row) accumulated down
//      the group's rows in registers; the group's column totals go to the
//      table row that ends the group;
//   B  per column: inclusive prefix over the group totals, in place, which
//      makes every group-end row final;
//   C  per group: the same row scans again, starting from the final row above
//      the group, writing the group's interior rows.
// HBM traffic: the planes are read twice and the tables written once.
//
// Four-corner pass: one thread per map column walks down the map; the
// difference of the two corner columns of a table row is a running
// column total of row-window sums, so a window sum is the difference of two
// such values K rows apart, kept in a register ring as in the band kernels.
#include "launch.hpp"
#include "box_band.hpp"
#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

namespace {

constexpr int kSNT = 512;  // max threads of a group-scan block

struct SatArgs {
  PlaneArg x, y;
  int W, H, G, n_groups;
  uint32_t* sat;
  int64_t rowlen, fstride, qstride;
  int vec_ok;  // CPT-element vector loads allowed
};

// CPT consecutive elements of row r from column c0 (zeros beyond W).
template <typename T, int CPT>
__device__ __forceinline__ void sat_load(const T* P, int64_t pitch, int W, int r, int c0, int vec_ok, uint32_t* v) {
  const T* s = P + (int64_t)r * pitch + c0;
  if (vec_ok && c0 + CPT <= W) {
    constexpr int NB = CPT * (int)sizeof(T);  // 4, 8, 16, 32 or 64 bytes
    uint32_t w[NB / 4];
    if constexpr (NB == 4) {
      w[0] = *(const uint32_t*)s;
    } else if constexpr (NB == 8) {
      const uint2 t = *(const uint2*)s;
      w[0] = t.x;
      w[1] = t.y;
    } else {
#pragma unroll
      for (int i = 0; i < NB / 16; ++i) {
        const uint4 t = ((const uint4*)s)[i];
        w[4 * i] = t.x;
        w[4 * i + 1] = t.y;
        w[4 * i + 2] = t.z;
        w[4 * i + 3] = t.w;
      }
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      if constexpr (sizeof(T) == 1) v[i] = (w[i >> 2] >> (8 * (i & 3))) & 0xffu;
      else v[i] = (w[i >> 1] >> (16 * (i & 1))) & 0xffffu;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < CPT; ++i) v[i] = c0 + i < W ? (uint32_t)s[i] : 0u;
}

// PHASE 0: group column totals -> the group's end row.  PHASE 1: interior rows.
template <typename T, int CPT, int PHASE>
__global__ __launch_bounds__(kSNT) void sat_group_kernel(SatArgs a) {
  __shared__ uint32_t wtot[2][kSNT / 64][5];
  __shared__ __align__(16) uint32_t tbuf[PHASE == 1 ? kSNT / 64 : 1][PHASE == 1 ? 64 * CPT : 4];
  const int g = blockIdx.x, frame = blockIdx.y;
  const int r0 = g * a.G, r1 = min(a.H, r0 + a.G);  // image rows; table rows r0+1 .. r1
  const int c0 = threadIdx.x * CPT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  const T* X = (const T*)a.x.data + (int64_t)frame * a.x.bstride;
  const T* Y = (const T*)a.y.data + (int64_t)frame * a.y.bstride;
  uint32_t* tab = a.sat + (int64_t)frame * a.fstride;

  uint32_t col[5][CPT];
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int i = 0; i < CPT; ++i)
      col[q][i] = (PHASE == 1 && c0 + i < a.W) ? tab[q * a.qstride + (int64_t)r0 * a.rowlen + c0 + i + 1] : 0u;

  // the next row's pixels are loaded while the current row is scanned
  uint32_t nx[CPT], ny[CPT];
  sat_load<T, CPT>(X, a.x.pitch, a.W, r0, c0, a.vec_ok, nx);
  sat_load<T, CPT>(Y, a.y.pitch, a.W, r0, c0, a.vec_ok, ny);
  for (int r = r0; r < r1; ++r) {
    uint32_t xv[CPT], yv[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      xv[i] = nx[i];
      yv[i] = ny[i];
    }
    if (r + 1 < r1) {
      sat_load<T, CPT>(X, a.x.pitch, a.W, r + 1, c0, a.vec_ok, nx);
      sat_load<T, CPT>(Y, a.y.pitch, a.W, r + 1, c0, a.vec_ok, ny);
    }
    uint32_t p[5][CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      // 8/16-bit samples: full-rate 24-bit products, exact below 2^32
      const uint32_t e[5] = {xv[i], yv[i], (uint32_t)__umul24(xv[i], xv[i]), (uint32_t)__umul24(yv[i], yv[i]),
                             (uint32_t)__umul24(xv[i], yv[i])};
#pragma unroll
      for (int q = 0; q < 5; ++q) p[q][i] = i ? p[q][i - 1] + e[q] : e[q];
    }
    // block-wide exclusive scan of the thread totals
    uint32_t t[5], own[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) own[q] = t[q] = p[q][CPT - 1];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const uint32_t v = __shfl_up(t[q], off, 64);
        if (lane >= off) t[q] += v;
      }
    }
    const int buf = r & 1;
    if (lane == 63)
#pragma unroll
      for (int q = 0; q < 5; ++q) wtot[buf][wid][q] = t[q];
    __syncthreads();
    uint32_t ex[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) ex[q] = t[q] - own[q];
    for (int w = 0; w < nwaves; ++w)
      if (w < wid)
#pragma unroll
        for (int q = 0; q < 5; ++q) ex[q] += wtot[buf][w][q];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int i = 0; i < CPT; ++i) col[q][i] += p[q][i] + ex[q];
    if (PHASE == 1 && r + 1 < r1) {
      // Each lane holds CPT consecutive columns; the row goes out through a
      // wave-private LDS slab so that every store instruction writes 64
      // consecutive entries (one lane per column).
      const int64_t ro = (int64_t)(r + 1) * a.rowlen;
      uint32_t* wb = tbuf[wid];
      const int wc0 = (threadIdx.x & ~63) * CPT;  // first column of this wave
#pragma unroll
      for (int q = 0; q < 5; ++q) {
#pragma unroll
        for (int i = 0; i < CPT; i += 4)
          *(uint4*)&wb[lane * CPT + i] = make_uint4(col[q][i], col[q][i + 1], col[q][i + 2], col[q][i + 3]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint32_t* d = tab + q * a.qstride + ro + 1;
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
          const int c = wc0 + i * 64 + lane;
          if (c < a.W) d[c] = wb[i * 64 + lane];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (threadIdx.x == 0) d[-1] = 0u;
      }
    }
  }
  if (PHASE == 0) {
    const int64_t ro = (int64_t)r1 * a.rowlen;
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int i = 0; i < CPT; ++i)
        if (c0 + i < a.W) tab[q * a.qstride + ro + c0 + i + 1] = col[q][i];
  }
}

// Pass B: inclusive prefix of the group totals down each column (column 0
// and row 0 are zero).
__global__ __launch_bounds__(BLOCK) void sat_carry_kernel(SatArgs a) {
  const int c = blockIdx.x * BLOCK + threadIdx.x;
  if (c > a.W) return;
  const int frame = blockIdx.y, q = blockIdx.z;
  uint32_t* t = a.sat + q * a.qstride + (int64_t)frame * a.fstride + c;
  t[0] = 0u;
  uint32_t carry = 0u;
  for (int g = 0; g < a.n_groups; ++g) {
    const int64_t e = (int64_t)min(a.H, (g + 1) * a.G) * a.rowlen;
    carry += c ? t[e] : 0u;
    t[e] = carry;
  }
}

template <typename T, int CPT>
int launch_groups(const SatArgs& a, int batch, hipStream_t st) {
  const int threads = ((a.W + CPT - 1) / CPT + 63) / 64 * 64;
  dim3 grid(a.n_groups, batch);
  hipLaunchKernelGGL((sat_group_kernel<T, CPT, 0>), grid, dim3(threads), 0, st, a);
  hipLaunchKernelGGL(sat_carry_kernel, dim3((a.W + 1 + BLOCK - 1) / BLOCK, batch, 5), dim3(BLOCK), 0, st, a);
  hipLaunchKernelGGL((sat_group_kernel<T, CPT, 1>), grid, dim3(threads), 0, st, a);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------- four-corner pass
struct SatSsimArgs {
  const uint32_t* sat;
  Geom g;                // TW = 256 map columns, TH map rows per tile
  int64_t rowlen, fstride, qstride;
  float C1, C2, inv_k4;
  int mode;
  float* map;
  int64_t map_pitch, map_bstride;
  float* partial;
};

constexpr int kRowsPerTile[] = {128, 256, 64, 512, 32, 1024};  // input rows per tile, per tile index

template <int K, int S>
__global__ __launch_bounds__(256) void sat_band_ssim_kernel(SatSsimArgs a) {
  constexpr int R = K / S + 1;
  __shared__ float red[4];
  int tile, frame;
  xcd_tile(tile, frame);
  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = __builtin_amdgcn_readfirstlane(txi * 256);
  const int oy0 = __builtin_amdgcn_readfirstlane(tyi * a.g.TH);
  const int oy_end = __builtin_amdgcn_readfirstlane(min(a.g.Ho, oy0 + a.g.TH));
  const int m_max = oy_end - oy0 + R - 2;
  const int oj = ox0 + threadIdx.x;
  const int c = S * min(oj, a.g.Wo - 1);  // inactive lanes read a valid column
  const uint32_t* T0 = a.sat + (int64_t)frame * a.fstride + c;
  uint32_t hist[R][5];
  float acc = 0.f;
  // sample m = table row S (oy0 + m); m0 runs over multiples of R, so sample
  // m sits in ring slot u and the sample K rows above it in slot (u + 1) % R
  // corner values of the next sample are loaded one sample ahead
  uint32_t lo[5], hi[5];
  {
    const uint32_t* p = T0 + (int64_t)(S * oy0) * a.rowlen;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      lo[q] = p[q * a.qstride];
      hi[q] = p[q * a.qstride + K];
    }
  }
  for (int m0 = 0; m0 <= m_max; m0 += R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
#pragma unroll
      for (int q = 0; q < 5; ++q) hist[u][q] = hi[q] - lo[q];
      {
        const int mn = min(m0 + u + 1, m_max);
        const uint32_t* p = T0 + (int64_t)(S * (oy0 + mn)) * a.rowlen;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          lo[q] = p[q * a.qstride];
          hi[q] = p[q * a.qstride + K];
        }
      }
      if (m0 + u <= m_max && m0 + u >= R - 1) {
        const int pv = (u + 1) % R;
        const int oi = oy0 + m0 + u - (R - 1);
        if (oj < a.g.Wo) {
          const SsimTerms t = bband::band_terms<K>(hist[u][0] - hist[pv][0], hist[u][1] - hist[pv][1],
                                                   hist[u][2] - hist[pv][2], hist[u][3] - hist[pv][3],
                                                   hist[u][4] - hist[pv][4], a.inv_k4, a.C1, a.C2);
          const float val = ssim_value(t, a.mode);
          if (a.map) a.map[(int64_t)frame * a.map_bstride + (int64_t)oi * a.map_pitch + oj] = val;
          acc += val;
        }
      }
    }
  }
  const float tot = block_sum<256>(acc, red);
  if (threadIdx.x == 0 && a.partial) a.partial[(int64_t)frame * gridDim.x + tile] = tot;
}

using SatKernel = void (*)(SatSsimArgs);

template <int S, int K>
constexpr SatKernel sat_entry() {
  if constexpr (K % S == 0) return sat_band_ssim_kernel<K, S>;
  else return nullptr;
}

template <int S, int... Ks>
constexpr void sat_fill_row(SatKernel* row, std::integer_sequence<int, Ks...>) {
  ((row[Ks + 2] = sat_entry<S, Ks + 2>()), ...);
}

struct SatTable {
  SatKernel k[3][17] = {};  // [stride 1, 2, 4][window 0..16]
  SatTable() {
    sat_fill_row<1>(k[0], std::make_integer_sequence<int, 15>{});
    sat_fill_row<2>(k[1], std::make_integer_sequence<int, 15>{});
    sat_fill_row<4>(k[2], std::make_integer_sequence<int, 15>{});
  }
};

SatKernel sat_band_kernel(int k, int s, int dtype_is_u8) {
  static const SatTable table;
  if (!dtype_is_u8 || !box_band_supported(k, s)) return nullptr;
  return table.k[s == 1 ? 0 : s == 2 ? 1 : 2][k];
}

Geom sat_band_geom(const Geom& g0, int tile_idx) {
  Geom g = g0;
  const int rows = kRowsPerTile[(tile_idx >= 0 && tile_idx < 6) ? tile_idx : 0];
  g.TW = 256;
  g.TH = max(1, rows / g.s);
  g.tiles_x = (g.Wo + 255) / 256;
  g.tiles_y = (g.Ho + g.TH - 1) / g.TH;
  return g;
}

}  // namespace

int launch_sat(int dtype, PlaneArg x, PlaneArg y, int W, int H, int batch, uint32_t* sat, hipStream_t st) {
  if (W > 16 * kSNT || (dtype != SSIMX_U8 && dtype != SSIMX_U16))
    return launch_sat_rowcol(dtype, x, y, W, H, batch, sat, st);
  SatArgs a{};
  a.x = x;
  a.y = y;
  a.W = W;
  a.H = H;
  a.rowlen = W + 1;
  a.fstride = (int64_t)(H + 1) * a.rowlen;
  a.qstride = (int64_t)batch * a.fstride;
  a.sat = sat;
  a.G = 32;
  while (a.G > 8 && (int64_t)((H + a.G - 1) / a.G) * batch < 1024) a.G /= 2;
  a.n_groups = (H + a.G - 1) / a.G;
  const int cpt = W <= 8 * kSNT ? 8 : 16;
  const int esz = dtype == SSIMX_U8 ? 1 : 2;
  const int vb = cpt * esz;  // bytes per vector load
  a.vec_ok = ((uintptr_t)x.data % (vb >= 16 ? 16 : vb)) == 0 && ((uintptr_t)y.data % (vb >= 16 ? 16 : vb)) == 0 &&
             (x.pitch * esz) % vb == 0 && (y.pitch * esz) % vb == 0 && (x.bstride * esz) % vb == 0 &&
             (y.bstride * esz) % vb == 0;
  if (dtype == SSIMX_U8)
    return cpt == 8 ? launch_groups<uint8_t, 8>(a, batch, st) : launch_groups<uint8_t, 16>(a, batch, st);
  return cpt == 8 ? launch_groups<uint16_t, 8>(a, batch, st) : launch_groups<uint16_t, 16>(a, batch, st);
}

int sat_ssim_tiles(const Geom& g, int dtype, int mode, int tile_idx) {
  if (mode != 2 && sat_band_kernel(g.k, g.s, dtype == SSIMX_U8)) {
    const Geom b = sat_band_geom(g, tile_idx);
    return b.tiles_x * b.tiles_y;
  }
  return (g.Wo * g.Ho + BLOCK - 1) / BLOCK;
}

int launch_sat_ssim(const uint32_t* sat, const Geom& g, int dtype, int batch, float C1, float C2, int mode,
                    float* map, int64_t map_pitch, int64_t map_bstride, float* partial, int32_t* sums, int tile_idx,
                    hipStream_t st) {
  // the ring pass forms its numerators in 24-bit products (K^2 255^2 < 2^24):
  // 8-bit planes only; 16-bit planes and the raw-sum output use the generic pass
  const SatKernel kern = mode != 2 ? sat_band_kernel(g.k, g.s, dtype == SSIMX_U8) : nullptr;
  if (!kern) return launch_sat_ssim_generic(sat, g, batch, C1, C2, mode, map, map_pitch, map_bstride, partial, sums, st);
  SatSsimArgs a{};
  a.sat = sat;
  a.g = sat_band_geom(g, tile_idx);
  a.rowlen = g.W + 1;
  a.fstride = (int64_t)(g.H + 1) * a.rowlen;
  a.qstride = (int64_t)batch * a.fstride;
  a.C1 = C1;
  a.C2 = C2;
  a.inv_k4 = (float)(1.0 / ((double)g.k * g.k * g.k * g.k));
  a.mode = mode;
  a.map = map;
  a.map_pitch = map_pitch;
  a.map_bstride = map_bstride;
  a.partial = partial;
  dim3 grid(a.g.tiles_x * a.g.tiles_y, batch);
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, a);
  return (int)hipGetLastError();
}

}  // namespace ssimx
