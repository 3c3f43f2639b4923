// Rectangular windows on integer planes (Performance-Efficiency subsection).
//
// Two ways to the same exact integer window sums S1x, S1y, S2x, S2y, S12:
//   * box_fwd_kernel: tile-local sums (row sums of the footprint in LDS, then
//     column sums), never leaving the chip;
//   * the paper's five integral images (eq. integral_image_start and the four
//     after it), built in HBM by a row scan and a column scan in uint32
//     wrap-around arithmetic, then the four-corner differences of
//     eq. integral_image_end.  Differences modulo 2^32 are exact because every
//     true window sum is non-negative and below 2^32.
// The statistics then follow eqs. mean_from_sum .. corr_from_sum with the
// variance numerators k^2 S2 - S1^2 formed exactly in int64 and rounded to
// float once.
#include "launch.hpp"
#include "box_tile.hpp"
#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

template <typename T>
__global__ __launch_bounds__(BLOCK) void box_fwd_kernel(BoxArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* red = (float*)(lds_raw + box_tile_lds_bytes(a.g, sizeof(typename BoxAcc<T>::type)));
  int tile, frame;
  xcd_tile(tile, frame);
  const float acc = box_fwd_tile<T>(a, frame, tile, lds_raw);
  const float tot = block_sum<BLOCK>(acc, red);
  if (threadIdx.x == 0 && a.partial) a.partial[(int64_t)frame * gridDim.x + tile] = tot;
}

static size_t box_lds_bytes(const Geom& g, int dtype) {
  const size_t acc = dtype == SSIMX_U8 ? 4 : 8;
  return acc * 5 * (size_t)g.IH * g.TW + 8 * (size_t)g.IH * g.IW + 4 * (BLOCK / 64);
}

int launch_box_fwd(int dtype, const BoxArgs& a, int batch, hipStream_t st) {
  dim3 grid(a.g.tiles_x * a.g.tiles_y, batch), block(BLOCK);
  const size_t lds = box_lds_bytes(a.g, dtype);
  if (dtype == SSIMX_U8)
    hipLaunchKernelGGL(box_fwd_kernel<uint8_t>, grid, block, lds, st, a);
  else if (dtype == SSIMX_U16)
    hipLaunchKernelGGL(box_fwd_kernel<uint16_t>, grid, block, lds, st, a);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------- integral images
// Layout: sat[q][frame][r][c], q = 0..4 (x, y, x^2, y^2, xy), r in [0, H],
// c in [0, W]; row 0 and column 0 are zero.

template <typename T>
__global__ __launch_bounds__(BLOCK) void sat_rows_kernel(PlaneArg xa, PlaneArg ya, int W, int H, uint32_t* sat,
                                                         int batch) {
  __shared__ uint32_t scan[5][BLOCK];
  const int r = blockIdx.x;  // 0..H
  const int frame = blockIdx.y;
  const int64_t rowlen = W + 1;
  const int64_t fstride = (int64_t)(H + 1) * rowlen;
  const int64_t qstride = (int64_t)batch * fstride;
  uint32_t* out = sat + (int64_t)frame * fstride + (int64_t)r * rowlen;
  if (r == 0) {
    for (int c = threadIdx.x; c <= W; c += BLOCK)
#pragma unroll
      for (int q = 0; q < 5; ++q) out[q * qstride + c] = 0u;
    return;
  }
  const T* X = (const T*)xa.data + (int64_t)frame * xa.bstride + (int64_t)(r - 1) * xa.pitch;
  const T* Y = (const T*)ya.data + (int64_t)frame * ya.bstride + (int64_t)(r - 1) * ya.pitch;
  const int chunk = (W + BLOCK - 1) / BLOCK;
  const int c0 = threadIdx.x * chunk, c1 = min(W, c0 + chunk);
  uint32_t loc[5] = {0u, 0u, 0u, 0u, 0u};
  for (int c = c0; c < c1; ++c) {
    const uint32_t xv = (uint32_t)X[c], yv = (uint32_t)Y[c];
    loc[0] += xv;
    loc[1] += yv;
    loc[2] += xv * xv;
    loc[3] += yv * yv;
    loc[4] += xv * yv;
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) scan[q][threadIdx.x] = loc[q];
  __syncthreads();
  // inclusive Hillis-Steele scan of the chunk totals
  for (int off = 1; off < BLOCK; off <<= 1) {
    uint32_t v[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] = threadIdx.x >= off ? scan[q][threadIdx.x - off] : 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 5; ++q) scan[q][threadIdx.x] += v[q];
    __syncthreads();
  }
  uint32_t run[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) run[q] = threadIdx.x ? scan[q][threadIdx.x - 1] : 0u;
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q * qstride] = 0u;
  for (int c = c0; c < c1; ++c) {
    const uint32_t xv = (uint32_t)X[c], yv = (uint32_t)Y[c];
    run[0] += xv;
    run[1] += yv;
    run[2] += xv * xv;
    run[3] += yv * yv;
    run[4] += xv * yv;
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q * qstride + c + 1] = run[q];
  }
}

__global__ __launch_bounds__(BLOCK) void sat_cols_kernel(uint32_t* sat, int W, int H, int batch) {
  const int c = blockIdx.x * BLOCK + threadIdx.x;
  if (c > W) return;
  const int frame = blockIdx.y, q = blockIdx.z;
  const int64_t rowlen = W + 1;
  const int64_t fstride = (int64_t)(H + 1) * rowlen;
  uint32_t* p = sat + ((int64_t)q * batch + frame) * fstride + c;
  uint32_t acc = 0u;
  for (int r = 1; r <= H; ++r) {
    acc += p[r * rowlen];
    p[r * rowlen] = acc;
  }
}

// Row scan then column scan (any width); the group-scan build in sat.hip
// takes frames up to 8192 columns.
int launch_sat_rowcol(int dtype, PlaneArg x, PlaneArg y, int W, int H, int batch, uint32_t* sat, hipStream_t st) {
  dim3 g1(H + 1, batch);
  if (dtype == SSIMX_U8)
    hipLaunchKernelGGL(sat_rows_kernel<uint8_t>, g1, dim3(BLOCK), 0, st, x, y, W, H, sat, batch);
  else if (dtype == SSIMX_U16)
    hipLaunchKernelGGL(sat_rows_kernel<uint16_t>, g1, dim3(BLOCK), 0, st, x, y, W, H, sat, batch);
  else
    return (int)hipErrorInvalidValue;
  dim3 g2((W + 1 + BLOCK - 1) / BLOCK, batch, 5);
  hipLaunchKernelGGL(sat_cols_kernel, g2, dim3(BLOCK), 0, st, sat, W, H, batch);
  return (int)hipGetLastError();
}

// Four-corner window sums (eq. integral_image_end) and the SSIM terms.
__global__ __launch_bounds__(BLOCK) void sat_ssim_kernel(const uint32_t* sat, Geom g, int batch, float C1, float C2,
                                                         int mode, float* map, int64_t map_pitch,
                                                         int64_t map_bstride, float* partial, int32_t* sums) {
  __shared__ float red[BLOCK / 64];
  const int frame = blockIdx.y;
  const int n = g.Ho * g.Wo;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  const int64_t rowlen = g.W + 1;
  const int64_t fstride = (int64_t)(g.H + 1) * rowlen;
  const int64_t qstride = (int64_t)batch * fstride;
  const int k = g.k;
  float val = 0.f;
  if (idx < n) {
    const int oi = idx / g.Wo, oj = idx - oi * g.Wo;
    const int r0 = oi * g.s, c0 = oj * g.s;  // window rows r0..r0+k-1
    const uint32_t* base = sat + (int64_t)frame * fstride;
    int64_t S[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const uint32_t* t = base + q * qstride;
      const uint32_t v = t[(r0 + k) * rowlen + c0 + k] + t[r0 * rowlen + c0] - t[(r0 + k) * rowlen + c0] -
                         t[r0 * rowlen + c0 + k];
      S[q] = (int64_t)v;  // window sums are non-negative and below 2^32
    }
    if (mode == 2) {
      const int64_t mstride = (int64_t)n;
#pragma unroll
      for (int q = 0; q < 5; ++q) sums[((int64_t)q * batch + frame) * mstride + idx] = (int32_t)S[q];
    } else {
      const int64_t kk = (int64_t)k * k;
      const SsimTerms t = ssim_terms_box(S[0], S[1], S[2], S[3], S[4], kk, (float)(kk * kk), C1, C2);
      val = ssim_value(t, mode);
      if (map) map[(int64_t)frame * map_bstride + (int64_t)oi * map_pitch + oj] = val;
    }
  }
  const float tot = block_sum<BLOCK>(val, red);
  if (threadIdx.x == 0 && partial) partial[(int64_t)frame * gridDim.x + blockIdx.x] = tot;
}

int launch_sat_ssim_generic(const uint32_t* sat, const Geom& g, int batch, float C1, float C2, int mode, float* map,
                            int64_t map_pitch, int64_t map_bstride, float* partial, int32_t* sums,
                            hipStream_t st) {
  const int n = g.Ho * g.Wo;
  dim3 grid((n + BLOCK - 1) / BLOCK, batch);
  hipLaunchKernelGGL(sat_ssim_kernel, grid, dim3(BLOCK), 0, st, sat, g, batch, C1, C2, mode, map, map_pitch,
                     map_bstride, partial, sums);
  return (int)hipGetLastError();
}

}  // namespace ssimx
