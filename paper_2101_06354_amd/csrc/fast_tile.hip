// Stride-1 tiled kernels with a compile-time window size K.
//
// A block owns a 64-column tile of the map and marches down it in chunks of
// 16 output rows.  Per chunk the footprint rows are staged in LDS, the row
// pass writes four row-statistics maps (row mean and row variance of u and
// v) into an LDS band of 16 + K - 1 rows, and the column pass consumes it.
// The K - 1 band rows shared with the next chunk are moved to the top of the
// band instead of being recomputed, so the row pass costs (16 n + K - 1) /
// (16 n) per output row for an n-chunk tile instead of (16 + K - 1) / 16.
// The next chunk's pixels are fetched into registers before the column pass
// so that their load latency is hidden behind it.
//
// Register blocking: a row-pass item computes 4 adjacent outputs of one row
// and a column-pass item 4 adjacent outputs of one column.  The 4 outputs of
// an item share the centring value (the input at window offset K/2 + 1 of
// the first output, i.e. offsets K/2+1 .. K/2-2 of the four windows), so the
// centred differences and their squares are formed once per input and then
// consumed by 4 FMAs per tap and output.  Sharing keeps every rounding error
// bounded by the local deviations: the shared value lies inside each window
// with weight g_t, and sum g (z - t)^2 <= V (1 + 1/g_t).
//
// Kernel: fast_stats_kernel<K, T, EPI>, EPI = 0: SSIM / cs map + pooled
// partials; EPI = 1: the three adjoint coefficient planes (the transposed
// window over them is in fast_adjoint.hip); EPI = 2: EPI 0 plus the next
// MS-SSIM scale's 2x2 means; EPI = 3: EPI 0 with luminance-weighted partials.
#include "fast_tile_body.hpp"

namespace ssimx {

using namespace fast;

template <int K, typename T, int EPI>
__global__ __launch_bounds__(kNT, sizeof(T) == 4 ? 3 : 4) void fast_stats_kernel(FastArgs a) {
  __shared__ __align__(16) float smem[fast_smem_floats<K>()];
  __shared__ float red[kNT / 64];
  int tile, frame;
  xcd_tile_rows_last(a.g.tiles_x, a.g.tiles_y, tile, frame);
  const float acc = fast_stats_tile<K, T, EPI>(a, frame, tile, smem);
  if constexpr (EPI != 1) {
    const float tot = block_sum<kNT>(acc, red);
    if (threadIdx.x == 0) a.partial[(int64_t)frame * gridDim.x + tile] = tot;
  }
}

template <int K, int EPI>
__global__ __launch_bounds__(kNT, 3) void fast_stats_segs_kernel(FastSegs m) {
  __shared__ __align__(16) float smem[fast_smem_floats<K>()];
  __shared__ float red[kNT / 64];
  const int s = seg_of(m.start, m.n);
  const FastArgs& a = m.seg[s];
  const int tiles = a.g.tiles_x * a.g.tiles_y;
  int tile, frame;
  seg_tile(m.start, s, tiles, tile, frame);
  const float acc = fast_stats_tile<K, float, EPI>(a, frame, tile, smem);
  if constexpr (EPI != 1) {
    const float tot = block_sum<kNT>(acc, red);
    if (threadIdx.x == 0) a.partial[(int64_t)frame * tiles + tile] = tot;
  }
}

// ---------------------------------------------------------------- dispatch
bool fast_supported(int k, int stride) {
  return stride == 1 && (k == 7 || k == 9 || k == 11 || k == 13);
}

template <int K, int EPI>
static int launch_stats_k(int dtype, const FastArgs& a, dim3 grid, hipStream_t st) {
  switch (dtype) {
    case SSIMX_U8: hipLaunchKernelGGL((fast_stats_kernel<K, uint8_t, EPI>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_U16: hipLaunchKernelGGL((fast_stats_kernel<K, uint16_t, EPI>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_F32: hipLaunchKernelGGL((fast_stats_kernel<K, float, EPI>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_BF16: hipLaunchKernelGGL((fast_stats_kernel<K, bf16_t, EPI>), grid, dim3(kNT), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_fast_stats_rgb(const FastArgs& a, int batch, hipStream_t st) {
  dim3 grid(a.g.tiles_x * a.g.tiles_y, 3 * batch);
  switch (a.g.k) {
    case 7: hipLaunchKernelGGL((fast_stats_kernel<7, Rgb8, 0>), grid, dim3(kNT), 0, st, a); break;
    case 9: hipLaunchKernelGGL((fast_stats_kernel<9, Rgb8, 0>), grid, dim3(kNT), 0, st, a); break;
    case 11: hipLaunchKernelGGL((fast_stats_kernel<11, Rgb8, 0>), grid, dim3(kNT), 0, st, a); break;
    case 13: hipLaunchKernelGGL((fast_stats_kernel<13, Rgb8, 0>), grid, dim3(kNT), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_fast_stats(int dtype, int epi, const FastArgs& a, int batch, hipStream_t st) {
  dim3 grid(a.g.tiles_x * a.g.tiles_y, batch);
#define SSIMX_K(KK)                                                                          \
  case KK:                                                                                   \
    return epi == 0   ? launch_stats_k<KK, 0>(dtype, a, grid, st)                            \
           : epi == 1 ? launch_stats_k<KK, 1>(dtype, a, grid, st)                            \
           : epi == 2 ? launch_stats_k<KK, 2>(dtype, a, grid, st)                            \
                      : launch_stats_k<KK, 3>(dtype, a, grid, st);
  switch (a.g.k) {
    SSIMX_K(7)
    SSIMX_K(9)
    SSIMX_K(11)
    SSIMX_K(13)
    default: return (int)hipErrorInvalidValue;
  }
#undef SSIMX_K
}

int launch_fast_stats_segs(int epi, const FastSegs& s, hipStream_t st) {
  if (s.n < 1 || s.n > kMaxSegs || (epi != 0 && epi != 1)) return (int)hipErrorInvalidValue;
  const dim3 grid(s.start[s.n]);
#define SSIMX_K(KK)                                                                                        \
  case KK:                                                                                                 \
    if (epi == 0)                                                                                          \
      hipLaunchKernelGGL((fast_stats_segs_kernel<KK, 0>), grid, dim3(kNT), 0, st, s);                     \
    else                                                                                                   \
      hipLaunchKernelGGL((fast_stats_segs_kernel<KK, 1>), grid, dim3(kNT), 0, st, s);                     \
    break;
  switch (s.seg[0].g.k) {
    SSIMX_K(7)
    SSIMX_K(9)
    SSIMX_K(11)
    SSIMX_K(13)
    default: return (int)hipErrorInvalidValue;
  }
#undef SSIMX_K
  return (int)hipGetLastError();
}

}  // namespace ssimx
