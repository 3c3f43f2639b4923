// Separable float path: windowed local statistics of a plane pair, the SSIM
// (or cs) map and per-tile pooled partial sums, for Gaussian windows and for
// rectangular windows on float planes.
//
// Local statistics (Background section, local_means .. local_corr) are formed
// in the basis u = x + y, v = x - y.  Cancellation in E[u^2] - mu_u^2 is kept
// bounded by centring both 1-D passes on a value inside each window (law of
// total variance):
//   row pass    : for an input row r and output column j, with t = u at the
//                 window's middle column, a = sum_t g_t (u - t),
//                 q = sum_t g_t (u - t)^2; the row mean is h = t + a and the
//                 row variance V = q - a^2 (both exact identities when the
//                 taps sum to one);
//   column pass : for output (i, j), with T = h of the window's middle row,
//                 M = sum_m g_m (h_m - T), S = sum_m g_m [V_m + (h_m - T)^2];
//                 mu = T + M and var = S - M^2.
// Every rounding error is then relative to local deviations, not to |u|, so
// flat regions far from any global shift stay exact.  For integer planes the
// row-pass differences and squares are exact integers in float32.
#include "sep_tile.hpp"
#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

size_t sep_lds_bytes(const Geom& g) {
  return sizeof(float) * (sep_tile_lds_floats(g.IH, g.IW, g.TW) + BLOCK / 64);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void sep_fwd_kernel(SepArgs a) {
  extern __shared__ float lds[];
  const int frame = blockIdx.y;
  const int tile = blockIdx.x;
  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = txi * a.g.TW, oy0 = tyi * a.g.TH;
  float* red = lds + sep_tile_lds_floats(a.g.IH, a.g.IW, a.g.TW);

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
  const float tot = block_sum<BLOCK>(acc, red);
  if (threadIdx.x == 0) a.partial[(int64_t)frame * gridDim.x + tile] = tot;
}

int launch_sep_fwd(int dtype, const SepArgs& a, int batch, size_t lds, hipStream_t st) {
  dim3 grid(a.g.tiles_x * a.g.tiles_y, batch), block(BLOCK);
  switch (dtype) {
    case SSIMX_U8:
      hipLaunchKernelGGL(sep_fwd_kernel<uint8_t>, grid, block, lds, st, a);
      break;
    case SSIMX_U16:
      hipLaunchKernelGGL(sep_fwd_kernel<uint16_t>, grid, block, lds, st, a);
      break;
    case SSIMX_F32:
      hipLaunchKernelGGL(sep_fwd_kernel<float>, grid, block, lds, st, a);
      break;
    case SSIMX_BF16:
      hipLaunchKernelGGL(sep_fwd_kernel<bf16_t>, grid, block, lds, st, a);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // namespace ssimx
