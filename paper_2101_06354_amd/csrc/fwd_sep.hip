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
#include "launch.hpp"
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
  float* red = lds + sep_tile_lds_floats(a.g.IH, a.g.IW, a.g.TW);
  int tile, frame;
  xcd_tile(tile, frame);
  const float acc = sep_fwd_tile<T>(a, frame, tile, lds);
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
