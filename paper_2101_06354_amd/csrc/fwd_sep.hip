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
#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

size_t sep_lds_bytes(const Geom& g) {
  return sizeof(float) * (2 * (size_t)g.IH * g.IW + 4 * (size_t)g.IH * g.TW + BLOCK / 64);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void sep_fwd_kernel(SepArgs a) {
  extern __shared__ float lds[];
  const int IW = a.g.IW, IH = a.g.IH, TW = a.g.TW, TH = a.g.TH, k = a.g.k, s = a.g.s;
  const int frame = blockIdx.y;
  const int tile = blockIdx.x;
  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = txi * TW, oy0 = tyi * TH;
  const int px0 = ox0 * s, py0 = oy0 * s;

  float* U = lds;
  float* V = U + IH * IW;
  float* HU = V + IH * IW;
  float* HV = HU + IH * TW;
  float* VU = HV + IH * TW;
  float* VV = VU + IH * TW;
  float* red = VV + IH * TW;

  const T* X = (const T*)a.x.data + (int64_t)frame * a.x.bstride;
  const T* Y = (const T*)a.y.data + (int64_t)frame * a.y.bstride;

  // 1. footprint of the tile -> u, v in LDS (zeros past the padded extent,
  //    which no valid output reads)
  for (int idx = threadIdx.x; idx < IH * IW; idx += BLOCK) {
    const int r = idx / IW, c = idx - r * IW;
    int sy, sx;
    float xv = 0.f, yv = 0.f;
    if (padded_source(py0 + r, px0 + c, a.g.H, a.g.W, a.g.pad, a.g.before, a.g.Hp, a.g.Wp, sy, sx)) {
      xv = to_f32<T>(X[(int64_t)sy * a.x.pitch + sx]);
      yv = to_f32<T>(Y[(int64_t)sy * a.y.pitch + sx]);
    }
    U[idx] = xv + yv;
    V[idx] = xv - yv;
  }
  __syncthreads();

  // 2. row pass at the tile's output columns, for every footprint row
  const int kc = k >> 1;
  for (int idx = threadIdx.x; idx < IH * TW; idx += BLOCK) {
    const int r = idx / TW, j = idx - r * TW;
    const float* ur = U + r * IW + j * s;
    const float* vr = V + r * IW + j * s;
    const float tu = ur[kc], tv = vr[kc];
    float au = 0.f, av = 0.f, qu = 0.f, qv = 0.f;
    for (int t = 0; t < k; ++t) {
      const float w = a.taps[t];
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

  // 3. column pass, SSIM terms, map store and pooling
  float acc = 0.f;
  for (int idx = threadIdx.x; idx < TH * TW; idx += BLOCK) {
    const int i = idx / TW, j = idx - i * TW;
    const int oi = oy0 + i, oj = ox0 + j;
    if (oi >= a.g.Ho || oj >= a.g.Wo) continue;
    const int r0 = i * s;
    const float Tu = HU[(r0 + kc) * TW + j], Tv = HV[(r0 + kc) * TW + j];
    float mu = 0.f, mv = 0.f, su = 0.f, sv = 0.f;
    for (int m = 0; m < k; ++m) {
      const float w = a.taps[m];
      const int o = (r0 + m) * TW + j;
      const float du = HU[o] - Tu, dv = HV[o] - Tv;
      const float wdu = w * du, wdv = w * dv;
      mu += wdu;
      mv += wdv;
      su = fmaf(wdu, du, fmaf(w, VU[o], su));
      sv = fmaf(wdv, dv, fmaf(w, VV[o], sv));
    }
    const SsimTerms t = ssim_terms_uv(Tu + mu, Tv + mv, su - mu * mu, sv - mv * mv, a.C1, a.C2);
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
