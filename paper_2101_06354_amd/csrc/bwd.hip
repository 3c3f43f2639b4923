// Adjoint of SSIM / MS-SSIM with respect to the distorted plane.
//
// In the basis u = x + y, v = x - y, each map position p depends on the
// window moments mean_u, mean_v, var_u = E[u^2] - mean_u^2, var_v.  With
// alpha = dT/dmean (variances held fixed) and beta = dT/dvar (T = Q or cs),
//   dT(p)/du(q) = w(q - s p) [alpha_u(p) + 2 beta_u(p) (u(q) - mean_u(p))]
// and likewise for v; dy = du - dv.  The backward therefore
//   1. recomputes the moments of every map position (same centred passes as
//      the forward; nothing is stored by the forward) and forms, centred on
//      a fixed shift t,
//        A_u = g (alpha_u - 2 beta_u (mean_u - t_u)),  B_u = 2 g beta_u
//      (g = upstream dL/dT(p)) and likewise for v; since the transposed
//      window W^T is linear, only three planes are written:
//        A = A_u - A_v, B_u, B_v;
//   2. applies the transposed window to them (a gather over the positions
//      whose window covers q) and combines
//        dL/dy(q) = (W^T A)(q) + (u(q) - t_u) (W^T B_u)(q) - (v(q) - t_v) (W^T B_v)(q).
// Border handling is adjoined by folding the padded gradient back onto its
// source pixels; the MS-SSIM pyramid by the transpose of 2x2 averaging.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "launch.hpp"
#include "fast_tile.hpp"
#include "host_common.hpp"
#include "sep_tile.hpp"
#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

struct CoefArgs {
  PlaneArg x, y;
  Geom g;
  float C1, C2;
  int mode;  // 0: Q, 1: cs, 3: g_l l + g_cs cs with per-frame upstreams
  const float* grad_map;
  int64_t gm_pitch, gm_bstride;
  const float* gscale;  // per-frame upstream scalars, gscale[frame * gscale_stride] * gmul (of cs in mode 3)
  int gscale_stride;
  const float* gscale2;  // mode 3: per-frame upstream of l
  int gscale2_stride;
  float gmul;
  float tu, tv;
  float* coef;  // planes A = A_u - A_v, B_u, B_v, each [batch][Ho][cpitch]
  int cpitch;
  int batch;
  float taps[KMAX_GAUSS];
};

template <typename T>
__global__ __launch_bounds__(BLOCK) void bwd_coef_kernel(CoefArgs a) {
  extern __shared__ float lds[];
  int tile, frame;
  xcd_tile(tile, frame);
  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  const int ox0 = txi * a.g.TW, oy0 = tyi * a.g.TH;
  sep_tile_rows<T>(a.g, a.taps, a.x, a.y, frame, ox0, oy0, lds);
  const float gframe = a.grad_map ? 0.f : a.gscale[(int64_t)frame * a.gscale_stride] * a.gmul;
  const float gl_frame = a.mode == 3 ? a.gscale2[(int64_t)frame * a.gscale2_stride] * a.gmul : 0.f;
  for (int idx = threadIdx.x; idx < a.g.TH * a.g.TW; idx += BLOCK) {
    const int i = idx / a.g.TW, j = idx - i * a.g.TW;
    const int oi = oy0 + i, oj = ox0 + j;
    if (oi >= a.g.Ho || oj >= a.g.Wo) continue;
    const TileStats st = sep_tile_column(a.g, a.taps, lds, i, j);
    const SsimTerms t = ssim_terms_uv(st.mean_u, st.mean_v, st.var_u, st.var_v, a.C1, a.C2);
    const float g = a.grad_map ? a.grad_map[(int64_t)frame * a.gm_bstride + (int64_t)oi * a.gm_pitch + oj] : gframe;
    const float ib2 = 1.f / t.B2;
    const float dcs_du = 0.5f * st.var_v * ib2 * ib2;        // d cs / d var_u
    const float dcs_dv = -0.5f * (t.A2 + t.B2) * ib2 * ib2;  // d cs / d var_v
    float au = 0.f, av = 0.f, bu, bv, gg = g;
    if (a.mode == 1) {
      bu = dcs_du;
      bv = dcs_dv;
    } else {
      // d(fl l + fc cs): Q = l cs takes fl = cs, fc = l; mode 3 the two upstreams
      const float ib1 = 1.f / t.B1;
      float fl = t.A2 * ib2, fc = t.A1 * ib1;
      if (a.mode == 3) {
        fl = gl_frame;
        fc = g;
        gg = 1.f;
      }
      au = fl * st.mean_u * (st.mean_v * st.mean_v) * ib1 * ib1;  // fl * d l / d mean_u
      av = -fl * st.mean_v * (t.A1 + t.B1) * ib1 * ib1;           // fl * d l / d mean_v
      bu = fc * dcs_du;
      bv = fc * dcs_dv;
    }
    const int64_t o = ((int64_t)frame * a.g.Ho + oi) * a.cpitch + oj;
    const int64_t qs = (int64_t)a.batch * a.g.Ho * a.cpitch;
    a.coef[o] = gg * ((au - 2.f * bu * (st.mean_u - a.tu)) - (av - 2.f * bv * (st.mean_v - a.tv)));
    a.coef[qs + o] = 2.f * gg * bu;
    a.coef[2 * qs + o] = 2.f * gg * bv;
  }
}

struct ScatArgs {
  PlaneArg x, y;
  Geom g;
  const float* coef;  // planes A, B_u, B_v, row pitch cpitch
  int cpitch;
  int batch;
  float tu, tv;
  int QW, QH, qtiles_x, MR, MC;
  float* out;
  int64_t out_pitch, out_bstride;
  const float* coarse;  // nullable: coarser-scale gradient [batch][Hc][Wc] added through the 2x2 transpose
  int Wc, Hc;
  float taps[KMAX_GAUSS];
};

__device__ __forceinline__ int ceil_div_i(int a, int s) { return a >= 0 ? (a + s - 1) / s : -((-a) / s); }

template <typename T>
__global__ __launch_bounds__(BLOCK) void bwd_scatter_kernel(ScatArgs a) {
  extern __shared__ float lds[];
  const Geom& g = a.g;
  int tile, frame;
  xcd_tile(tile, frame);
  const int tyi = tile / a.qtiles_x, txi = tile - tyi * a.qtiles_x;
  const int qx0 = txi * a.QW, qy0 = tyi * a.QH;
  const int k = g.k, s = g.s;
  // map positions whose window reaches the tile
  const int pr_lo = max(0, ceil_div_i(qy0 - k + 1, s));
  const int pr_hi = min(g.Ho - 1, (qy0 + a.QH - 1) / s);
  const int pc_lo = max(0, ceil_div_i(qx0 - k + 1, s));
  const int pc_hi = min(g.Wo - 1, (qx0 + a.QW - 1) / s);
  const int nr = max(0, pr_hi - pr_lo + 1), nc = max(0, pc_hi - pc_lo + 1);
  const int MR = a.MR, MC = a.MC, QW = a.QW;
  float* C = lds;                  // [3][MR][MC]
  float* Hm = C + 3 * MR * MC;     // [3][MR][QW]
  const int64_t qs = (int64_t)a.batch * g.Ho * a.cpitch;
  for (int idx = threadIdx.x; idx < nr * nc; idx += BLOCK) {
    const int r = idx / nc, c = idx - r * nc;
    const int64_t o = ((int64_t)frame * g.Ho + pr_lo + r) * a.cpitch + pc_lo + c;
    C[r * MC + c] = a.coef[o];
    C[(MR + r) * MC + c] = a.coef[qs + o];
    C[(2 * MR + r) * MC + c] = a.coef[2 * qs + o];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nr * QW; idx += BLOCK) {
    const int r = idx / QW, qx = idx - r * QW;
    const int px = qx0 + qx;
    const int ca = max(pc_lo, ceil_div_i(px - k + 1, s)), cb = min(pc_hi, px / s);
    float h0 = 0.f, h1 = 0.f, h2 = 0.f;
    for (int pc = ca; pc <= cb; ++pc) {
      const float w = a.taps[px - s * pc];
      const int o = r * MC + (pc - pc_lo);
      h0 = fmaf(w, C[o], h0);
      h1 = fmaf(w, C[MR * MC + o], h1);
      h2 = fmaf(w, C[2 * MR * MC + o], h2);
    }
    const int o = r * QW + qx;
    Hm[o] = h0;
    Hm[MR * QW + o] = h1;
    Hm[2 * MR * QW + o] = h2;
  }
  __syncthreads();
  const T* X = (const T*)a.x.data + (int64_t)frame * a.x.bstride;
  const T* Y = (const T*)a.y.data + (int64_t)frame * a.y.bstride;
  for (int idx = threadIdx.x; idx < a.QH * QW; idx += BLOCK) {
    const int qy = idx / QW, qx = idx - qy * QW;
    const int py = qy0 + qy, px = qx0 + qx;
    if (py >= g.Hp || px >= g.Wp) continue;
    const int ra = max(pr_lo, ceil_div_i(py - k + 1, s)), rb = min(pr_hi, py / s);
    float ga = 0.f, gb = 0.f, gc = 0.f;
    for (int pr = ra; pr <= rb; ++pr) {
      const float w = a.taps[py - s * pr];
      const int o = (pr - pr_lo) * QW + qx;
      ga = fmaf(w, Hm[o], ga);
      gb = fmaf(w, Hm[MR * QW + o], gb);
      gc = fmaf(w, Hm[2 * MR * QW + o], gc);
    }
    int sy, sx;
    float xv = 0.f, yv = 0.f;
    if (padded_source(py, px, g.H, g.W, g.pad, g.before, g.Hp, g.Wp, sy, sx)) {
      xv = to_f32<T>(X[(int64_t)sy * a.x.pitch + sx]);
      yv = to_f32<T>(Y[(int64_t)sy * a.y.pitch + sx]);
    }
    float gy = fmaf((xv + yv) - a.tu, gb, ga) - ((xv - yv) - a.tv) * gc;
    if (a.coarse) {
      const int cy = py >> 1, cx = px >> 1;
      if (cy < a.Hc && cx < a.Wc) gy += 0.25f * a.coarse[((int64_t)frame * a.Hc + cy) * a.Wc + cx];
    }
    a.out[(int64_t)frame * a.out_bstride + (int64_t)py * a.out_pitch + px] = gy;
  }
}

// Adjoint of zero / reflect border extension: every source pixel gathers the
// padded-gradient cells that map onto it, plus the coarser-scale term.
__global__ __launch_bounds__(BLOCK) void bwd_fold_kernel(const float* gpad, int Hp, int Wp, int H, int W, int before,
                                                         int pad, float* out, int64_t out_pitch, int64_t out_bstride,
                                                         const float* coarse, int Wc, int Hc) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= H * W) return;
  const int frame = blockIdx.y;
  const int r = idx / W, c = idx - r * W;
  const float* G = gpad + (int64_t)frame * Hp * Wp;
  float acc = 0.f;
  if (pad == SSIMX_PAD_ZERO) {
    acc = G[(int64_t)(r + before) * Wp + c + before];
  } else {
    // padded index p maps to source reflect(p - before) with period 2n; the
    // preimages of source index r are p - before = r + 2nt and -r - 1 + 2nt
    // (never equal: one is even-offset, the other odd)
    const int Tr = Hp / (2 * H) + 2, Tc = Wp / (2 * W) + 2;
    for (int br = 0; br < 2; ++br) {
      const int rb = br ? -r - 1 : r;
      for (int t = -Tr; t <= Tr; ++t) {
        const int py = rb + 2 * H * t + before;
        if (py < 0 || py >= Hp) continue;
        for (int bc = 0; bc < 2; ++bc) {
          const int cbase = bc ? -c - 1 : c;
          for (int u = -Tc; u <= Tc; ++u) {
            const int px = cbase + 2 * W * u + before;
            if (px < 0 || px >= Wp) continue;
            acc += G[(int64_t)py * Wp + px];
          }
        }
      }
    }
  }
  if (coarse) {
    const int cy = r >> 1, cx = c >> 1;
    if (cy < Hc && cx < Wc) acc += 0.25f * coarse[((int64_t)frame * Hc + cy) * Wc + cx];
  }
  out[(int64_t)frame * out_bstride + (int64_t)r * out_pitch + c] = acc;
}

struct UpArgs {
  float w[MAX_SCALES];
  float inv_count[MAX_SCALES];
};

// dL/dT for the pooled term of each scale: grad * MS * w_j / val_j / N_j for
// the weighted product (zero where a clamped value is not positive), grad *
// w_j / N_j for the weighted average.  With lv (the coarsest term read as
// mean(l) * mean(cs), lv = mean(l)), the coarsest upstream is split: up holds
// that of mean(cs) (dS * mean(l)) and up2 that of mean(l) (dS * mean(cs)).
__global__ void ms_upstream_kernel(const float* vals, const float* ms, const float* gscore, UpArgs u, int M,
                                   int clamp, int sum, int batch, const float* lv, float* up, float* up2) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= batch) return;
  ms_upstream_frame(vals + (int64_t)f * M, M, lv ? lv[f] : 1.f, lv != nullptr, ms[f], gscore[f], u.w, u.inv_count,
                    clamp, sum, up + (int64_t)f * M, up2 + f);
}

// ---------------------------------------------------------------- host side
float shift_guess(const ssimx_params* p) {
  // t_u = 2 * mid-range, with the range L recovered from C2 = (0.03 L)^2.
  // Only the rounding of the combine step depends on it.
  return (float)(sqrt(p->C2) / 0.03);
}

// Pixel tiles of the fast adjoint: the tallest of 512, 256 and 128 rows
// (fewer K - 1 prologue rows per pixel) whose launch still holds >= 4096
// workgroups; smaller launches take 128 rows, halved down to 32 while they
// would hold fewer than 1024 workgroups.
void adjoint_tiles(FastArgs& fa, int W, int H, int batch) {
  fa.qtiles_x = (W + 63) / 64;
  fa.QH = 512;
  while (fa.QH > 128 && (int64_t)fa.qtiles_x * ((H + fa.QH - 1) / fa.QH) * batch < 4096) fa.QH /= 2;
  while (fa.QH > 32 && (int64_t)fa.qtiles_x * ((H + fa.QH - 1) / fa.QH) * batch < 1024) fa.QH /= 2;
  fa.qtiles_y = (H + fa.QH - 1) / fa.QH;
}

static Geom scat_geom_fit(const Geom& g, int& QW, int& QH, int& MR, int& MC, int& qtx, int& qty) {
  QW = 32;
  QH = 32;
  while (true) {
    MR = (QH + g.k - 2) / g.s + 1;
    MC = (QW + g.k - 2) / g.s + 1;
    const size_t bytes = sizeof(float) * (3 * (size_t)MR * MC + 3 * (size_t)MR * QW);
    if (bytes <= kLdsLimit || (QW == 1 && QH == 1)) break;
    if (QH >= QW && QH > 1)
      QH /= 2;
    else
      QW = std::max(1, QW / 2);
  }
  qtx = (g.Wp + QW - 1) / QW;
  qty = (g.Hp + QH - 1) / QH;
  return g;
}

struct BwdLevel {
  int dtype;
  PlaneArg x, y;
  int W, H;
};

// Coefficients + transposed filter (+ fold) for one scale.
static ssimx_status bwd_level(const ssimx_params* p, const BwdLevel& lv, int batch, int mode, const float* grad_map,
                              int64_t gm_pitch, int64_t gm_bstride, const float* gscale, int gscale_stride,
                              const float* gscale2, float gmul, float* coef, float* gpad, float* out, int64_t out_pitch,
                              int64_t out_bstride, const float* coarse, int Wc, int Hc, hipStream_t st) {
  ssimx_params pf = *p;
  pf.algo = SSIMX_ALGO_SEPARABLE;
  // statistics through the float separable path (box windows use taps 1/k)
  Geom g = make_geom_path(&pf, SSIMX_F32, lv.W, lv.H, 0);
  const bool valid = p->padding == SSIMX_PAD_VALID;
  const bool fast = use_fast(&pf, SSIMX_F32);
  const int cpitch = (g.Wo + 3) & ~3;
  const float tu = shift_guess(p), tv = 0.f;
  int err = 0;
  FastArgs fa{};
  if (fast) {
    fill_fast_common(fa, &pf, lv.dtype, lv.x, lv.y, coef_geom(&pf, lv.W, lv.H, batch));
    fa.mode = mode;
    fa.grad_map = grad_map;
    fa.gm_pitch = gm_pitch;
    fa.gm_bstride = gm_bstride;
    fa.gscale = gscale;
    fa.gscale_stride = gscale_stride;
    fa.gscale2 = gscale2;
    fa.gscale2_stride = 1;
    fa.gmul = gmul;
    fa.tu = tu;
    fa.tv = tv;
    fa.coef = coef;
    fa.cpitch = cpitch;
    fa.batch = batch;
    err = launch_fast_stats(lv.dtype, 1, fa, batch, st);
    if (err) return hip_status(err);
  } else {
    CoefArgs ca{};
    ca.x = lv.x;
    ca.y = lv.y;
    ca.g = g;
    ca.C1 = (float)p->C1;
    ca.C2 = (float)p->C2;
    ca.mode = mode;
    ca.grad_map = grad_map;
    ca.gm_pitch = gm_pitch;
    ca.gm_bstride = gm_bstride;
    ca.gscale = gscale;
    ca.gscale_stride = gscale_stride;
    ca.gscale2 = gscale2;
    ca.gscale2_stride = 1;
    ca.gmul = gmul;
    ca.tu = tu;
    ca.tv = tv;
    ca.coef = coef;
    ca.cpitch = cpitch;
    ca.batch = batch;
    gaussian_taps_f32(p->window, p->k, p->sigma, ca.taps);
    const size_t lds1 = sizeof(float) * sep_tile_lds_floats(g.IH, g.IW, g.TW);
    dim3 grid1(g.tiles_x * g.tiles_y, batch);
    switch (lv.dtype) {
      case SSIMX_U8: hipLaunchKernelGGL(bwd_coef_kernel<uint8_t>, grid1, dim3(BLOCK), lds1, st, ca); break;
      case SSIMX_U16: hipLaunchKernelGGL(bwd_coef_kernel<uint16_t>, grid1, dim3(BLOCK), lds1, st, ca); break;
      case SSIMX_F32: hipLaunchKernelGGL(bwd_coef_kernel<float>, grid1, dim3(BLOCK), lds1, st, ca); break;
      case SSIMX_BF16: hipLaunchKernelGGL(bwd_coef_kernel<bf16_t>, grid1, dim3(BLOCK), lds1, st, ca); break;
      default: return SSIMX_EDTYPE;
    }
    err = (int)hipGetLastError();
    if (err) return hip_status(err);
  }
  if (fast && valid && cpitch < kFastMaxPitch) {  // coefficient offsets: 24-bit multiplies of cpitch
    adjoint_tiles(fa, lv.W, lv.H, batch);
    fa.out = out;
    fa.out_pitch = out_pitch;
    fa.out_bstride = out_bstride;
    fa.coarse = coarse;
    fa.Wc = Wc;
    fa.Hc = Hc;
    return hip_status(launch_fast_adjoint(lv.dtype, fa, batch, st));
  }

  ScatArgs sa{};
  sa.x = lv.x;
  sa.y = lv.y;
  sa.g = g;
  sa.coef = coef;
  sa.cpitch = cpitch;
  sa.batch = batch;
  sa.tu = tu;
  sa.tv = tv;
  int qtx, qty;
  scat_geom_fit(g, sa.QW, sa.QH, sa.MR, sa.MC, qtx, qty);
  sa.qtiles_x = qtx;
  if (valid) {
    sa.out = out;
    sa.out_pitch = out_pitch;
    sa.out_bstride = out_bstride;
    sa.coarse = coarse;
    sa.Wc = Wc;
    sa.Hc = Hc;
  } else {
    sa.out = gpad;
    sa.out_pitch = g.Wp;
    sa.out_bstride = (int64_t)g.Wp * g.Hp;
  }
  gaussian_taps_f32(p->window, p->k, p->sigma, sa.taps);
  const size_t lds2 = sizeof(float) * (3 * (size_t)sa.MR * sa.MC + 3 * (size_t)sa.MR * sa.QW);
  dim3 grid2(qtx * qty, batch);
  switch (lv.dtype) {
    case SSIMX_U8: hipLaunchKernelGGL(bwd_scatter_kernel<uint8_t>, grid2, dim3(BLOCK), lds2, st, sa); break;
    case SSIMX_U16: hipLaunchKernelGGL(bwd_scatter_kernel<uint16_t>, grid2, dim3(BLOCK), lds2, st, sa); break;
    case SSIMX_F32: hipLaunchKernelGGL(bwd_scatter_kernel<float>, grid2, dim3(BLOCK), lds2, st, sa); break;
    case SSIMX_BF16: hipLaunchKernelGGL(bwd_scatter_kernel<bf16_t>, grid2, dim3(BLOCK), lds2, st, sa); break;
    default: return SSIMX_EDTYPE;
  }
  err = (int)hipGetLastError();
  if (err) return hip_status(err);
  if (!valid) {
    dim3 grid3((lv.W * lv.H + BLOCK - 1) / BLOCK, batch);
    hipLaunchKernelGGL(bwd_fold_kernel, grid3, dim3(BLOCK), 0, st, gpad, g.Hp, g.Wp, lv.H, lv.W, g.before,
                       p->padding, out, out_pitch, out_bstride, coarse, Wc, Hc);
    err = (int)hipGetLastError();
    if (err) return hip_status(err);
  }
  return SSIMX_OK;
}

static ssimx_status check_bwd(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                              float* grad, int64_t gp, int64_t gb) {
  ssimx_status s;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if ((s = check_images(ref, dis, batch)) != SSIMX_OK) return s;
  if (p->k > KMAX_GAUSS) return SSIMX_ENOTSUP;
  if (!grad || gp < ref->width || (batch > 1 && gb < gp * (int64_t)ref->height)) return SSIMX_EINVAL;
  int Wo, Ho;
  map_dims(p, ref->width, ref->height, Wo, Ho);
  if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  return SSIMX_OK;
}

struct SsimBwdLayout {
  size_t coef, gpad, total;
};

static SsimBwdLayout ssim_bwd_layout(const ssimx_params* p, int W, int H, int batch) {
  int Wo, Ho;
  map_dims(p, W, H, Wo, Ho);
  const int Wp = p->padding == SSIMX_PAD_VALID ? W : W + p->k - 1;
  const int Hp = p->padding == SSIMX_PAD_VALID ? H : H + p->k - 1;
  Ws ws;
  SsimBwdLayout L;
  L.coef = ws.take(sizeof(float) * 3 * (size_t)batch * ((Wo + 3) & ~3) * Ho);
  L.gpad = p->padding == SSIMX_PAD_VALID ? 0 : ws.take(sizeof(float) * (size_t)batch * Wp * Hp);
  L.total = ws.used;
  return L;
}

MsBwdLayout ms_bwd_layout(const ssimx_params* p, int dtype, int W, int H, int batch, int M) {
  MsBwdLayout L{};
  L.fwd = ms_layout(p, dtype, W, H, batch, M);
  Ws ws;
  ws.used = L.fwd.total;
  L.msval = ws.take(sizeof(float) * batch);
  L.up = ws.take(sizeof(float) * batch * M);
  L.up2 = ws.take(sizeof(float) * batch);
  int Wo, Ho;
  map_dims(p, W, H, Wo, Ho);
  L.coef = ws.take(sizeof(float) * 3 * (size_t)batch * ((Wo + 3) & ~3) * Ho);
  const int Wp = p->padding == SSIMX_PAD_VALID ? W : W + p->k - 1;
  const int Hp = p->padding == SSIMX_PAD_VALID ? H : H + p->k - 1;
  L.gpad = p->padding == SSIMX_PAD_VALID ? 0 : ws.take(sizeof(float) * (size_t)batch * Wp * Hp);
  for (int j = 1; j < M; ++j) L.glev[j] = ws.take(sizeof(float) * (size_t)batch * L.fwd.W[j] * L.fwd.H[j]);
  L.total = ws.used;
  return L;
}

size_t bwd_ws_bytes(const ssimx_params* p, int op, int dtype, int W, int H, int batch, int M) {
  if (op == SSIMX_OP_MSSSIM_BACKWARD) return ms_bwd_layout(p, dtype, W, H, batch, M).total;
  return ssim_bwd_layout(p, W, H, batch).total;
}

static ssimx_status ssim_bwd_entry(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                                   const float* grad_map, int64_t gm_pitch, int64_t gm_bstride,
                                   const float* grad_score, float* grad, int64_t gp, int64_t gb, void* ws,
                                   size_t ws_bytes, hipStream_t st) {
  ssimx_status s = check_bwd(p, ref, dis, batch, grad, gp, gb);
  if (s != SSIMX_OK) return s;
  int Wo, Ho;
  map_dims(p, ref->width, ref->height, Wo, Ho);
  if (grad_map && (gm_pitch < Wo || (batch > 1 && gm_bstride < gm_pitch * (int64_t)Ho))) return SSIMX_EINVAL;
  const SsimBwdLayout L = ssim_bwd_layout(p, ref->width, ref->height, batch);
  if (!ws || ws_bytes < L.total) return SSIMX_EWORKSPACE;
  BwdLevel lv{ref->dtype, PlaneArg{ref->data, ref->pitch, ref->batch_stride},
              PlaneArg{dis->data, dis->pitch, dis->batch_stride}, ref->width, ref->height};
  char* base = (char*)ws;
  return bwd_level(p, lv, batch, 0, grad_map, gm_pitch, gm_bstride, grad_score, 1, nullptr,
                   1.f / ((float)Wo * (float)Ho),
                   (float*)(base + L.coef), (float*)(base + L.gpad), grad, gp, gb, nullptr, 0, 0, st);
}

// MS-SSIM adjoint.  With fwd_score / fwd_cs (the score_out and cs_out of a
// forward call on the same inputs and flags) the forward's windowed passes are
// not repeated: only the 2x2 pyramid is rebuilt, and the per-scale values feed
// the upstream factors directly.
static ssimx_status ms_bwd_impl(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                const ssimx_image* ref, const ssimx_image* dis, int batch, const float* fwd_score,
                                const float* fwd_cs, const float* grad_score, float* grad_dis, int64_t grad_pitch,
                                int64_t grad_batch_stride, void* ws, size_t ws_bytes, hipStream_t st) {
  ssimx_status s = check_bwd(p, ref, dis, batch, grad_dis, grad_pitch, grad_batch_stride);
  if (s != SSIMX_OK) return s;
  if (!grad_score) return SSIMX_EINVAL;
  if ((s = check_ms(p, weights, n_scales, flags, ref->width, ref->height)) != SSIMX_OK) return s;
  // the split coarsest term (mean l, mean cs) is not in a forward's cs_out
  if (fwd_cs && (flags & SSIMX_MS_COARSE_SEPARATE)) return SSIMX_ENOTSUP;
  if ((s = check_path(p, ref->dtype)) != SSIMX_OK) return s;
  if ((s = check_path(p, SSIMX_F32)) != SSIMX_OK) return s;
  const MsBwdLayout L = ms_bwd_layout(p, ref->dtype, ref->width, ref->height, batch, n_scales);
  if (!ws || ws_bytes < L.total) return SSIMX_EWORKSPACE;
  char* base = (char*)ws;
  float w[MAX_SCALES];
  ms_weights(weights, n_scales, flags, w);
  const float* vals = fwd_cs;
  const float* msv = fwd_score;
  if (fwd_cs) {
    for (int j = 1; j < n_scales; ++j) {
      const PlaneArg x = j == 1 ? PlaneArg{ref->data, ref->pitch, ref->batch_stride}
                                : PlaneArg{base + L.fwd.lvl_x_off[j - 1], L.fwd.W[j - 1],
                                           (int64_t)L.fwd.W[j - 1] * L.fwd.H[j - 1]};
      const PlaneArg y = j == 1 ? PlaneArg{dis->data, dis->pitch, dis->batch_stride}
                                : PlaneArg{base + L.fwd.lvl_y_off[j - 1], L.fwd.W[j - 1],
                                           (int64_t)L.fwd.W[j - 1] * L.fwd.H[j - 1]};
      const int err = launch_downsample(j == 1 ? ref->dtype : SSIMX_F32, x, L.fwd.W[j - 1], L.fwd.H[j - 1],
                                        (float*)(base + L.fwd.lvl_x_off[j]), (float*)(base + L.fwd.lvl_y_off[j]), y,
                                        batch, st);
      if (err) return hip_status(err);
    }
  } else {
    s = ms_forward(p, w, n_scales, flags, ref, dis, batch, (float*)(base + L.msval), nullptr, ws, L.fwd, st);
    if (s != SSIMX_OK) return s;
    vals = (const float*)(base + L.fwd.vals_off);
    msv = (const float*)(base + L.msval);
  }
  return ms_bwd_levels(p, w, n_scales, flags, ref, dis, batch, vals, msv, grad_score, grad_dis, grad_pitch,
                       grad_batch_stride, base, L, st);
}

// The per-scale part of the MS-SSIM adjoint, once the workspace holds the
// pyramid levels (L.fwd) of a forward on these planes: the upstream of every
// scale's pooled term from the per-scale values `vals` [batch][M], the scores
// `msv` [batch] and dL/dscore `grad_score`, then coefficients and the
// transposed window from the coarsest scale down, each finer scale adding the
// 2x2 transpose of the coarser gradient.
ssimx_status ms_bwd_levels(const ssimx_params* p, const float* w, int n_scales, int flags, const ssimx_image* ref,
                           const ssimx_image* dis, int batch, const float* vals, const float* msv,
                           const float* grad_score, float* grad_dis, int64_t grad_pitch, int64_t grad_batch_stride,
                           char* base, const MsBwdLayout& L, hipStream_t st, bool up_ready) {
  ssimx_status s;
  UpArgs u{};
  for (int j = 0; j < n_scales; ++j) {
    int Wo, Ho;
    map_dims(p, L.fwd.W[j], L.fwd.H[j], Wo, Ho);
    u.w[j] = w[j];
    u.inv_count[j] = (float)(1.0 / ((double)Wo * Ho));
  }
  float* up = (float*)(base + L.up);
  float* up2 = (float*)(base + L.up2);
  const bool sep = (flags & SSIMX_MS_COARSE_SEPARATE) != 0;
  if (!up_ready) {
    hipLaunchKernelGGL(ms_upstream_kernel, dim3((batch + 63) / 64), dim3(64), 0, st, vals, msv, grad_score, u,
                       n_scales, (flags & SSIMX_MS_CS_CLAMP) ? 1 : 0, (flags & SSIMX_MS_SUM) ? 1 : 0, batch,
                       sep ? (const float*)(base + L.fwd.lvals_off) : nullptr, up, up2);
    const int err = (int)hipGetLastError();
    if (err) return hip_status(err);
  }
  for (int j = n_scales - 1; j >= 0; --j) {
    BwdLevel lv;
    float* out;
    int64_t op, ob;
    if (j == 0) {
      lv = BwdLevel{ref->dtype, PlaneArg{ref->data, ref->pitch, ref->batch_stride},
                    PlaneArg{dis->data, dis->pitch, dis->batch_stride}, ref->width, ref->height};
      out = grad_dis;
      op = grad_pitch;
      ob = grad_batch_stride;
    } else {
      const int64_t pl = (int64_t)L.fwd.W[j] * L.fwd.H[j];
      lv = BwdLevel{SSIMX_F32, PlaneArg{base + L.fwd.lvl_x_off[j], L.fwd.W[j], pl},
                    PlaneArg{base + L.fwd.lvl_y_off[j], L.fwd.W[j], pl}, L.fwd.W[j], L.fwd.H[j]};
      out = (float*)(base + L.glev[j]);
      op = L.fwd.W[j];
      ob = pl;
    }
    const float* coarse = j + 1 < n_scales ? (const float*)(base + L.glev[j + 1]) : nullptr;
    const int Wc = j + 1 < n_scales ? L.fwd.W[j + 1] : 0, Hc = j + 1 < n_scales ? L.fwd.H[j + 1] : 0;
    const int mode = j == n_scales - 1 ? (sep ? 3 : 0) : 1;
    s = bwd_level(p, lv, batch, mode, nullptr, 0, 0, up + j, n_scales, mode == 3 ? up2 : nullptr, 1.f,
                  (float*)(base + L.coef),
                  (float*)(base + L.gpad), out, op, ob, coarse, Wc, Hc, st);
    if (s != SSIMX_OK) return s;
  }
  return SSIMX_OK;
}

}  // namespace ssimx

using namespace ssimx;

extern "C" {

ssimx_status ssim_map_backward(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                               const float* grad_map, int64_t map_pitch, int64_t map_batch_stride, float* grad_dis,
                               int64_t grad_pitch, int64_t grad_batch_stride, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!grad_map) return SSIMX_EINVAL;
  return ssim_bwd_entry(p, ref, dis, batch, grad_map, map_pitch, map_batch_stride, nullptr, grad_dis, grad_pitch,
                        grad_batch_stride, ws, ws_bytes, (hipStream_t)stream);
}

ssimx_status ssim_pooled_backward(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                                  const float* grad_score, float* grad_dis, int64_t grad_pitch,
                                  int64_t grad_batch_stride, void* ws, size_t ws_bytes, void* stream) {
  if (!grad_score) return SSIMX_EINVAL;
  return ssim_bwd_entry(p, ref, dis, batch, nullptr, 0, 0, grad_score, grad_dis, grad_pitch, grad_batch_stride, ws,
                        ws_bytes, (hipStream_t)stream);
}

ssimx_status msssim_backward(const ssimx_params* p, const float* weights, int n_scales, int flags,
                             const ssimx_image* ref, const ssimx_image* dis, int batch, const float* grad_score,
                             float* grad_dis, int64_t grad_pitch, int64_t grad_batch_stride, void* ws,
                             size_t ws_bytes, void* stream) {
  return ms_bwd_impl(p, weights, n_scales, flags, ref, dis, batch, nullptr, nullptr, grad_score, grad_dis,
                     grad_pitch, grad_batch_stride, ws, ws_bytes, (hipStream_t)stream);
}

ssimx_status msssim_backward_values(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                    const ssimx_image* ref, const ssimx_image* dis, int batch, const float* fwd_score,
                                    const float* fwd_cs, const float* grad_score, float* grad_dis, int64_t grad_pitch,
                                    int64_t grad_batch_stride, void* ws, size_t ws_bytes, void* stream) {
  if (!fwd_score || !fwd_cs) return SSIMX_EINVAL;
  return ms_bwd_impl(p, weights, n_scales, flags, ref, dis, batch, fwd_score, fwd_cs, grad_score, grad_dis,
                     grad_pitch, grad_batch_stride, ws, ws_bytes, (hipStream_t)stream);
}

ssimx_status ssimx_workspace_size(const ssimx_params* p, int op, int dtype, int width, int height, int batch,
                                  int n_scales, size_t* bytes) {
  ssimx_status s = check_params(p);
  if (s != SSIMX_OK) return s;
  if (!bytes || width < 1 || height < 1 || batch < 1 || batch > kMaxGridY) return SSIMX_EINVAL;
  if ((int64_t)width * height > kMaxPlaneElems) return SSIMX_EINVAL;
  if (dtype < SSIMX_U8 || dtype > SSIMX_BF16) return SSIMX_EDTYPE;
  const bool ms = op == SSIMX_OP_MSSSIM || op == SSIMX_OP_MSSSIM_BACKWARD;
  if (ms && (n_scales < 1 || n_scales > MAX_SCALES)) return SSIMX_EINVAL;
  switch (op) {
    case SSIMX_OP_MAP:
    case SSIMX_OP_POOLED: *bytes = fwd_ws_bytes(p, dtype, width, height, batch); return SSIMX_OK;
    case SSIMX_OP_MSSSIM: *bytes = ms_layout(p, dtype, width, height, batch, n_scales).total; return SSIMX_OK;
    case SSIMX_OP_MAP_BACKWARD:
    case SSIMX_OP_POOLED_BACKWARD:
    case SSIMX_OP_MSSSIM_BACKWARD: *bytes = bwd_ws_bytes(p, op, dtype, width, height, batch, n_scales); return SSIMX_OK;
    default: return SSIMX_EINVAL;
  }
}

}  // extern "C"
