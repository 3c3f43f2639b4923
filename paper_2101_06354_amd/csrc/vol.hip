// SSIM-3D and MS-SSIM-3D (Spatio-Temporal SSIM subsection): SSIM whose local
// mean, variance and covariance are taken over k x k x kt rectangular
// spatio-temporal boxes, computed with rolling temporal sums so that the work
// per frame does not grow with kt.
//
// Each workgroup owns one spatial tile (64 x OH map positions, i.e. an input
// footprint of (64 + k - 1) x (OH + k - 1) pixels) and walks a run of frames.
// Every thread keeps, in registers, the temporal sums of x, y, x^2, y^2 and
// x*y over the last kt frames for the footprint pixels it owns, updated per
// frame by adding the entering frame and subtracting the one that leaves (the
// recurrence T(k) = T(k-1) - I(k - kt) + I(k)).  Per frame the sums go to LDS,
// a horizontal pass forms k-wide running sums along the rows, a vertical pass
// forms k-tall running sums down the columns, and the SSIM epilogue writes the
// map and the tile's share of the per-frame mean.
//
// 8-bit clips accumulate in uint32 (exact while k^2 kt 255^2 < 2^32); other
// dtypes accumulate in float64 (exact for integer-valued planes, such as the
// 2x2-average pyramid levels of integer clips).  The variance numerators
// N S2 - S1^2 (N = k^2 kt) are formed in float64 and are exact for 8-bit
// clips, so identical clips give Q == 1 exactly.
#include "launch.hpp"
#include "ssimx_internal.hpp"
#include "ssim_epilogue.hpp"
#include "host_common.hpp"

#include <algorithm>
#include <type_traits>

namespace ssimx {

namespace {

constexpr int kVolNT = 256;
constexpr int kVolOW = 64;   // map columns per tile
constexpr int kVolSeg = 16;  // map columns per horizontal task
constexpr int kVolKMax = 16;
constexpr int kVolKtMax = 64;
constexpr int kVolWaves = kVolNT / 64;  // pooled partials per tile and map frame

struct VolArgs {
  PlaneArg x, y;
  int W, H;          // frame size
  int Wo, Ho;        // map frame size
  int k, kt;
  int tiles_x, tiles_y;
  int n_out;         // map frames (frames - kt + 1)
  int seg_len;       // map frames per workgroup
  double N;          // k * k * kt
  float invN2;       // 1 / N^2
  float C1, C2;
  int mode;          // 0: l*cs, 1: cs
  float* map;        // nullable: [n_out][Ho][map_pitch], frame stride map_fstride
  int64_t map_pitch, map_fstride;
  float* partial;    // [n_out][tiles][waves]
};

template <typename Acc, int OH, int KCAP>
struct VolShape {
  static constexpr int IH = OH + KCAP - 1;
  static constexpr int IW = kVolOW + KCAP - 1;
  static constexpr int IWP = IW | 1;     // odd row stride of the sums
  static constexpr int HSP = kVolOW + 1; // odd row stride of the row sums
  static constexpr int T_WORDS = 5 * IH * IWP;
  static constexpr int H_WORDS = 5 * IH * HSP;
  static constexpr int PPT = (IH * IW + kVolNT - 1) / kVolNT;  // footprint pixels per thread
  static constexpr size_t LDS = sizeof(Acc) * (size_t)(T_WORDS + H_WORDS);
};

// Raw sample as loaded: the byte for 8-bit clips, float otherwise.
template <typename T, typename Acc>
using Raw = typename std::conditional<std::is_same<Acc, uint32_t>::value, uint32_t, float>::type;

// Element `off` of a frame whose base is `fb` (block-uniform).
template <typename T, typename Acc>
__device__ __forceinline__ Raw<T, Acc> vol_load(const T* fb, int64_t off) {
  const T* p = fb + off;
  if constexpr (std::is_same<Acc, uint32_t>::value)
    return (uint32_t)*p;
  else
    return to_f32<T>(*p);
}

template <typename Acc, typename R>
__device__ __forceinline__ Acc widen(R v) {
  return (Acc)v;
}

// Product of two samples in the accumulation type.  Integer sums take
// samples below 2^24 whose products stay below 2^32 (8-bit values and sums of
// four of them), so the full-rate 24-bit multiply is exact.
template <typename Acc>
__device__ __forceinline__ Acc sprod(Acc a, Acc b) {
  if constexpr (std::is_same<Acc, uint32_t>::value)
    return __umul24(a, b);
  else
    return a * b;
}

// SSIM terms from the five box sums (as float64 values, exact for 8-bit clips).
__device__ __forceinline__ float vol_value(double sx, double sy, double sxx, double syy, double sxy, double N,
                                           float invN2, float C1, float C2, int mode) {
  const double nxx = N * sxx - sx * sx;
  const double nyy = N * syy - sy * sy;
  const double nxy = N * sxy - sx * sy;
  const double d = sx - sy;
  SsimTerms t;
  t.A1 = (float)(2.0 * sx * sy) * invN2 + C1;
  t.B1 = (float)(sx * sx + sy * sy) * invN2 + C1;
  t.A2 = (float)(2.0 * nxy) * invN2 + C2;
  t.B2 = (float)(nxx + nyy) * invN2 + C2;
  t.D1 = (float)(d * d) * invN2;                  // (mu_x - mu_y)^2
  t.D2 = (float)(nxx + nyy - 2.0 * nxy) * invN2;  // variance of x - y
  return ssim_value(t, mode);
}

// KC > 0: the window size is the compile-time constant KC (loops unroll);
// KC == 0: runtime k <= KCAP.  G map rows per column task (OH = multiple of G,
// 64 * OH / G <= 256 tasks).
template <typename T, typename Acc, int OH, int G, int KC, int KCAP>
__global__ __launch_bounds__(kVolNT) void vol_kernel(VolArgs a) {
  static_assert(OH % G == 0 && kVolOW * (OH / G) <= kVolNT, "column tasks must fit the workgroup");
  using S = VolShape<Acc, OH, (KC > 0 ? KC : KCAP)>;
  using RawT = Raw<T, Acc>;
  __shared__ Acc tsum[S::T_WORDS];  // [5][IH][IWP] temporal sums of the footprint
  __shared__ Acc hsum[S::H_WORDS];  // [5][IH][HSP] k-wide row sums

  int tile, seg;
  xcd_tile(tile, seg);
  const int t0 = seg * a.seg_len;
  const int nseg = min(a.seg_len, a.n_out - t0);
  if (nseg <= 0) return;  // uniform over the workgroup
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int col0 = tx * kVolOW, row0 = ty * OH;
  const int k = KC > 0 ? KC : a.k;
  const int kt = a.kt;
  const int IW = kVolOW + k - 1, IH = OH + k - 1;
  const int npx = IW * IH;
  const int tid = threadIdx.x;

  // footprint pixels owned by this thread: p = tid + i * NT, and their
  // element offsets within a frame (fixed for the tile: a frame's loads only
  // change the block-uniform frame base)
  int pr[S::PPT], pc[S::PPT];
  bool pin[S::PPT];
  int64_t xoff[S::PPT], yoff[S::PPT];
#pragma unroll
  for (int i = 0; i < S::PPT; ++i) {
    const int p = tid + i * kVolNT;
    pr[i] = p / IW;
    pc[i] = p - pr[i] * IW;
    pin[i] = p < npx && row0 + pr[i] < a.H && col0 + pc[i] < a.W;
    xoff[i] = (int64_t)(row0 + pr[i]) * a.x.pitch + col0 + pc[i];
    yoff[i] = (int64_t)(row0 + pr[i]) * a.y.pitch + col0 + pc[i];
  }

  Acc st[S::PPT][5];
#pragma unroll
  for (int i = 0; i < S::PPT; ++i)
#pragma unroll
    for (int m = 0; m < 5; ++m) st[i][m] = (Acc)0;

  RawT nx[S::PPT], ny[S::PPT], ox[S::PPT], oy[S::PPT];
  auto fetch = [&](int f, RawT* vx, RawT* vy) {
    const T* fx = (const T*)a.x.data + (int64_t)f * a.x.bstride;
    const T* fy = (const T*)a.y.data + (int64_t)f * a.y.bstride;
#pragma unroll
    for (int i = 0; i < S::PPT; ++i) {
      vx[i] = (RawT)0;
      vy[i] = (RawT)0;
      if (pin[i]) {
        vx[i] = vol_load<T, Acc>(fx, xoff[i]);
        vy[i] = vol_load<T, Acc>(fy, yoff[i]);
      }
    }
  };

  const int f_first_out = t0 + kt - 1;
  const int f_last = t0 + nseg + kt - 2;
  fetch(t0, nx, ny);
  for (int f = t0; f <= f_last; ++f) {
    const bool drop = f - kt >= t0;  // frame f - kt leaves the box
#pragma unroll
    for (int i = 0; i < S::PPT; ++i) {
      const Acc xn = widen<Acc>(nx[i]), yn = widen<Acc>(ny[i]);
      st[i][0] += xn;
      st[i][1] += yn;
      st[i][2] += sprod(xn, xn);
      st[i][3] += sprod(yn, yn);
      st[i][4] += sprod(xn, yn);
      if (drop) {
        const Acc xo = widen<Acc>(ox[i]), yo = widen<Acc>(oy[i]);
        st[i][0] -= xo;
        st[i][1] -= yo;
        st[i][2] -= sprod(xo, xo);
        st[i][3] -= sprod(yo, yo);
        st[i][4] -= sprod(xo, yo);
      }
    }
    // prefetch the next entering and leaving frames
    if (f + 1 <= f_last) {
      fetch(f + 1, nx, ny);
      if (f + 1 - kt >= t0) fetch(f + 1 - kt, ox, oy);
    }
    if (f < f_first_out) continue;  // warm-up frames: sums only

    // temporal sums of the footprint to LDS
#pragma unroll
    for (int i = 0; i < S::PPT; ++i) {
      const int p = tid + i * kVolNT;
      if (p < npx) {
        const int l = pr[i] * S::IWP + pc[i];
#pragma unroll
        for (int m = 0; m < 5; ++m) tsum[m * IH * S::IWP + l] = st[i][m];
      }
    }
    __syncthreads();

    // k-wide running sums along the rows: task = (row, 16-column segment, moment)
    const int ntask = IH * (kVolOW / kVolSeg) * 5;
    for (int q = tid; q < ntask; q += kVolNT) {
      const int r = q % IH;
      const int rest = q / IH;
      const int sg = rest % (kVolOW / kVolSeg), m = rest / (kVolOW / kVolSeg);
      const Acc* src = tsum + (m * IH + r) * S::IWP + sg * kVolSeg;
      Acc* dst = hsum + (m * IH + r) * S::HSP + sg * kVolSeg;
      Acc s = (Acc)0;
#pragma unroll
      for (int c = 0; c < (KC > 0 ? KC : KCAP); ++c)
        if (KC > 0 || c < k) s += src[c];
      dst[0] = s;
#pragma unroll
      for (int j = 1; j < kVolSeg; ++j) {
        s += src[j + k - 1] - src[j - 1];
        dst[j] = s;
      }
    }
    __syncthreads();

    // k-tall running sums down the columns and the epilogue: task = (column, 4 rows)
    const int t = f - f_first_out + t0;  // map frame
    float part = 0.f;
    const int j = tid % kVolOW, g = __builtin_amdgcn_readfirstlane(tid / kVolOW);  // g: wave-uniform
    if (g < OH / G) {
      Acc acc[G][5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const Acc* col = hsum + (m * IH + G * g) * S::HSP + j;
        Acc s = (Acc)0;
#pragma unroll
        for (int r = 0; r < (KC > 0 ? KC : KCAP); ++r)
          if (KC > 0 || r < k) s += col[r * S::HSP];
        acc[0][m] = s;
#pragma unroll
        for (int i = 1; i < G; ++i) {
          s += col[(i + k - 1) * S::HSP] - col[(i - 1) * S::HSP];
          acc[i][m] = s;
        }
      }
      const int oj = col0 + j;
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int oi = row0 + G * g + i;
        if (oi < a.Ho && oj < a.Wo) {
          const float v = vol_value((double)acc[i][0], (double)acc[i][1], (double)acc[i][2], (double)acc[i][3],
                                    (double)acc[i][4], a.N, a.invN2, a.C1, a.C2, a.mode);
          if (a.map) {
            char* row = (char*)(a.map + (int64_t)t * a.map_fstride + (int64_t)oi * a.map_pitch);  // wave-uniform
            *(float*)(row + 4u * (uint32_t)oj) = v;
          }
          part += v;
        }
      }
    }
    // one partial per wave (no barrier); the finalize adds them in a fixed order
    const float tot = wave_sum(part);
    if ((tid & 63) == 0)
      a.partial[((int64_t)t * (a.tiles_x * a.tiles_y) + tile) * kVolWaves + (tid >> 6)] = tot;
  }
}

// Rows of map positions per tile (LDS budget): 16 for integer sums, 8 for
// float64 sums.  (15-row tiles for the 11 x 11 window, whose 500 row-sum
// tasks fill exactly two rounds of the workgroup, measured no faster.)
constexpr int kVolOHInt = 16, kVolOHF64 = 8;

int vol_tile_rows(bool int_acc, int) { return int_acc ? kVolOHInt : kVolOHF64; }

template <typename T, typename Acc>
int launch_vol_t(const VolArgs& a, int nsegs, hipStream_t st) {
  constexpr bool kInt = std::is_same<Acc, uint32_t>::value;
  constexpr int OH = kInt ? kVolOHInt : kVolOHF64;
  const dim3 grid(a.tiles_x * a.tiles_y, nsegs);
  if (a.k == 11) {
    hipLaunchKernelGGL((vol_kernel<T, Acc, OH, 4, 11, 11>), grid, dim3(kVolNT), 0, st, a);
  } else if (a.k < 11) {
    hipLaunchKernelGGL((vol_kernel<T, Acc, OH, 4, 0, 11>), grid, dim3(kVolNT), 0, st, a);
  } else {
    hipLaunchKernelGGL((vol_kernel<T, Acc, OH, 4, 0, kVolKMax>), grid, dim3(kVolNT), 0, st, a);
  }
  return (int)hipGetLastError();
}

// Geometry of a launch over a clip of `frames` frames.
struct VolGeom {
  int Wo, Ho, n_out, tiles_x, tiles_y, seg_len, nsegs;
};

// Internal plane kind of the second MS-SSIM-3D scale of 8-bit clips: uint16
// sums of 2x2 blocks (four times the 2x2 mean), accumulated in uint32.
constexpr int kVolU16Sum = 100;

bool vol_int_acc(int dtype) { return dtype == SSIMX_U8 || dtype == kVolU16Sum; }

VolGeom vol_geom(int W, int H, int frames, int k, int kt, int dtype) {
  VolGeom g{};
  g.Wo = W - k + 1;
  g.Ho = H - k + 1;
  g.n_out = frames - kt + 1;
  const int OH = vol_tile_rows(vol_int_acc(dtype), k);
  g.tiles_x = (g.Wo + kVolOW - 1) / kVolOW;
  g.tiles_y = (g.Ho + OH - 1) / OH;
  // Split the frames into runs so that the grid holds about 4096 workgroups,
  // keeping every run at least 2 kt map frames long (warm-up frames are
  // accumulated but not emitted).
  const int tiles = g.tiles_x * g.tiles_y;
  int want = (4096 + tiles - 1) / tiles;
  const int max_runs = std::max(1, g.n_out / std::max(2 * kt, 4));
  want = std::max(1, std::min(want, max_runs));
  g.seg_len = (g.n_out + want - 1) / want;
  g.nsegs = (g.n_out + g.seg_len - 1) / g.seg_len;
  return g;
}

ssimx_status check_vol(const ssimx_params* p, int kt) {
  ssimx_status s = check_params(p);
  if (s != SSIMX_OK) return s;
  if (p->window != SSIMX_WIN_BOX || p->stride != 1 || p->padding != SSIMX_PAD_VALID) return SSIMX_ENOTSUP;
  if (p->k > kVolKMax) return SSIMX_ENOTSUP;
  if (kt < 1 || kt > kVolKtMax) return SSIMX_EINVAL;
  return SSIMX_OK;
}

// cscale multiplies C1 and C2: planes holding s times the pixel values give
// the same SSIM with the constants scaled by s^2.
ssimx_status vol_pass(const ssimx_params* p, int kt, int dtype, double cscale, PlaneArg x, PlaneArg y, int W, int H,
                      int frames, int mode, float* map, int64_t map_pitch, int64_t map_fstride, float* out,
                      int64_t out_stride, float* partial, hipStream_t st) {
  const VolGeom g = vol_geom(W, H, frames, p->k, kt, dtype);
  VolArgs a{};
  a.x = x;
  a.y = y;
  a.W = W;
  a.H = H;
  a.Wo = g.Wo;
  a.Ho = g.Ho;
  a.k = p->k;
  a.kt = kt;
  a.tiles_x = g.tiles_x;
  a.tiles_y = g.tiles_y;
  a.n_out = g.n_out;
  a.seg_len = g.seg_len;
  a.N = (double)p->k * p->k * kt;
  a.invN2 = (float)(1.0 / (a.N * a.N));
  a.C1 = (float)(p->C1 * cscale);
  a.C2 = (float)(p->C2 * cscale);
  a.mode = mode;
  a.map = map;
  a.map_pitch = map_pitch;
  a.map_fstride = map_fstride;
  a.partial = partial;
  int err;
  switch (dtype) {
    case SSIMX_U8: err = launch_vol_t<uint8_t, uint32_t>(a, g.nsegs, st); break;
    case SSIMX_U16: err = launch_vol_t<uint16_t, double>(a, g.nsegs, st); break;
    case SSIMX_F32: err = launch_vol_t<float, double>(a, g.nsegs, st); break;
    case SSIMX_BF16: err = launch_vol_t<bf16_t, double>(a, g.nsegs, st); break;
    case kVolU16Sum: err = launch_vol_t<uint16_t, uint32_t>(a, g.nsegs, st); break;
    default: return SSIMX_EDTYPE;
  }
  if (err) return hip_status(err);
  if (out) {
    err = launch_finalize(partial, g.tiles_x * g.tiles_y * kVolWaves, g.n_out, g.Wo * g.Ho, 1.f, out, out_stride,
                          st);
    if (err) return hip_status(err);
  }
  return SSIMX_OK;
}

size_t vol_partial_floats(int W, int H, int frames, int k, int kt, int dtype) {
  const VolGeom g = vol_geom(W, H, frames, k, kt, dtype);
  return (size_t)g.n_out * g.tiles_x * g.tiles_y * kVolWaves;
}

size_t vol_ws_bytes(int W, int H, int frames, int k, int kt, int dtype) {
  Ws ws;
  ws.take(sizeof(float) * vol_partial_floats(W, H, frames, k, kt, dtype));
  return ws.used;
}

ssimx_status check_vol_images(const ssimx_params* p, int kt, const ssimx_image* ref, const ssimx_image* dis,
                              int frames) {
  ssimx_status s;
  if ((s = check_vol(p, kt)) != SSIMX_OK) return s;
  if ((s = check_images(ref, dis, frames)) != SSIMX_OK) return s;
  if (frames < kt || ref->width < p->k || ref->height < p->k) return SSIMX_ETOOSMALL;
  return SSIMX_OK;
}

// 2x2 block sums of 8-bit planes as uint16 (exact): four times the 2x2 mean.
__global__ __launch_bounds__(BLOCK) void sum4_kernel(PlaneArg xa, PlaneArg ya, int W2, int H2, uint16_t* ox,
                                                     uint16_t* oy) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= W2 * H2) return;
  const int frame = blockIdx.y;
  const int r = idx / W2, c = idx - r * W2;
  const uint8_t* px = (const uint8_t*)xa.data + (int64_t)frame * xa.bstride + (int64_t)(2 * r) * xa.pitch + 2 * c;
  const uint8_t* py = (const uint8_t*)ya.data + (int64_t)frame * ya.bstride + (int64_t)(2 * r) * ya.pitch + 2 * c;
  const int64_t o = (int64_t)frame * W2 * H2 + idx;
  ox[o] = (uint16_t)(px[0] + px[1] + px[xa.pitch] + px[xa.pitch + 1]);
  oy[o] = (uint16_t)(py[0] + py[1] + py[ya.pitch] + py[ya.pitch + 1]);
}

struct Ms3Layout {
  int W[MAX_SCALES], H[MAX_SCALES];
  int dt[MAX_SCALES];         // plane kind of each scale
  double cscale[MAX_SCALES];  // C1, C2 multiplier of each scale
  size_t lvl_x[MAX_SCALES], lvl_y[MAX_SCALES];
  size_t partial, vals, lvals, total;
};

// For 8-bit clips the second scale is kept as exact uint16 2x2 sums (4x the
// means) and accumulated in uint32 while k^2 kt 1020^2 < 2^32; the coarser
// scales are float 2x2 means of it (still 4x the pixel values), so their
// constants are scaled by 16.  Everything else uses float 2x2 means.
Ms3Layout ms3_layout(const ssimx_params* p, int kt, int dtype, int W, int H, int frames, int M) {
  Ms3Layout L{};
  scale_dims(W, H, M, L.W, L.H);
  const bool sum16 = dtype == SSIMX_U8 && M > 1 && (double)p->k * p->k * kt * 1020.0 * 1020.0 < 4294967296.0;
  Ws ws;
  size_t np = 0;
  for (int j = 0; j < M; ++j) {
    L.dt[j] = j == 0 ? dtype : (j == 1 && sum16) ? kVolU16Sum : SSIMX_F32;
    L.cscale[j] = (sum16 && j > 0) ? 16.0 : 1.0;
    if (j > 0) {
      const size_t es = L.dt[j] == kVolU16Sum ? sizeof(uint16_t) : sizeof(float);
      L.lvl_x[j] = ws.take(es * (size_t)frames * L.W[j] * L.H[j]);
      L.lvl_y[j] = ws.take(es * (size_t)frames * L.W[j] * L.H[j]);
    }
    np = std::max(np, vol_partial_floats(L.W[j], L.H[j], frames, p->k, kt, L.dt[j]));
  }
  L.partial = ws.take(sizeof(float) * np);
  L.vals = ws.take(sizeof(float) * (size_t)(frames - kt + 1) * M);
  L.lvals = ws.take(sizeof(float) * (size_t)(frames - kt + 1));
  L.total = ws.used;
  return L;
}

}  // namespace

}  // namespace ssimx

using namespace ssimx;

extern "C" {

ssimx_status ssimx_ssim3d_workspace_size(const ssimx_params* p, int kt, int dtype, int width, int height, int frames,
                                         size_t* bytes) {
  ssimx_status s;
  if ((s = check_vol(p, kt)) != SSIMX_OK) return s;
  if (!bytes || frames > kMaxGridY) return SSIMX_EINVAL;
  if (dtype < SSIMX_U8 || dtype > SSIMX_BF16) return SSIMX_EDTYPE;
  if (frames < kt || width < p->k || height < p->k) return SSIMX_ETOOSMALL;
  *bytes = vol_ws_bytes(width, height, frames, p->k, kt, dtype);
  return SSIMX_OK;
}

ssimx_status ssimx_ssim3d(const ssimx_params* p, int kt, const ssimx_image* ref, const ssimx_image* dis, int frames,
                          float* map_out, long long map_pitch, long long map_frame_stride, float* score_out,
                          void* ws, size_t ws_bytes, void* stream) {
  ssimx_status s;
  if ((s = check_vol_images(p, kt, ref, dis, frames)) != SSIMX_OK) return s;
  if (!map_out && !score_out) return SSIMX_EINVAL;
  const int Wo = ref->width - p->k + 1, Ho = ref->height - p->k + 1, n_out = frames - kt + 1;
  if (map_out && (map_pitch < Wo || (n_out > 1 && map_frame_stride < map_pitch * (long long)Ho)))
    return SSIMX_EINVAL;
  const size_t need = vol_ws_bytes(ref->width, ref->height, frames, p->k, kt, ref->dtype);
  if (!ws || ws_bytes < need) return SSIMX_EWORKSPACE;
  PlaneArg x{ref->data, ref->pitch, ref->batch_stride}, y{dis->data, dis->pitch, dis->batch_stride};
  return vol_pass(p, kt, ref->dtype, 1.0, x, y, ref->width, ref->height, frames, 0, map_out, map_pitch, map_frame_stride,
                  score_out, 1, (float*)ws, (hipStream_t)stream);
}

ssimx_status ssimx_msssim3d_workspace_size(const ssimx_params* p, int kt, int n_scales, int dtype, int width,
                                           int height, int frames, size_t* bytes) {
  ssimx_status s;
  if ((s = check_vol(p, kt)) != SSIMX_OK) return s;
  if (!bytes || n_scales < 1 || n_scales > MAX_SCALES || frames > kMaxGridY) return SSIMX_EINVAL;
  if (dtype < SSIMX_U8 || dtype > SSIMX_BF16) return SSIMX_EDTYPE;
  if (frames < kt || width < 1 || height < 1) return SSIMX_ETOOSMALL;
  int Wj[MAX_SCALES], Hj[MAX_SCALES];
  scale_dims(width, height, n_scales, Wj, Hj);
  for (int j = 0; j < n_scales; ++j)
    if (Wj[j] < p->k || Hj[j] < p->k) return SSIMX_ETOOSMALL;
  *bytes = ms3_layout(p, kt, dtype, width, height, frames, n_scales).total;
  return SSIMX_OK;
}

ssimx_status ssimx_msssim3d(const ssimx_params* p, int kt, const float* weights, int n_scales, int flags,
                            const ssimx_image* ref, const ssimx_image* dis, int frames, float* score_out,
                            float* cs_out, void* ws, size_t ws_bytes, void* stream) {
  ssimx_status s;
  if ((s = check_vol_images(p, kt, ref, dis, frames)) != SSIMX_OK) return s;
  if (!score_out) return SSIMX_EINVAL;
  if ((s = check_ms(p, weights, n_scales, flags, ref->width, ref->height)) != SSIMX_OK) return s;
  const Ms3Layout L = ms3_layout(p, kt, ref->dtype, ref->width, ref->height, frames, n_scales);
  if (!ws || ws_bytes < L.total) return SSIMX_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  float w[MAX_SCALES];
  ms_weights(weights, n_scales, flags, w);
  float* vals = (float*)(base + L.vals);
  for (int j = 0; j < n_scales; ++j) {
    PlaneArg x, y;
    const int dt = L.dt[j];
    if (j == 0) {
      x = PlaneArg{ref->data, ref->pitch, ref->batch_stride};
      y = PlaneArg{dis->data, dis->pitch, dis->batch_stride};
    } else {
      x = PlaneArg{base + L.lvl_x[j], L.W[j], (int64_t)L.W[j] * L.H[j]};
      y = PlaneArg{base + L.lvl_y[j], L.W[j], (int64_t)L.W[j] * L.H[j]};
    }
    if (j + 1 < n_scales) {
      int err;
      if (L.dt[j + 1] == kVolU16Sum) {
        const int W2 = L.W[j + 1], H2 = L.H[j + 1];
        hipLaunchKernelGGL(sum4_kernel, dim3((W2 * H2 + BLOCK - 1) / BLOCK, frames), dim3(BLOCK), 0, st, x, y, W2,
                           H2, (uint16_t*)(base + L.lvl_x[j + 1]), (uint16_t*)(base + L.lvl_y[j + 1]));
        err = (int)hipGetLastError();
      } else {
        err = launch_downsample(dt == kVolU16Sum ? SSIMX_U16 : dt, x, L.W[j], L.H[j],
                                (float*)(base + L.lvl_x[j + 1]), (float*)(base + L.lvl_y[j + 1]), y, frames, st);
      }
      if (err) return hip_status(err);
    }
    const bool sep = j + 1 == n_scales && (flags & SSIMX_MS_COARSE_SEPARATE);
    s = vol_pass(p, kt, dt, L.cscale[j], x, y, L.W[j], L.H[j], frames, (j + 1 < n_scales || sep) ? 1 : 0, nullptr, 0,
                 0, vals + j, n_scales, (float*)(base + L.partial), st);
    if (s != SSIMX_OK) return s;
    if (sep) {  // coarsest term mean(l) * mean(cs): the mean of l as well
      s = vol_pass(p, kt, dt, L.cscale[j], x, y, L.W[j], L.H[j], frames, 3, nullptr, 0, 0,
                   (float*)(base + L.lvals), 1, (float*)(base + L.partial), st);
      if (s != SSIMX_OK) return s;
    }
  }
  const int err = launch_ms_combine(vals, n_scales, frames - kt + 1, w, flags, score_out, cs_out,
                                    (flags & SSIMX_MS_COARSE_SEPARATE) ? (const float*)(base + L.lvals) : nullptr, st);
  return err ? hip_status(err) : SSIMX_OK;
}

}  // extern "C"
