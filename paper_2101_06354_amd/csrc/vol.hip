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
// recurrence T(k) = T(k-1) - I(k - kt) + I(k)).  Per frame the sums go to one
// LDS array, a column pass turns each column into k-tall running sums in
// place (one thread per column and moment), and a row pass forms the k-wide
// running sums of 4 adjacent outputs from 16-byte aligned row reads and runs
// the SSIM epilogue (map and the tile's share of the per-frame mean).  One
// array instead of separate input and partial-sum arrays halves the LDS of a
// workgroup, so twice as many workgroups share a CU.  Footprint pixels
// outside the frame hold arbitrary (loaded) values: they only enter windows
// of positions outside the map, which are neither written nor pooled, and
// every running sum reaches them only after the last in-map position of its
// row or column.
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
constexpr int kVolKMax = 16;
constexpr int kVolKtMax = 64;
constexpr int kVolWaves = kVolNT / 64;  // pooled partials per tile and map frame
constexpr int64_t kVolMaxPitch = int64_t(1) << 26;  // elements per row

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
  static constexpr int IWP = (IW + 3) & ~3;  // row stride of the sums: 16-byte aligned rows
  static constexpr int T_WORDS = 5 * IH * IWP;
  static constexpr int PPT = (IH * IW + kVolNT - 1) / kVolNT;  // footprint pixels per thread
};

// Raw sample as loaded: the byte for 8-bit clips, float otherwise.
template <typename T, typename Acc>
using Raw = typename std::conditional<std::is_same<Acc, uint32_t>::value, uint32_t, float>::type;

// Element `off` of a frame whose base is `fb` (block-uniform).
template <typename T, typename Acc>
__device__ __forceinline__ Raw<T, Acc> vol_load(const T* fb, uint32_t off) {
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

// Entering or leaving samples of a thread's footprint pixels, one register
// per sample (combining them at load time would make each load wait).
template <typename Acc, int PPT>
struct VolSamples {
  using R = Raw<void, Acc>;
  R xs[PPT], ys[PPT];
  __device__ __forceinline__ void set(int i, R x, R y) {
    xs[i] = x;
    ys[i] = y;
  }
  __device__ __forceinline__ Acc x(int i) const { return (Acc)xs[i]; }
  __device__ __forceinline__ Acc y(int i) const { return (Acc)ys[i]; }
};

typedef unsigned short vol_us2 __attribute__((ext_vector_type(2)));
// Temporal sums of one footprint pixel: sum x, sum y, sum x^2, sum y^2,
// sum x y over the frames in the box.  Integer sums keep sum x and sum y as
// one pair of 16-bit halves (at most 64 frames of samples below 1021 stay
// below 2^16), updated by one packed 16-bit add per frame.
template <typename Acc>
struct VolSums {
  Acc v[5];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int m = 0; m < 5; ++m) v[m] = (Acc)0;
  }
  template <class Sm>
  __device__ __forceinline__ void add(const Sm& sm, int i) {
    const Acc x = sm.x(i), y = sm.y(i);
    v[0] += x;
    v[1] += y;
    v[2] += x * x;
    v[3] += y * y;
    v[4] += x * y;
  }
  template <class Sm>
  __device__ __forceinline__ void sub(const Sm& sm, int i) {
    const Acc x = sm.x(i), y = sm.y(i);
    v[0] -= x;
    v[1] -= y;
    v[2] -= x * x;
    v[3] -= y * y;
    v[4] -= x * y;
  }
  __device__ __forceinline__ Acc get(int m) const { return v[m]; }
};
template <>
struct VolSums<uint32_t> {
  vol_us2 s01;
  uint32_t s2, s3, s4;
  __device__ __forceinline__ void zero() {
    s01 = vol_us2{0, 0};
    s2 = s3 = s4 = 0u;
  }
  // integer samples are below 2^16, so the 24-bit multiplies are exact
  __device__ __forceinline__ void add(uint32_t x, uint32_t y) {
    s01 += vol_us2{(unsigned short)x, (unsigned short)y};
    s2 += __umul24(x, x);
    s3 += __umul24(y, y);
    s4 += __umul24(x, y);
  }
  __device__ __forceinline__ void sub(uint32_t x, uint32_t y) {
    s01 -= vol_us2{(unsigned short)x, (unsigned short)y};
    s2 -= __umul24(x, x);
    s3 -= __umul24(y, y);
    s4 -= __umul24(x, y);
  }
  template <class Sm>
  __device__ __forceinline__ void add(const Sm& sm, int i) {
    add(sm.x(i), sm.y(i));
  }
  template <class Sm>
  __device__ __forceinline__ void sub(const Sm& sm, int i) {
    sub(sm.x(i), sm.y(i));
  }
  __device__ __forceinline__ uint32_t get(int m) const {
    return m == 0 ? (uint32_t)s01.x : m == 1 ? (uint32_t)s01.y : m == 2 ? s2 : m == 3 ? s3 : s4;
  }
};

// SSIM terms from the five box sums (as float64 values, exact for 8-bit clips).
__device__ __forceinline__ float vol_value(double sx, double sy, double sxx, double syy, double sxy, double N,
                                           float invN2, float C1, float C2, int mode) {
  // With P = sx sy and Q = sx^2 + sy^2: N^2 (mu_x^2 + mu_y^2) = Q,
  // N^2 (sigma_x^2 + sigma_y^2) = N (sxx + syy) - Q, N^2 sigma_xy = N sxy - P,
  // N^2 (mu_x - mu_y)^2 = Q - 2 P and N^2 var(x - y) = the variance sum - 2
  // N^2 sigma_xy.  Exact for integer sums; for x == y both differences are 0.
  const double P = sx * sy;
  const double Q = fma(sx, sx, sy * sy);
  const double nxy = fma(N, sxy, -P);
  const double n2 = fma(N, sxx + syy, -Q);
  SsimTerms t;
  t.A1 = (float)(2.0 * P) * invN2 + C1;
  t.B1 = (float)Q * invN2 + C1;
  t.A2 = (float)(2.0 * nxy) * invN2 + C2;
  t.B2 = (float)n2 * invN2 + C2;
  t.D1 = (float)fma(-2.0, P, Q) * invN2;    // (mu_x - mu_y)^2
  t.D2 = (float)fma(-2.0, nxy, n2) * invN2;  // variance of x - y
  return ssim_value(t, mode);
}

// The footprint pixels a thread owns, their temporal sums and the samples
// of the entering and leaving frames.  Pixel path: pixels p = tid + i NT of
// the row-major footprint, each loaded on its own.  Per pixel its element
// offset from the tile origin within an x frame (32-bit: the host keeps row
// pitches below 2^26), 0 outside the frame, and its LDS slot or -1 past the
// footprint; the y offset is the same for equal pitches, else it is derived
// from the slot.  Pixels outside the frame load the tile origin (always
// inside), so that no load sits behind a branch.
template <typename T, typename Acc, class S>
struct VolPixels {
  uint32_t xo[S::PPT];
  int li[S::PPT];
  VolSums<Acc> st[S::PPT];
  VolSamples<Acc, S::PPT> en, lv;

  __device__ __forceinline__ void init(const VolArgs& a, int tid, int row0, int col0, int IW, int IH) {
#pragma unroll
    for (int i = 0; i < S::PPT; ++i) {
      const int p = tid + i * kVolNT;
      const int pr = p / IW, pc = p - pr * IW;
      const bool in = p < IW * IH && row0 + pr < a.H && col0 + pc < a.W;
      li[i] = p < IW * IH ? pr * S::IWP + pc : -1;
      xo[i] = in ? (uint32_t)(pr * (int)a.x.pitch + pc) : 0u;
      st[i].zero();
    }
  }
  // fx, fy: the frame's tile origin (block-uniform)
  __device__ __forceinline__ void fetch(const T* fx, const T* fy, int dpitch, VolSamples<Acc, S::PPT>& v) {
    if (dpitch == 0) {
#pragma unroll
      for (int i = 0; i < S::PPT; ++i) v.set(i, vol_load<T, Acc>(fx, xo[i]), vol_load<T, Acc>(fy, xo[i]));
    } else {
#pragma unroll
      for (int i = 0; i < S::PPT; ++i) {
        const uint32_t oy = xo[i] ? xo[i] + (uint32_t)((li[i] / S::IWP) * dpitch) : 0u;
        v.set(i, vol_load<T, Acc>(fx, xo[i]), vol_load<T, Acc>(fy, oy));
      }
    }
  }
  __device__ __forceinline__ void update(bool drop) {
#pragma unroll
    for (int i = 0; i < S::PPT; ++i) {
      st[i].add(en, i);
      if (drop) st[i].sub(lv, i);
    }
  }
  __device__ __forceinline__ void store(Acc* tsum, int IH) const {
#pragma unroll
    for (int i = 0; i < S::PPT; ++i)
      if (li[i] >= 0) {
#pragma unroll
        for (int m = 0; m < 5; ++m) tsum[m * IH * S::IWP + li[i]] = st[i].get(m);
      }
  }
};

// Quad path (integer clips, 8-bit or the 16-bit 2x2 sums, whose rows hold
// whole quads: base, row and frame strides aligned to 4 elements, width a
// multiple of 4): a thread owns quads of 4 adjacent footprint pixels,
// q = tid + i NT over rows of IWP / 4 quads, so a frame costs one 4- or
// 8-byte load per quad and plane and each moment of a quad goes to LDS as one
// 16-byte store.  A quad lies wholly inside or outside the frame; outside
// quads load the tile origin.  The columns of the last quad of a row past
// the footprint land in the row's padding.
template <typename T, class S>
struct VolQuads {
  static constexpr int IWQ = S::IWP / 4;
  static constexpr int QPT = (S::IH * IWQ + kVolNT - 1) / kVolNT;
  using Q = typename std::conditional<sizeof(T) == 1, uint32_t, uint2>::type;  // 4 samples
  uint32_t xo[QPT], yo[QPT];
  int li[QPT];
  VolSums<uint32_t> st[QPT][4];
  Q enx[QPT], eny[QPT], lvx[QPT], lvy[QPT];

  static __device__ __forceinline__ uint32_t sample(const Q& q, int j) {
    if constexpr (sizeof(T) == 1)
      return (q >> (8 * j)) & 0xffu;
    else
      return ((j < 2 ? q.x : q.y) >> (16 * (j & 1))) & 0xffffu;
  }
  __device__ __forceinline__ void init(const VolArgs& a, int tid, int row0, int col0, int IW, int IH) {
    const int nq = (IW + 3) >> 2;
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      const int q = tid + i * kVolNT;
      const int pr = q / nq, qc = q - pr * nq;
      const bool slot = q < nq * IH;
      const bool in = slot && row0 + pr < a.H && col0 + 4 * qc < a.W;
      li[i] = slot ? pr * S::IWP + 4 * qc : -1;
      xo[i] = in ? (uint32_t)(pr * (int)a.x.pitch + 4 * qc) : 0u;
      yo[i] = in ? (uint32_t)(pr * (int)a.y.pitch + 4 * qc) : 0u;
#pragma unroll
      for (int j = 0; j < 4; ++j) st[i][j].zero();
    }
  }
  __device__ __forceinline__ void fetch(const T* fx, const T* fy, Q* vx, Q* vy) const {
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      vx[i] = *(const Q*)(fx + xo[i]);
      vy[i] = *(const Q*)(fy + yo[i]);
    }
  }
  __device__ __forceinline__ void update(bool drop) {
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        st[i][j].add(sample(enx[i], j), sample(eny[i], j));
        if (drop) st[i][j].sub(sample(lvx[i], j), sample(lvy[i], j));
      }
  }
  __device__ __forceinline__ void store(uint32_t* tsum, int IH) const {
#pragma unroll
    for (int i = 0; i < QPT; ++i)
      if (li[i] >= 0) {
#pragma unroll
        for (int m = 0; m < 5; ++m)
          *(uint4*)&tsum[m * IH * S::IWP + li[i]] =
              make_uint4(st[i][0].get(m), st[i][1].get(m), st[i][2].get(m), st[i][3].get(m));
      }
  }
};

// KC > 0: the window size is the compile-time constant KC (loops unroll and
// the column pass keeps the last KC sums of its column in registers);
// KC == 0: runtime k <= KCAP (the column pass leaves prefix sums and the row
// pass takes their differences).
template <typename T, typename Acc, int OH, int KC, int KCAP, bool QUAD>
__global__ __launch_bounds__(kVolNT, (QUAD && KC > 0) ? 4 : 2) void vol_kernel(VolArgs a) {
  static_assert(OH * (kVolOW / 4) <= kVolNT && OH % 4 == 0, "one row task per thread, 4 rows per wave");
  static_assert(!QUAD || std::is_same<Acc, uint32_t>::value, "quads: integer sums");
  using S = VolShape<Acc, OH, (KC > 0 ? KC : KCAP)>;
  __shared__ __align__(16) Acc tsum[S::T_WORDS];  // [5][IH][IWP] temporal sums, then their column sums

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
  const int tid = threadIdx.x;

  using Own = typename std::conditional<QUAD, VolQuads<T, S>, VolPixels<T, Acc, S>>::type;
  Own own;
  own.init(a, tid, row0, col0, IW, IH);
  const int dpitch = (int)(a.y.pitch - a.x.pitch);  // block-uniform
  const int64_t xorg = (int64_t)row0 * a.x.pitch + col0, yorg = (int64_t)row0 * a.y.pitch + col0;
  auto fetch = [&](int f, bool entering) {
    const T* fx = (const T*)a.x.data + (f * a.x.bstride + xorg);
    const T* fy = (const T*)a.y.data + (f * a.y.bstride + yorg);
    if constexpr (QUAD) {
      if (entering)
        own.fetch(fx, fy, own.enx, own.eny);
      else
        own.fetch(fx, fy, own.lvx, own.lvy);
    } else {
      own.fetch(fx, fy, dpitch, entering ? own.en : own.lv);
    }
  };

  const int f_first_out = t0 + kt - 1;
  const int f_last = t0 + nseg + kt - 2;
  fetch(t0, true);
  for (int f = t0; f <= f_last; ++f) {
    own.update(f - kt >= t0);  // frame f enters, frame f - kt leaves the box
    // prefetch the next entering and leaving frames
    if (f + 1 <= f_last) {
      fetch(f + 1, true);
      if (f + 1 - kt >= t0) fetch(f + 1 - kt, false);
    }
    if (f < f_first_out) continue;  // warm-up frames: sums only

    // temporal sums of the footprint to LDS, once the previous map frame's
    // row pass has read the array
    if (f > f_first_out) __syncthreads();
    own.store(tsum, IH);
    __syncthreads();

    // k-tall sums down the columns, in place: task = (moment, column), one
    // thread walking the column (output row i lands in row i after the sums
    // it needs have been read)
    for (int q = tid; q < 5 * IW; q += kVolNT) {
      const int m = q / IW, c = q - m * IW;
      Acc* col = tsum + m * IH * S::IWP + c;
      if constexpr (KC > 0) {
        Acc ring[KC];  // the sums of rows i - 1 .. i + KC - 2, slot r % KC
        Acc s = (Acc)0;
#pragma unroll
        for (int r = 0; r < KC; ++r) {
          ring[r] = col[r * S::IWP];
          s += ring[r];
        }
        col[0] = s;
#pragma unroll
        for (int i = 1; i < OH; ++i) {
          const Acc nv = col[(i + KC - 1) * S::IWP];
          s += nv - ring[(i - 1) % KC];
          ring[(i - 1) % KC] = nv;
          col[i * S::IWP] = s;
        }
      } else {
        Acc s = (Acc)0;  // inclusive prefix sums; the row pass differences them
        for (int r = 0; r < IH; ++r) {
          s += col[r * S::IWP];
          col[r * S::IWP] = s;
        }
      }
    }
    __syncthreads();

    // k-wide running sums along the rows and the epilogue: task = (map row,
    // 4 adjacent columns); wave w takes rows 4 w .. 4 w + 3
    const int t = f - f_first_out + t0;  // map frame
    float part = 0.f;
    const int i = tid >> 4, j0 = 4 * (tid & 15);
    if (i < OH) {
      const Acc* rows = tsum + i * S::IWP + j0;
      // column sum (rows i .. i + k - 1) of moment m at column j0 + c
      auto cs = [&](int m, int c) -> Acc {
        const Acc* r = rows + m * IH * S::IWP + c;
        if constexpr (KC > 0) {
          return r[0];
        } else {
          Acc v = r[(k - 1) * S::IWP];
          if (i > 0) v -= r[-S::IWP];
          return v;
        }
      };
      // the window sums of the 4 outputs one at a time, so that only one
      // output's five sums are live through the epilogue
      Acc acc[5];
      // KC > 0: the KC + 3 column sums of each moment, read as 16-byte
      // vectors (row starts and j0 are multiples of 4 elements)
      constexpr int NV = KC > 0 ? (KC + 3 + 3) / 4 * 4 : 1;
      static_assert(KC == 0 || NV <= S::IWP - (kVolOW - 4), "vector reads stay inside the row");
      Acc cv[5][NV];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        acc[m] = (Acc)0;
        if constexpr (KC > 0) {
          const Acc* r = rows + m * IH * S::IWP;
#pragma unroll
          for (int c = 0; c < NV; c += 16 / (int)sizeof(Acc)) {
            if constexpr (sizeof(Acc) == 4) {
              const uint4 q = *(const uint4*)(r + c);
              cv[m][c] = q.x;
              cv[m][c + 1] = q.y;
              cv[m][c + 2] = q.z;
              cv[m][c + 3] = q.w;
            } else {
              const double2 q = *(const double2*)(r + c);
              cv[m][c] = q.x;
              cv[m][c + 1] = q.y;
            }
          }
#pragma unroll
          for (int c = 0; c < KC; ++c) acc[m] += cv[m][c];
        } else {
#pragma unroll 1
          for (int c = 0; c < k; ++c) acc[m] += cs(m, c);
        }
      }
      const int oi = row0 + i;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u > 0) {
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            if constexpr (KC > 0)
              acc[m] += cv[m][u + KC - 1] - cv[m][u - 1];
            else
              acc[m] += cs(m, u + k - 1) - cs(m, u - 1);
          }
        }
        const int oj = col0 + j0 + u;
        if (oi < a.Ho && oj < a.Wo) {
          const float v = vol_value((double)acc[0], (double)acc[1], (double)acc[2], (double)acc[3],
                                    (double)acc[4], a.N, a.invN2, a.C1, a.C2, a.mode);
          if (a.map) {
            char* row = (char*)(a.map + (int64_t)t * a.map_fstride + (int64_t)oi * a.map_pitch);
            *(float*)(row + 4u * (uint32_t)oj) = v;
          }
          part += v;
        }
      }
    }
    // one partial per wave; the finalize adds them in a fixed order
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

template <typename T, typename Acc, bool QUAD>
void launch_vol_q(const VolArgs& a, dim3 grid, hipStream_t st) {
  constexpr int OH = std::is_same<Acc, uint32_t>::value ? kVolOHInt : kVolOHF64;
  if (a.k == 11)
    hipLaunchKernelGGL((vol_kernel<T, Acc, OH, 11, 11, QUAD>), grid, dim3(kVolNT), 0, st, a);
  else if (a.k < 11)
    hipLaunchKernelGGL((vol_kernel<T, Acc, OH, 0, 11, QUAD>), grid, dim3(kVolNT), 0, st, a);
  else
    hipLaunchKernelGGL((vol_kernel<T, Acc, OH, 0, kVolKMax, QUAD>), grid, dim3(kVolNT), 0, st, a);
}

// Integer clips whose rows are whole quads take the quad loads.
bool vol_quads_ok(const VolArgs& a, int esize) {
  for (const PlaneArg* pl : {&a.x, &a.y})
    if (((uintptr_t)pl->data & (4 * esize - 1)) || (pl->pitch & 3) || (pl->bstride & 3)) return false;
  return (a.W & 3) == 0;
}

template <typename T, typename Acc>
int launch_vol_t(const VolArgs& a, int nsegs, hipStream_t st) {
  const dim3 grid(a.tiles_x * a.tiles_y, nsegs);
  if constexpr (std::is_same<Acc, uint32_t>::value) {
    if (vol_quads_ok(a, (int)sizeof(T))) {
      launch_vol_q<T, Acc, true>(a, grid, st);
      return (int)hipGetLastError();
    }
  }
  launch_vol_q<T, Acc, false>(a, grid, st);
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
  // the kernel forms in-frame offsets in 32 bits (at most 31 rows of a tile)
  if (ref->pitch > kVolMaxPitch || dis->pitch > kVolMaxPitch) return SSIMX_EINVAL;
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
