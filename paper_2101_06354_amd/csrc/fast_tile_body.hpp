// Tile bodies of the stride-1, compile-time-K band kernels (shared by the
// per-frame kernels and the persistent ragged-batch kernel).
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
// Kernels:
//   fast_stats_kernel<K, T, EPI>  EPI = 0: SSIM / cs map + pooled partials
//                                 EPI = 1: the four adjoint coefficient maps
//   fast_adjoint_kernel<K, T>     transposed window over the coefficient
//                                 maps and the per-pixel combine (valid
//                                 borders), optionally adding the 2x2
//                                 transpose of a coarser-scale gradient.
#pragma once

#include <type_traits>

#include "fast_tile.hpp"
#include "ssim_epilogue.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {
namespace fast {


constexpr int kTW = 64;   // map columns per tile
constexpr int kTWP = 68;  // LDS row stride of the adjoint's coefficient band (4 floats of padding keep
                          // rows and planes off a common bank)
constexpr int kCH = 16;   // output rows per chunk
constexpr int kNT = 256;  // threads per block

template <int K>
struct Shape {
  static constexpr int HALO = K - 1;
  static constexpr int NREAD = (K + 3 + 3) / 4;        // float4 reads per row-pass item
  static constexpr int IWP = kTW - 4 + 4 * NREAD;      // LDS row length of the footprint
  static constexpr int NQ = IWP / 4;                   // float4 quads per footprint row
  static constexpr int BAND = kCH + HALO;              // rows of the row-statistics band
  static constexpr int RS = 4 * (kTW + kTW / 8);       // floats per band row: a float4 per map column,
                                                       // one float4 of padding after every 8 columns
  static constexpr int BANDF = BAND * RS;              // floats of the band
  static constexpr int SHIFT = K / 2 + 1;              // centring offset of an item
  static_assert(IWP >= kTW + K - 1, "footprint row too short");
  static_assert(kCH >= HALO, "band copy needs CH >= K - 1");
  static_assert(SHIFT - 3 >= 0 && SHIFT < K, "shared centring value must lie in all 4 windows");
};

// Raw footprint quad held in registers between the global load and the LDS
// store (4 elements in the plane's own packing), so that the load latency of
// the next chunk overlaps the column pass.  Border elements are gathered one
// by one (zero outside the padded plane) and packed the same way.
template <typename T>
struct Quad {
  static constexpr int NW = sizeof(T);  // 32-bit words for 4 elements
  uint32_t w[NW];
};

template <typename T>
__device__ __forceinline__ uint32_t elem_bits(T v) {
  if constexpr (sizeof(T) == 4) {
    uint32_t b;
    __builtin_memcpy(&b, &v, 4);
    return b;
  } else if constexpr (sizeof(T) == 2) {
    uint16_t b;
    __builtin_memcpy(&b, &v, 2);
    return (uint32_t)b;
  } else {
    uint8_t b;
    __builtin_memcpy(&b, &v, 1);
    return (uint32_t)b;
  }
}

template <typename T>
__device__ __forceinline__ void fetch4(const T* P, int64_t pitch, const Geom& g, int vec_ok, int py, int px,
                                       Quad<T>& q) {
  if (vec_ok && g.pad == SSIMX_PAD_VALID && py < g.H && px + 3 < g.W) {
    const T* s = P + (int64_t)py * pitch + px;
    if constexpr (sizeof(T) == 1) {
      q.w[0] = *(const uint32_t*)s;
    } else if constexpr (sizeof(T) == 2) {
      const uint2 v = *(const uint2*)s;
      q.w[0] = v.x;
      q.w[1] = v.y;
    } else {
      const uint4 v = *(const uint4*)s;
      q.w[0] = v.x;
      q.w[1] = v.y;
      q.w[2] = v.z;
      q.w[3] = v.w;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < Quad<T>::NW; ++i) q.w[i] = 0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int sy, sx;
    const uint32_t e =
        padded_source(py, px + i, g.H, g.W, g.pad, g.before, g.Hp, g.Wp, sy, sx) ? elem_bits<T>(P[(int64_t)sy * pitch + sx])
                                                                                 : 0u;
    if constexpr (sizeof(T) == 1) q.w[0] |= e << (8 * i);
    else if constexpr (sizeof(T) == 2) q.w[i >> 1] |= e << (16 * (i & 1));
    else q.w[i] = e;
  }
}

// A 16-bit element given as the low bits of a word, as float.
template <typename T>
__device__ __forceinline__ float bits16_to_f32(uint32_t b) {
  static_assert(sizeof(T) == 2, "16-bit element types only");
  if constexpr (std::is_same<T, bf16_t>::value) return __uint_as_float(b << 16);
  else return (float)b;
}

template <typename T>
__device__ __forceinline__ void unpack4(const Quad<T>& q, float* o) {
  if constexpr (sizeof(T) == 1) {
    o[0] = (float)(q.w[0] & 0xffu);
    o[1] = (float)((q.w[0] >> 8) & 0xffu);
    o[2] = (float)((q.w[0] >> 16) & 0xffu);
    o[3] = (float)(q.w[0] >> 24);
  } else if constexpr (sizeof(T) == 2) {
    // the 16-bit elements are taken out of the words by shifts (reading the
    // word array through a 16-bit pointer would break type-based aliasing)
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = bits16_to_f32<T>((q.w[i >> 1] >> (16 * (i & 1))) & 0xffffu);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = __uint_as_float(q.w[i]);
  }
}

// ---- 8-bit planar RGB sources (colour path)
template <>
struct Quad<Rgb8> {
  static constexpr int NW = 3;  // the R, G, B words of 4 pixels
  uint32_t w[3];
};

// Channel c of BT.709 YCbCr as printed (0 Y, 1 Cb, 2 Cr), in the operation
// order of the stand-alone transform kernel.
__device__ __forceinline__ float ycbcr709(float R, float G, float B, int c) {
  const float Y = fmaf(0.213f, R, fmaf(0.715f, G, 0.072f * B));
  return c == 0 ? Y : (c == 1 ? 0.539f * (B - Y) : 0.635f * (R - Y));
}

__device__ __forceinline__ void fetch4_rgb(const uint8_t* P, int64_t pitch, int64_t cs, const Geom& g, int vec_ok,
                                           int py, int px, Quad<Rgb8>& q) {
  if (vec_ok && g.pad == SSIMX_PAD_VALID && py < g.H && px + 3 < g.W) {
    const uint8_t* s = P + (int64_t)py * pitch + px;
    q.w[0] = *(const uint32_t*)s;
    q.w[1] = *(const uint32_t*)(s + cs);
    q.w[2] = *(const uint32_t*)(s + 2 * cs);
    return;
  }
  q.w[0] = q.w[1] = q.w[2] = 0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int sy, sx;
    if (padded_source(py, px + i, g.H, g.W, g.pad, g.before, g.Hp, g.Wp, sy, sx)) {
      const uint8_t* s = P + (int64_t)sy * pitch + sx;
      q.w[0] |= (uint32_t)s[0] << (8 * i);
      q.w[1] |= (uint32_t)s[cs] << (8 * i);
      q.w[2] |= (uint32_t)s[2 * cs] << (8 * i);
    }
  }
}

__device__ __forceinline__ void unpack4_rgb(const Quad<Rgb8>& q, int c, float* o) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
    o[i] = ycbcr709((float)((q.w[0] >> (8 * i)) & 0xffu), (float)((q.w[1] >> (8 * i)) & 0xffu),
                    (float)((q.w[2] >> (8 * i)) & 0xffu), c);
}

template <typename T>
constexpr bool is_rgb() {
  return std::is_same<T, Rgb8>::value;
}

// Chunk staging split in two halves: fetch_chunk issues the global loads of
// kCH footprint rows into registers, store_chunk converts them to u, v and
// writes LDS.  A thread's items are fixed for the whole tile: item 0 is row
// t / 16, quad t % 16 (the 16 quads of the tile's 64 columns, 16 lanes per
// row); item 1 covers the NQ - 16 quads past them, four lanes per row in the
// first wave.  Only the row base of a chunk changes; it is block-uniform, so
// a vector load adds a 32-bit in-chunk offset to a scalar base (the host
// allows vector loads only for row pitches below 2^24 elements, so 16 rows of
// any element type stay below 2^32 bytes).
template <int K>
struct ChunkItems {
  static constexpr int NQ = Shape<K>::NQ;
  static constexpr int PER_THREAD = 2;
  static_assert(kCH == 16 && kNT == 256 && NQ >= 16 && NQ - 16 <= 4, "item layout");
};

template <int K>
__device__ __forceinline__ bool chunk_item(int i, int& r, int& q) {
  if (i == 0) {
    r = threadIdx.x >> 4;
    q = threadIdx.x & 15;
    return true;
  }
  r = (threadIdx.x >> 2) & 15;
  q = 16 + (threadIdx.x & 3);
  return threadIdx.x < 64 && (threadIdx.x & 3) < ChunkItems<K>::NQ - 16;
}

// The per-thread part of a chunk load, fixed for the whole tile: the byte
// offsets of the thread's quads from the chunk's row base, and whether each
// quad lies inside the plane's columns and may take one vector load.
template <int K>
struct ChunkLoad {
  uint32_t xo[ChunkItems<K>::PER_THREAD], yo[ChunkItems<K>::PER_THREAD];
  bool vec[ChunkItems<K>::PER_THREAD];
};

template <int K, typename T>
__device__ __forceinline__ ChunkLoad<K> chunk_load_init(const FastArgs& a, int px0) {
  ChunkLoad<K> cl;
  constexpr uint32_t ES = is_rgb<T>() ? 1u : (uint32_t)sizeof(T);
  const bool vec = a.vec_ok && a.g.pad == SSIMX_PAD_VALID;
#pragma unroll
  for (int i = 0; i < ChunkItems<K>::PER_THREAD; ++i) {
    int r, q;
    const bool live = chunk_item<K>(i, r, q);
    const int px = px0 + 4 * q;
    cl.vec[i] = live && vec && px + 3 < a.g.W;
    cl.xo[i] = (__umul24((uint32_t)r, (uint32_t)a.x.pitch) + (uint32_t)px) * ES;
    cl.yo[i] = (__umul24((uint32_t)r, (uint32_t)a.y.pitch) + (uint32_t)px) * ES;
  }
  return cl;
}

// EDGE = false: the tile reads only inside the plane's columns with vector
// loads (valid borders, aligned planes), so no element-wise border path is
// compiled in; rows past the plane (below the last valid window) read zero.
// One quad of 4 elements (the R, G, B words for RGB sources) with vector
// loads from p (aligned).
template <typename T>
__device__ __forceinline__ Quad<T> load_quad(const char* p, int64_t cs) {
  Quad<T> q;
  if constexpr (is_rgb<T>()) {
    q.w[0] = *(const uint32_t*)p;
    q.w[1] = *(const uint32_t*)(p + cs);
    q.w[2] = *(const uint32_t*)(p + 2 * cs);
  } else if constexpr (sizeof(T) == 1) {
    q.w[0] = *(const uint32_t*)p;
  } else if constexpr (sizeof(T) == 2) {
    const uint2 v = *(const uint2*)p;
    q.w[0] = v.x;
    q.w[1] = v.y;
  } else {
    const uint4 v = *(const uint4*)p;
    q.w[0] = v.x;
    q.w[1] = v.y;
    q.w[2] = v.z;
    q.w[3] = v.w;
  }
  return q;
}

template <typename T>
__device__ __forceinline__ Quad<T> zero_quad() {
  Quad<T> q;
#pragma unroll
  for (int w = 0; w < Quad<T>::NW; ++w) q.w[w] = 0u;
  return q;
}

// EDGE = false: the tile reads only inside the plane's columns with vector
// loads (valid borders, aligned planes), so no element-wise border path is
// compiled in; rows past the plane (below the last valid window) read zero.
// Every branch yields whole quad values that are stored once (stores to the
// register arrays from several branches would keep them out of registers).
template <int K, typename T, bool EDGE>
__device__ __forceinline__ void fetch_chunk(const FastArgs& a, const T* X, const T* Y, int py0, int px0,
                                            const ChunkLoad<K>& cl, Quad<T>* qx, Quad<T>* qy, int nrows = kCH) {
  // block-uniform row bases of the chunk
  const char* xr = (const char*)(X + (int64_t)py0 * a.x.pitch);
  const char* yr = (const char*)(Y + (int64_t)py0 * a.y.pitch);
#pragma unroll
  for (int i = 0; i < ChunkItems<K>::PER_THREAD; ++i) {
    int r, q;
    if (!chunk_item<K>(i, r, q) || r >= nrows) continue;
    Quad<T> nx = zero_quad<T>(), ny = zero_quad<T>();
    if (!EDGE || cl.vec[i]) {
      if (py0 + r < a.g.H) {
        nx = load_quad<T>(xr + cl.xo[i], a.cstride);
        ny = load_quad<T>(yr + cl.yo[i], a.cstride);
      }
    } else if constexpr (EDGE) {
      const int px = px0 + 4 * q;
      if constexpr (is_rgb<T>()) {
        fetch4_rgb((const uint8_t*)X, a.x.pitch, a.cstride, a.g, a.vec_ok, py0 + r, px, nx);
        fetch4_rgb((const uint8_t*)Y, a.y.pitch, a.cstride, a.g, a.vec_ok, py0 + r, px, ny);
      } else {
        fetch4<T>(X, a.x.pitch, a.g, a.vec_ok, py0 + r, px, nx);
        fetch4<T>(Y, a.y.pitch, a.g, a.vec_ok, py0 + r, px, ny);
      }
    }
    qx[i] = nx;
    qy[i] = ny;
  }
}

template <int K, typename T>
__device__ __forceinline__ void store_chunk(const Quad<T>* qx, const Quad<T>* qy, float* U, float* V, int ch,
                                            int nrows = kCH) {
  using S = Shape<K>;
#pragma unroll
  for (int i = 0; i < ChunkItems<K>::PER_THREAD; ++i) {
    int r, q;
    if (!chunk_item<K>(i, r, q) || r >= nrows) continue;
    float xv[4], yv[4];
    if constexpr (is_rgb<T>()) {
      unpack4_rgb(qx[i], ch, xv);
      unpack4_rgb(qy[i], ch, yv);
    } else {
      unpack4<T>(qx[i], xv);
      unpack4<T>(qy[i], yv);
    }
    *(float4*)&U[r * S::IWP + 4 * q] = make_float4(xv[0] + yv[0], xv[1] + yv[1], xv[2] + yv[2], xv[3] + yv[3]);
    *(float4*)&V[r * S::IWP + 4 * q] = make_float4(xv[0] - yv[0], xv[1] - yv[1], xv[2] - yv[2], xv[3] - yv[3]);
  }
}

// 2x2 means of the staged rows rbase .. rbase + nrows - 1 (LDS rows 0 ..) that
// the tile owns: input rows [own_r0, own_r1) and columns [ox0, own_c1).  With
// u = x + y and v = x - y staged, the x mean is the sum of u + v over the
// block / 8 and the y mean the sum of u - v / 8: exact, and equal to the
// stand-alone down-sampling, for integer-valued planes and their pyramid
// levels.  Every boundary is even, so no block straddles two tiles or chunks.
template <int K>
__device__ __forceinline__ void emit_down(const FastArgs& a, const float* U, const float* V, int rbase, int nrows,
                                          int ox0, int own_r0, int own_r1, int own_c1, int frame) {
  using S = Shape<K>;
  const int W2 = a.g.W / 2, H2 = a.g.H / 2;
  const int r_lo = max(rbase, own_r0), r_hi = min(min(rbase + nrows, own_r1), 2 * H2);
  const int c_hi = min(own_c1, 2 * W2);
  if (r_hi <= r_lo || c_hi <= ox0) return;  // uniform over the block
  const int npr = (r_hi - r_lo) / 2, npc = (c_hi - ox0) / 2;
  for (int it = threadIdx.x; it < npr * npc; it += kNT) {
    const int pr = it / npc, pc = it - pr * npc;
    const int ri = r_lo - rbase + 2 * pr, ci = 2 * pc;
    const float2 u0 = *(const float2*)&U[ri * S::IWP + ci], u1 = *(const float2*)&U[(ri + 1) * S::IWP + ci];
    const float2 v0 = *(const float2*)&V[ri * S::IWP + ci], v1 = *(const float2*)&V[(ri + 1) * S::IWP + ci];
    const float sx = ((u0.x + v0.x) + (u0.y + v0.y)) + ((u1.x + v1.x) + (u1.y + v1.y));
    const float sy = ((u0.x - v0.x) + (u0.y - v0.y)) + ((u1.x - v1.x) + (u1.y - v1.y));
    const int64_t o = ((int64_t)frame * H2 + (r_lo / 2 + pr)) * W2 + (ox0 / 2 + pc);
    a.ds_x[o] = 0.125f * sx;
    a.ds_y[o] = 0.125f * sy;
  }
}

// Row pass over `nrows` staged rows into band rows [band0, band0 + nrows).
template <int K>
__device__ __forceinline__ void row_pass(const float* taps, const float* U, const float* V, int nrows, float* HM,
                                         int band0) {
  using S = Shape<K>;
  constexpr int NG = kTW / 4;
  for (int it = threadIdx.x; it < nrows * NG; it += kNT) {
    const int r = it / NG, gq = it - r * NG;
    float u[4 * S::NREAD], v[4 * S::NREAD];
#pragma unroll
    for (int n = 0; n < S::NREAD; ++n) {
      *(float4*)&u[4 * n] = *(const float4*)&U[r * S::IWP + 4 * gq + 4 * n];
      *(float4*)&v[4 * n] = *(const float4*)&V[r * S::IWP + 4 * gq + 4 * n];
    }
    const float tu = u[S::SHIFT], tv = v[S::SHIFT];
    float du[K + 3], dv[K + 3], pu[K + 3], pv[K + 3];
#pragma unroll
    for (int n = 0; n < K + 3; ++n) {
      du[n] = u[n] - tu;
      dv[n] = v[n] - tv;
      pu[n] = du[n] * du[n];
      pv[n] = dv[n] * dv[n];
    }
    float hu[4], hv[4], vu[4], vv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float au = 0.f, av = 0.f, qu = 0.f, qv = 0.f;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        // the centring element's own terms are 0 for finite inputs; a
        // non-finite one already makes t, and so every output, non-finite
        if (j + t == S::SHIFT) continue;
        const float w = taps[t];
        au = fmaf(w, du[j + t], au);
        av = fmaf(w, dv[j + t], av);
        qu = fmaf(w, pu[j + t], qu);
        qv = fmaf(w, pv[j + t], qv);
      }
      hu[j] = tu + au;
      hv[j] = tv + av;
      vu[j] = fmaf(-au, au, qu);
      vv[j] = fmaf(-av, av, qv);
    }
    // (mean_u, mean_v, var_u, var_v) of a column side by side: the column
    // pass reads a band row of its column with one 16-byte load.  Column p
    // sits in slot p + p / 8, so the 8 lanes of a 16-byte store phase (4
    // columns apart) hit distinct banks.
    float* o = HM + (band0 + r) * S::RS + 4 * (4 * gq + gq / 2);
#pragma unroll
    for (int j = 0; j < 4; ++j) *(float4*)&o[4 * j] = make_float4(hu[j], hv[j], vu[j], vv[j]);
  }
}

// Move band rows [CH, CH + HALO) to [0, HALO): HALO contiguous rows of
// float4, dealt round-robin to the threads (a thread's copies are the same for
// every chunk of the tile).
template <int K>
struct BandCopy {
  static constexpr int N = Shape<K>::HALO * Shape<K>::RS / 4;  // float4 copies
  static constexpr int PER = (N + kNT - 1) / kNT;
};

template <int K>
__device__ __forceinline__ void band_shift(float* HM) {
  using B = BandCopy<K>;
  float4* d = (float4*)HM;
#pragma unroll
  for (int i = 0; i < B::PER; ++i) {
    const int it = threadIdx.x + i * kNT;
    if ((i + 1) * kNT <= B::N || it < B::N) d[it] = d[it + kCH * Shape<K>::RS / 4];
  }
}


template <int K>
__host__ __device__ constexpr int fast_smem_floats() {
  return 2 * kCH * Shape<K>::IWP + Shape<K>::BANDF;
}

// One map tile: returns this thread's share of the tile's pooled sum (EPI 0:
// forward; EPI 2: forward that also writes the 2x2 means of its input to
// a.ds_x, a.ds_y; EPI 3: forward with luminance-weighted values) or 0 (EPI 1:
// adjoint coefficients).  `smem` holds
// fast_smem_floats<K>() floats.
// GMAP (EPI 1): the upstream is a per-position map (a.grad_map) rather than
// per-frame scalars.  It is a separate body because a load in the epilogue
// makes the compiler wait there for every older memory operation (the next
// chunk's prefetch and the previous outputs' stores) on both paths of a
// runtime branch.
// MODE >= 0 (EPI 1, interior tiles): the coefficient mode (0 Q, 1 cs, 3 the
// two upstreams) fixed at compile time, so that the four outputs' epilogues
// form one block; MODE = -1 reads a.mode per output.
template <int K, typename T, int EPI, bool EDGE, bool GMAP = false, int MODE = -1>
__device__ __forceinline__ float fast_stats_tile_body(const FastArgs& a, int frame, int tile, float* smem) {
  using S = Shape<K>;
  float* U = smem;
  float* V = U + kCH * S::IWP;
  float* HM = V + kCH * S::IWP;

  const int tyi = tile / a.g.tiles_x, txi = tile - tyi * a.g.tiles_x;
  // block-uniform tile origin and chunk-loop bound (scalar loop control)
  const int ox0 = __builtin_amdgcn_readfirstlane(txi * kTW), oy0 = __builtin_amdgcn_readfirstlane(tyi * a.g.TH);
  // RGB sources: staged frame 3 b + c is channel c of RGB frame b
  const int src = is_rgb<T>() ? frame / 3 : frame;
  const int ch = is_rgb<T>() ? frame - 3 * src : 0;
  const T* X = (const T*)a.x.data + (int64_t)src * a.x.bstride;
  const T* Y = (const T*)a.y.data + (int64_t)src * a.y.bstride;
  float taps[K];
#pragma unroll
  for (int t = 0; t < K; ++t) taps[t] = a.taps[t];

  // input rows and columns whose 2x2 means this tile writes (down-sampling)
  constexpr bool down = EPI == 2;  // forward plus the next scale's 2x2 means
  const int own_r1 = tyi == a.g.tiles_y - 1 ? a.g.H : oy0 + a.g.TH;
  const int own_c1 = txi == a.g.tiles_x - 1 ? a.g.W : ox0 + kTW;

  // prologue: the first K-1 footprint rows
  Quad<T> qx[ChunkItems<K>::PER_THREAD], qy[ChunkItems<K>::PER_THREAD];
  const ChunkLoad<K> cl = chunk_load_init<K, T>(a, ox0);
  fetch_chunk<K, T, EDGE>(a, X, Y, oy0, ox0, cl, qx, qy, S::HALO);
  store_chunk<K, T>(qx, qy, U, V, ch, S::HALO);
  __syncthreads();
  if constexpr (down) emit_down<K>(a, U, V, oy0, S::HALO, ox0, oy0, own_r1, own_c1, frame);
  row_pass<K>(taps, U, V, S::HALO, HM, 0);

  const float gframe = (EPI == 1 && !GMAP) ? a.gscale[(int64_t)frame * a.gscale_stride] * a.gmul : 0.f;
  const float gl_frame = (EPI == 1 && a.mode == 3) ? a.gscale2[(int64_t)frame * a.gscale2_stride] * a.gmul : 0.f;
  float acc = 0.f;
  const float c1x2 = 2.f * a.C1, c2x2 = 2.f * a.C2;
  const int oy_end = __builtin_amdgcn_readfirstlane(min(a.g.Ho, oy0 + a.g.TH));
  fetch_chunk<K, T, EDGE>(a, X, Y, oy0 + S::HALO, ox0, cl, qx, qy);
  if constexpr (EPI == 1 && !GMAP) {
    // as many dropped stores as a chunk's epilogue issues: on entry to the
    // chunk loop the prefetch then lies as far behind the newest memory
    // operation as in every later iteration, so the one wait for it at the
    // top of the loop can leave the previous chunk's twelve coefficient
    // stores in flight (the forward's four stores measured better waited for)
#pragma unroll
    for (int i = 0; i < 12; ++i) store_row_f32(nullptr, kStoreDrop + 4u * i, 0.f);  // distinct: none merged
  }
  for (int cy = oy0; cy < oy_end; cy += kCH) {
    __syncthreads();  // U, V free; band rows [0, HALO) ready
    store_chunk<K, T>(qx, qy, U, V, ch);
    // the next chunk's pixels are loaded while this chunk's row and column
    // passes run (the registers were just staged; with down-sampling, after
    // the 2x2 means are written, which keeps those registers free for it)
    if constexpr (!down)
      if (cy + kCH < oy_end) fetch_chunk<K, T, EDGE>(a, X, Y, cy + kCH + S::HALO, ox0, cl, qx, qy);
    __syncthreads();
    if constexpr (down) {
      emit_down<K>(a, U, V, cy + S::HALO, kCH, ox0, oy0, own_r1, own_c1, frame);
      if (cy + kCH < oy_end) fetch_chunk<K, T, EDGE>(a, X, Y, cy + kCH + S::HALO, ox0, cl, qx, qy);
    }
    row_pass<K>(taps, U, V, kCH, HM, S::HALO);
    __syncthreads();
    // column pass: item = (4 output rows, 1 column); the block's 256 items
    // are one per thread, wave w taking output rows cy + 4 w .. cy + 4 w + 3,
    // so the row base of every store is wave-uniform and a store only adds
    // the lane's column
    static_assert((kCH / 4) * kTW == kNT && kTW == 64, "one column-pass item per thread, one row group per wave");
    {
      const int gr = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), c = threadIdx.x & 63;
      const int oj = ox0 + c;
      const bool col_in = oj < a.g.Wo;
      const uint32_t cb = 4u * (uint32_t)c;  // byte offset of the lane's column from the tile's first
      // coefficient stores: the same, or the dropped offset past the map's last
      // column; a row past the tile's last ORs in the dropped offset too (a
      // uniform choice, so no store is split into exec-masked branches)
      const uint32_t lane_off = col_in ? cb : kStoreDrop;
      const float4* hb = (const float4*)(HM + 4 * gr * S::RS) + (c + c / 8);  // (mean_u, mean_v, var_u, var_v)
      const float Tu = hb[S::SHIFT * (S::RS / 4)].x, Tv = hb[S::SHIFT * (S::RS / 4)].y;
      float Mu[4] = {0.f, 0.f, 0.f, 0.f}, Mv[4] = {0.f, 0.f, 0.f, 0.f};
      // the second moments of u start at 2 C2: every use of var_u below takes
      // var_u + 2 C2, which the fma that removes the squared mean then yields
      float Su[4] = {c2x2, c2x2, c2x2, c2x2}, Sv[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < K + 3; ++m) {
        const float4 h = hb[m * (S::RS / 4)];
        // the centring row (m == SHIFT) adds only its variances: its mean
        // deviations are 0 for finite values, and a non-finite one already
        // makes T, and so every output, non-finite
        constexpr int kSelf = S::SHIFT;
        const bool self = m == kSelf;
        const float du = h.x - Tu, dv = h.y - Tv;
        const float su = self ? h.z : fmaf(du, du, h.z);
        const float sv = self ? h.w : fmaf(dv, dv, h.w);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int t = m - j;
          if (t >= 0 && t < K) {
            const float w = taps[t];
            if (!self) {
              Mu[j] = fmaf(w, du, Mu[j]);
              Mv[j] = fmaf(w, dv, Mv[j]);
            }
            Su[j] = fmaf(w, su, Su[j]);
            Sv[j] = fmaf(w, sv, Sv[j]);
          }
        }
      }
      // value epilogue, with the (uniform) mode resolved once per chunk
      auto values = [&](auto mode_c) {
        constexpr int M = decltype(mode_c)::value;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int oi = cy + 4 * gr + j;  // wave-uniform
          if (oi >= oy_end || !col_in) continue;
          const float s2 = fmaf(-Mu[j], Mu[j], Su[j]), var_v = fmaf(-Mv[j], Mv[j], Sv[j]);  // s2 = var_u + 2 C2
          const float val = ssim_value_uv_s<M>(Tu + Mu[j], Tv + Mv[j], s2, var_v, c1x2);
          if (a.map) {
            store_row_f32(a.map + (int64_t)frame * a.map_bstride + (int64_t)oi * a.map_pitch + ox0, cb, val);
          }
          if constexpr (EPI == 3) {
            // Luminance-Weighted Pooling: weight of the reference's local mean
            // mu_x = (mu_u + mu_v) / 2, 0 below a_s, a ramp over b_s, then 1
            const float mx = 0.5f * ((Tu + Mu[j]) + (Tv + Mv[j]));
            const float wgt = a.lw_b > 0.f ? fminf(fmaxf((mx - a.lw_a) / a.lw_b, 0.f), 1.f)
                                           : (mx >= a.lw_a ? 1.f : 0.f);
            acc = fmaf(wgt, val, acc);
          } else {
            acc += val;
          }
        }
      };
      if constexpr (EPI != 1) {
        if (a.mode == 1) values(std::integral_constant<int, 1>{});
        else if (a.mode == 3) values(std::integral_constant<int, 3>{});
        else values(std::integral_constant<int, 0>{});
      }
#pragma unroll
      for (int j = 0; j < 4 && EPI == 1; ++j) {
        const int oi = cy + 4 * gr + j;  // wave-uniform
        if constexpr (GMAP)
          if (oi >= oy_end || !col_in) continue;  // the upstream map is read only inside the map
        const float mean_u = Tu + Mu[j], mean_v = Tv + Mv[j];
        const float s2 = fmaf(-Mu[j], Mu[j], Su[j]), var_v = fmaf(-Mv[j], Mv[j], Sv[j]);  // s2 = var_u + 2 C2
        {
          float g = gframe;
          if constexpr (GMAP) {
            const char* row = (const char*)(a.grad_map + (int64_t)frame * a.gm_bstride + (int64_t)oi * a.gm_pitch + ox0);
            g = *(const float*)(row + cb);
          }
          // reciprocal estimates (about 1 ulp) suffice for the adjoint.
          // d(f_l l + f_c cs) with upstream g: Q = l cs takes f_l = cs,
          // f_c = l (both times g); cs alone f_l = 0, f_c = g; mode 3 the
          // two upstreams.  With k_l = f_l / B1^2 and k_c = f_c / B2^2:
          //   B_u = k_c var_v,  B_v = -k_c (A2 + B2),
          //   A   = k_l m_v (m_u m_v + A1 + B1) - B_u (m_u - t_u) + B_v (m_v - t_v)
          // (the three planes are A = A_u - A_v, B_u, B_v of the transpose).
          // In doubled terms, e = A1 + B1 = m_u^2 + 2 C1 and s = A2 + B2 =
          // var_u + 2 C2 give 2 B1 = e + m_v^2, 2 A1 = e - m_v^2,
          // 2 B2 = s + var_v, 2 A2 = s - var_v; with r1 = 1 / (2 B1) and
          // r2 = 1 / (2 B2), 1 / B = 2 r and, for Q,
          //   k_l = 4 g (2 A2) r2 r1^2,  k_c = 4 g (2 A1) r1 r2^2
          // (cs: k_l = 0, k_c = 4 g r2^2; two upstreams: k_l = 4 g_l r1^2).
          const float e = fmaf(mean_u, mean_u, c1x2);
          const float r1 = __builtin_amdgcn_rcpf(fmaf(mean_v, mean_v, e)), r2 = __builtin_amdgcn_rcpf(s2 + var_v);
          const float g4 = 4.f * g;
          float kl, kc;
          const int mode = MODE >= 0 ? MODE : a.mode;
          if (mode == 1) {
            kl = 0.f;
            kc = (g4 * r2) * r2;
          } else if (mode == 3) {
            kl = ((4.f * gl_frame) * r1) * r1;
            kc = (g4 * r2) * r2;
          } else {
            const float q = g4 * (r1 * r2);
            kl = (q * r1) * (s2 - var_v);
            kc = (q * r2) * fmaf(-mean_v, mean_v, e);
          }
          const float bu = kc * var_v, bv = -kc * s2;
          const float ca = fmaf(kl * mean_v, fmaf(mean_u, mean_v, e), fmaf(-bu, mean_u - a.tu, bv * (mean_v - a.tv)));
          // W^T is linear: the two A maps are combined before the transpose
          const int64_t qs = (int64_t)a.batch * a.g.Ho * a.cpitch;
          // every row and lane stores, outside the map with the dropped
          // offset: a fixed twelve stores per chunk, which the wait for the
          // next chunk's loads at the top of the loop leaves in flight
          float* row = a.coef + ((int64_t)frame * a.g.Ho + min(oi, oy_end - 1)) * a.cpitch + ox0;
          const uint32_t off = lane_off | (oi < oy_end ? 0u : kStoreDrop);
          store_row_f32(row, off, ca);
          store_row_f32(row + qs, off, bu);
          store_row_f32(row + 2 * qs, off, bv);
        }
      }
    }
    __syncthreads();
    band_shift<K>(HM);
  }
  __syncthreads();  // the caller may reuse smem for the next tile
  return acc;
}


// A tile whose footprint columns lie inside an aligned plane with valid
// borders takes the body without the element-wise border path (the common
// case); edge tiles, other borders and unaligned planes take the full one.
// The choice is uniform over the workgroup.
template <int K, typename T, int EPI>
__device__ __forceinline__ float fast_stats_tile(const FastArgs& a, int frame, int tile, float* smem) {
  const int txi = tile % a.g.tiles_x;
  const bool interior = a.vec_ok && a.g.pad == SSIMX_PAD_VALID && txi * kTW + Shape<K>::IWP <= a.g.W;
  if constexpr (EPI == 1) {
    if (a.grad_map)
      return interior ? fast_stats_tile_body<K, T, EPI, false, true>(a, frame, tile, smem)
                      : fast_stats_tile_body<K, T, EPI, true, true>(a, frame, tile, smem);
    if (interior) {  // one body per coefficient mode
      if (a.mode == 1) return fast_stats_tile_body<K, T, EPI, false, false, 1>(a, frame, tile, smem);
      if (a.mode == 3) return fast_stats_tile_body<K, T, EPI, false, false, 3>(a, frame, tile, smem);
      return fast_stats_tile_body<K, T, EPI, false, false, 0>(a, frame, tile, smem);
    }
  }
  return interior ? fast_stats_tile_body<K, T, EPI, false>(a, frame, tile, smem)
                  : fast_stats_tile_body<K, T, EPI, true>(a, frame, tile, smem);
}

}  // namespace fast
}  // namespace ssimx
