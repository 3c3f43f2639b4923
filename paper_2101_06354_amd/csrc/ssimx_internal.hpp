// Internal declarations shared by the HIP translation units of libssimx.
// Not part of the public ABI (include/ssimx.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ssimx.h"

namespace ssimx {

constexpr int KMAX_GAUSS = 41;  // largest Gaussian window (odd)
constexpr int KMAX_BOX = 64;    // largest rectangular window
constexpr int BLOCK = 256;      // threads per block of the tiled kernels
constexpr int MAX_SCALES = 8;
// BT.601 luma weights of the differentiable-loss workload (R, G, B).
constexpr float kBt601R = 0.299f, kBt601G = 0.587f, kBt601B = 0.114f;
// Launch limits checked on the host before any launch: frames go on grid.y
// (65535 at most; the colour path puts 3 channel frames per RGB frame
// there), and per-plane element grids are formed in 32-bit ints.
constexpr int kMaxGridY = 65535;
constexpr int64_t kMaxPlaneElems = (1ll << 31) - (1ll << 16);

struct bf16_t {
  uint16_t bits;
};

// ---------------------------------------------------------------- scalars
template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<uint8_t>(uint8_t v) { return (float)v; }
template <>
__device__ __forceinline__ float to_f32<uint16_t>(uint16_t v) { return (float)v; }
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<bf16_t>(bf16_t v) { return __uint_as_float(((uint32_t)v.bits) << 16); }

template <typename T>
__device__ __forceinline__ int32_t to_i32(T v) { return (int32_t)v; }

// Half-sample symmetric reflection of index i into [0, n) (period 2n).
__device__ __forceinline__ int reflect_index(int i, int n) {
  const int p = 2 * n;
  int m = i % p;
  if (m < 0) m += p;
  return m < n ? m : p - 1 - m;
}

// Source pixel of padded coordinate (py, px); returns false for zero padding
// outside the plane and for coordinates past the padded extent.
__device__ __forceinline__ bool padded_source(int py, int px, int H, int W, int pad, int before, int Hp, int Wp,
                                              int& sy, int& sx) {
  if (py >= Hp || px >= Wp) return false;
  if (pad == SSIMX_PAD_VALID) {
    sy = py;
    sx = px;
    return true;
  }
  int yy = py - before, xx = px - before;
  if (pad == SSIMX_PAD_ZERO) {
    if (yy < 0 || yy >= H || xx < 0 || xx >= W) return false;
    sy = yy;
    sx = xx;
    return true;
  }
  sy = reflect_index(yy, H);
  sx = reflect_index(xx, W);
  return true;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Error-free transformation a + b = s + e.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Mean of one frame's tile partials in a fixed-order compensated (TwoSum) tree
// over the block: (hi + lo) * inv_count with the low part kept through the
// product.  hs, ls: LDS arrays of blockDim.x floats.  Result valid in thread 0.
__device__ __forceinline__ float tile_mean(const float* p, int tiles, float inv_count, float* hs, float* ls) {
  float s = 0.f, c = 0.f;
  for (int i = threadIdx.x; i < tiles; i += blockDim.x) {
    float e;
    two_sum(s, p[i], s, e);
    c += e;
  }
  hs[threadIdx.x] = s;
  ls[threadIdx.x] = c;
  __syncthreads();
  for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      float e, t;
      two_sum(hs[threadIdx.x], hs[threadIdx.x + w], t, e);
      hs[threadIdx.x] = t;
      ls[threadIdx.x] += ls[threadIdx.x + w] + e;
    }
    __syncthreads();
  }
  const float hi = hs[0], lo = ls[0];
  const float ph = hi * inv_count;
  const float pe = fmaf(hi, inv_count, -ph);
  return ph + (pe + lo * inv_count);
}

// MS-SSIM of one frame from its per-scale values v[0..M-1] (CS_j, then the
// coarsest term): the weighted product S_M^{w_M} prod CS_j^{w_j} (clamp: of
// max(v, 0)), or (sum) the weighted average sum w_j v_j.  With `split` the
// coarsest term is v[M-1] * lval (mean(l) * mean(cs)).  cs (nullable) gets the
// terms as combined.
__device__ __forceinline__ float ms_combine_frame(const float* v, int M, const float* w, int clamp, int sum,
                                                  float lval, bool split, float* cs) {
  float score = sum ? 0.f : 1.f;
  for (int j = 0; j < M; ++j) {
    float t = v[j];
    if (split && j == M - 1) t *= lval;
    if (cs) cs[j] = t;
    if (sum) {
      score = fmaf(w[j], t, score);
      continue;
    }
    if (clamp) t = fmaxf(t, 0.f);
    score *= powf(t, w[j]);
  }
  return score;
}

// Upstream of every pooled per-scale term of one frame's MS-SSIM, from its
// values c[0..M-1] (split: the coarsest term is c[M-1] * lval), the score ms
// and dL/dscore g, with weights w and 1/(map positions) inv: for the weighted
// product g ms w_j / T_j / N_j (zero where a clamped term is not positive), for
// the weighted average g w_j / N_j.  With split, up[M-1] is the upstream of
// mean(cs) and *up2 that of mean(l).
__device__ __forceinline__ void ms_upstream_frame(const float* c, int M, float lval, bool split, float ms, float g,
                                                  const float* w, const float* inv, int clamp, int sum, float* up,
                                                  float* up2) {
  for (int j = 0; j < M; ++j) {
    const bool sp = split && j == M - 1;
    const float v = sp ? c[j] * lval : c[j];
    float r = sum ? g * w[j] * inv[j] : g * ms * w[j] / v * inv[j];
    if (!sum && clamp && !(v > 0.f)) r = 0.f;
    if (sp) {
      up[j] = r * lval;
      *up2 = r * c[j];
    } else {
      up[j] = r;
    }
  }
}

// Deterministic block sum of one float per thread (fixed shuffle order, then
// fixed order across waves).  Result valid in thread 0.
template <int NT>
__device__ __forceinline__ float block_sum(float v, float* lds_scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds_scratch[wid] = v;
  __syncthreads();
  float r = 0.f;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += lds_scratch[w];
  }
  return r;
}

// ---------------------------------------------------------------- arguments
// Workgroups of a launch are handed to the 8 XCDs round-robin in dispatch
// order, and each XCD has its own L2.  The i-th workgroup that lands on XCD x
// takes logical index x * per + i instead (XCDs 0 .. rem-1 take per + 1), so
// each XCD walks a contiguous range of tiles and neighbouring tiles, which
// read the same halo cache lines, meet in the same L2.  Returns (tile, frame)
// for a (tiles, frames) grid; the mapping is a bijection on [0, n).
__device__ __forceinline__ int xcd_perm(int b, int n) {
  const int per = n >> 3, rem = n & 7, x = b & 7, i = b >> 3;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

__device__ __forceinline__ void xcd_tile(int& tile, int& frame) {
  const int nx = gridDim.x;
  const int l = xcd_perm(blockIdx.x + nx * blockIdx.y, nx * gridDim.y);
  frame = l / nx;
  tile = l - frame * nx;
}

// The same XCD ranges for a (tiles_x * tiles_y, frames) grid, with each
// XCD taking the tiles of its range that lie in a frame's last tile row
// after all its other tiles.  The last row is usually shorter (the map
// height is rarely a multiple of the tile height), so the launch ends on
// short tiles instead of full ones that would leave CUs idle.  Within the
// XCD's range [lo, lo + cnt), the i-th workgroup takes the i-th tile of the
// range's full rows, in order, then the range's last-row tiles in order (a
// bijection on the range).
__device__ __forceinline__ void xcd_tile_rows_last(int tiles_x, int tiles_y, int& tile, int& frame) {
  const int T = gridDim.x;  // tiles per frame, tiles_x * tiles_y
  const int n = T * gridDim.y;
  const int b = blockIdx.x + T * blockIdx.y;
  const int per = n >> 3, rem = n & 7, x = b & 7, i = b >> 3;
  const int lo = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
  const int cnt = x < rem ? per + 1 : per;
  const int body = tiles_x * (tiles_y - 1);  // tiles above the last row, per frame
  // tiles of the full rows among logical indices [0, m)
  auto full_before = [&](int m) { return (m / T) * body + min(m - (m / T) * T, body); };
  const int f0 = full_before(lo), nf = full_before(lo + cnt) - f0;
  int l;
  if (i < nf) {
    const int c = f0 + i;  // the c-th full-row tile of the grid (body > 0 here)
    l = (c / body) * T + c % body;
  } else {
    const int c = (lo - f0) + (i - nf);  // the c-th last-row tile of the grid
    l = (c / tiles_x) * T + body + c % tiles_x;
  }
  frame = l / T;
  tile = l - frame * T;
}

// A launch made of segments, segment s owning workgroups [start[s],
// start[s + 1]) of a one-dimensional grid (start[0] = 0), each laid over its
// own (tiles, frames) grid with the XCD mapping above taken within the
// segment (a segment that does not start on a multiple of 8 keeps each XCD's
// share contiguous, shifted by the start).
__device__ __forceinline__ int seg_of(const int* start, int nseg) {
  int s = 0;
  while (s + 1 < nseg && (int)blockIdx.x >= start[s + 1]) ++s;
  return __builtin_amdgcn_readfirstlane(s);
}

__device__ __forceinline__ void seg_tile(const int* start, int s, int tiles, int& tile, int& frame) {
  const int l = xcd_perm((int)blockIdx.x - start[s], start[s + 1] - start[s]);
  frame = l / tiles;
  tile = l - frame * tiles;
}

// Store of one float at byte offset `off` from a wave-uniform address (a
// row's first column of the tile): a raw buffer store takes the 32-bit lane
// offset as is, where a global store would form a 64-bit address per lane
// with vector instructions.  `off` must stay below 2^31.
// An offset store_row_f32 drops (past the buffer's range, so the hardware
// discards the store): a loop can then issue the same number of stores on
// every path, and the compiler's wait for its loads need not include them.
constexpr uint32_t kStoreDrop = 0x80000000u;

__device__ __forceinline__ void store_row_f32(float* row, uint32_t off, float v) {
  // gfx9 raw buffer: stride 0, range check against num_records only
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(row, 0, 0x7fffffff, 0x00020000);
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}

struct PlaneArg {
  const void* data;
  int64_t pitch, bstride;
};

// Geometry of a windowed pass over one plane pair.
struct Geom {
  int W, H;        // unpadded plane
  int Wp, Hp;      // padded extent (== W, H for valid)
  int Wo, Ho;      // map
  int k, s, pad, before;
  int TW, TH;      // outputs per tile
  int IW, IH;      // input footprint of a tile
  int tiles_x, tiles_y;
};

struct SepArgs {
  PlaneArg x, y;
  Geom g;
  float C1, C2;
  int mode;            // 0: Q = l*cs, 1: cs only
  float* map;          // nullable
  int64_t map_pitch, map_bstride;
  float* partial;      // [batch][tiles] tile sums of the pooled term
  float taps[KMAX_GAUSS];
};

struct BoxArgs {
  PlaneArg x, y;
  Geom g;
  float C1, C2;
  int mode;            // 0: Q, 1: cs, 2: emit the five sums
  float* map;
  int64_t map_pitch, map_bstride;
  float* partial;
  int32_t* sums;       // mode 2: [5][batch][Ho][Wo]
  int batch;
};

}  // namespace ssimx
