// Stride-1 adjoint band kernel with a compile-time window size K: the
// transposed window over the coefficient planes written by
// fast_stats_kernel<K, T, 1> and the per-pixel combine (valid borders),
// optionally adding the 2x2 transpose of a coarser-scale gradient.
#include "fast_tile_body.hpp"

namespace ssimx {

using namespace fast;

// ---------------------------------------------------------------- adjoint
// Transposed window over the coefficient planes (valid borders, stride 1):
// G_q(y) = sum_{p in map, y - p in [0, K)} w(y - p) C_q(p), a plain K x K
// correlation of the zero-extended planes with the (symmetric) window.  Three
// planes arrive (A = A_u - A_v, B_u, B_v), each with a row pitch that is a
// multiple of 4; the footprint origin is aligned to 4 map columns so that an
// interior footprint quad is one aligned 16-byte load per plane.  The next
// chunk's quads are fetched into registers as soon as the current chunk is
// staged, so the loads overlap both passes.
namespace {

constexpr int kNM = 3;  // coefficient planes

template <int K>
struct AShape {
  static constexpr int HALO = K - 1;
  static constexpr int LP = (4 - HALO % 4) % 4;          // left pad aligning the footprint origin
  static constexpr int NREAD = (LP + K + 3 + 3) / 4;     // float4 LDS reads per row-pass item
  static constexpr int IWP = kTW - 4 + 4 * NREAD;
  static constexpr int NQ = IWP / 4;
  static constexpr int CH = 16;                           // pixel rows per chunk
  static constexpr int BAND = CH + HALO;
  static constexpr int PL = BAND * kTWP;
  static_assert(CH >= HALO, "band copy needs CH >= K - 1");
  static_assert(IWP >= LP + kTW + K - 1, "footprint row too short");
};

struct CQuad {
  float4 v[kNM];  // four consecutive map positions of each plane
};

// Item i of a thread in a chunk of coefficient rows: row r and quad q of the
// footprint.  Item 0 is row t / 16, quad t % 16; item 1 covers the NQ - 16
// quads past them, four lanes per row in the first wave.
template <int K>
__device__ __forceinline__ bool coef_item(int i, int& r, int& q) {
  if (i == 0) {
    r = threadIdx.x >> 4;
    q = threadIdx.x & 15;
    return true;
  }
  r = (threadIdx.x >> 2) & 15;
  q = 16 + (threadIdx.x & 3);
  return threadIdx.x < 64 && (threadIdx.x & 3) < AShape<K>::NQ - 16;
}

// Map rows r0 .. r0+nrows-1, footprint columns from c0 (a multiple of 4),
// into registers.  The rows' base is block-uniform; an interior quad adds a
// 32-bit offset to it (the host runs this kernel only for coefficient row
// pitches below 2^24 floats).
template <int K>
__device__ __forceinline__ void fetch_coef(const FastArgs& a, int frame, int r0, int c0, int nrows, CQuad* q) {
  using S = AShape<K>;
  static_assert(S::CH == 16 && kNT == 256 && S::NQ >= 16 && S::NQ - 16 <= 4, "item layout");
  const int64_t qs = (int64_t)a.batch * a.g.Ho * a.cpitch;
  const float* base = a.coef + (int64_t)frame * a.g.Ho * a.cpitch;
  const char* rb = (const char*)(base + (int64_t)r0 * a.cpitch);  // may point before the plane; read only in range
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    int r, qq;
    if (!coef_item<K>(i, r, qq) || r >= nrows) continue;
    const int pr = r0 + r, pc = c0 + 4 * qq;
    if (pr >= 0 && pr < a.g.Ho && pc >= 0 && pc + 3 < a.g.Wo) {
      const uint32_t off = 4u * (__umul24((uint32_t)r, (uint32_t)a.cpitch) + (uint32_t)pc);
#pragma unroll
      for (int m = 0; m < kNM; ++m) q[i].v[m] = *(const float4*)(rb + 4 * m * qs + off);
    } else {
#pragma unroll
      for (int m = 0; m < kNM; ++m) {
        float e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const bool in = pr >= 0 && pr < a.g.Ho && pc + k >= 0 && pc + k < a.g.Wo;
          e[k] = in ? base[m * qs + (int64_t)pr * a.cpitch + pc + k] : 0.f;
        }
        q[i].v[m] = make_float4(e[0], e[1], e[2], e[3]);
      }
    }
  }
}

// Pixel quads of the chunk's rows (the 64 output columns of the tile), one
// quad per thread and plane, held in registers until the chunk is staged
// (valid borders: pixels outside the plane read as zero and are not used).
// Vector loads add a 32-bit offset to the block-uniform row base of the
// chunk (vec_ok implies row pitches below 2^24 elements).
template <typename T>
__device__ __forceinline__ void fetch_quad_valid(const T* P, int64_t pitch, int W, int H, int vec_ok, int py0, int r,
                                                 int px, fast::Quad<T>& q) {
#pragma unroll
  for (int i = 0; i < fast::Quad<T>::NW; ++i) q.w[i] = 0u;
  const int py = py0 + r;
  if (py >= H) return;
  if (vec_ok && px + 3 < W) {
    const char* s = (const char*)(P + (int64_t)py0 * pitch) +
                    (__umul24((uint32_t)r, (uint32_t)pitch) + (uint32_t)px) * (uint32_t)sizeof(T);
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
  const T* s = P + (int64_t)py * pitch + px;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (px + e >= W) break;
    const uint32_t b = fast::elem_bits<T>(s[e]);
    if constexpr (sizeof(T) == 1) q.w[0] |= b << (8 * e);
    else if constexpr (sizeof(T) == 2) q.w[e >> 1] |= b << (16 * (e & 1));
    else q.w[e] = b;
  }
}

template <typename T>
__device__ __forceinline__ void fetch_xy(const FastArgs& a, const T* X, const T* Y, int py0, int px0,
                                         fast::Quad<T>& qx, fast::Quad<T>& qy) {
  const int r = threadIdx.x >> 4, q = threadIdx.x & 15;  // 16 rows x 16 quads
  fetch_quad_valid<T>(X, a.x.pitch, a.g.W, a.g.H, a.vec_ok, py0, r, px0 + 4 * q, qx);
  fetch_quad_valid<T>(Y, a.y.pitch, a.g.W, a.g.H, a.vec_ok, py0, r, px0 + 4 * q, qy);
}

// Registers -> the LDS planes C[m][r][col].
template <int K>
__device__ __forceinline__ void store_coef(const CQuad* q, int nrows, float* C) {
  using S = AShape<K>;
  constexpr int PLC = S::CH * S::IWP;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    int r, qq;
    if (!coef_item<K>(i, r, qq) || r >= nrows) continue;
    float* d = C + r * S::IWP + 4 * qq;
#pragma unroll
    for (int m = 0; m < kNM; ++m) *(float4*)&d[m * PLC] = q[i].v[m];
  }
}

// Row pass of the transposed window: thread t takes row t / 16 and the 4
// adjacent outputs of column group t % 16, in all three planes (a fixed
// mapping: no index arithmetic per item).  Consecutive lanes take
// consecutive 4-column groups of the same row, so every 8-lane phase of a
// 16-byte LDS read touches 32 distinct banks.
template <int K>
__device__ __forceinline__ void coef_row_pass(const float* taps, const float* C, int nrows, float* HM, int band0) {
  using S = AShape<K>;
  constexpr int PLC = S::CH * S::IWP;
  static_assert(kTW / 4 == 16 && kNT == 16 * S::CH, "one row and column group per thread");
  const int r = threadIdx.x >> 4, gq = threadIdx.x & 15;
  if (r >= nrows) return;
  const float* src = C + r * S::IWP + 4 * gq;
  float* dst = HM + (band0 + r) * kTWP + 4 * gq;
#pragma unroll
  for (int m = 0; m < kNM; ++m) {
    float z[4 * S::NREAD];
#pragma unroll
    for (int n = 0; n < S::NREAD; ++n) *(float4*)&z[4 * n] = *(const float4*)&src[m * PLC + 4 * n];
    float h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int t = 0; t < K; ++t) acc = fmaf(taps[t], z[S::LP + j + t], acc);
      h[j] = acc;
    }
    *(float4*)&dst[m * S::PL] = make_float4(h[0], h[1], h[2], h[3]);
  }
}

// The band's last K - 1 rows move to its top (thread t: row t / 16, column
// group t % 16, all planes; the source rows CH.. and the destination rows
// 0..K-2 do not overlap).
template <int K>
__device__ __forceinline__ void coef_band_shift(float* HM) {
  using S = AShape<K>;
  static_assert(S::HALO <= S::CH && kNT == 16 * S::CH, "one row and column group per thread");
  const int row = threadIdx.x >> 4, q = threadIdx.x & 15;
  if (row >= S::HALO) return;
  float4 v[kNM];
#pragma unroll
  for (int m = 0; m < kNM; ++m) v[m] = *(const float4*)&HM[m * S::PL + (S::CH + row) * kTWP + 4 * q];
#pragma unroll
  for (int m = 0; m < kNM; ++m) *(float4*)&HM[m * S::PL + row * kTWP + 4 * q] = v[m];
}

}  // namespace

// LDS of the adjoint tile, declared once per kernel (the tile bodies of one
// kernel share it).  8- and 16-bit planes: the chunk's x, y quads are staged
// through LDS in their own packing (one 4- or 8-byte load per quad); float
// planes are loaded straight into the output stage's layout (one coalesced
// element per lane and row), which frees the 8 KB that would keep them at
// three workgroups per CU (staging 16-bit planes fits four anyway and
// measured faster than direct loads).
template <int K, typename T>
struct AdjSmem {
  static constexpr bool kStage = sizeof(T) <= 2;
  __align__(16) float C[kNM * AShape<K>::CH * AShape<K>::IWP];
  __align__(16) float HM[kNM * AShape<K>::PL];
  __align__(16) uint32_t XY[2][kStage ? AShape<K>::CH * kTW * sizeof(T) / 4 : 1];
};

// The adjoint of one (tile, frame): 64 pixel columns by a.QH pixel rows.
// COARSE: a coarser scale's gradient is added through the 2x2 transpose.  It
// is a separate body because its load in the output stage makes the
// compiler wait there for every older memory operation; without it the
// output stage issues a fixed four stores per chunk (rows past the tile and
// columns past the plane with the dropped offset), and the wait for the next
// chunk's loads at the top of the loop leaves them in flight.
template <int K, typename T, bool COARSE>
__device__ __forceinline__ void fast_adjoint_tile(const FastArgs& a, int frame, int tile, AdjSmem<K, T>& sm) {
  using S = AShape<K>;
  static_assert(S::CH == 16 && kTW == 64 && kNT == 256, "one pixel quad per thread and plane per chunk");
  float* C = sm.C;
  float* HM = sm.HM;
  auto& XY = sm.XY;
  constexpr bool kStage = AdjSmem<K, T>::kStage;
  constexpr int PL = S::PL;
  const int tyi = tile / a.qtiles_x, txi = tile - tyi * a.qtiles_x;
  const int qx0 = __builtin_amdgcn_readfirstlane(txi * kTW), qy0 = __builtin_amdgcn_readfirstlane(tyi * a.QH);
  const int c0 = qx0 - S::HALO - S::LP;
  float taps[K];
#pragma unroll
  for (int t = 0; t < K; ++t) taps[t] = a.taps[t];
  const T* X = (const T*)a.x.data + (int64_t)frame * a.x.bstride;
  const T* Y = (const T*)a.y.data + (int64_t)frame * a.y.bstride;

  // pixel row y reads map rows y-K+1 .. y; prologue = the first K-1 of them
  CQuad q[2];
  fetch_coef<K>(a, frame, qy0 - S::HALO, c0, S::HALO, q);
  store_coef<K>(q, S::HALO, C);
  __syncthreads();
  coef_row_pass<K>(taps, C, S::HALO, HM, 0);
  const int qy_end = __builtin_amdgcn_readfirstlane(min(a.g.H, qy0 + a.QH));
  fetch_coef<K>(a, frame, qy0, c0, S::CH, q);
  fast::Quad<T> px4, py4;
  if constexpr (kStage) fetch_xy<T>(a, X, Y, qy0, qx0, px4, py4);
  if constexpr (!COARSE) {
    // as many dropped stores as a chunk's output stage issues: the loop's
    // entry then has the prefetch as far behind the newest memory operation
    // as every later iteration (distinct offsets, so none is merged)
#pragma unroll
    for (int i = 0; i < 4; ++i) store_row_f32(nullptr, kStoreDrop + 4u * i, 0.f);
  }
  const int gr = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), c = threadIdx.x & 63;
  const int px = qx0 + c;
  const uint32_t lane_off = px < a.g.W ? 4u * (uint32_t)c : kStoreDrop;
  for (int cy = qy0; cy < qy_end; cy += S::CH) {
    __syncthreads();
    store_coef<K>(q, S::CH, C);
    T xd[4], yd[4];  // direct path: this chunk's pixels of the lane's output column
    if constexpr (kStage) {
#pragma unroll
      for (int w = 0; w < fast::Quad<T>::NW; ++w) {
        XY[0][threadIdx.x * fast::Quad<T>::NW + w] = px4.w[w];
        XY[1][threadIdx.x * fast::Quad<T>::NW + w] = py4.w[w];
      }
    } else {
      // issued here so that the row pass hides their latency
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int py = cy + 4 * gr + j;  // wave-uniform
        xd[j] = T{};
        yd[j] = T{};
        if (py < qy_end && px < a.g.W) {
          xd[j] = (X + (int64_t)py * a.x.pitch)[px];
          yd[j] = (Y + (int64_t)py * a.y.pitch)[px];
        }
      }
    }
    // the next chunk's quads are loaded while this chunk's row and column
    // passes run (the registers were just staged)
    if (cy + S::CH < qy_end) {
      fetch_coef<K>(a, frame, cy + S::CH, c0, S::CH, q);
      if constexpr (kStage) fetch_xy<T>(a, X, Y, cy + S::CH, qx0, px4, py4);
    }
    __syncthreads();
    coef_row_pass<K>(taps, C, S::CH, HM, S::HALO);
    __syncthreads();
    // item = (4 pixel rows, 1 column), one per thread; wave w takes rows
    // cy + 4 w .. cy + 4 w + 3, so every output row base is wave-uniform
    static_assert((S::CH / 4) * kTW == kNT, "one column-pass item per thread, one row group per wave");
    {
      float G[kNM][4];
#pragma unroll
      for (int m = 0; m < kNM; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) G[m][j] = 0.f;
#pragma unroll
      for (int r = 0; r < K + 3; ++r) {
        float h[kNM];
#pragma unroll
        for (int m = 0; m < kNM; ++m) h[m] = HM[m * PL + (4 * gr + r) * kTWP + c];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int t = r - j;
          if (t >= 0 && t < K) {
#pragma unroll
            for (int m = 0; m < kNM; ++m) G[m][j] = fmaf(taps[t], h[m], G[m][j]);
          }
        }
      }
      // elements read back by byte copies (well defined for any element type)
      const char* xs = (const char*)XY[0];
      const char* ys = (const char*)XY[1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int py = cy + 4 * gr + j;  // wave-uniform
        if constexpr (COARSE)
          if (py >= qy_end || px >= a.g.W) continue;
        T xe, ye;
        if constexpr (kStage) {
          // staged row 4 gr + j, column c (quads are stored row-major, 16 per row)
          const int e = ((4 * gr + j) * kTW + c) * (int)sizeof(T);
          __builtin_memcpy(&xe, xs + e, sizeof(T));
          __builtin_memcpy(&ye, ys + e, sizeof(T));
        } else {
          xe = xd[j];
          ye = yd[j];
        }
        const float xv = to_f32<T>(xe), yv = to_f32<T>(ye);
        // dL/dy = W^T A + (u - t_u) W^T B_u - (v - t_v) W^T B_v
        float gy = fmaf((xv + yv) - a.tu, G[1][j], G[0][j]) - ((xv - yv) - a.tv) * G[2][j];
        if constexpr (COARSE) {
          const int cyy = py >> 1, cxx = px >> 1;
          if (cyy < a.Hc && cxx < a.Wc) {
            const char* crow = (const char*)(a.coarse + ((int64_t)frame * a.Hc + cyy) * a.Wc);
            gy += 0.25f * *(const float*)(crow + 4u * (uint32_t)cxx);
          }
        }
        const uint32_t off = lane_off | (py < qy_end ? 0u : kStoreDrop);
        store_row_f32(a.out + (int64_t)frame * a.out_bstride + (int64_t)min(py, qy_end - 1) * a.out_pitch + qx0, off, gy);
      }
    }
    __syncthreads();
    coef_band_shift<K>(HM);
  }
}

template <int K, typename T>
__global__ __launch_bounds__(kNT, 4) void fast_adjoint_kernel(FastArgs a) {
  __shared__ AdjSmem<K, T> sm;
  int tile, frame;
  xcd_tile_rows_last(a.qtiles_x, a.qtiles_y, tile, frame);
  if (a.coarse) fast_adjoint_tile<K, T, true>(a, frame, tile, sm);
  else fast_adjoint_tile<K, T, false>(a, frame, tile, sm);
}

template <int K>
__global__ __launch_bounds__(kNT, 4) void fast_adjoint_segs_kernel(FastSegs m) {
  const int s = seg_of(m.start, m.n);
  const FastArgs& a = m.seg[s];
  int tile, frame;
  __shared__ AdjSmem<K, float> sm;
  seg_tile(m.start, s, a.qtiles_x * a.qtiles_y, tile, frame);
  if (a.coarse) fast_adjoint_tile<K, float, true>(a, frame, tile, sm);
  else fast_adjoint_tile<K, float, false>(a, frame, tile, sm);
}

// ---------------------------------------------------------------- dispatch
template <int K>
static int launch_adj_k(int dtype, const FastArgs& a, dim3 grid, hipStream_t st) {
  switch (dtype) {
    case SSIMX_U8: hipLaunchKernelGGL((fast_adjoint_kernel<K, uint8_t>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_U16: hipLaunchKernelGGL((fast_adjoint_kernel<K, uint16_t>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_F32: hipLaunchKernelGGL((fast_adjoint_kernel<K, float>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_BF16: hipLaunchKernelGGL((fast_adjoint_kernel<K, bf16_t>), grid, dim3(kNT), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_fast_adjoint(int dtype, const FastArgs& a, int batch, hipStream_t st) {
  dim3 grid(a.qtiles_x * a.qtiles_y, batch);
  switch (a.g.k) {
    case 7: return launch_adj_k<7>(dtype, a, grid, st);
    case 9: return launch_adj_k<9>(dtype, a, grid, st);
    case 11: return launch_adj_k<11>(dtype, a, grid, st);
    case 13: return launch_adj_k<13>(dtype, a, grid, st);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_fast_adjoint_segs(const FastSegs& s, hipStream_t st) {
  if (s.n < 1 || s.n > kMaxSegs) return (int)hipErrorInvalidValue;
  const dim3 grid(s.start[s.n]);
  switch (s.seg[0].g.k) {
    case 7: hipLaunchKernelGGL((fast_adjoint_segs_kernel<7>), grid, dim3(kNT), 0, st, s); break;
    case 9: hipLaunchKernelGGL((fast_adjoint_segs_kernel<9>), grid, dim3(kNT), 0, st, s); break;
    case 11: hipLaunchKernelGGL((fast_adjoint_segs_kernel<11>), grid, dim3(kNT), 0, st, s); break;
    case 13: hipLaunchKernelGGL((fast_adjoint_segs_kernel<13>), grid, dim3(kNT), 0, st, s); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // namespace ssimx
