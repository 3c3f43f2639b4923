// Spatial pooling of quality maps (Spatial and Temporal Aggregation section):
// mean, coefficient of variation, mean deviation, Minkowski and
// distortion-weighted pooling as sums over the map, and the five-number
// summary and percentile pooling from exact order statistics.
//
// Sums: each block takes map rows round-robin and accumulates up to two
// float64 sums per frame; a finishing kernel adds the block sums of a frame in
// a fixed order (deterministic) and forms the pooled value.
//
// Order statistics: radix select on the order-preserving uint32 image of the
// float map values, 8 bits per pass from the top.  Per pass every block
// histograms the keys that match each target's prefix in LDS and adds its
// histogram to the frame's global histogram; a step kernel then picks, per
// target, the bin that holds the wanted rank, extends the prefix and clears
// the histogram for the next pass.  After four passes the prefix is the exact
// key of the order statistic.
#include "launch.hpp"
#include "ssimx_internal.hpp"
#include "host_common.hpp"

#include <math.h>

namespace ssimx {

namespace {

constexpr int kPoolNT = 256;
constexpr int kMaxTargets = 8;

// Per-frame selection state, kStateWords uint32 words: the targets' key
// prefixes and remaining ranks, the histogram slot of each target, and the
// distinct prefixes (one histogram each).  Distinct prefixes of the same
// length select disjoint key sets, so every key adds to at most one histogram.
constexpr int kStateWords = 64;
constexpr int kPre = 0, kRank = 8, kSlot = 16, kUniq = 24, kNUniq = 32;

struct MapArg {
  const float* map;
  int w, h;
  int64_t pitch, bstride;
};

__device__ __forceinline__ uint32_t ordered_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// d^p for d >= 0: repeated products for small integer p, else powf.
__device__ __forceinline__ double pow_term(double d, double p, int ip) {
  if (ip >= 0) {
    double r = 1.0;
    for (int i = 0; i < ip; ++i) r *= d;
    return r;
  }
  return (double)powf((float)d, (float)p);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// kind: 0 sum Q | 1 sum Q, Q^2 | 2 sum |Q - mu|^p | 3 sum (1-Q)^p | 4 sum (1-Q)^p Q, (1-Q)^p
// | 5 sum of Q below the per-frame threshold, and their count | 6 sum log Q | 7 sum 1/Q over
// the non-zero values, and the number of zeros
// Calls f(v) on every value of the frame rows blockIdx.x, blockIdx.x +
// gridDim.x, ...; thread t takes columns t, t + NT, ... of a row in that order,
// with eight loads in flight before their values are used.
template <class F>
__device__ __forceinline__ void for_each_value(const MapArg& a, const float* m, F& f) {
  for (int r = blockIdx.x; r < a.h; r += gridDim.x) {
    const float* row = m + (int64_t)r * a.pitch;
    for (int c0 = threadIdx.x; c0 < a.w; c0 += 8 * kPoolNT) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = c0 + j * kPoolNT < a.w ? row[c0 + j * kPoolNT] : 0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (c0 + j * kPoolNT < a.w) f(v[j]);
    }
  }
}

__global__ __launch_bounds__(kPoolNT) void pool_sums_kernel(MapArg a, int kind, double p, int ip, const double* mu,
                                                            const uint32_t* thr_key, double* partial) {
  __shared__ double red[2][kPoolNT / 64];
  const int frame = blockIdx.y;
  const float* m = a.map + (int64_t)frame * a.bstride;
  const double muf = mu ? mu[frame] : 0.0;
  const uint32_t tk = thr_key ? thr_key[(int64_t)frame * kStateWords + kPre] : 0u;  // target 0's key
  double s0 = 0.0, s1 = 0.0;
  auto acc = [&](float qf) {
    const double q = (double)qf;
    switch (kind) {
      case 0: s0 += q; break;
      case 1: s0 += q; s1 += q * q; break;
      case 2: s0 += pow_term(fabs(q - muf), p, ip); break;
      case 3: s0 += pow_term(1.0 - q, p, ip); break;
      case 4: {
        const double wgt = pow_term(1.0 - q, p, ip);
        s0 += wgt * q;
        s1 += wgt;
        break;
      }
      case 5:  // below the m-th smallest value of the frame
        if (ordered_key(qf) < tk) {
          s0 += q;
          s1 += 1.0;
        }
        break;
      case 6: s0 += (double)logf(qf); break;
      default:  // reciprocals; zeros (of either sign) are counted instead
        if (q == 0.0)
          s1 += 1.0;
        else
          s0 += 1.0 / q;
        break;
    }
  };
  for_each_value(a, m, acc);
  s0 = wave_sum_d(s0);
  s1 = wave_sum_d(s1);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wid] = s0;
    red[1][wid] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int w = 0; w < kPoolNT / 64; ++w) {
      t0 += red[0][w];
      t1 += red[1][w];
    }
    double* o = partial + ((int64_t)frame * gridDim.x + blockIdx.x) * 2;
    o[0] = t0;
    o[1] = t1;
  }
}

// Fixed-order sum of a frame's block sums.
__device__ __forceinline__ void frame_sums(const double* partial, int nblk, int frame, double& s0, double& s1) {
  s0 = s1 = 0.0;
  const double* p = partial + (int64_t)frame * nblk * 2;
  for (int b = 0; b < nblk; ++b) {
    s0 += p[2 * b];
    s1 += p[2 * b + 1];
  }
}

struct FinishArgs {
  int kind;      // ssimx_pool_kind
  int stage;     // 0: final value; 1: store mu (first pass of the mean deviation)
  double p, o, r;
  double n;
  int m;         // percentile pooling: number of values divided by r
  int nt;        // order-statistic targets
  double frac[kMaxTargets];  // interpolation weights for the five-number summary
};

__global__ void pool_finish_kernel(const double* partial, const double* total, int nblk, int batch, FinishArgs f,
                                   const uint32_t* keys, double* mu_out, float* out, int64_t out_stride) {
  const int frame = blockIdx.x * blockDim.x + threadIdx.x;
  if (frame >= batch) return;
  double s0 = 0.0, s1 = 0.0;
  if (partial) frame_sums(partial, nblk, frame, s0, s1);
  double v = 0.0;
  switch (f.kind) {
    case SSIMX_POOL_MEAN: v = s0 / f.n; break;
    case SSIMX_POOL_COV: {
      const double mean = s0 / f.n;
      const double var = fmax(s1 / f.n - mean * mean, 0.0);
      v = sqrt(var) / mean;
      break;
    }
    case SSIMX_POOL_MEAN_DEV:
      if (f.stage == 1) {
        mu_out[frame] = s0 / f.n;
        return;
      }
      v = pow(pow(s0 / f.n, 1.0 / f.p), f.o);
      break;
    case SSIMX_POOL_MINKOWSKI: v = s0 / f.n; break;
    case SSIMX_POOL_DIST_WEIGHTED: v = s1 == 0.0 ? 1.0 : s0 / s1; break;
    case SSIMX_POOL_FIVE_NUMBER: {
      const uint32_t* k = keys + (int64_t)frame * kStateWords + kPre;  // selected keys
      double q[kMaxTargets];
      for (int t = 0; t < f.nt; ++t) q[t] = (double)key_value(k[t]);
      // targets: min, max, then (lo, hi) pairs of Q1, median, Q3
      double acc = q[0] + q[1];
      for (int j = 0; j < 3; ++j) acc += q[2 + 2 * j] + f.frac[j] * (q[3 + 2 * j] - q[2 + 2 * j]);
      v = acc / 5.0;
      break;
    }
    case SSIMX_POOL_GEOMETRIC: v = exp(s0 / f.n); break;
    case SSIMX_POOL_HARMONIC: v = s1 > 0.0 ? 0.0 : f.n / s0; break;
    case SSIMX_POOL_MEDIAN: {
      const uint32_t* k = keys + (int64_t)frame * kStateWords + kPre;
      const double lo = (double)key_value(k[0]), hi = (double)key_value(k[1]);
      v = lo + f.frac[0] * (hi - lo);
      break;
    }
    case SSIMX_POOL_PERCENTILE: {
      double tot = 0.0, tmp = 0.0;
      frame_sums(total, nblk, frame, tot, tmp);
      if (f.m == 0) {
        v = tot / f.n;
      } else {
        const double thr = (double)key_value(keys[(int64_t)frame * kStateWords + kPre]);
        // s0 = sum of the values strictly below the m-th smallest, s1 = their count
        const double low = s0 + ((double)f.m - s1) * thr;
        v = (low / f.r + (tot - low)) / f.n;
      }
      break;
    }
    default: v = 0.0; break;
  }
  out[(int64_t)frame * out_stride] = (float)v;
}

// ---------------------------------------------------------------- radix select
struct SelArgs {
  MapArg a;
  int nt;
  uint32_t* state;  // [batch][kStateWords]
  uint32_t* hist;   // [batch][kMaxTargets][256]
};

struct Ranks {
  uint32_t r[kMaxTargets];
};

__global__ void sel_init_kernel(SelArgs s, int batch, Ranks ranks) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch * kMaxTargets * 256) s.hist[i] = 0u;
  if (i < batch) {
    uint32_t* st = s.state + (int64_t)i * kStateWords;
    for (int t = 0; t < kMaxTargets; ++t) {
      st[kPre + t] = 0u;
      st[kRank + t] = ranks.r[t];
      st[kSlot + t] = 0u;
      st[kUniq + t] = 0u;
    }
    st[kNUniq] = 1u;
  }
}

// Adds `cnt` to LDS bin `idx` (skipped for idx < 0).
__device__ __forceinline__ void flush_run(uint32_t* h, int idx, uint32_t cnt) {
  if (idx >= 0) atomicAdd(&h[idx], cnt);
}

__global__ __launch_bounds__(kPoolNT) void sel_hist_kernel(SelArgs s, int shift) {
  __shared__ uint32_t h[kMaxTargets * 256];
  const int frame = blockIdx.y;
  const uint32_t* st = s.state + (int64_t)frame * kStateWords;
  for (int i = threadIdx.x; i < kMaxTargets * 256; i += kPoolNT) h[i] = 0u;
  const uint32_t himask = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
  // The distinct prefixes are the same for the whole block: held in registers
  // and matched by a fixed compare-select. Unused slots hold a word whose low
  // (shift + 8) bits are set, which no masked key equals.
  const int nu = (int)st[kNUniq];
  uint32_t pm[kMaxTargets];
#pragma unroll
  for (int u = 0; u < kMaxTargets; ++u) pm[u] = u < nu ? (st[kUniq + u] & himask) : 0xffffffffu;
  __syncthreads();
  const float* m = s.a.map + (int64_t)frame * s.a.bstride;
  // Neighbouring map values are strongly correlated, so runs of equal bins in
  // a thread's keys are merged before they reach the (contended) LDS bins.
  int cur = -1;
  uint32_t cnt = 0u;
  auto add = [&](float v) {
    const uint32_t k = ordered_key(v);
    const uint32_t kp = k & himask;
    int base = -1;
#pragma unroll
    for (int u = 0; u < kMaxTargets; ++u) base = kp == pm[u] ? u * 256 : base;
    const int idx = base < 0 ? -1 : base + (int)((k >> shift) & 255u);
    if (idx != cur) {
      flush_run(h, cur, cnt);
      cur = idx;
      cnt = 0u;
    }
    ++cnt;
  };
  for_each_value(s.a, m, add);
  flush_run(h, cur, cnt);
  __syncthreads();
  uint32_t* g = s.hist + (int64_t)frame * kMaxTargets * 256;
  for (int i = threadIdx.x; i < nu * 256; i += kPoolNT) {
    const uint32_t v = h[i];
    if (v) atomicAdd(&g[i], v);
  }
}

// One block of 256 threads per frame, one thread per bin: scan each distinct
// prefix's histogram, extend the prefix of every target that uses it by the
// bin holding its remaining rank, clear the histogram, then regroup the new
// prefixes into distinct histograms for the next pass.
__global__ __launch_bounds__(256) void sel_step_kernel(SelArgs s, int shift) {
  __shared__ uint32_t wtot[4];
  __shared__ uint32_t npre[kMaxTargets], nrank[kMaxTargets];
  const int frame = blockIdx.x, b = threadIdx.x, lane = b & 63, wid = b >> 6;
  uint32_t* st = s.state + (int64_t)frame * kStateWords;
  uint32_t* g = s.hist + (int64_t)frame * kMaxTargets * 256;
  const int nu = (int)st[kNUniq];
  if (b < s.nt) {  // fallback, replaced below by the thread whose bin holds the rank
    npre[b] = st[kPre + b] | (255u << shift);
    nrank[b] = st[kRank + b];
  }
  __syncthreads();
  for (int u = 0; u < nu; ++u) {
    const uint32_t c = g[u * 256 + b];
    uint32_t v = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (lane == 63) wtot[wid] = v;
    __syncthreads();
    for (int w = 0; w < wid; ++w) v += wtot[w];
    const uint32_t incl = v, excl = v - c;
    for (int t = 0; t < s.nt; ++t) {
      if ((int)st[kSlot + t] != u) continue;
      const uint32_t r = st[kRank + t];
      if (r >= excl && r < incl) {
        npre[t] = st[kPre + t] | ((uint32_t)b << shift);
        nrank[t] = r - excl;
      }
    }
    g[u * 256 + b] = 0u;
    __syncthreads();
  }
  if (b == 0) {
    uint32_t uqv[kMaxTargets];
    int n = 0;
    for (int t = 0; t < s.nt; ++t) {
      int j = 0;
      while (j < n && uqv[j] != npre[t]) ++j;
      if (j == n) uqv[n++] = npre[t];
      st[kPre + t] = npre[t];
      st[kRank + t] = nrank[t];
      st[kSlot + t] = (uint32_t)j;
    }
    for (int j = 0; j < n; ++j) st[kUniq + j] = uqv[j];
    st[kNUniq] = (uint32_t)n;
  }
}

// Windowed means of a single-row map (a series of frame scores): one block
// per series, thread t takes the windows t, t + NT, ...; every window value is
// summed directly in float64, then the block adds its windows in a fixed order.
// mean: 0 AM | 1 GM | 2 HM | 3 CoV.
__global__ __launch_bounds__(kPoolNT) void pool_window_kernel(MapArg a, int win, int mean, float* out,
                                                              int64_t out_stride) {
  __shared__ double red[kPoolNT / 64];
  const int frame = blockIdx.x;
  const float* s = a.map + (int64_t)frame * a.bstride;
  const int nw = a.w - win + 1;
  double acc = 0.0;
  for (int t = threadIdx.x; t < nw; t += kPoolNT) {
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < win; ++i) {
      const float vf = s[t + i];
      const double v = (double)vf;
      if (mean == 0) {
        s1 += v;
      } else if (mean == 1) {
        s1 += (double)logf(vf);
      } else if (mean == 2) {
        if (v == 0.0)
          s2 += 1.0;  // zeros counted
        else
          s1 += 1.0 / v;
      } else {
        s1 += v;
        s2 += v * v;
      }
    }
    double r;
    if (mean == 0) {
      r = s1 / win;
    } else if (mean == 1) {
      r = exp(s1 / win);
    } else if (mean == 2) {
      r = s2 > 0.0 ? 0.0 : win / s1;
    } else {
      const double mu = s1 / win;
      r = sqrt(fmax(s2 / win - mu * mu, 0.0)) / mu;
    }
    acc += r;
  }
  acc = wave_sum_d(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kPoolNT / 64; ++w) t += red[w];
    out[(int64_t)frame * out_stride] = (float)(t / nw);
  }
}

bool windowed(int kind) { return kind >= SSIMX_POOL_WIN_AM && kind <= SSIMX_POOL_WIN_COV; }

bool order_stat(int kind) {
  return kind == SSIMX_POOL_FIVE_NUMBER || kind == SSIMX_POOL_PERCENTILE || kind == SSIMX_POOL_MEDIAN;
}

int blocks_per_frame(int h) { return h < 64 ? h : 64; }

}  // namespace

size_t pool_ws_bytes(const ssimx_pool* pl, int w, int h, int batch) {
  (void)w;
  Ws ws;
  const int nblk = blocks_per_frame(h);
  ws.take(sizeof(double) * 2 * (size_t)batch * nblk);  // block sums
  ws.take(sizeof(double) * 2 * (size_t)batch * nblk);  // second set (totals)
  ws.take(sizeof(double) * (size_t)batch);              // per-frame mean
  if (order_stat(pl->kind)) {
    ws.take(sizeof(uint32_t) * kStateWords * (size_t)batch);
    ws.take(sizeof(uint32_t) * 256 * kMaxTargets * (size_t)batch);
  }
  return ws.used;
}

ssimx_status check_pool(const ssimx_pool* pl) {
  if (!pl) return SSIMX_EINVAL;
  if (!isfinite(pl->p) || !isfinite(pl->o) || !isfinite(pl->r)) return SSIMX_EINVAL;
  switch (pl->kind) {
    case SSIMX_POOL_MEAN:
    case SSIMX_POOL_COV:
    case SSIMX_POOL_FIVE_NUMBER: return SSIMX_OK;
    case SSIMX_POOL_MEAN_DEV: return pl->p > 0.0 ? SSIMX_OK : SSIMX_EINVAL;
    case SSIMX_POOL_MINKOWSKI: return pl->p > 0.0 ? SSIMX_OK : SSIMX_EINVAL;
    case SSIMX_POOL_DIST_WEIGHTED: return pl->p >= 0.0 ? SSIMX_OK : SSIMX_EINVAL;
    case SSIMX_POOL_PERCENTILE: return (pl->p >= 0.0 && pl->p <= 100.0 && pl->r > 0.0) ? SSIMX_OK : SSIMX_EINVAL;
    case SSIMX_POOL_GEOMETRIC:
    case SSIMX_POOL_HARMONIC:
    case SSIMX_POOL_MEDIAN: return SSIMX_OK;
    case SSIMX_POOL_WIN_AM:
    case SSIMX_POOL_WIN_GM:
    case SSIMX_POOL_WIN_HM:
    case SSIMX_POOL_WIN_COV: return (pl->p >= 1.0 && pl->p == floor(pl->p) && pl->p < 2147483648.0) ? SSIMX_OK
                                                                                                  : SSIMX_EINVAL;
    default: return SSIMX_EINVAL;
  }
}

static int int_power(double p) {
  return (p == floor(p) && p >= 0.0 && p <= 16.0) ? (int)p : -1;
}

ssimx_status pool_run(const ssimx_pool* pl, const float* map, int w, int h, int64_t pitch, int64_t bstride,
                      int batch, float* out, int64_t out_stride, void* ws, hipStream_t st) {
  const int nblk = blocks_per_frame(h);
  Ws lay;
  double* partial = (double*)((char*)ws + lay.take(sizeof(double) * 2 * (size_t)batch * nblk));
  double* total = (double*)((char*)ws + lay.take(sizeof(double) * 2 * (size_t)batch * nblk));
  double* mu = (double*)((char*)ws + lay.take(sizeof(double) * (size_t)batch));
  MapArg a{map, w, h, pitch, bstride};
  const double n = (double)w * (double)h;
  FinishArgs f{};
  f.kind = pl->kind;
  f.p = pl->p;
  f.o = pl->o;
  f.r = pl->r;
  f.n = n;
  const dim3 grid(nblk, batch), fin((batch + 63) / 64);
  const int ip = int_power(pl->p);
  int err = 0;
  switch (pl->kind) {
    case SSIMX_POOL_WIN_AM:
    case SSIMX_POOL_WIN_GM:
    case SSIMX_POOL_WIN_HM:
    case SSIMX_POOL_WIN_COV:
      hipLaunchKernelGGL(pool_window_kernel, dim3(batch), dim3(kPoolNT), 0, st, a, (int)pl->p,
                         (int)pl->kind - SSIMX_POOL_WIN_AM, out, out_stride);
      break;
    case SSIMX_POOL_MEAN:
    case SSIMX_POOL_COV:
    case SSIMX_POOL_MINKOWSKI:
    case SSIMX_POOL_DIST_WEIGHTED:
    case SSIMX_POOL_GEOMETRIC:
    case SSIMX_POOL_HARMONIC: {
      const int k = pl->kind == SSIMX_POOL_MEAN ? 0 : pl->kind == SSIMX_POOL_COV ? 1
                  : pl->kind == SSIMX_POOL_MINKOWSKI ? 3 : pl->kind == SSIMX_POOL_DIST_WEIGHTED ? 4
                  : pl->kind == SSIMX_POOL_GEOMETRIC ? 6 : 7;
      hipLaunchKernelGGL(pool_sums_kernel, grid, dim3(kPoolNT), 0, st, a, k, pl->p, ip, nullptr, nullptr, partial);
      hipLaunchKernelGGL(pool_finish_kernel, fin, dim3(64), 0, st, partial, nullptr, nblk, batch, f, nullptr, nullptr,
                         out, out_stride);
      break;
    }
    case SSIMX_POOL_MEAN_DEV: {
      hipLaunchKernelGGL(pool_sums_kernel, grid, dim3(kPoolNT), 0, st, a, 0, 0.0, 1, nullptr, nullptr, partial);
      f.stage = 1;
      hipLaunchKernelGGL(pool_finish_kernel, fin, dim3(64), 0, st, partial, nullptr, nblk, batch, f, nullptr, mu,
                         out, out_stride);
      hipLaunchKernelGGL(pool_sums_kernel, grid, dim3(kPoolNT), 0, st, a, 2, pl->p, ip, mu, nullptr, partial);
      f.stage = 0;
      hipLaunchKernelGGL(pool_finish_kernel, fin, dim3(64), 0, st, partial, nullptr, nblk, batch, f, nullptr, nullptr,
                         out, out_stride);
      break;
    }
    default: {  // order statistics
      uint32_t* state = (uint32_t*)((char*)ws + lay.take(sizeof(uint32_t) * kStateWords * (size_t)batch));
      uint32_t* hist = (uint32_t*)((char*)ws + lay.take(sizeof(uint32_t) * 256 * kMaxTargets * (size_t)batch));
      uint32_t ranks[kMaxTargets] = {};
      const uint32_t last = (uint32_t)(w * (int64_t)h - 1);
      int nt = 0;
      if (pl->kind == SSIMX_POOL_FIVE_NUMBER) {
        ranks[0] = 0;
        ranks[1] = last;
        const double qs[3] = {0.25, 0.5, 0.75};
        for (int j = 0; j < 3; ++j) {
          const double hpos = (double)last * qs[j];
          const uint32_t lo = (uint32_t)floor(hpos);
          ranks[2 + 2 * j] = lo;
          ranks[3 + 2 * j] = lo < last ? lo + 1 : lo;
          f.frac[j] = hpos - (double)lo;
        }
        nt = 8;
      } else if (pl->kind == SSIMX_POOL_MEDIAN) {
        const double hpos = (double)last * 0.5;
        const uint32_t lo = (uint32_t)floor(hpos);
        ranks[0] = lo;
        ranks[1] = lo < last ? lo + 1 : lo;
        f.frac[0] = hpos - (double)lo;
        nt = 2;
      } else {
        f.m = (int)ceil(pl->p * n / 100.0);
        if (f.m > (int)(last + 1)) f.m = (int)(last + 1);
        ranks[0] = f.m > 0 ? (uint32_t)(f.m - 1) : 0u;
        nt = 1;
      }
      f.nt = nt;
      SelArgs s{a, nt, state, hist};
      const int ninit = batch * kMaxTargets * 256;
      Ranks rk{};
      for (int t = 0; t < kMaxTargets; ++t) rk.r[t] = ranks[t];
      hipLaunchKernelGGL(sel_init_kernel, dim3((ninit + 255) / 256), dim3(256), 0, st, s, batch, rk);
      for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(sel_hist_kernel, grid, dim3(kPoolNT), 0, st, s, shift);
        hipLaunchKernelGGL(sel_step_kernel, dim3(batch), dim3(256), 0, st, s, shift);
      }
      if (pl->kind == SSIMX_POOL_PERCENTILE) {
        // totals, then the sum and count of the values below the threshold
        hipLaunchKernelGGL(pool_sums_kernel, grid, dim3(kPoolNT), 0, st, a, 0, 0.0, 1, nullptr, nullptr, total);
        hipLaunchKernelGGL(pool_sums_kernel, grid, dim3(kPoolNT), 0, st, a, 5, 0.0, 1, nullptr, state, partial);
      }
      hipLaunchKernelGGL(pool_finish_kernel, fin, dim3(64), 0, st,
                         pl->kind == SSIMX_POOL_PERCENTILE ? partial : nullptr, total, nblk, batch, f, state, nullptr,
                         out, out_stride);
      break;
    }
  }
  err = (int)hipGetLastError();
  return hip_status(err);
}

}  // namespace ssimx

using namespace ssimx;

extern "C" {

ssimx_status ssimx_pool_workspace_size(const ssimx_pool* pool, int w, int h, int batch, size_t* bytes) {
  ssimx_status s;
  if ((s = check_pool(pool)) != SSIMX_OK) return s;
  if (!bytes || batch < 1 || batch > kMaxGridY) return SSIMX_EINVAL;
  if (w < 1 || h < 1) return SSIMX_ETOOSMALL;
  *bytes = pool_ws_bytes(pool, w, h, batch);
  return SSIMX_OK;
}

ssimx_status ssimx_pool_map(const ssimx_pool* pool, const float* map, int w, int h, long long pitch,
                            long long batch_stride, int batch, float* out, void* ws, size_t ws_bytes, void* stream) {
  ssimx_status s;
  if ((s = check_pool(pool)) != SSIMX_OK) return s;
  if (!map || !out || batch < 1 || batch > kMaxGridY) return SSIMX_EINVAL;
  if (w < 1 || h < 1) return SSIMX_ETOOSMALL;
  if (pitch < w || (batch > 1 && batch_stride < pitch * (long long)h)) return SSIMX_EINVAL;
  if ((long long)w * h >= (1ll << 31)) return SSIMX_ENOTSUP;
  if (windowed(pool->kind)) {
    if (h != 1) return SSIMX_EINVAL;
    if (pool->p > (double)w) return SSIMX_ETOOSMALL;
  }
  if (!ws || ws_bytes < pool_ws_bytes(pool, w, h, batch)) return SSIMX_EWORKSPACE;
  return pool_run(pool, map, w, h, pitch, batch_stride, batch, out, 1, ws, (hipStream_t)stream);
}

}  // extern "C"
