// Tile-shape autotuner for the forward kernels and its process-wide cache.
//
// A cache entry maps (architecture, dtype, window, k, stride, padding, algo,
// width x height, batch class) to the index of the fastest tile shape.  The
// cache is filled by ssimx_autotune (timed with HIP events on the caller's
// stream) or loaded from a JSON file, and read by every later call.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "launch.hpp"
#include "host_common.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {

// Timing frames: independent pseudo-random samples over the dtype's range
// (8-bit full range, 16-bit 10-bit video range, floats in [0, 1)), from the
// lowbias32 integer hash of the element index, so that candidates are timed
// on data with the value spread of real frames rather than on constants.
__device__ __forceinline__ uint32_t tune_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(BLOCK) void tune_fill_kernel(void* out, int dtype, size_t n, uint32_t seed) {
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * BLOCK) {
    const uint32_t h = tune_hash((uint32_t)i * 0x9e3779b9u + seed);
    switch (dtype) {
      case SSIMX_U8: ((uint8_t*)out)[i] = (uint8_t)(h >> 24); break;
      case SSIMX_U16: ((uint16_t*)out)[i] = (uint16_t)(h >> 22); break;
      case SSIMX_F32: ((float*)out)[i] = (float)(h >> 8) * (1.f / 16777216.f); break;
      default: ((uint16_t*)out)[i] = (uint16_t)(__float_as_uint((float)(h >> 8) * (1.f / 16777216.f)) >> 16); break;
    }
  }
}

static int tune_fill(void* out, int dtype, size_t n, uint32_t seed, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + BLOCK - 1) / BLOCK, 4096);
  hipLaunchKernelGGL(tune_fill_kernel, dim3(std::max(1u, blocks)), dim3(BLOCK), 0, st, out, dtype, n, seed);
  return (int)hipGetLastError();
}

static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune_cache;
static int g_tile_override = -1;

static int batch_class(int batch) {
  int c = 0;
  while ((1 << c) < batch && c < 20) ++c;
  return c;
}

static std::string tune_key(const ssimx_params* p, int dtype, int W, int H, int batch) {
  char buf[192];
  snprintf(buf, sizeof(buf), "gfx950|dt%d|win%d|k%d|s%d|pad%d|algo%d|%dx%d|b%d", dtype, p->window, p->k, p->stride,
           p->padding, p->algo, W, H, batch_class(batch));
  return buf;
}

// ---- cache file: the JSON object the save call writes,
//   {"version": <int>, "entries": {"<key>": <tile index>, ...}}
// read by a strict recursive-descent parser: whitespace anywhere between
// tokens, keys are plain strings (printable ASCII, no quote or backslash,
// at most 191 bytes), values decimal integers naming a tile configuration,
// "version" must equal SSIMX_VERSION, nothing may follow the object.  A file
// that breaks any rule loads nothing.
constexpr size_t kCacheMaxBytes = 1 << 20;

namespace {

struct CacheParser {
  const std::string& t;
  size_t i = 0;
  void ws() {
    while (i < t.size() && (t[i] == ' ' || t[i] == '\t' || t[i] == '\n' || t[i] == '\r')) ++i;
  }
  bool lit(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    if (!lit('"')) return false;
    out.clear();
    while (i < t.size() && t[i] != '"') {
      const unsigned char c = (unsigned char)t[i];
      if (c < 0x20 || c > 0x7e || c == '\\' || out.size() >= 191) return false;
      out.push_back((char)c);
      ++i;
    }
    if (i >= t.size()) return false;
    ++i;  // closing quote
    return true;
  }
  bool integer(long& v) {
    ws();
    const size_t b = i;
    if (i < t.size() && t[i] == '-') ++i;
    const size_t d = i;
    while (i < t.size() && t[i] >= '0' && t[i] <= '9' && i - d < 9) ++i;
    if (i == d || (i < t.size() && t[i] >= '0' && t[i] <= '9')) return false;  // no digits, or too many
    v = strtol(t.c_str() + b, nullptr, 10);
    return true;
  }
};

}  // namespace

static bool parse_cache(const std::string& text, std::map<std::string, int>& out) {
  CacheParser P{text};
  if (!P.lit('{')) return false;
  bool have_version = false, have_entries = false;
  std::string key;
  do {
    if (!P.str(key) || !P.lit(':')) return false;
    if (key == "version") {
      long v;
      if (have_version || !P.integer(v) || v != SSIMX_VERSION) return false;
      have_version = true;
    } else if (key == "entries") {
      if (have_entries || !P.lit('{')) return false;
      have_entries = true;
      if (!P.lit('}')) {
        do {
          long v;
          if (!P.str(key) || !P.lit(':') || !P.integer(v)) return false;
          if (v < 0 || v >= num_tile_cfgs() || out.count(key)) return false;
          out[key] = (int)v;
        } while (P.lit(','));
        if (!P.lit('}')) return false;
      }
    } else {
      return false;
    }
  } while (P.lit(','));
  if (!P.lit('}') || !have_version || !have_entries) return false;
  P.ws();
  return P.i == text.size();
}

// SSIMX_TUNE_CACHE names a cache file: it is loaded once, before the first
// tile choice or autotune call of the process (a missing or malformed file
// loads nothing), and every autotune call writes the whole cache back to it.
static std::once_flag g_env_once;

static const char* env_cache_path() {
  const char* e = getenv("SSIMX_TUNE_CACHE");
  return (e && *e) ? e : nullptr;
}

static void load_env_cache() {
  std::call_once(g_env_once, [] {
    if (const char* path = env_cache_path()) (void)ssimx_tune_cache_load(path);
  });
}

int pick_tile(const ssimx_params* p, int dtype, int W, int H, int batch) {
  load_env_cache();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tile_override >= 0) return g_tile_override;
  auto it = g_tune_cache.find(tune_key(p, dtype, W, H, batch));
  return it == g_tune_cache.end() ? 0 : it->second;
}

}  // namespace ssimx

using namespace ssimx;

extern "C" {

int ssimx_num_tile_configs(void) { return num_tile_cfgs(); }

ssimx_status ssimx_set_tile_override(int tile) {
  if (tile < -1 || tile >= num_tile_cfgs()) return SSIMX_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tile_override = tile;
  return SSIMX_OK;
}

ssimx_status ssimx_autotune(const ssimx_params* p, int dtype, int width, int height, int batch, void* stream,
                            int* best_tile_out) {
  load_env_cache();
  ssimx_status s = check_params(p);
  if (s != SSIMX_OK) return s;
  if (width < 1 || height < 1 || batch < 1 || batch > kMaxGridY || dtype < SSIMX_U8 || dtype > SSIMX_BF16)
    return SSIMX_EINVAL;
  if ((int64_t)width * height > kMaxPlaneElems) return SSIMX_EINVAL;
  if ((s = check_path(p, dtype)) != SSIMX_OK) return s;
  int Wo, Ho;
  map_dims(p, width, height, Wo, Ho);
  if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  hipStream_t st = (hipStream_t)stream;
  const size_t plane = (size_t)width * height * batch * ssimx::dtype_size(dtype);
  const size_t wsb = fwd_ws_bytes(p, dtype, width, height, batch);
  void *x = nullptr, *y = nullptr, *ws = nullptr, *score = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = 0;
  float best_ms = 1e30f;
  int err = (int)hipMalloc(&x, plane);
  if (!err) err = (int)hipMalloc(&y, plane);
  if (!err) err = (int)hipMalloc(&ws, wsb);
  if (!err) err = (int)hipMalloc(&score, sizeof(float) * batch);
  const size_t nel = (size_t)width * height * batch;
  if (!err) err = tune_fill(x, dtype, nel, 0x2545f491u, st);
  if (!err) err = tune_fill(y, dtype, nel, 0x9e3779b9u, st);
  if (!err) err = (int)hipEventCreate(&e0);
  if (!err) err = (int)hipEventCreate(&e1);
  if (!err) {
    PlaneArg xa{x, width, (int64_t)width * height}, ya{y, width, (int64_t)width * height};
    const Path path = choose_path(p, dtype);
    const int ncfg = path == Path::kSat ? 1 : num_tile_cfgs();
    for (int t = 0; t < ncfg && s == SSIMX_OK; ++t) {
      std::vector<float> times;
      for (int rep = 0; rep < 7 && s == SSIMX_OK; ++rep) {
        (void)hipEventRecord(e0, st);
        s = fwd_pass(p, dtype, xa, ya, width, height, batch, 0, nullptr, 0, 0, (float*)score, 1, (float*)ws,
                     path == Path::kSat ? (uint32_t*)((char*)ws + ((sizeof(float) * batch *
                                                                    max_partials(p, dtype, width, height) + 255) &
                                                                   ~(size_t)255))
                                        : nullptr,
                     t, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep >= 2) times.push_back(ms);
      }
      if (s != SSIMX_OK) break;
      std::sort(times.begin(), times.end());
      const float med = times[times.size() / 2];
      if (med < best_ms) {
        best_ms = med;
        best = t;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (x) (void)hipFree(x);
  if (y) (void)hipFree(y);
  if (ws) (void)hipFree(ws);
  if (score) (void)hipFree(score);
  if (err) return hip_status(err);
  if (s != SSIMX_OK) return s;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[tune_key(p, dtype, width, height, batch)] = best;
  }
  if (const char* path = env_cache_path()) (void)ssimx_tune_cache_save(path);
  if (best_tile_out) *best_tile_out = best;
  return SSIMX_OK;
}

ssimx_status ssimx_tune_cache_save(const char* path) {
  if (!path) return SSIMX_EINVAL;
  load_env_cache();
  FILE* f = fopen(path, "w");
  if (!f) return SSIMX_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  fprintf(f, "{\n  \"version\": %d,\n  \"entries\": {", SSIMX_VERSION);
  bool first = true;
  for (const auto& kv : g_tune_cache) {
    fprintf(f, "%s\n    \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  fprintf(f, "\n  }\n}\n");
  fclose(f);
  return SSIMX_OK;
}

ssimx_status ssimx_tune_cache_load(const char* path) {
  if (!path) return SSIMX_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return SSIMX_EINVAL;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0 && text.size() < kCacheMaxBytes) text.append(buf, n);
  fclose(f);
  if (text.size() >= kCacheMaxBytes) return SSIMX_EINVAL;
  std::map<std::string, int> loaded;
  if (!parse_cache(text, loaded)) return SSIMX_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : loaded) g_tune_cache[kv.first] = kv.second;
  return SSIMX_OK;
}

}  // extern "C"
