// Tile-shape autotuner for the forward kernels and its process-wide cache.
//
// A cache entry maps (architecture, dtype, window, k, stride, padding, algo,
// width x height, batch class) to the index of the fastest tile shape.  The
// cache is filled by ssimx_autotune (timed with HIP events on the caller's
// stream) or loaded from a JSON file, and read by every later call.
#include <stdio.h>
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

int pick_tile(const ssimx_params* p, int dtype, int W, int H, int batch) {
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
  ssimx_status s = check_params(p);
  if (s != SSIMX_OK) return s;
  if (width < 1 || height < 1 || batch < 1 || dtype < SSIMX_U8 || dtype > SSIMX_BF16) return SSIMX_EINVAL;
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
  if (!err) err = (int)hipMemsetAsync(x, 0x35, plane, st);
  if (!err) err = (int)hipMemsetAsync(y, 0x3a, plane, st);
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
  if (best_tile_out) *best_tile_out = best;
  return SSIMX_OK;
}

ssimx_status ssimx_tune_cache_save(const char* path) {
  if (!path) return SSIMX_EINVAL;
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
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  fclose(f);
  const size_t ent = text.find("\"entries\"");
  if (ent == std::string::npos) return SSIMX_EINVAL;
  size_t pos = text.find('{', ent);
  if (pos == std::string::npos) return SSIMX_EINVAL;
  std::map<std::string, int> loaded;
  while (true) {
    const size_t q0 = text.find('"', pos + 1);
    const size_t close = text.find('}', pos + 1);
    if (q0 == std::string::npos || (close != std::string::npos && close < q0)) break;
    const size_t q1 = text.find('"', q0 + 1);
    if (q1 == std::string::npos) return SSIMX_EINVAL;
    const size_t colon = text.find(':', q1);
    if (colon == std::string::npos) return SSIMX_EINVAL;
    const int v = atoi(text.c_str() + colon + 1);
    if (v < 0 || v >= num_tile_cfgs()) return SSIMX_EINVAL;
    loaded[text.substr(q0 + 1, q1 - q0 - 1)] = v;
    pos = colon + 1;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : loaded) g_tune_cache[kv.first] = kv.second;
  return SSIMX_OK;
}

}  // extern "C"
