// ssim_pooled_noalloc: mean SSIM per frame pair without a caller workspace,
// for callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid allocation).
//
// The forward's only scratch, the per-tile partial sums the fixed-order
// finalize reduces (and, for 8-bit box windows with the integral-image
// algorithm, the five tables), lives in one file-scope device array.  Host
// code never passes the array's name to a kernel: the name is a host-side
// stand-in, not a device address.  The first call on a device, with that
// device current, resolves the array's device address once with
// hipGetSymbolAddress and keeps it per device; every launch then takes that
// address.  Each GPU holds its own copy of the array until the process ends.
//
// Every call on a GPU shares that GPU's array: calls that overlap on one GPU
// (two streams, two host threads) race on it.  Every partial slot a launch
// reads was written by the same launch, so nothing needs clearing between
// calls.
#include <mutex>

#include "launch.hpp"
#include "host_common.hpp"
#include "ssimx_internal.hpp"

namespace ssimx {
namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;  // 8 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's array (resolved once per device).
ssimx_status scratch_address(void** out) {
  int dev = -1;
  int err = (int)hipGetDevice(&dev);
  if (err) return hip_status(err);
  if (dev < 0 || dev >= kMaxDevices) return SSIMX_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    err = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err) return hip_status(err);
    if (!p) return SSIMX_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SSIMX_OK;
}

}  // namespace
}  // namespace ssimx

using namespace ssimx;

extern "C" {

size_t ssimx_noalloc_scratch_bytes(void) { return kScratchBytes; }

ssimx_status ssim_pooled_noalloc(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                                 float* score_out, void* stream) {
  ssimx_status s;
  if (!score_out) return SSIMX_EINVAL;
  if ((s = check_params(p)) != SSIMX_OK) return s;
  if ((s = check_images(ref, dis, batch)) != SSIMX_OK) return s;
  if ((s = check_path(p, ref->dtype)) != SSIMX_OK) return s;
  int Wo, Ho;
  map_dims(p, ref->width, ref->height, Wo, Ho);
  if (Wo < 1 || Ho < 1) return SSIMX_ETOOSMALL;
  if (fwd_ws_bytes(p, ref->dtype, ref->width, ref->height, batch) > kScratchBytes) return SSIMX_ESCRATCH;
  void* base = nullptr;
  if ((s = scratch_address(&base)) != SSIMX_OK) return s;
  // the same slices as the workspace of ssim_pooled
  Ws lay;
  float* partial = (float*)((char*)base + lay.take(sizeof(float) * (size_t)batch *
                                                   max_partials(p, ref->dtype, ref->width, ref->height)));
  uint32_t* sat = nullptr;
  if (choose_path(p, ref->dtype) == Path::kSat)
    sat = (uint32_t*)((char*)base + lay.take(sizeof(uint32_t) * 5 * (size_t)batch * (ref->width + 1) *
                                             (size_t)(ref->height + 1)));
  PlaneArg x{ref->data, ref->pitch, ref->batch_stride}, y{dis->data, dis->pitch, dis->batch_stride};
  const int tile = pick_tile(p, ref->dtype, ref->width, ref->height, batch);
  return fwd_pass(p, ref->dtype, x, y, ref->width, ref->height, batch, 0, nullptr, 0, 0, score_out, 1, partial, sat,
                  tile, (hipStream_t)stream);
}

}  // extern "C"
