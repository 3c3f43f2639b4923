// Strided Gaussian band kernels (see strided_tile.hpp).
#include "launch.hpp"
#include "strided_tile.hpp"

namespace ssimx {

using namespace strided;

template <int K, int S, typename T>
__global__ __launch_bounds__(kNT, 3) void strided_kernel(FastArgs a) {
  __shared__ __align__(16) float smem[strided_smem_floats<K, S>()];
  __shared__ float red[kNT / 64];
  int tile, frame;
  xcd_tile(tile, frame);
  const float acc = strided_tile<K, S, T>(a, frame, tile, smem);
  const float tot = block_sum<kNT>(acc, red);
  if (threadIdx.x == 0 && a.partial) a.partial[(int64_t)frame * gridDim.x + tile] = tot;
}

bool strided_supported(int k, int stride) {
  return (k == 7 || k == 9 || k == 11 || k == 13) && (stride == 2 || stride == 3 || stride == 4);
}

namespace {

template <int K, int S>
int launch_ks(int dtype, const FastArgs& a, dim3 grid, hipStream_t st) {
  switch (dtype) {
    case SSIMX_U8: hipLaunchKernelGGL((strided_kernel<K, S, uint8_t>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_U16: hipLaunchKernelGGL((strided_kernel<K, S, uint16_t>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_F32: hipLaunchKernelGGL((strided_kernel<K, S, float>), grid, dim3(kNT), 0, st, a); break;
    case SSIMX_BF16: hipLaunchKernelGGL((strided_kernel<K, S, bf16_t>), grid, dim3(kNT), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <int K>
int launch_k(int dtype, const FastArgs& a, dim3 grid, hipStream_t st) {
  switch (a.g.s) {
    case 2: return launch_ks<K, 2>(dtype, a, grid, st);
    case 3: return launch_ks<K, 3>(dtype, a, grid, st);
    case 4: return launch_ks<K, 4>(dtype, a, grid, st);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

int launch_strided(int dtype, const FastArgs& a, int batch, hipStream_t st) {
  dim3 grid(a.g.tiles_x * a.g.tiles_y, batch);
  switch (a.g.k) {
    case 7: return launch_k<7>(dtype, a, grid, st);
    case 9: return launch_k<9>(dtype, a, grid, st);
    case 11: return launch_k<11>(dtype, a, grid, st);
    case 13: return launch_k<13>(dtype, a, grid, st);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace ssimx
