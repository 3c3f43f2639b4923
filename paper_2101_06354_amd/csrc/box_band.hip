// Rectangular-window band kernels on 8-bit planes (see box_band.hpp).
#include "launch.hpp"
#include "box_band.hpp"

namespace ssimx {

using namespace bband;

template <int K, int S>
__global__ __launch_bounds__(kNT, 2) void box_band_kernel(BandArgs a) {
  __shared__ uint32_t lds[band_lds_dwords<K, S>()];
  __shared__ float red[kNT / 64];
  int tile, frame;
  xcd_tile(tile, frame);
  const float acc = box_band_tile<K, S>(a, frame, tile, lds);
  const float tot = block_sum<kNT>(acc, red);
  if (threadIdx.x == 0 && a.partial) a.partial[(int64_t)frame * gridDim.x + tile] = tot;
}

bool box_band_supported(int k, int s) {
  if (k < 2 || k > 16) return false;
  if (s == 1) return true;
  if (s == 2 || s == 4) return k % s == 0;
  return false;
}

namespace {

using BandKernel = void (*)(BandArgs);

template <int S, int K>
constexpr BandKernel band_entry() {
  if constexpr (K % S == 0) return box_band_kernel<K, S>;
  else return nullptr;
}

template <int S, int... Ks>
constexpr void fill_row(BandKernel* row, std::integer_sequence<int, Ks...>) {
  ((row[Ks + 2] = band_entry<S, Ks + 2>()), ...);
}

struct BandTable {
  BandKernel k[3][17] = {};  // [stride 1, 2, 4][window 0..16]
  BandTable() {
    fill_row<1>(k[0], std::make_integer_sequence<int, 15>{});
    fill_row<2>(k[1], std::make_integer_sequence<int, 15>{});
    fill_row<4>(k[2], std::make_integer_sequence<int, 15>{});
  }
};

}  // namespace

int launch_box_band(const BandArgs& a, int batch, hipStream_t st) {
  static const BandTable table;
  if (!box_band_supported(a.g.k, a.g.s)) return (int)hipErrorInvalidValue;
  const int si = a.g.s == 1 ? 0 : a.g.s == 2 ? 1 : 2;
  const BandKernel kern = table.k[si][a.g.k];
  if (!kern) return (int)hipErrorInvalidValue;
  dim3 grid(a.g.tiles_x * a.g.tiles_y, batch), block(kNT);
  hipLaunchKernelGGL(kern, grid, block, 0, st, a);
  return (int)hipGetLastError();
}

}  // namespace ssimx
