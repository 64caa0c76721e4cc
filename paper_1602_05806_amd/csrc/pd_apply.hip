// Dispatch of the operator-apply launches to the per-(precision, degree) instantiations of
// pd_apply_kernels.h (see pd_apply_inst.hip), and the tile-count queries.
#include <hip/hip_runtime.h>

#include "pd_apply2d.h"
#include "pd_launch.h"

namespace pdk {

// defined in pd_apply_kernels.h, instantiated once per (T, N) in pd_apply_inst.hip
template <typename T, int N>
hipError_t launch_apply_N(const ApplyLaunch& L, hipStream_t s);
template <typename T, int N>
unsigned blocks_N(const ApplyLaunch& L);

template <typename T>
static hipError_t launch_apply_T(const ApplyLaunch& L, hipStream_t s) {
  switch (L.N) {
    case 0: return launch_apply_N<T, 0>(L, s);
    case 1: return launch_apply_N<T, 1>(L, s);
    case 2: return launch_apply_N<T, 2>(L, s);
    case 3: return launch_apply_N<T, 3>(L, s);
    case 4: return launch_apply_N<T, 4>(L, s);
    case 5: return launch_apply_N<T, 5>(L, s);
    case 6: return launch_apply_N<T, 6>(L, s);
    case 7: return launch_apply_N<T, 7>(L, s);
    case 8: return launch_apply_N<T, 8>(L, s);
    default: return hipErrorInvalidValue;
  }
}

void tiles2d(int N, bool fp32, int variant, int nx, int ny, int* ntx, int* nty) {
  ApplyLaunch L;
  L.dim = 2;
  L.N = N;
  L.fp32 = fp32;
  L.tile_variant = variant;
  L.nc[0] = nx;
  L.nc[1] = ny;
  L.tiles_per_wg = 1;
  *ntx = *nty = 0;
  const unsigned blocks = apply_blocks(L);
  (void)blocks;
#define PD_T2D(NN)                                                                   \
  case NN: {                                                                         \
    int tx, ty;                                                                      \
    if (fp32) {                                                                      \
      tx = variant == 1 ? Tile2D<float, NN, 1>::TX : variant == 2 ? Tile2D<float, NN, 2>::TX \
                                                                  : Tile2D<float, NN, 0>::TX; \
      ty = variant == 1 ? Tile2D<float, NN, 1>::TY : variant == 2 ? Tile2D<float, NN, 2>::TY \
                                                                  : Tile2D<float, NN, 0>::TY; \
    } else {                                                                         \
      tx = variant == 1 ? Tile2D<double, NN, 1>::TX : variant == 2 ? Tile2D<double, NN, 2>::TX \
                                                                   : Tile2D<double, NN, 0>::TX; \
      ty = variant == 1 ? Tile2D<double, NN, 1>::TY : variant == 2 ? Tile2D<double, NN, 2>::TY \
                                                                   : Tile2D<double, NN, 0>::TY; \
    }                                                                                \
    *ntx = (nx + tx - 1) / tx;                                                       \
    *nty = (ny + ty - 1) / ty;                                                       \
    break;                                                                           \
  }
  switch (N) { PD_T2D(0) PD_T2D(1) PD_T2D(2) PD_T2D(3) PD_T2D(4) PD_T2D(5) PD_T2D(6) PD_T2D(7) PD_T2D(8) }
#undef PD_T2D
}

hipError_t launch_apply(const ApplyLaunch& L, hipStream_t s) {
  return L.fp32 ? launch_apply_T<float>(L, s) : launch_apply_T<double>(L, s);
}

template <typename T>
static unsigned apply_blocks_T(const ApplyLaunch& L) {
  switch (L.N) {
    case 0: return blocks_N<T, 0>(L);
    case 1: return blocks_N<T, 1>(L);
    case 2: return blocks_N<T, 2>(L);
    case 3: return blocks_N<T, 3>(L);
    case 4: return blocks_N<T, 4>(L);
    case 5: return blocks_N<T, 5>(L);
    case 6: return blocks_N<T, 6>(L);
    case 7: return blocks_N<T, 7>(L);
    case 8: return blocks_N<T, 8>(L);
    default: return 0;
  }
}

unsigned apply_blocks(const ApplyLaunch& L) {
  return L.fp32 ? apply_blocks_T<float>(L) : apply_blocks_T<double>(L);
}

}  // namespace pdk
