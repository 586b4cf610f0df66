// Shared-query kernel instances (I32).
#include "sw_device.h"
#include "sw_menus.h"

namespace swk {
namespace {
using O = dev::OpsI32;

template <int M, bool CH, bool LZ>
hipError_t launch_m(const KArgs &a, int grid, hipStream_t st, uint32_t mask, size_t lds) {
  constexpr SharedMenu mm = kSharedMenus[M];
  auto k = dev::shared_kernel<O, mm.seg16, mm.seg32, mm.seg64, CH, LZ>;
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWavesPerGroup * kWave), lds, st, a, mask);
  return hipGetLastError();
}

template <bool CH, bool LZ>
hipError_t dispatch(int menu, const KArgs &a, int grid, hipStream_t st, uint32_t mask, size_t lds) {
  switch (menu) {
    case 0: return launch_m<0, CH, LZ>(a, grid, st, mask, lds);
    case 1: return launch_m<1, CH, LZ>(a, grid, st, mask, lds);
    case 2: return launch_m<2, CH, LZ>(a, grid, st, mask, lds);
    case 3: return launch_m<3, CH, LZ>(a, grid, st, mask, lds);
    case 4: return launch_m<4, CH, LZ>(a, grid, st, mask, lds);
    case 5: return launch_m<5, CH, LZ>(a, grid, st, mask, lds);
  }
  return hipErrorInvalidValue;
}
template <int K>
hipError_t launch_d(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  constexpr DirectShape ds = kDirectShapes[K];
  auto k = dev::shared_direct_kernel<O, ds.seg, ds.lanes>;
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWavesPerGroup * kWave), lds, st, a);
  return hipGetLastError();
}
template <int M, bool CH>
hipError_t launch_dual_m(const KArgs &a, int grid, hipStream_t st, uint32_t mask, size_t lds) {
  constexpr SharedMenu mm = kSharedMenus[M];
  auto k = dev::shared_dual_kernel<mm.seg16, mm.seg32, mm.seg64, CH>;
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWavesPerGroup * kWave), lds, st, a, mask);
  return hipGetLastError();
}

template <bool CH>
hipError_t dispatch_dual(int menu, const KArgs &a, int grid, hipStream_t st, uint32_t mask,
                         size_t lds) {
  switch (menu) {
    case 0: return launch_dual_m<0, CH>(a, grid, st, mask, lds);
    case 1: return launch_dual_m<1, CH>(a, grid, st, mask, lds);
    case 2: return launch_dual_m<2, CH>(a, grid, st, mask, lds);
    case 3: return launch_dual_m<3, CH>(a, grid, st, mask, lds);
    case 4: return launch_dual_m<4, CH>(a, grid, st, mask, lds);
    case 5: return launch_dual_m<5, CH>(a, grid, st, mask, lds);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_shared_dual_i32(int menu, bool chunked, const KArgs &a, int grid,
                                  hipStream_t st, uint32_t mask, size_t lds) {
  return chunked ? dispatch_dual<true>(menu, a, grid, st, mask, lds)
                 : dispatch_dual<false>(menu, a, grid, st, mask, lds);
}

hipError_t launch_direct_i32(int shape, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  static_assert(kNumDirectShapes == 6, "direct shapes");
  switch (shape) {
    case 0: return launch_d<0>(a, grid, st, lds);
    case 1: return launch_d<1>(a, grid, st, lds);
    case 2: return launch_d<2>(a, grid, st, lds);
    case 3: return launch_d<3>(a, grid, st, lds);
    case 4: return launch_d<4>(a, grid, st, lds);
    case 5: return launch_d<5>(a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_shared_i32(Alg alg, int menu, bool chunked, const KArgs &a, int grid,
                              hipStream_t st, uint32_t mask, size_t lds) {
  if (alg == ALG_LAZYF)
    return chunked ? dispatch<true, true>(menu, a, grid, st, mask, lds)
                   : dispatch<false, true>(menu, a, grid, st, mask, lds);
  return chunked ? dispatch<true, false>(menu, a, grid, st, mask, lds)
                 : dispatch<false, false>(menu, a, grid, st, mask, lds);
}

}  // namespace swk
