// Per-pair kernel instances (I32).
#include "sw_device.h"
#include "sw_menus.h"

namespace swk {
namespace {
using O = dev::OpsI32;

template <int SEG, int PMAX, bool CH>
hipError_t launch_t(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  auto k = dev::pair_kernel<O, SEG, PMAX, CH>;
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWave), lds, st, a);
  return hipGetLastError();
}
template <int SEG, bool CH>
hipError_t launch_p(int pmax, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  switch (pmax) {
    case 16: return launch_t<SEG, 16, CH>(a, grid, st, lds);
    case 32: return launch_t<SEG, 32, CH>(a, grid, st, lds);
    case 64: return launch_t<SEG, 64, CH>(a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}
template <bool CH>
hipError_t launch_s(int seg, int pmax, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  switch (seg) {
    case 4: return launch_p<4, CH>(pmax, a, grid, st, lds);
    case 6: return launch_p<6, CH>(pmax, a, grid, st, lds);
    case 8: return launch_p<8, CH>(pmax, a, grid, st, lds);
    case 10: return launch_p<10, CH>(pmax, a, grid, st, lds);
    case 12: return launch_p<12, CH>(pmax, a, grid, st, lds);
    case 16: return launch_p<16, CH>(pmax, a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}
template <int SEG>
hipError_t launch_d(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  auto k = dev::pair_direct_kernel<O, SEG, 16, 4>;
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWave), lds, st, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_pair_direct_i32(int seg, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  switch (seg) {
    case 4: return launch_d<4>(a, grid, st, lds);
    case 6: return launch_d<6>(a, grid, st, lds);
    case 8: return launch_d<8>(a, grid, st, lds);
    case 10: return launch_d<10>(a, grid, st, lds);
    case 12: return launch_d<12>(a, grid, st, lds);
    case 16: return launch_d<16>(a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pair_i32(int seg, int pmax, bool chunked, const KArgs &a, int grid,
                            hipStream_t st, size_t lds) {
  return chunked ? launch_s<true>(seg, pmax, a, grid, st, lds)
                 : launch_s<false>(seg, pmax, a, grid, st, lds);
}

}  // namespace swk
