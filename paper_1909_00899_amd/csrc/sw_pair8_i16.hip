// Device-planned per-pair kernel instances with eight-lane sub-groups (I16,
// byte profiles): sixteen alignments per wavefront for short queries.
#include "sw_device.h"
#include "sw_menus.h"

namespace swk {
namespace {
using O = dev::OpsI16;

template <int SEG>
hipError_t launch_d8(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  auto k = dev::pair_direct_kernel<O, SEG, 8, 1>;
  (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWave), lds, st, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_pair_direct8_i16(int seg, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  static_assert(kNumPair8Segs == 5, "menu and switch agree");
  switch (seg) {
    case 8: return launch_d8<8>(a, grid, st, lds);
    case 10: return launch_d8<10>(a, grid, st, lds);
    case 13: return launch_d8<13>(a, grid, st, lds);
    case 16: return launch_d8<16>(a, grid, st, lds);
    case 19: return launch_d8<19>(a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}

}  // namespace swk
