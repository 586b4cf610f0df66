// Swapped-striping kernel instances (int32): the reference striped over one
// 64-lane wavefront, SEG rows per lane, the query streamed as columns.
#include "sw_device.h"

namespace swk {
namespace {
template <int SEG>
hipError_t launch_s(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  auto k = dev::swap_kernel<SEG>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWave), lds, st, a);
  return hipGetLastError();
}
}  // namespace

bool swap_has(int seg) {
  for (int s : kSwapSegs)
    if (s == seg) return true;
  return false;
}

size_t swap_lds_bytes(int alpha, int seg) {
  return (size_t)dev::swap_snap_offset(alpha) + (size_t)seg * kWave * sizeof(uint32_t);
}

hipError_t launch_swap(int seg, const KArgs &a, int grid, hipStream_t st) {
  if (a.ntasks <= 0 || grid <= 0) return hipSuccess;
  const size_t lds = swap_lds_bytes(a.alpha, seg);
  switch (seg) {
    case 4: return launch_s<4>(a, grid, st, lds);
    case 8: return launch_s<8>(a, grid, st, lds);
    case 12: return launch_s<12>(a, grid, st, lds);
    case 16: return launch_s<16>(a, grid, st, lds);
    case 20: return launch_s<20>(a, grid, st, lds);
    case 24: return launch_s<24>(a, grid, st, lds);
    case 28: return launch_s<28>(a, grid, st, lds);
    case 32: return launch_s<32>(a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}

}  // namespace swk
