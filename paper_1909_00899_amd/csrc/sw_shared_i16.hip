// Shared-query kernel instances (I16).
#include "sw_device.h"
#include "sw_menus.h"

namespace swk {
namespace {
using O = dev::OpsI16;

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
template <int SEG, bool LREC, bool MASKED>
hipError_t launch_rp(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  // grid: wavefronts wanted
  auto k = dev::shared_rowpair_kernel<SEG, LREC, MASKED>;
  constexpr int wpg = dev::rowpair_waves_per_group(LREC);
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3((grid + wpg - 1) / wpg), dim3(wpg * kWave), lds, st, a);
  return hipGetLastError();
}

template <bool LREC, bool MASKED>
hipError_t launch_rps(int seg, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  switch (seg) {
    case 4: return launch_rp<4, LREC, MASKED>(a, grid, st, lds);
    case 8: return launch_rp<8, LREC, MASKED>(a, grid, st, lds);
    case 12: return launch_rp<12, LREC, MASKED>(a, grid, st, lds);
    case 16: return launch_rp<16, LREC, MASKED>(a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}
}  // namespace

// masked: a.first_row gives each pair's first query row (start-cell passes)
hipError_t launch_rowpair_i16(int seg, bool lds_records, const KArgs &a, int grid,
                              hipStream_t st, size_t lds) {
  const bool masked = a.first_row != nullptr;
  if (masked)
    return lds_records ? launch_rps<true, true>(seg, a, grid, st, lds)
                       : launch_rps<false, true>(seg, a, grid, st, lds);
  return lds_records ? launch_rps<true, false>(seg, a, grid, st, lds)
                     : launch_rps<false, false>(seg, a, grid, st, lds);
}

hipError_t launch_direct_i16(int shape, const KArgs &a, int grid, hipStream_t st, size_t lds) {
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

hipError_t launch_shared_i16(Alg alg, int menu, bool chunked, const KArgs &a, int grid,
                              hipStream_t st, uint32_t mask, size_t lds) {
  if (alg != ALG_SCAN) return hipErrorInvalidValue;
  return chunked ? dispatch<true, false>(menu, a, grid, st, mask, lds)
                 : dispatch<false, false>(menu, a, grid, st, mask, lds);
}

}  // namespace swk
