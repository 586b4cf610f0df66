// Per-pair kernel instances (I16).
#include "sw_device.h"
#include "sw_menus.h"

namespace swk {
namespace {
using O = dev::OpsI16;

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
template <int SEG, int ES>
hipError_t launch_d(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  auto k = dev::pair_direct_kernel<O, SEG, 16, ES>;
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kWave), lds, st, a);
  return hipGetLastError();
}
// grid: wavefronts wanted; workgroups of 8 wavefronts (4 where the kernel
// runs three wavefronts per SIMD, so that three workgroups share a CU)
template <int SEG, bool CH, int P>
hipError_t launch_rp(const KArgs &a, int grid, hipStream_t st, size_t lds) {
  auto k = dev::pair_rowpair_kernel<SEG, CH, P>;
  constexpr int wpg = dev::rp_pair_waves_per_eu(SEG, CH) == 3 ? 4 : kWavesPerGroup;
  hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3((grid + wpg - 1) / wpg), dim3(wpg * kWave), lds, st, a);
  return hipGetLastError();
}
template <bool CH, int P>
hipError_t launch_rps(int seg, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  switch (seg) {
    case 4: return launch_rp<4, CH, P>(a, grid, st, lds);
    case 8: return launch_rp<8, CH, P>(a, grid, st, lds);
    case 12: return launch_rp<12, CH, P>(a, grid, st, lds);
    case 16: return launch_rp<16, CH, P>(a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}
template <bool CH>
hipError_t launch_rpp(int seg, int lanes, const KArgs &a, int grid, hipStream_t st, size_t lds) {
  switch (lanes) {
    case 16: return launch_rps<CH, 16>(seg, a, grid, st, lds);
    case 32: return launch_rps<CH, 32>(seg, a, grid, st, lds);
    case 64: return launch_rps<CH, 64>(seg, a, grid, st, lds);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_pair_rowpair_i16(int seg, int lanes, bool chunked, const KArgs &a, int grid,
                                   hipStream_t st, size_t lds) {
  return chunked ? launch_rpp<true>(seg, lanes, a, grid, st, lds)
                 : launch_rpp<false>(seg, lanes, a, grid, st, lds);
}

hipError_t launch_pair_direct_i16(int seg, int es, const KArgs &a, int grid, hipStream_t st,
                                  size_t lds) {
  if (es == 1) {
    switch (seg) {
      case 4: return launch_d<4, 1>(a, grid, st, lds);
      case 6: return launch_d<6, 1>(a, grid, st, lds);
      case 8: return launch_d<8, 1>(a, grid, st, lds);
      case 10: return launch_d<10, 1>(a, grid, st, lds);
      case 12: return launch_d<12, 1>(a, grid, st, lds);
      case 16: return launch_d<16, 1>(a, grid, st, lds);
    }
  } else if (es == 2) {
    switch (seg) {
      case 4: return launch_d<4, 2>(a, grid, st, lds);
      case 6: return launch_d<6, 2>(a, grid, st, lds);
      case 8: return launch_d<8, 2>(a, grid, st, lds);
      case 10: return launch_d<10, 2>(a, grid, st, lds);
      case 12: return launch_d<12, 2>(a, grid, st, lds);
      case 16: return launch_d<16, 2>(a, grid, st, lds);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pair_i16(int seg, int pmax, bool chunked, const KArgs &a, int grid,
                            hipStream_t st, size_t lds) {
  return chunked ? launch_s<true>(seg, pmax, a, grid, st, lds)
                 : launch_s<false>(seg, pmax, a, grid, st, lds);
}

}  // namespace swk
