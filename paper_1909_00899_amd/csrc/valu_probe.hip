// Integer VALU issue-rate probe (measurement aid, not part of the alignment
// library): every lane of every wavefront runs long streams of independent
// packed int16 saturating adds and subtracts (v_pk_add_i16 / v_pk_sub_u16
// with clamp, the instructions of the column step), so the achieved rate is
// the chip's sustained int16x2 VALU rate under this load, to set beside the
// rate derived from unit counts and clock.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr int kAcc = 8;       // independent accumulators per lane
constexpr int kUnroll = 8;    // steps per loop trip, two instructions per accumulator each

__global__ __launch_bounds__(256) void valu_probe_kernel(uint32_t *out, int trips) {
  s16x2 acc[kAcc], add[kAcc];
  u16x2 sub[kAcc];
  const uint32_t seed = threadIdx.x * 2654435761u ^ blockIdx.x;
#pragma unroll
  for (int k = 0; k < kAcc; ++k) {
    acc[k] = __builtin_bit_cast(s16x2, seed + 977u * k);
    add[k] = __builtin_bit_cast(s16x2, (seed >> 3) | 0x00070003u);
    sub[k] = __builtin_bit_cast(u16x2, ((seed >> 5) & 0x00050005u) + 0x00020001u);
  }
  for (int t = 0; t < trips; ++t) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kAcc; ++k) {
        acc[k] = __builtin_elementwise_add_sat(acc[k], add[k]);
        acc[k] = __builtin_bit_cast(
            s16x2, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, acc[k]), sub[k]));
      }
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < kAcc; ++k) x ^= __builtin_bit_cast(uint32_t, acc[k]);
  out[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

// The same for 32-bit integer adds and maxima (v_add_u32 / v_max_i32, the
// instructions of the int32 path and end-to-end kernels): one op per lane per
// instruction.  Each step is written as the two instructions themselves, so
// the count is exact: in plain C++ the chain max(acc + a, b) composes into one
// add and one maximum over any number of unrolled steps (max-plus algebra with
// loop-invariant operands), and the compiler folds it.
__global__ __launch_bounds__(256) void valu_probe_i32_kernel(uint32_t *out, int trips) {
  int acc[kAcc], add[kAcc], lim[kAcc];
  const uint32_t seed = threadIdx.x * 2654435761u ^ blockIdx.x;
#pragma unroll
  for (int k = 0; k < kAcc; ++k) {
    acc[k] = (int)(seed + 977u * k);
    add[k] = (int)((seed >> 3) | 7u) + k;
    lim[k] = (int)(seed >> 7) - k;
  }
  for (int t = 0; t < trips; ++t) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kAcc; ++k) {
        asm volatile("v_add_u32 %0, %0, %1\n\tv_max_i32 %0, %0, %2"
                     : "+v"(acc[k])
                     : "v"(add[k]), "v"(lim[k]));
      }
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < kAcc; ++k) x ^= (uint32_t)acc[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

}  // namespace

// Runs `grid` workgroups of 256 threads, `trips` loop trips each, and returns
// the packed int16 operations per second (two per instruction per lane) in
// *ops_per_s.  0 on success, else the HIP error code.
extern "C" int swprobe_valu(int grid, int trips, double *ops_per_s) {
  if (grid <= 0 || trips <= 0 || ops_per_s == nullptr) return (int)hipErrorInvalidValue;
  uint32_t *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void **)&out, (size_t)grid * 256 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0.f;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(valu_probe_kernel, dim3(grid), dim3(256), 0, nullptr, out, 1);  // warm-up
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(valu_probe_kernel, dim3(grid), dim3(256), 0, nullptr, out, trips);
    hipEventRecord(e1, nullptr);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  }
  if (e == hipSuccess) {
    const double instr = (double)grid * 256 * trips * kUnroll * kAcc * 2;
    *ops_per_s = ms > 0.f ? 2.0 * instr / (ms * 1e-3) : 0.0;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (out) hipFree(out);
  return (int)e;
}

// As swprobe_valu for the 32-bit kernel: *ops_per_s receives int32 operations
// per second (one v_add_u32 and one v_max_i32 per step and lane, each one
// operation per lane).  0 on success, else the HIP error.
extern "C" int swprobe_valu_i32(int grid, int trips, double *ops_per_s) {
  if (grid <= 0 || trips <= 0 || ops_per_s == nullptr) return (int)hipErrorInvalidValue;
  uint32_t *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void **)&out, (size_t)grid * 256 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0.f;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(valu_probe_i32_kernel, dim3(grid), dim3(256), 0, nullptr, out, 1);
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(valu_probe_i32_kernel, dim3(grid), dim3(256), 0, nullptr, out, trips);
    hipEventRecord(e1, nullptr);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  }
  if (e == hipSuccess) {
    const double ops = (double)grid * 256 * trips * kUnroll * kAcc * 2;
    *ops_per_s = ms > 0.f ? ops / (ms * 1e-3) : 0.0;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (out) hipFree(out);
  return (int)e;
}
