// sw_align_batch_noalloc: the device-planned batch call for callers that
// cannot allocate (code under stream capture, tight serving loops, hosts that
// forbid hipMalloc).  Every buffer of the call lives in one file-scope device
// array of fixed size; its device address is looked up once per device when
// the library initialises that device, and only that address is ever handed
// to kernels or copies (the array's name in host code is a host-side stand-in,
// not device memory).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "sw.h"
#include "sw_runtime.h"

namespace {

constexpr size_t kScratchBytes = swrt::noalloc_scratch_bytes(SW_NOALLOC_MAX_PAIRS);
constexpr int kMaxDevices = 64;

// Shared by every call of the process on a device; the calls serialise on
// the library's lock, so one call's contents never meet another's.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace swrt {

int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d: no scratch slot (at most %d devices)", device, kMaxDevices);
    return SW_EDEVICE;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return SW_OK;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != device) e = hipSetDevice(device);
  void *p = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", device,
              hipGetErrorString(e));
    return SW_EDEVICE;
  }
  g_scratch_ptr[device] = (unsigned char *)p;
  return SW_OK;
}

}  // namespace swrt

extern "C" {

int sw_align_batch_noalloc(const sw_batch *b, const sw_scoring *sc, sw_result *out,
                           sw_stats *stats) {
  using namespace swrt;
  const double t0 = now_ms();
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!b || !out) { set_error("batch or out is NULL"); return SW_EINVAL; }
  Scoring S;
  int rc = prepare_scoring(sc, S);
  if (rc) return rc;
  if (b->n_pairs < 0 || b->n_queries < 0 || b->n_refs < 0) { set_error("negative count"); return SW_EINVAL; }
  if (b->precision != SW_PREC_AUTO && b->precision != SW_PREC_I32) { set_error("bad precision"); return SW_EINVAL; }
  if (!b->device_resident) {
    set_error("sw_align_batch_noalloc needs device-resident inputs (device_resident = 1)");
    return SW_EINVAL;
  }
  if (b->n_pairs > SW_NOALLOC_MAX_PAIRS) {
    set_error("sw_align_batch_noalloc: %d pairs, at most %d", b->n_pairs, SW_NOALLOC_MAX_PAIRS);
    return SW_EINVAL;
  }
  if (b->n_pairs == 0) return SW_OK;
  if (!b->query_res || !b->query_off || !b->ref_res || !b->ref_off || !b->pair_ref ||
      b->n_queries < 1 || b->n_refs < 1) {
    set_error("NULL sequence pointer or empty query/reference set");
    return SW_EINVAL;
  }
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_ctx.mu);
  Context &C = g_ctx;
  if (hipSetDevice(C.device) != hipSuccess) { set_error("hipSetDevice failed"); return SW_EDEVICE; }
  unsigned char *scr = C.device >= 0 && C.device < kMaxDevices ? g_scratch_ptr[C.device] : nullptr;
  if (!scr) { set_error("scratch array of device %d not set up", C.device); return SW_EDEVICE; }
  return run_device_plan_noalloc(b, S, C, scr, SW_NOALLOC_MAX_PAIRS, out, stats, t0);
}

}  // extern "C"
