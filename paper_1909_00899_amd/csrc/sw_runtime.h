// Host runtime internals of libswscan.so (shared by the batch path and the
// request server).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "sw.h"
#include "sw_internal.h"

namespace swrt {

void set_error(const char *fmt, ...);
extern thread_local std::string g_last_error;

// Grow-only device allocation.
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes);
  void release();
  template <class T> T *as() const { return (T *)p; }
};

// Grow-only pinned host allocation.
struct HostBuf {
  void *p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes);
  void release();
  template <class T> T *as() const { return (T *)p; }
};

struct Scoring {
  int alpha = 0;
  std::vector<int> M;   // alpha*alpha, [query code][ref code]
  int go = 0, ge = 0;   // ge already min(ge, go)
  int max_s = 0;        // max(0, max entry)
  bool fits_i16 = false;
};
int prepare_scoring(const sw_scoring *sc, Scoring &out);

// One pair as the planner sees it.
struct PlanItem {
  int pair;        // index into the PairInfo array (== result index)
  int query;       // query id
  int m, n;
};

// Everything one execution needs on the device, independent of who owns the
// sequence buffers (the caller's device memory or the library's copies).
struct ExecInput {
  const uint8_t *d_qres = nullptr;   // device
  const uint8_t *d_rres = nullptr;   // device
  std::vector<swk::PairInfo> pairs;  // host PairInfo (index = pair id), or empty when
  const swk::PairInfo *d_pairs = nullptr;  // ... they are already on the device
  int n_pairs = 0;                   // size of the PairInfo array
  std::vector<PlanItem> items;       // pairs with m > 0 and n > 0
  int n_queries = 0;
  std::vector<int64_t> q_off_of_query;  // query start offsets
  std::vector<int> m_of_query;
};

struct ExecOptions {
  int algorithm = SW_ALG_SCAN;
  int force_lanes = 0, force_seglen = 0, force_kernel = 0, mixed_layout = 0;
  int int16_cap = 32767;
};

struct ExecStats {
  double kernel_ms = 0;
  double plan_ms = 0, launch_ms = 0, finish_ms = 0;
  int64_t padded_cells = 0;
  int launches = 0;
  int lanes_used[3] = {0, 0, 0};
  int seglen_max = 0;
  unsigned long long dev_stats[3] = {0, 0, 0};
};

double now_ms();

// Work buffers used by one execution (the batch path owns one; the request
// server one per in-flight batch).
struct Workspace {
  DevBuf tasks, pairs, streams, results, bnd, misc, matrix, offs;
  HostBuf staging;
  void release() {
    for (DevBuf *b : {&tasks, &pairs, &streams, &results, &bnd, &misc, &matrix, &offs})
      b->release();
    staging.release();
  }
};

struct Context {
  std::mutex mu;
  int device = -1;
  bool inited = false;
  int num_cus = 256;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evx = nullptr;
  DevBuf qres, rres, flag;
  Workspace ws;
  int init(int dev);
  void shutdown();
};

extern Context g_ctx;
int ensure_init(int dev = -1);

// Plans and runs every item of `in` with the given precision on `st`,
// writing swk::DevResult entries into ws.results (indexed by pair id).
// Synchronous.  results must already hold n_results entries (zeroed for
// pairs that are not run).
int execute(const ExecInput &in, const Scoring &sc, swk::Prec prec, const ExecOptions &opt,
            Workspace &ws, int n_results, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
            int num_cus, ExecStats &stats, bool reset_results);

// Full batch semantics (int16 pass + int32 rerun) on prepared input.
int run_batch(const ExecInput &in, const Scoring &sc, int precision, const ExecOptions &opt,
              Workspace &ws, int n_pairs, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
              int num_cus, sw_result *out, sw_stats *stats);

}  // namespace swrt
