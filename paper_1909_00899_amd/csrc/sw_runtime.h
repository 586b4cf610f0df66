// Host runtime internals of libswscan.so (shared by the batch path and the
// request server).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <mutex>
#include <string>
#include <unordered_map>
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
  int grow_pct = 25;          // slack added on growth, percent of the request
  // when set, an outgrown buffer is kept here instead of freed (a free waits
  // for the whole device; the owner frees the list when it is done)
  std::vector<void *> *retired = nullptr;
  int ensure(size_t bytes);
  void release();
  template <class T> T *as() const { return (T *)p; }
};

// Grow-only pinned host allocation.
struct HostBuf {
  void *p = nullptr;
  size_t cap = 0;
  int grow_pct = 25;          // slack added on growth, percent of the request
  std::vector<void *> *retired = nullptr;   // as DevBuf::retired (pinned host memory)
  int ensure(size_t bytes);
  void release();
  template <class T> T *as() const { return (T *)p; }
};

// alpha*alpha matrix entries in fixed storage (preparing a scoring scheme
// touches no heap, which the no-allocation batch call relies on).
struct MatrixWords {
  int v[swk::kMaxAlpha * swk::kMaxAlpha];
  size_t n = 0;
  void assign(const int *b, const int *e) {
    n = (size_t)(e - b);
    for (size_t k = 0; k < n; ++k) v[k] = b[k];
  }
  const int *data() const { return v; }
  size_t size() const { return n; }
  const int *begin() const { return v; }
  const int *end() const { return v + n; }
};

struct Scoring {
  int alpha = 0;
  MatrixWords M;        // alpha*alpha, [query code][ref code]
  int go = 0, ge = 0;   // ge already min(ge, go)
  int max_s = 0;        // max(0, max entry)
  bool fits_i16 = false;
  bool fits_i8 = false;  // every entry in [-128, 127]: byte profile entries
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
  bool use_tuning = true;   // consult the autotuner's table for unforced shapes
  int algorithm = SW_ALG_SCAN;
  int force_lanes = 0, force_seglen = 0, force_kernel = 0, mixed_layout = 0, use_graph = 0;
  int int16_cap = 32767;
  int lane_pairing = 0;     // SW_PAIRING_*
  int int32_chains = 0;     // SW_CHAINS_*
  int striping = 0;         // SW_STRIPE_*
  int lds_records = -1;     // device-planned row pairs: -1 as LDS allows, 0 registers, 1 LDS
};

struct ExecStats {
  double kernel_ms = 0;
  double plan_ms = 0, launch_ms = 0, finish_ms = 0;
  int64_t padded_cells = 0;
  int launches = 0;
  int graph_hits = 0;
  int lanes_used[3] = {0, 0, 0};
  int row_pairs = 0;
  int seglen_max = 0;
  unsigned long long dev_stats[3] = {0, 0, 0};
};

double now_ms();

// Dense index of the distinct query lengths of a batch.
struct LengthIndex {
  std::vector<int> dense;               // m -> slot + 1 (0: not seen) for small m
  std::unordered_map<int, int> sparse;  // larger m
  std::vector<int> ms;                  // distinct lengths in first-seen order
  void reset(int max_m);
  int slot(int m);
};

// A pair as the per-pair packer reads it (sorted, compact).
struct PackRec {
  int pair, n, P, nch;
};

// Planner scratch kept between calls, so that large batches do not pay for
// fresh allocations (and their page faults) every time.
struct HostScratch {
  std::vector<int> order, count, bounds, slot, qstart, qcount, nlen, mlen;
  std::vector<PackRec> packed;
  std::vector<double> nsum;
  std::vector<int> nmax;
  std::vector<PlanItem> shared_items, per_pair;
  std::vector<swk::Task> tasks;
  LengthIndex lengths;
};

// Host threads for the planner's large passes, and a helper that runs
// fn(t, begin, end) over T contiguous ranges of [0, n) (the caller runs t = 0).
int host_threads();
void parallel_ranges(size_t n, int T, const std::function<void(int, size_t, size_t)> &fn);

// Sub-group widths (lanes) of a wavefront layout (bit r set <=> a sub-group
// starts at lane 16*r); returns their number.
int layout_groups(int layout, int widths[4]);
// Layouts the kernels run: 32-lane groups start at lane 0 or 32, no 48-lane
// groups, none wider than pmax.
bool layout_valid(int layout, int pmax);

// Instantiated graphs of recent executions, keyed by the full parameter
// signature of their device operations (least recently used evicted).
struct GraphCache {
  static constexpr size_t kMaxEntries = 8;
  struct Entry {
    std::vector<uint64_t> sig;
    hipGraphExec_t exec;
    uint64_t stamp;
  };
  std::vector<Entry> entries;
  uint64_t clock = 0;
  hipGraphExec_t find(const std::vector<uint64_t> &sig);
  void put(const std::vector<uint64_t> &sig, hipGraphExec_t exec);
  void clear();
};

constexpr int kSideStreams = 3;

// Work buffers used by one execution (the batch path owns one; the request
// server one per in-flight batch).
struct Workspace {
  DevBuf tasks, pairs, streams, results, bnd, misc, matrix, offs, plan;
  HostBuf staging;
  HostScratch host;
  GraphCache graphs;
  // side streams for concurrent per-pair launches (created on first use, on
  // the device current at that time), fork/join events
  hipStream_t side[kSideStreams] = {};
  hipEvent_t fork = nullptr, join[kSideStreams] = {};
  bool side_ready = false;
  int ensure_side_streams();
  // Sets the growth slack of every buffer (a long-lived caller whose batches
  // grow, such as a server worker, reallocates less often with more slack;
  // each reallocation frees the old buffer, which waits for the device).
  void set_growth(int pct, std::vector<void *> *dev_retired = nullptr,
                  std::vector<void *> *host_retired = nullptr) {
    for (DevBuf *b : {&tasks, &pairs, &streams, &results, &bnd, &misc, &matrix, &offs, &plan}) {
      b->grow_pct = pct;
      b->retired = dev_retired;
    }
    staging.grow_pct = pct;
    staging.retired = host_retired;
  }
  void release() {
    graphs.clear();
    if (side_ready) {
      for (int k = 0; k < kSideStreams; ++k) {
        (void)hipStreamDestroy(side[k]);
        (void)hipEventDestroy(join[k]);
      }
      (void)hipEventDestroy(fork);
      side_ready = false;
    }
    for (DevBuf *b : {&tasks, &pairs, &streams, &results, &bnd, &misc, &matrix, &offs, &plan})
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

// Checks a public batch description, builds the planner items and puts the
// PairInfo records, sequences and the residue check on the device.  The
// caller holds C.mu; `out` receives the empty result of every pair.
int prepare_batch(const sw_batch *b, const Scoring &S, Context &C, ExecInput &in,
                  sw_result *out, int64_t &cells);
// 1 if prepare_batch's residue check found a code >= alphabet_size, 0 if
// not, -1 on a device error.
int residue_flag(Context &C);

// Autotuner table (process-wide).  Lookups return false when no entry applies.
bool tune_lookup(int kind, swk::Prec prec, int alpha, int m, sw_tune_entry &e);
bool tune_mixed(swk::Prec prec, int alpha, int m_min, int m_max, sw_tune_entry &e);
int tune_validate(const sw_tune_entry &e);
// The per-pair (lanes, rows per lane) shapes of least modelled cost for items,
// best first; and the rows per lane of least modelled cost for mixed layouts.
std::vector<std::pair<int, int>> pair_candidates(swk::Prec prec, int alpha, const PlanItem *items,
                                                 size_t cnt, int max_cands);
std::vector<int> pair_mixed_candidates(swk::Prec prec, int alpha, const PlanItem *items,
                                       size_t cnt, int max_cands);

// Device-planned batch (one query, a compiled shape that holds it in one
// chunk): planner 0 = use it when the batch qualifies and has at least 4096
// pairs, 1 = never, 2 = always (SW_EINVAL when the batch does not qualify).
// `handled` is false when the caller must run the host planner instead (then
// nothing was launched and `out` is untouched).  The caller holds C.mu.
// first_row (start-cell passes; device memory, one int per pair, planner 2):
// one query, int16 row pairs, each pair aligning the query rows from
// first_row[k] on; saturated pairs are not rerun but keep kFlagNeedsI32.
int run_device_plan(const sw_batch *b, const Scoring &S, const ExecOptions &eo, int planner,
                    Context &C, sw_result *out, sw_stats *stats, double t0, bool &handled,
                    const int32_t *first_row = nullptr);
// Rows per virtual lane of the device planner's row-pair layout for a query of
// m residues (false if no compiled shape holds it in one chunk).
bool rowpair_shape(int m, int alpha, int &seg);
// The row-pair rows per lane force_seg if it holds a query of m residues
// within the planner's LDS budget.
bool rowpair_shape_forced(int m, int alpha, int force_seg, int &seg);

// The no-allocation batch call's scratch region for up to max_pairs pairs:
// the plan words, PairInfo records, the int32 rerun's results and the
// matrix, each 256-byte aligned.
constexpr size_t noalloc_align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t noalloc_scratch_bytes(size_t max_pairs) {
  return noalloc_align256(((size_t)swk::kPlanOrder + max_pairs) * sizeof(int32_t)) +
         noalloc_align256(max_pairs * sizeof(swk::PairInfo) + 4096) +
         noalloc_align256(max_pairs * sizeof(swk::DevResult)) +
         noalloc_align256(sizeof(int32_t) * swk::kMaxAlpha * swk::kMaxAlpha);
}
// sw_align_batch's device plan with every buffer in `scr` (a region of
// noalloc_scratch_bytes(max_pairs) bytes of device memory) and the results
// written to the device array `out`: allocates nothing.  The caller holds
// C.mu and has checked that b is device-resident with at most max_pairs pairs.
int run_device_plan_noalloc(const sw_batch *b, const Scoring &S, Context &C, unsigned char *scr,
                            int max_pairs, sw_result *out, sw_stats *stats, double t0);
// Looks up the scratch array's device address on the current device (once
// per device; the library's init calls it).  Defined beside the array.
int noalloc_setup(int device);

// Full batch semantics (int16 pass + int32 rerun) on prepared input.
int run_batch(const ExecInput &in, const Scoring &sc, int precision, const ExecOptions &opt,
              Workspace &ws, int n_pairs, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
              int num_cus, sw_result *out, sw_stats *stats);

}  // namespace swrt
