// Start cells and paths of a batch's alignments, and end-to-end scores of a
// batch (include/sw.h: sw_align_batch_starts, sw_align_batch_cigar,
// sw_align_batch_global).  The three share the batch loading and validation
// below and one set of work buffers, so their calls are serialised.
//
// The start of the reported alignment of a pair is the end cell of the same
// local alignment problem on the reversed prefixes q[0..query_end] and
// r[0..ref_end]: every optimal alignment inside the prefixes ends at the
// reported end cell (an alignment ending earlier would precede it in the
// (ref_end, query_end) order the end cell is chosen by), and the smallest end
// of the reversed problem is the largest start of the forward one.  The
// reversed prefixes are cut out on the device and aligned by the library's own
// kernels:
//
// * one query (the batch's pairs share it): every reversed query prefix is a
//   suffix of the reversed query, so all pairs run in one device-planned
//   row-pair launch on the whole reversed query, each pair with the rows
//   before its suffix masked (profile scores capped at 0); pairs whose int16
//   lanes saturate, and batches that do not fit that kernel, take the next path;
// * otherwise each reversed query prefix is a query of its own, through the
//   batch path (device or host planner, int32 reruns).
//
// Paths and end-to-end scores run the kernels of sw_trace.hip; this file
// builds their pair tables (validated on the host), sizes their scratch, and
// packs the paths' runs for the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <mutex>
#include <vector>

#include "sw.h"
#include "sw_internal.h"
#include "sw_trace.h"
#include "sw_runtime.h"

using namespace swrt;

namespace {

#define HIPCHK(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                __LINE__);                                                       \
      return SW_EDEVICE;                                                         \
    }                                                                            \
  } while (0)

// Grow-only device buffers and a stream of their own; one call at a time.
struct StartsWork {
  std::mutex mu;
  hipStream_t st = nullptr;
  DevBuf src_q, src_r;   // host-resident residue sets, uploaded
  DevBuf rev_q, rev_r;   // reversed query / prefixes
  DevBuf tab;            // offsets (int64), pair ids and first rows (int32)
  // paths
  DevBuf tr_pairs, tr_mat, tr_runs, tr_packed, tr_nruns, tr_off;
  HostBuf tr_host, tr_hcounts;   // pinned: the pair table, the run counts
  HostBuf ld_stage;              // pinned: a device-resident batch's offsets and indices
  DevBuf tr_res;                 // end-to-end results
  DevBuf tr_rstart;              // end-to-end paths: reference starts
  DevBuf tr_qstart;              // end-to-end paths: query starts
  HostBuf tr_hres;
  // host scratch of the path tables: each pair's rectangle and class (the
  // tables are built by host threads in two passes)
  std::vector<swk::TracePair> tr_rect;
  std::vector<uint8_t> tr_cls;
  // device-memory rectangles: the largest group, the second, the rest each on
  // a stream of their own, so the long poles of the largest rectangles (one
  // wavefront each) overlap instead of adding up
  static constexpr int kTraceStreams = 3;
  hipStream_t tr_st[kTraceStreams] = {};
  hipEvent_t tr_ready = nullptr, tr_done[kTraceStreams] = {};
  DevBuf tr_bits[kTraceStreams], tr_carry[kTraceStreams];
};
StartsWork g_starts;


// What every path needs: the batch's offsets and ids on the host, its residues
// on the device.
struct Batch {
  const sw_batch *b;
  const sw_result *ends;
  // offsets and pair indices on the host: the caller's arrays, or (device-
  // resident batches) a pinned copy; pq is all zeros without pair_query
  const int64_t *qoff = nullptr, *roff = nullptr;
  const int32_t *pq = nullptr, *pr = nullptr;
  std::vector<int32_t> pq_zero;
  const uint8_t *d_q = nullptr, *d_r = nullptr;
};

int upload(const std::vector<int64_t> *v64[4], size_t L1, const std::vector<int32_t> *v32[2],
           size_t L, StartsWork &W, int64_t *&d64, int32_t *&d32) {
  const size_t bytes = 4 * L1 * sizeof(int64_t) + 2 * L * sizeof(int32_t) + 64;
  int rc = W.tab.ensure(bytes);
  if (rc) return rc;
  d64 = W.tab.as<int64_t>();
  d32 = (int32_t *)(d64 + 4 * L1);
  for (int k = 0; k < 4; ++k)
    if (v64[k]) HIPCHK(hipMemcpyAsync(d64 + k * L1, v64[k]->data(), L1 * sizeof(int64_t),
                                      hipMemcpyHostToDevice, W.st));
  for (int k = 0; k < 2; ++k)
    if (v32[k] && L) HIPCHK(hipMemcpyAsync(d32 + k * L, v32[k]->data(), L * sizeof(int32_t),
                                           hipMemcpyHostToDevice, W.st));
  return SW_OK;
}

// One query: the masked row-pair launch on the reversed query.  Pairs it
// cannot finish (int16 saturation) are appended to `rest`.
int starts_masked(const Batch &B, const sw_scoring *sc, const Scoring &S,
                  const std::vector<int> &live, StartsWork &W, int32_t *query_start,
                  int32_t *ref_start, std::vector<int> &rest) {
  const int L = (int)live.size();
  const int q0 = B.pq[live[0]];   // every live pair's query
  const int64_t m = B.qoff[q0 + 1] - B.qoff[q0];
  std::vector<int64_t> rsrc, rdst{0};
  std::vector<int32_t> ids(L), first(L);
  for (int t = 0; t < L; ++t) {
    const int k = live[t];
    ids[t] = t;
    first[t] = (int32_t)(m - 1 - B.ends[k].query_end);
    rsrc.push_back(B.roff[B.pr[k]]);
    rdst.push_back(rdst.back() + B.ends[k].ref_end + 1);
  }
  rsrc.push_back(0);
  int rc;
  if ((rc = W.rev_q.ensure((size_t)m)) || (rc = W.rev_r.ensure((size_t)rdst.back()))) return rc;
  const size_t L1 = (size_t)L + 1;
  // table rows: [0] the query's source offset, [1] its reversed copy's
  // offsets {0, m}, [2] reference sources, [3] reversed prefix offsets
  std::vector<int64_t> qsrcL(L1, 0), qdstL(L1, 0);
  qsrcL[0] = B.qoff[q0];
  qdstL[1] = m;
  const std::vector<int64_t> *v64[4] = {&qsrcL, &qdstL, &rsrc, &rdst};
  const std::vector<int32_t> *v32[2] = {&ids, &first};
  int64_t *d64;
  int32_t *d32;
  if ((rc = upload(v64, L1, v32, (size_t)L, W, d64, d32))) return rc;
  HIPCHK(swk::launch_reverse_segments(1, B.d_q, d64, d64 + L1, W.rev_q.as<uint8_t>(), W.st));
  HIPCHK(swk::launch_reverse_segments(L, B.d_r, d64 + 2 * L1, d64 + 3 * L1,
                                      W.rev_r.as<uint8_t>(), W.st));
  HIPCHK(hipStreamSynchronize(W.st));
  sw_batch nb;
  std::memset(&nb, 0, sizeof(nb));
  nb.n_pairs = L;
  nb.query_res = W.rev_q.as<uint8_t>();
  nb.query_off = d64 + L1;          // {0, m}
  nb.n_queries = 1;
  nb.ref_res = W.rev_r.as<uint8_t>();
  nb.ref_off = d64 + 3 * L1;
  nb.n_refs = L;
  nb.pair_ref = d32;
  nb.precision = SW_PREC_AUTO;
  nb.device_resident = 1;
  nb.stream = W.st;
  std::vector<sw_result> rev(L);
  {
    std::lock_guard<std::mutex> g(g_ctx.mu);
    HIPCHK(hipSetDevice(g_ctx.device));
    ExecOptions eo;
    bool handled = false;
    rc = run_device_plan(&nb, S, eo, 2, g_ctx, rev.data(), nullptr, now_ms(), handled, d32 + L);
  }
  if (rc) return rc;
  (void)sc;
  for (int t = 0; t < L; ++t) {
    const int k = live[t];
    if (rev[t].flags & swk::kFlagNeedsI32) {
      rest.push_back(k);
      continue;
    }
    if (rev[t].score != B.ends[k].score) {
      set_error("pair %d: score %d is not this pair's optimum at its end cell (%d found)", k,
                B.ends[k].score, rev[t].score);
      return SW_EINVAL;
    }
    // reported rows count from the reversed query's first row
    query_start[k] = B.ends[k].query_end - (rev[t].query_end - first[t]);
    ref_start[k] = B.ends[k].ref_end - rev[t].ref_end;
  }
  return SW_OK;
}

// Each reversed query prefix as a query of its own, through the batch path.
int starts_per_pair(const Batch &B, const sw_scoring *sc, const std::vector<int> &live,
                    StartsWork &W, int32_t *query_start, int32_t *ref_start) {
  const int L = (int)live.size();
  std::vector<int64_t> qsrc, qdst{0}, rsrc, rdst{0};
  std::vector<int32_t> ids(L);
  for (int t = 0; t < L; ++t) {
    const int k = live[t];
    const int q = B.b->pair_query ? B.pq[k] : 0;
    ids[t] = t;
    qsrc.push_back(B.qoff[q]);
    qdst.push_back(qdst.back() + B.ends[k].query_end + 1);
    rsrc.push_back(B.roff[B.pr[k]]);
    rdst.push_back(rdst.back() + B.ends[k].ref_end + 1);
  }
  qsrc.push_back(0);
  rsrc.push_back(0);
  int rc;
  if ((rc = W.rev_q.ensure((size_t)qdst.back())) || (rc = W.rev_r.ensure((size_t)rdst.back())))
    return rc;
  const size_t L1 = (size_t)L + 1;
  const std::vector<int64_t> *v64[4] = {&qsrc, &qdst, &rsrc, &rdst};
  const std::vector<int32_t> *v32[2] = {&ids, nullptr};
  int64_t *d64;
  int32_t *d32;
  if ((rc = upload(v64, L1, v32, (size_t)L, W, d64, d32))) return rc;
  HIPCHK(swk::launch_reverse_segments(L, B.d_q, d64, d64 + L1, W.rev_q.as<uint8_t>(), W.st));
  HIPCHK(swk::launch_reverse_segments(L, B.d_r, d64 + 2 * L1, d64 + 3 * L1,
                                      W.rev_r.as<uint8_t>(), W.st));
  HIPCHK(hipStreamSynchronize(W.st));
  sw_batch nb;
  std::memset(&nb, 0, sizeof(nb));
  nb.n_pairs = L;
  nb.query_res = W.rev_q.as<uint8_t>();
  nb.query_off = d64 + L1;
  nb.n_queries = L;
  nb.ref_res = W.rev_r.as<uint8_t>();
  nb.ref_off = d64 + 3 * L1;
  nb.n_refs = L;
  nb.pair_query = d32;
  nb.pair_ref = d32;
  nb.precision = B.b->precision;
  nb.device_resident = 1;
  nb.stream = W.st;
  std::vector<sw_result> rev(L);
  if ((rc = sw_align_batch(&nb, sc, rev.data()))) return rc;
  for (int t = 0; t < L; ++t) {
    const int k = live[t];
    if (rev[t].score != B.ends[k].score) {
      set_error("pair %d: score %d is not this pair's optimum at its end cell (%d found)", k,
                B.ends[k].score, rev[t].score);
      return SW_EINVAL;
    }
    query_start[k] = B.ends[k].query_end - rev[t].query_end;
    ref_start[k] = B.ends[k].ref_end - rev[t].ref_end;
  }
  return SW_OK;
}

// The batch's offsets and pair ids on the host (validated), its residues on
// the device (uploaded when host-resident), in the order of the caller's
// stream.  Entry checks common to the starts and path calls.
int load_batch(const sw_batch *b, StartsWork &W, Batch &B) {
  const int np = b->n_pairs;
  HIPCHK(hipSetDevice(g_ctx.device));
  if (!W.st) HIPCHK(hipStreamCreateWithFlags(&W.st, hipStreamNonBlocking));
  const bool dev = b->device_resident != 0;
  if (dev && b->stream) {
    // the caller's stream produced the inputs
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, (hipStream_t)b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(W.st, ev, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(W.st);
    (void)hipEventDestroy(ev);
    HIPCHK(e);
  }
  B.b = b;
  const int64_t nq = b->n_queries, nr = b->n_refs;
  if (dev) {
    // one pinned staging area, four asynchronous copies, one wait
    const size_t bytes = (size_t)(nq + 1 + nr + 1) * 8 + (size_t)np * 8;
    int rc = W.ld_stage.ensure(std::max<size_t>(bytes, 8));
    if (rc) return rc;
    unsigned char *h = W.ld_stage.as<unsigned char>();
    int64_t *hq = (int64_t *)h, *hr = hq + nq + 1;
    int32_t *hpr = (int32_t *)(hr + nr + 1), *hpq = hpr + np;
    HIPCHK(hipMemcpyAsync(hq, b->query_off, (size_t)(nq + 1) * 8, hipMemcpyDeviceToHost, W.st));
    HIPCHK(hipMemcpyAsync(hr, b->ref_off, (size_t)(nr + 1) * 8, hipMemcpyDeviceToHost, W.st));
    if (np) HIPCHK(hipMemcpyAsync(hpr, b->pair_ref, (size_t)np * 4, hipMemcpyDeviceToHost, W.st));
    if (np && b->pair_query)
      HIPCHK(hipMemcpyAsync(hpq, b->pair_query, (size_t)np * 4, hipMemcpyDeviceToHost, W.st));
    HIPCHK(hipStreamSynchronize(W.st));
    B.qoff = hq;
    B.roff = hr;
    B.pr = hpr;
    B.pq = b->pair_query ? hpq : nullptr;
  } else {
    B.qoff = b->query_off;
    B.roff = b->ref_off;
    B.pr = b->pair_ref;
    B.pq = b->pair_query;
  }
  if (!B.pq) {
    B.pq_zero.assign(np, 0);
    B.pq = B.pq_zero.data();
  }
  // validation on host threads; each check reports the first failing entry
  const int T = std::max<int64_t>({nq, nr, (int64_t)np}) >= 65536 ? host_threads() : 1;
  auto first_bad = [&](int64_t n, auto bad) -> int64_t {
    std::vector<int64_t> at(T, INT64_MAX);
    parallel_ranges((size_t)n, T, [&](int t, size_t lo, size_t hi) {
      for (size_t k = lo; k < hi; ++k)
        if (bad((int64_t)k)) { at[t] = (int64_t)k; return; }
    });
    return *std::min_element(at.begin(), at.end());
  };
  if (first_bad(nq, [&](int64_t k) { return B.qoff[k] < 0 || B.qoff[k + 1] < B.qoff[k]; }) != INT64_MAX) {
    set_error("query offsets not nondecreasing");
    return SW_EINVAL;
  }
  if (first_bad(nr, [&](int64_t k) { return B.roff[k] < 0 || B.roff[k + 1] < B.roff[k]; }) != INT64_MAX) {
    set_error("reference offsets not nondecreasing");
    return SW_EINVAL;
  }
  const int64_t kp = first_bad(np, [&](int64_t k) {
    return B.pq[k] < 0 || B.pq[k] >= nq || B.pr[k] < 0 || B.pr[k] >= nr;
  });
  if (kp != INT64_MAX) {
    set_error("pair %d refers to a query or reference out of range", (int)kp);
    return SW_EINVAL;
  }
  B.d_q = b->query_res;
  B.d_r = b->ref_res;
  if (!dev) {
    const size_t qb = (size_t)B.qoff[b->n_queries], rb = (size_t)B.roff[b->n_refs];
    int rc;
    if ((rc = W.src_q.ensure(qb + 1)) || (rc = W.src_r.ensure(rb + 1))) return rc;
    if (qb) HIPCHK(hipMemcpyAsync(W.src_q.p, b->query_res, qb, hipMemcpyHostToDevice, W.st));
    if (rb) HIPCHK(hipMemcpyAsync(W.src_r.p, b->ref_res, rb, hipMemcpyHostToDevice, W.st));
    B.d_q = W.src_q.as<uint8_t>();
    B.d_r = W.src_r.as<uint8_t>();
  }
  return SW_OK;
}

int check_batch_args(const sw_batch *b) {
  if (!b) { set_error("batch is NULL"); return SW_EINVAL; }
  if (b->n_pairs < 0 || b->n_queries < 0 || b->n_refs < 0) { set_error("negative count"); return SW_EINVAL; }
  if (b->precision != SW_PREC_AUTO && b->precision != SW_PREC_I32) { set_error("bad precision"); return SW_EINVAL; }
  if (b->n_pairs > 0 && (!b->query_off || !b->ref_off || !b->pair_ref || b->n_queries < 1 || b->n_refs < 1)) {
    set_error("batch arrays are NULL or empty");
    return SW_EINVAL;
  }
  return SW_OK;
}

}  // namespace

extern "C" int sw_align_batch_starts(const sw_batch *b, const sw_scoring *sc,
                                     const sw_result *ends, int32_t *query_start,
                                     int32_t *ref_start) {
  int rc = check_batch_args(b);
  if (rc) return rc;
  Scoring S;
  if ((rc = prepare_scoring(sc, S))) return rc;
  const int np = b->n_pairs;
  if (np == 0) return SW_OK;
  if (!ends || !query_start || !ref_start) { set_error("ends or an output array is NULL"); return SW_EINVAL; }
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_starts.mu);
  StartsWork &W = g_starts;
  Batch B;
  B.ends = ends;
  if ((rc = load_batch(b, W, B))) return rc;
  std::vector<int> live;
  bool one_query = true;
  for (int k = 0; k < np; ++k) {
    const sw_result &e = ends[k];
    query_start[k] = ref_start[k] = -1;
    if (e.score <= 0) continue;
    const int64_t m = B.qoff[B.pq[k] + 1] - B.qoff[B.pq[k]];
    const int64_t n = B.roff[B.pr[k] + 1] - B.roff[B.pr[k]];
    if (e.query_end < 0 || e.query_end >= m || e.ref_end < 0 || e.ref_end >= n) {
      set_error("pair %d: end cell (%d, %d) outside its %lld x %lld sequences", k, e.query_end,
                e.ref_end, (long long)m, (long long)n);
      return SW_EINVAL;
    }
    one_query = one_query && B.pq[k] == B.pq[live.empty() ? k : live[0]];
    live.push_back(k);
  }
  if (live.empty()) return SW_OK;
  std::vector<int> rest;
  int seg = 0;
  const int q0 = B.pq[live[0]];
  const int64_t m0 = B.qoff[q0 + 1] - B.qoff[q0];
  if (one_query && b->precision == SW_PREC_AUTO && S.fits_i16 && m0 <= 512 &&
      rowpair_shape((int)m0, S.alpha, seg)) {
    rc = starts_masked(B, sc, S, live, W, query_start, ref_start, rest);
  } else {
    rest = live;
  }
  if (!rc && !rest.empty()) rc = starts_per_pair(B, sc, rest, W, query_start, ref_start);
  if (rc) {
    for (int u = 0; u < np; ++u) query_start[u] = ref_start[u] = -1;
    return rc;
  }
  return SW_OK;
}

// ------------------------------------------------------------------ paths

namespace {

constexpr int64_t kTraceScratchBytes = 1ll << 30;    // device-memory decision bits per launch
constexpr int kTraceMaxWaves = 4096;
constexpr int kDualCols = 160;   // end-to-end queries up to this length run two per wavefront

// Runs a path can have between start and end: every run but the first is
// preceded by a change of operation, M runs alternate with one or two gap
// runs, and a rectangle of A x B cells holds at most min(A, B) pairs.
int64_t run_bound(int64_t A, int64_t B) {
  return std::min(A + B - 1, 3 * std::min(A, B) - 2);
}

// 2-byte units of a rectangle's decision words: rows x tiles x 64 lanes x
// the word width of its variant
int64_t trace_slot_words(const swk::TracePair &P) {
  int64_t tiles;
  switch (swk::trace_cols(P.pad)) {   // constant divisors (the tables hold millions)
    case 1: tiles = (P.B + 63) / 64; break;
    case 2: tiles = (P.B + 127) / 128; break;
    case 3: tiles = (P.B + 191) / 192; break;
    case 8: tiles = (P.B + 511) / 512; break;
    default: tiles = (P.B + 255) / 256; break;
  }
  return (int64_t)P.A * tiles * 64 * (swk::trace_word_bytes(P.pad) / 2);
}

// Size class of a device-memory rectangle: its variant and the power of two
// below its slot, largest first.  Every member of a class needs more than
// half the largest member's slot, so one class is one launch group.
constexpr int kSlotBuckets = 40;   // slots below 2^40 words
int trace_size_class(int64_t slot, int variant) {
  const int b = std::min(kSlotBuckets - 1, 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(slot, 1)));
  return (kSlotBuckets - 1 - b) * 3 + variant;
}

}  // namespace

// Paths of a batch: mode 0 the local alignments between start and end cells
// (sw_align_batch_cigar), modes 1-4 whole end-to-end alignments (the API's
// mode + 1: global, semi-global query fitted, semi-global reference fitted,
// overlap) from their end cells (sw_align_batch_global_cigar;
// query_start_out / ref_start_out receive the start element + 1).
namespace {
int paths_impl(const sw_batch *b, const sw_scoring *sc, int mode, const sw_result *ends,
               const int32_t *query_start, const int32_t *ref_start, int32_t *query_start_out,
               int32_t *ref_start_out, uint32_t *cigar, int64_t cigar_cap, int64_t *cigar_off) {
  int rc = check_batch_args(b);
  if (rc) return rc;
  Scoring S;
  if ((rc = prepare_scoring(sc, S))) return rc;
  const int np = b->n_pairs;
  if (!cigar_off) { set_error("cigar_off is NULL"); return SW_EINVAL; }
  cigar_off[0] = 0;
  if (np == 0) return SW_OK;
  if (!ends || (mode == 0 && (!query_start || !ref_start)) ||
      (mode != 0 && (!ref_start_out || !query_start_out))) {
    set_error("ends, starts or the start outputs are NULL");
    return SW_EINVAL;
  }
  // end-to-end modes: which prefixes are free (virtual start elements (v, -1)
  // and (-1, w)) and where an end cell may lie
  const bool col_free = mode == 2 || mode == 4, row_free = mode == 3 || mode == 4;
  static const char *const kModeName[] = {"local", "global", "semi-global (query fitted)",
                                          "semi-global (reference fitted)", "overlap"};
  if (cigar_cap < 0 || (cigar_cap > 0 && !cigar)) { set_error("cigar is NULL or its capacity negative"); return SW_EINVAL; }
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_starts.mu);
  StartsWork &W = g_starts;
  Batch B;
  B.ends = ends;
  if ((rc = load_batch(b, W, B))) return rc;
  int64_t maxabs = 0;
  for (int v : S.M) maxabs = std::max<int64_t>(maxabs, v < 0 ? -(int64_t)v : v);
  // the table lives in pinned memory (one fast upload)
  if ((rc = W.tr_host.ensure((size_t)np * sizeof(swk::TracePair))) ||
      (rc = W.tr_hcounts.ensure((size_t)np * sizeof(int32_t))))
    return rc;
  swk::TracePair *htab = W.tr_host.as<swk::TracePair>();
  int64_t region = 0;
  // ---- one rectangle per pair with a positive score, built by host threads:
  // pass 1 classifies every pair (its rectangle, kernel variant and size
  // class, or an error, or runs made here), pass 2 lays the classes out
  // (LDS rectangles by variant, then device-memory ones by size class,
  // largest first; within a class in pair order) and assigns run regions in
  // pair order, pass 3 writes the table straight into pinned memory
  auto gap = [&](int64_t L) -> int64_t { return L <= 0 ? 0 : S.go + (L - 1) * (int64_t)S.ge; };
  // end-to-end alignments with an empty side: at most a D and an I run
  struct HostRun { int k; int n; uint32_t run[2]; };
  constexpr int NCLS = 3 + kSlotBuckets * 3;     // LDS variants, then size classes
  constexpr uint8_t kSkip = 0xff, kHost = 0xfe;
  // classifies pair k: kSkip (no path), kHost (runs in *hr), a class with the
  // rectangle in *tp, or an error (returns its code; with report, sets the message)
  auto classify = [&](int k, bool report, swk::TracePair *tp, HostRun *hr,
                      uint8_t *cls) -> int {
    const sw_result &e = ends[k];
    const int64_t m = B.qoff[B.pq[k] + 1] - B.qoff[B.pq[k]];
    const int64_t n = B.roff[B.pr[k] + 1] - B.roff[B.pr[k]];
    int qs = 0, rs = 0;
    *cls = kSkip;
    if (mode == 0) {
      if (e.score <= 0) return SW_OK;
      qs = query_start[k];
      rs = ref_start[k];
      if (qs < 0 || qs > e.query_end || e.query_end >= m || rs < 0 || rs > e.ref_end ||
          e.ref_end >= n) {
        if (report)
          set_error("pair %d: start (%d, %d) and end (%d, %d) are not a rectangle of its %lld x "
                    "%lld sequences", k, qs, rs, e.query_end, e.ref_end, (long long)m, (long long)n);
        return SW_EINVAL;
      }
    } else {
      const bool in = e.ref_end >= -1 && e.ref_end < n && e.query_end >= -1 && e.query_end < m;
      const bool on_q = e.query_end == m - 1, on_r = e.ref_end == n - 1;
      const bool ok = mode == 1 ? on_q && on_r : mode == 2 ? on_q : mode == 3 ? on_r : on_q || on_r;
      if (!in || !ok) {
        if (report)
          set_error("pair %d: end (%d, %d) is not the end cell of a %s alignment of its %lld x "
                    "%lld sequences", k, e.query_end, e.ref_end, kModeName[mode], (long long)m,
                    (long long)n);
        return SW_EINVAL;
      }
      if (e.query_end < 0 || e.ref_end < 0) {
        // nothing to pair: runs from the best virtual start element -- the
        // largest (ref, query) one -- to the end cell
        const int64_t A0 = e.ref_end + 1, B0 = e.query_end + 1;
        int64_t best = INT64_MIN, bx = 0, by = 0;
        auto consider = [&](int64_t x, int64_t y) {   // element (x, y): its value at the end
          const int64_t v = -gap(A0 - 1 - x) - gap(B0 - 1 - y);
          if (v > best || (v == best && (x > bx || (x == bx && y > by)))) {
            best = v;
            bx = x;
            by = y;
          }
        };
        consider(-1, -1);
        for (int64_t x = 0; col_free && x < A0; ++x) consider(x, -1);
        for (int64_t y = 0; row_free && y < B0; ++y) consider(-1, y);
        if (e.score != best) {
          if (report)
            set_error("pair %d: score %d is not the optimum at the end cell (%d, %d)", k, e.score,
                      e.query_end, e.ref_end);
          return SW_EINVAL;
        }
        hr->k = k;
        hr->n = 0;
        if (A0 - 1 - bx) hr->run[hr->n++] = (uint32_t)(A0 - 1 - bx) << 4 | swk::kCigarD;
        if (B0 - 1 - by) hr->run[hr->n++] = (uint32_t)(B0 - 1 - by) << 4 | swk::kCigarI;
        ref_start_out[k] = (int32_t)(bx + 1);
        query_start_out[k] = (int32_t)(by + 1);
        *cls = kHost;
        return SW_OK;
      }
    }
    const int64_t A = e.ref_end - rs + 1, Bq = e.query_end - qs + 1;
    // every reachable value stays above -2^28 and every row term below 2^30,
    // so unreachable values (near -2^30) never meet reachable ones
    const int64_t lo = 2 * (maxabs + S.go) + (A + Bq + 2 * swk::kTraceTileCols) * (S.ge + 1);
    const int64_t hi = std::min(A, Bq) * (int64_t)S.max_s + (Bq + swk::kTraceTileCols) * S.ge;
    if (lo >= (1ll << 27) || hi >= (1ll << 30)) {
      if (report)
        set_error("pair %d: a %lld x %lld rectangle leaves the int32 range of the path kernel", k,
                  (long long)A, (long long)Bq);
      return SW_EOVERFLOW;
    }
    tp->q = B.qoff[B.pq[k]] + qs;
    tp->r = B.roff[B.pr[k]] + rs;
    tp->out = 0;
    tp->A = (int32_t)A;
    tp->B = (int32_t)Bq;
    tp->score = e.score;
    // end-to-end: k <= min(A, B) pairs, k M runs and two gap runs in each of the
    // k + 1 gaps (start, between pairs, end)
    tp->cap = (int32_t)(mode == 0 ? run_bound(A, Bq) : std::min(A + Bq + 2, 3 * std::min(A, Bq) + 2));
    tp->id = k;
    // columns per lane: the fewest that hold a one-tile query (4 beyond), so
    // a one-tile query's slot of 64-lane rows is the same at any count
    tp->pad = (int32_t)std::min<int64_t>(4, (Bq + 63) / 64);
    // 16-bit values (4 or 8 columns per lane) when the rectangle's range
    // provably fits: every reachable value -- a pair and two gap runs from
    // the start or a boundary, plus a gap opening, or a scan term with its
    // tile offset -- stays above every value derived from an unreachable
    // edge (-32768 plus a score, a tile's scan offsets and an opening), and
    // the largest chain score with its tile offset stays below 32767
    if (Bq > 64) {
      const int64_t tc = Bq <= 256 ? 256 : 512;
      const int64_t span = 5 * (maxabs + S.go) + (A + Bq + 3 + tc) * (int64_t)S.ge + 256;
      const int64_t top = std::min(A, Bq) * (int64_t)S.max_s + tc * S.ge + maxabs + 256;
      if (span < 32768 && top < 32767) tp->pad = swk::kTracePad16 | (int32_t)(tc / 64);
    }
    const int64_t slot = trace_slot_words(*tp);
    const int variant = swk::trace_variant(tp->pad);
    if (slot <= (int64_t)swk::kTraceLdsRowTiles * 64) {
      // LDS rectangles in runs of one kernel variant (one launch each), the
      // common 16-bit four-column one first
      *cls = (uint8_t)(variant == swk::kTraceV16x4 ? 0 : variant == swk::kTraceV32 ? 1 : 2);
    } else {
      if (slot * 2 > (2ll << 30)) {
        if (report)
          set_error("pair %d: a %lld x %lld rectangle needs more than 2 GiB of path scratch", k,
                    (long long)A, (long long)Bq);
        return SW_ENOMEM;
      }
      *cls = (uint8_t)(3 + trace_size_class(slot, variant));
    }
    return SW_OK;
  };

  if (W.tr_rect.size() < (size_t)np) W.tr_rect.resize(np);
  if (W.tr_cls.size() < (size_t)np) W.tr_cls.resize(np);
  swk::TracePair *rect = W.tr_rect.data();
  uint8_t *cls = W.tr_cls.data();
  const int T = np >= 65536 ? host_threads() : 1;
  struct Part {
    int64_t count[NCLS] = {}, caps = 0, cslot[NCLS] = {};
    int crows[NCLS] = {};
    int first_err = INT32_MAX;
    std::vector<HostRun> host;
  };
  std::vector<Part> part(T);
  parallel_ranges((size_t)np, T, [&](int t, size_t lo, size_t hi) {
    Part &P = part[t];
    for (size_t k = lo; k < hi; ++k) {
      if (mode != 0) {
        ref_start_out[k] = 0;
        query_start_out[k] = 0;
      }
      HostRun hr;
      if (classify((int)k, false, &rect[k], &hr, &cls[k]) != SW_OK) {
        P.first_err = (int)k;
        return;
      }
      const uint8_t c = cls[k];
      if (c == kHost) {
        P.host.push_back(hr);
      } else if (c != kSkip) {
        ++P.count[c];
        P.caps += rect[k].cap;
        P.cslot[c] = std::max(P.cslot[c], trace_slot_words(rect[k]));
        P.crows[c] = std::max(P.crows[c], rect[k].A);
      }
    }
  });
  {
    int first = INT32_MAX;
    for (const Part &P : part) first = std::min(first, P.first_err);
    if (first != INT32_MAX) {   // the first failing pair, as a serial pass finds it
      swk::TracePair tp;
      HostRun hr;
      uint8_t c;
      return classify(first, true, &tp, &hr, &c);
    }
  }
  // class layout, and each thread's first slot in every class and region
  int64_t cstart[NCLS + 1] = {}, cslot[NCLS] = {};
  int crows[NCLS] = {};
  for (int c = 0; c < NCLS; ++c) {
    int64_t cnt = 0;
    for (const Part &P : part) {
      cnt += P.count[c];
      cslot[c] = std::max(cslot[c], P.cslot[c]);
      crows[c] = std::max(crows[c], P.crows[c]);
    }
    cstart[c + 1] = cstart[c] + cnt;
  }
  const int nl = (int)cstart[3], nt = (int)cstart[NCLS], ng = nt - nl;
  std::vector<std::array<int64_t, NCLS>> tpos(T);
  std::vector<int64_t> treg(T);
  {
    int64_t run[NCLS];
    std::memcpy(run, cstart, sizeof(run));
    int64_t reg = 0;
    for (int t = 0; t < T; ++t) {
      for (int c = 0; c < NCLS; ++c) {
        tpos[t][c] = run[c];
        run[c] += part[t].count[c];
      }
      treg[t] = reg;
      reg += part[t].caps;
    }
    region = reg;
  }
  parallel_ranges((size_t)np, T, [&](int t, size_t lo, size_t hi) {
    int64_t reg = treg[t];
    std::array<int64_t, NCLS> &pos = tpos[t];
    for (size_t k = lo; k < hi; ++k) {
      const uint8_t c = cls[k];
      if (c >= NCLS) continue;
      swk::TracePair tp = rect[k];
      tp.out = reg;
      reg += tp.cap;
      htab[pos[c]++] = tp;
    }
  });
  std::vector<HostRun> host_runs;
  for (Part &P : part) host_runs.insert(host_runs.end(), P.host.begin(), P.host.end());
  // one launch group per device-memory size class
  struct Group { int first, count, waves; int64_t slot_words; int carry_rows; int variant; };
  std::vector<Group> groups;
  constexpr int NS = StartsWork::kTraceStreams;
  int64_t bits_words[NS] = {}, carry_ints[NS] = {};
  for (int c = 3; c < NCLS; ++c) {
    const int64_t cnt = cstart[c + 1] - cstart[c];
    if (!cnt) continue;
    const int64_t slot = cslot[c];
    const int carry_rows = std::max(1, crows[c]);
    const int64_t per_wave = slot * 2 + 6ll * carry_rows * 4;
    const int waves = (int)std::max<int64_t>(
        1, std::min<int64_t>({cnt, kTraceScratchBytes / per_wave, kTraceMaxWaves}));
    const int sk = std::min((int)groups.size(), NS - 1);
    groups.push_back({(int)(cstart[c] - nl), (int)cnt, waves, slot, carry_rows, (c - 3) % 3});
    bits_words[sk] = std::max<int64_t>(bits_words[sk], slot * waves);
    carry_ints[sk] = std::max<int64_t>(carry_ints[sk], 6ll * carry_rows * waves);
  }
  (void)ng;
  std::vector<int32_t> counts(np, 0);
  if (nt > 0) {
    if ((rc = W.tr_pairs.ensure((size_t)nt * sizeof(swk::TracePair))) ||
        (rc = W.tr_mat.ensure((size_t)S.alpha * S.alpha * sizeof(int32_t))) ||
        (rc = W.tr_runs.ensure((size_t)std::max<int64_t>(region, 1) * sizeof(uint32_t))) ||
        (rc = W.tr_nruns.ensure((size_t)np * sizeof(int32_t))) ||
        (rc = W.tr_off.ensure((size_t)(np + 1) * sizeof(int64_t))) ||
        (rc = W.tr_rstart.ensure((size_t)np * sizeof(int32_t))) ||
        (rc = W.tr_qstart.ensure((size_t)np * sizeof(int32_t))))
      return rc;
    for (int k = 0; k < NS && k < (int)groups.size(); ++k) {
      if ((rc = W.tr_bits[k].ensure((size_t)std::max<int64_t>(bits_words[k], 1) * sizeof(uint16_t))) ||
          (rc = W.tr_carry[k].ensure((size_t)std::max<int64_t>(carry_ints[k], 1) * sizeof(int32_t))))
        return rc;
      if (!W.tr_st[k]) HIPCHK(hipStreamCreateWithFlags(&W.tr_st[k], hipStreamNonBlocking));
      if (!W.tr_done[k]) HIPCHK(hipEventCreateWithFlags(&W.tr_done[k], hipEventDisableTiming));
    }
    if (!W.tr_ready) HIPCHK(hipEventCreateWithFlags(&W.tr_ready, hipEventDisableTiming));
    swk::TracePair *dp = W.tr_pairs.as<swk::TracePair>();
    HIPCHK(hipMemcpyAsync(dp, htab, (size_t)nt * sizeof(swk::TracePair), hipMemcpyHostToDevice,
                          W.st));
    HIPCHK(hipMemcpyAsync(W.tr_mat.p, S.M.data(), (size_t)S.alpha * S.alpha * sizeof(int32_t),
                          hipMemcpyHostToDevice, W.st));
    swk::TraceArgs ta;
    ta.qres = B.d_q;
    ta.rres = B.d_r;
    ta.matrix = W.tr_mat.as<int32_t>();
    ta.alpha = S.alpha;
    ta.go = S.go;
    ta.ge = S.ge;
    ta.cigar = W.tr_runs.as<uint32_t>();
    ta.n_runs = W.tr_nruns.as<int32_t>();
    ta.mode = mode;
    ta.ref_start = W.tr_rstart.as<int32_t>();
    ta.query_start = W.tr_qstart.as<int32_t>();
    ta.pairs = dp;
    ta.n = nl;
    ta.slot_words = 0;
    ta.carry_rows = 0;
    ta.gbits = nullptr;
    ta.gcarry = nullptr;
    const int used = std::min((int)groups.size(), NS);
    if (used) HIPCHK(hipEventRecord(W.tr_ready, W.st));
    for (int k = 0; k < used; ++k) HIPCHK(hipStreamWaitEvent(W.tr_st[k], W.tr_ready, 0));
    for (int lo = 0; lo < nl;) {                   // one LDS launch per variant
      const int v = swk::trace_variant(htab[lo].pad);
      int hi = lo;
      while (hi < nl && swk::trace_variant(htab[hi].pad) == v) ++hi;
      ta.pairs = dp + lo;
      ta.n = hi - lo;
      HIPCHK(swk::launch_trace(true, v, ta, hi - lo, W.st));
      lo = hi;
    }
    for (int g = 0; g < (int)groups.size(); ++g) {
      const Group &gr = groups[g];
      const int k = std::min(g, NS - 1);
      ta.pairs = dp + nl + gr.first;
      ta.n = gr.count;
      ta.slot_words = gr.slot_words;
      ta.carry_rows = gr.carry_rows;
      ta.gbits = W.tr_bits[k].as<uint16_t>();
      ta.gcarry = W.tr_carry[k].as<int32_t>();
      HIPCHK(swk::launch_trace(false, gr.variant, ta, gr.waves, W.tr_st[k]));
    }
    for (int k = 0; k < used; ++k) {
      HIPCHK(hipEventRecord(W.tr_done[k], W.tr_st[k]));
      HIPCHK(hipStreamWaitEvent(W.st, W.tr_done[k], 0));
    }
    int32_t *dev_counts = W.tr_hcounts.as<int32_t>();
    HIPCHK(hipMemcpyAsync(dev_counts, W.tr_nruns.p, (size_t)np * sizeof(int32_t),
                          hipMemcpyDeviceToHost, W.st));
    std::vector<int32_t> dev_rstart, dev_qstart;
    if (mode != 0) {
      dev_rstart.resize(np);
      dev_qstart.resize(np);
      HIPCHK(hipMemcpyAsync(dev_rstart.data(), W.tr_rstart.p, (size_t)np * sizeof(int32_t),
                            hipMemcpyDeviceToHost, W.st));
      HIPCHK(hipMemcpyAsync(dev_qstart.data(), W.tr_qstart.p, (size_t)np * sizeof(int32_t),
                            hipMemcpyDeviceToHost, W.st));
    }
    HIPCHK(hipStreamSynchronize(W.st));
    // run counts by pair; the first entry of the table (LDS rectangles, then
    // device-memory ones) with an error is reported
    auto check = [&](int t, bool report) -> int {
      const swk::TracePair &P = htab[t];
      const int c = dev_counts[P.id];
      if (c == swk::kTraceBadResidue) {
        if (report)
          set_error("pair %d: a residue code inside its alignment is not below alphabet_size", P.id);
        return SW_EINVAL;
      }
      if (c == swk::kTraceInconsistent) {
        if (!report) return SW_EINVAL;
        if (mode == 0)
          set_error("pair %d: no alignment of score %d runs from its start (%d, %d) to its end "
                    "(%d, %d)", P.id, P.score, query_start[P.id], ref_start[P.id],
                    ends[P.id].query_end, ends[P.id].ref_end);
        else
          set_error("pair %d: score %d is not the optimum at the end cell (%d, %d)", P.id,
                    P.score, ends[P.id].query_end, ends[P.id].ref_end);
        return SW_EINVAL;
      }
      if (c < 1 || c > P.cap) {
        if (report) set_error("pair %d: internal path error (%d runs, bound %d)", P.id, c, P.cap);
        return SW_EDEVICE;
      }
      counts[P.id] = c;
      if (mode != 0) {
        ref_start_out[P.id] = dev_rstart[P.id];
        query_start_out[P.id] = dev_qstart[P.id];
      }
      return SW_OK;
    };
    const int TT = nt >= 65536 ? host_threads() : 1;
    std::vector<int> bad(TT, INT32_MAX);
    parallel_ranges((size_t)nt, TT, [&](int th, size_t lo, size_t hi) {
      for (size_t t = lo; t < hi; ++t)
        if (check((int)t, false) != SW_OK) { bad[th] = (int)t; return; }
    });
    const int first = *std::min_element(bad.begin(), bad.end());
    if (first != INT32_MAX) return check(first, true);
  }
  for (const HostRun &hr : host_runs) counts[hr.k] = hr.n;
  {  // cigar_off: an exclusive prefix sum of the counts, two passes on host threads
    const int TP = np >= 65536 ? host_threads() : 1;
    std::vector<int64_t> base(TP + 1, 0);
    parallel_ranges((size_t)np, TP, [&](int t, size_t lo, size_t hi) {
      int64_t sum = 0;
      for (size_t k = lo; k < hi; ++k) sum += counts[k];
      base[t + 1] = sum;
    });
    for (int t = 0; t < TP; ++t) base[t + 1] += base[t];
    parallel_ranges((size_t)np, TP, [&](int t, size_t lo, size_t hi) {
      int64_t run = base[t];
      for (size_t k = lo; k < hi; ++k) cigar_off[k + 1] = run += counts[k];
    });
  }
  if (cigar_off[np] > cigar_cap) {
    set_error("the paths need %lld runs, cigar holds %lld", (long long)cigar_off[np],
              (long long)cigar_cap);
    return SW_EINVAL;
  }
  if (nt > 0 && cigar_off[np] > 0) {
    if ((rc = W.tr_packed.ensure((size_t)cigar_off[np] * sizeof(uint32_t)))) return rc;
    HIPCHK(hipMemcpyAsync(W.tr_off.p, cigar_off, (size_t)(np + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, W.st));
    HIPCHK(swk::launch_pack_runs(W.tr_pairs.as<swk::TracePair>(), nt, W.tr_nruns.as<int32_t>(),
                                 W.tr_off.as<int64_t>(), W.tr_runs.as<uint32_t>(),
                                 W.tr_packed.as<uint32_t>(), W.st));
    HIPCHK(hipMemcpyAsync(cigar, W.tr_packed.p, (size_t)cigar_off[np] * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, W.st));
    HIPCHK(hipStreamSynchronize(W.st));
  }
  for (const HostRun &hr : host_runs) std::copy(hr.run, hr.run + hr.n, cigar + cigar_off[hr.k]);
  return SW_OK;
}
}  // namespace

extern "C" int sw_align_batch_cigar(const sw_batch *b, const sw_scoring *sc,
                                    const sw_result *ends, const int32_t *query_start,
                                    const int32_t *ref_start, uint32_t *cigar,
                                    int64_t cigar_cap, int64_t *cigar_off) {
  return paths_impl(b, sc, 0, ends, query_start, ref_start, nullptr, nullptr, cigar, cigar_cap,
                    cigar_off);
}

extern "C" int sw_align_batch_global_cigar(const sw_batch *b, const sw_scoring *sc, int32_t mode,
                                           const sw_result *ends, int32_t *query_start,
                                           int32_t *ref_start, uint32_t *cigar,
                                           int64_t cigar_cap, int64_t *cigar_off) {
  if (mode < SW_MODE_GLOBAL || mode > SW_MODE_OVERLAP) {
    set_error("bad mode %d", mode);
    if (cigar_off) cigar_off[0] = 0;
    return SW_EINVAL;
  }
  return paths_impl(b, sc, mode + 1, ends, nullptr, nullptr, query_start, ref_start, cigar,
                    cigar_cap, cigar_off);
}


// ------------------------------------------------------------------ end-to-end scores

extern "C" int sw_align_batch_global(const sw_batch *b, const sw_scoring *sc, int32_t mode,
                                     sw_result *out) {
  int rc = check_batch_args(b);
  if (rc) return rc;
  if (mode < SW_MODE_GLOBAL || mode > SW_MODE_OVERLAP) { set_error("bad mode %d", mode); return SW_EINVAL; }
  Scoring S;
  if ((rc = prepare_scoring(sc, S))) return rc;
  const int np = b->n_pairs;
  if (np == 0) return SW_OK;
  if (!out) { set_error("out is NULL"); return SW_EINVAL; }
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_starts.mu);
  StartsWork &W = g_starts;
  Batch B;
  if ((rc = load_batch(b, W, B))) return rc;
  int64_t maxabs = 0;
  for (int v : S.M) maxabs = std::max<int64_t>(maxabs, v < 0 ? -(int64_t)v : v);
  auto gap = [&](int64_t L) -> int64_t { return L <= 0 ? 0 : S.go + (L - 1) * (int64_t)S.ge; };
  if ((rc = W.tr_host.ensure((size_t)np * sizeof(swk::TracePair)))) return rc;
  swk::TracePair *htab = W.tr_host.as<swk::TracePair>();
  int n1 = 0;                        // one-tile pairs first, then the rest
  std::vector<swk::TracePair> single, multi;   // one-tile pairs with m > 160; longer ones
  int carry_rows = 0;
  for (int k = 0; k < np; ++k) {
    const int64_t m = B.qoff[B.pq[k] + 1] - B.qoff[B.pq[k]];
    const int64_t n = B.roff[B.pr[k] + 1] - B.roff[B.pr[k]];
    if (m == 0 || n == 0) {          // a side with nothing to align: one gap run (or none)
      // the charged sides' runs; ends where the charged sides are used up,
      // the smallest (ref_end, query_end) among the free choices
      const bool qc = mode == SW_MODE_GLOBAL || mode == SW_MODE_SEMIGLOBAL;
      const bool rc_ = mode == SW_MODE_GLOBAL || mode == SW_MODE_SEMIGLOBAL_REF;
      const int64_t s = -(qc ? gap(m) : 0) - (rc_ ? gap(n) : 0);
      out[k].score = (int32_t)s;
      out[k].query_end = qc ? (int32_t)(m - 1) : -1;
      out[k].ref_end = rc_ ? (int32_t)(n - 1) : -1;
      out[k].flags = 0;
      if (s < INT32_MIN) { set_error("pair %d: score below the int32 range", k); return SW_EOVERFLOW; }
      continue;
    }
    const int64_t lo = 2 * (maxabs + S.go) + (m + n + 2 * swk::kTraceTileCols) * (S.ge + 1);
    const int64_t hi = std::min(m, n) * (int64_t)S.max_s + (m + swk::kTraceTileCols) * S.ge;
    if (lo >= (1ll << 27) || hi >= (1ll << 30)) {
      set_error("pair %d: %lld x %lld leaves the int32 range of the end-to-end kernel", k,
                (long long)m, (long long)n);
      return SW_EOVERFLOW;
    }
    swk::TracePair tp;
    tp.q = B.qoff[B.pq[k]];
    tp.r = B.roff[B.pr[k]];
    tp.out = 0;
    tp.A = (int32_t)n;
    tp.B = (int32_t)m;
    tp.score = 0;
    tp.cap = 0;
    tp.id = k;
    // query columns per lane: 32 lanes per pair up to 160 columns (two pairs
    // per wavefront), 64 lanes per pair up to 256, 256-column tiles beyond
    if (m <= kDualCols) {
      tp.pad = (int32_t)((m + 31) / 32);
      htab[n1++] = tp;
    } else if (m <= swk::kTraceTileCols) {
      tp.pad = (int32_t)((m + 63) / 64);
      single.push_back(tp);
    } else {
      tp.pad = 4;
      multi.push_back(tp);
      carry_rows = std::max(carry_rows, (int)n);
    }
  }
  const int n_one = (int)single.size();
  if (n_one) std::memcpy(htab + n1, single.data(), (size_t)n_one * sizeof(swk::TracePair));
  const int nm = (int)multi.size(), nt = n1 + n_one + nm;
  if (nt == 0) return SW_OK;
  if (nm) std::memcpy(htab + n1 + n_one, multi.data(), (size_t)nm * sizeof(swk::TracePair));
  const int64_t per_wave = 4ll * carry_rows * (int64_t)sizeof(int32_t);
  const int waves_m = nm == 0 ? 0 : (int)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)nm, kTraceScratchBytes / std::max<int64_t>(per_wave, 1),
                            kTraceMaxWaves}));
  if ((rc = W.tr_pairs.ensure((size_t)nt * sizeof(swk::TracePair))) ||
      (rc = W.tr_mat.ensure((size_t)S.alpha * S.alpha * sizeof(int32_t))) ||
      (rc = W.tr_carry[0].ensure((size_t)std::max<int64_t>(per_wave * waves_m, 4))) ||
      (rc = W.tr_res.ensure((size_t)np * sizeof(swk::DevResult))) ||
      (rc = W.tr_hres.ensure((size_t)np * sizeof(swk::DevResult))))
    return rc;
  swk::TracePair *dp = W.tr_pairs.as<swk::TracePair>();
  HIPCHK(hipMemcpyAsync(dp, htab, (size_t)nt * sizeof(swk::TracePair), hipMemcpyHostToDevice, W.st));
  HIPCHK(hipMemcpyAsync(W.tr_mat.p, S.M.data(), (size_t)S.alpha * S.alpha * sizeof(int32_t),
                        hipMemcpyHostToDevice, W.st));
  swk::EndArgs ea;
  ea.qres = B.d_q;
  ea.rres = B.d_r;
  ea.matrix = W.tr_mat.as<int32_t>();
  ea.alpha = S.alpha;
  ea.go = S.go;
  ea.ge = S.ge;
  ea.gcarry = W.tr_carry[0].as<int32_t>();
  ea.out = W.tr_res.as<swk::DevResult>();
  ea.pairs = dp;
  ea.n = n1;
  ea.carry_rows = 0;
  HIPCHK(swk::launch_endtoend2(mode, ea, W.st));   // a workgroup per two pairs
  ea.pairs = dp + n1;
  ea.n = n_one;
  HIPCHK(swk::launch_endtoend(mode, ea, n_one, W.st));   // a workgroup per pair
  ea.pairs = dp + n1 + n_one;
  ea.n = nm;
  ea.carry_rows = carry_rows;
  HIPCHK(swk::launch_endtoend(mode, ea, waves_m, W.st));
  swk::DevResult *hres = W.tr_hres.as<swk::DevResult>();
  HIPCHK(hipMemcpyAsync(hres, W.tr_res.p, (size_t)np * sizeof(swk::DevResult),
                        hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipStreamSynchronize(W.st));
  for (int t = 0; t < nt; ++t) {
    const int k = htab[t].id;
    const swk::DevResult &r = hres[k];
    if (r.flags & swk::kFlagBadResidue) {
      set_error("pair %d: a residue code is not below alphabet_size", k);
      return SW_EINVAL;
    }
    out[k].score = r.score;
    out[k].query_end = r.qend;
    out[k].ref_end = r.rend;
    out[k].flags = 0;
  }
  return SW_OK;
}
