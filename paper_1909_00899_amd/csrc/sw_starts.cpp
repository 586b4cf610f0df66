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
#include <climits>
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
  HostBuf ld_stage;              // pinned: a device-resident batch's offsets and indices
  // pinned staging of the caller's pageable arrays (see stage_up / stage_down)
  struct Pending {
    void *dst;
    const void *src;
    size_t bytes;
  };
  HostBuf up_stage, dn_stage;
  DevBuf sp_src, sp_dst;         // start cells: reversed prefixes' sources and offsets
  HostBuf rev_res;               // pinned: the reversed prefixes' results
  size_t up_used = 0, dn_used = 0;
  std::vector<Pending> dn_pending;
  DevBuf tr_res;                 // end-to-end results
  DevBuf e2e_sorted, e2e_hist;   // end-to-end: the two-pairs-per-wavefront entries reordered
  DevBuf tr_rstart;              // end-to-end paths: reference starts
  DevBuf tr_qstart;              // end-to-end paths: query starts
  // path tables built on the device: the caller's inputs (results, start
  // cells; a host batch's offsets and indices), per-pair scratch, the
  // planner's workgroup arrays, its summaries (pinned)
  DevBuf tr_ends, tr_qs, tr_rs, tr_qoff, tr_roff, tr_pq, tr_pr;
  DevBuf tr_rect, tr_cls, tr_hruns, tr_blk, tr_blkcaps, tr_clsmax, tr_err, tr_sum, tr_bsum;
  HostBuf tr_hsum;
  // device-memory rectangles: the largest group, the second, the rest each on
  // a stream of their own, so the long poles of the largest rectangles (one
  // wavefront each) overlap instead of adding up
  static constexpr int kTraceStreams = 3;
  hipStream_t tr_st[kTraceStreams] = {};
  hipEvent_t tr_ready = nullptr, tr_done[kTraceStreams] = {};
  DevBuf tr_bits[kTraceStreams], tr_carry[kTraceStreams];
};
StartsWork g_starts;

// Transfers between the caller's pageable host arrays and the device go
// through pinned staging memory: the host side copies on several threads and
// the DMA runs at the bus rate (the runtime's path for pageable memory stages
// chunk by chunk with one thread copying in between: about 7.5 GB/s).  The
// regions a call stages do not overlap; a staging buffer grows only after the
// stream has drained.  Transfers below kStageMin go directly.
constexpr size_t kStageMin = 1 << 20;

size_t stage_round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

void host_copy(void *dst, const void *src, size_t bytes) {
  constexpr size_t kPerThread = 4u << 20;
  const int T = (int)std::min<size_t>((size_t)host_threads(), (bytes + kPerThread - 1) / kPerThread);
  if (T <= 1) {
    std::memcpy(dst, src, bytes);
    return;
  }
  parallel_ranges(bytes, T, [&](int, size_t lo, size_t hi) {
    std::memcpy((char *)dst + lo, (const char *)src + lo, hi - lo);
  });
}

// A call's staging starts empty (earlier calls' copies have finished).
int stage_begin(StartsWork &W) {
  HIPCHK(hipStreamSynchronize(W.st));
  W.up_used = W.dn_used = 0;
  W.dn_pending.clear();
  return SW_OK;
}

int stage_up(StartsWork &W, void *dst, const void *src, size_t bytes) {
  if (bytes < kStageMin) {
    if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, W.st));
    return SW_OK;
  }
  if (W.up_used + stage_round(bytes) > W.up_stage.cap) {
    const size_t need = W.up_used + stage_round(bytes);
    HIPCHK(hipStreamSynchronize(W.st));   // the regions staged so far are consumed
    const int rc = W.up_stage.ensure(need);
    if (rc) return rc;
    W.up_used = 0;
  }
  char *p = W.up_stage.as<char>() + W.up_used;
  host_copy(p, src, bytes);
  HIPCHK(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, W.st));
  W.up_used += stage_round(bytes);
  return SW_OK;
}

// The staged downloads to their destinations, once the stream has drained.
void stage_complete(StartsWork &W) {
  for (const auto &x : W.dn_pending) host_copy(x.dst, x.src, x.bytes);
  W.dn_pending.clear();
  W.dn_used = 0;
}

// Queues a download; dst holds the data after the stream is synchronised and
// stage_complete has run.
int stage_down(StartsWork &W, void *dst, const void *src, size_t bytes) {
  if (bytes < kStageMin) {
    if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, W.st));
    return SW_OK;
  }
  if (W.dn_used + stage_round(bytes) > W.dn_stage.cap) {
    const size_t need = W.dn_used + stage_round(bytes);
    HIPCHK(hipStreamSynchronize(W.st));
    stage_complete(W);                    // the pending ones leave the old buffer first
    const int rc = W.dn_stage.ensure(need);
    if (rc) return rc;
  }
  char *p = W.dn_stage.as<char>() + W.dn_used;
  HIPCHK(hipMemcpyAsync(p, src, bytes, hipMemcpyDeviceToHost, W.st));
  W.dn_pending.push_back({dst, p, bytes});
  W.dn_used += stage_round(bytes);
  return SW_OK;
}


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
  {
    const int rc0 = stage_begin(W);
    if (rc0) return rc0;
  }
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
    if ((rc = stage_up(W, W.src_q.p, b->query_res, qb)) || (rc = stage_up(W, W.src_r.p, b->ref_res, rb)))
      return rc;
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

namespace {
int starts_device(const sw_batch *b, const sw_scoring *sc, const Scoring &S, StartsWork &W,
                  const sw_result *ends, int32_t *query_start, int32_t *ref_start, bool &handled);
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
  if (b->pair_query && b->n_queries > 1) {
    // one query per pair: the tables on the device (unless every aligned
    // pair turns out to share one query: the one-query launch below)
    bool handled = false;
    rc = starts_device(b, sc, S, W, ends, query_start, ref_start, handled);
    if (handled) return rc;
  }
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
// Wavefronts of a device-memory path launch, by measurement on 1M DNA pairs
// and the 100k protein search: 8192 (local, semi-global, overlap paths: 3-5
// ms faster than 4096 per DNA call, 2048 far slower); global paths, whose
// rectangles are whole pairs, ran fastest at 4096 (79 ms; 2048: 94, 5120:
// 98.5, 6144: 93, 8192: 86.5).
constexpr int kTraceMaxWaves = 8192;
constexpr int kTraceGlobalWaves = 4096;
// The end-to-end kernel for queries of several tiles keeps only a per-row
// carry per wavefront (no decision bits), so its launch takes up to twice as
// many wavefronts as the 4096 it had (about five fit per SIMD at its register
// count).
constexpr int kEndMaxWaves = 8192;

int launch_waves(int64_t count, int64_t per_wave, int max_waves) {
  per_wave = std::max<int64_t>(per_wave, 1);
  return (int)std::max<int64_t>(
      1, std::min<int64_t>({count, kTraceScratchBytes / per_wave, (int64_t)max_waves}));
}

}  // namespace

// Paths of a batch: mode 0 the local alignments between start and end cells
// (sw_align_batch_cigar), modes 1-4 whole end-to-end alignments (the API's
// mode + 1: global, semi-global query fitted, semi-global reference fitted,
// overlap) from their end cells (sw_align_batch_global_cigar;
// query_start_out / ref_start_out receive the start element + 1).
namespace {
// Lengths of pair k's sequences (for messages): from the host arrays, or read
// from a device-resident batch.
void pair_lengths(const sw_batch *b, int k, int64_t &m, int64_t &n) {
  m = n = -1;
  int32_t q = 0, r = 0;
  int64_t qo[2] = {0, 0}, ro[2] = {0, 0};
  if (b->device_resident) {
    if (b->pair_query && hipMemcpy(&q, b->pair_query + k, 4, hipMemcpyDeviceToHost) != hipSuccess) return;
    if (hipMemcpy(&r, b->pair_ref + k, 4, hipMemcpyDeviceToHost) != hipSuccess) return;
    if (q < 0 || q >= b->n_queries || r < 0 || r >= b->n_refs) return;
    if (hipMemcpy(qo, b->query_off + q, 16, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ro, b->ref_off + r, 16, hipMemcpyDeviceToHost) != hipSuccess)
      return;
  } else {
    q = b->pair_query ? b->pair_query[k] : 0;
    r = b->pair_ref[k];
    if (q < 0 || q >= b->n_queries || r < 0 || r >= b->n_refs) return;
    qo[0] = b->query_off[q];
    qo[1] = b->query_off[q + 1];
    ro[0] = b->ref_off[r];
    ro[1] = b->ref_off[r + 1];
  }
  m = qo[1] - qo[0];
  n = ro[1] - ro[0];
}

const char *const kModeName[] = {"local", "global", "semi-global (query fitted)",
                                 "semi-global (reference fitted)", "overlap"};

// The message and status of the planner's error word for pair k.
int path_error(const sw_batch *b, int mode, const sw_result *ends, const int32_t *query_start,
               const int32_t *ref_start, int k, int code) {
  const sw_result &e = ends[k];
  int64_t m, n;
  pair_lengths(b, k, m, n);
  const int qs = mode == 0 ? query_start[k] : 0, rs = mode == 0 ? ref_start[k] : 0;
  switch (code) {
    case swk::kTrErrPair:
      set_error("pair %d refers to a query or reference out of range", k);
      return SW_EINVAL;
    case swk::kTrErrQoff:
      set_error("query offsets not nondecreasing");
      return SW_EINVAL;
    case swk::kTrErrRoff:
      set_error("reference offsets not nondecreasing");
      return SW_EINVAL;
    case swk::kTrErrRect:
      set_error("pair %d: start (%d, %d) and end (%d, %d) are not a rectangle of its %lld x "
                "%lld sequences", k, qs, rs, e.query_end, e.ref_end, (long long)m, (long long)n);
      return SW_EINVAL;
    case swk::kTrErrEnd:
      set_error("pair %d: end (%d, %d) is not the end cell of a %s alignment of its %lld x %lld "
                "sequences", k, e.query_end, e.ref_end, kModeName[mode], (long long)m,
                (long long)n);
      return SW_EINVAL;
    case swk::kTrErrOptimum:
      set_error("pair %d: score %d is not the optimum at the end cell (%d, %d)", k, e.score,
                e.query_end, e.ref_end);
      return SW_EINVAL;
    case swk::kTrErrRange:
      set_error("pair %d: a %lld x %lld rectangle leaves the int32 range of the path kernel", k,
                (long long)(e.ref_end - rs + 1), (long long)(e.query_end - qs + 1));
      return SW_EOVERFLOW;
    case swk::kTrErrScratch:
      set_error("pair %d: a %lld x %lld rectangle needs more than 2 GiB of path scratch", k,
                (long long)(e.ref_end - rs + 1), (long long)(e.query_end - qs + 1));
      return SW_ENOMEM;
    case swk::kTrErrResidue:
      set_error("pair %d: a residue code inside its alignment is not below alphabet_size", k);
      return SW_EINVAL;
    case swk::kTrErrInconsistent:
      if (mode == 0)
        set_error("pair %d: no alignment of score %d runs from its start (%d, %d) to its end "
                  "(%d, %d)", k, e.score, qs, rs, e.query_end, e.ref_end);
      else
        set_error("pair %d: score %d is not the optimum at the end cell (%d, %d)", k, e.score,
                  e.query_end, e.ref_end);
      return SW_EINVAL;
    default:
      set_error("pair %d: internal path error (run count outside its bound)", k);
      return SW_EDEVICE;
  }
}

// The batch on W.st's device: a host batch's offsets, pair indices and
// residues uploaded on W.st, a device batch's own arrays (W.st first waits
// for the stream that produced them).  Offsets are checked by the device
// planners, pair by pair.
struct DevInputs {
  const int64_t *qoff, *roff;
  const int32_t *pq, *pr;   // pq null: query 0 for every pair
  const uint8_t *q, *r;
};

int device_inputs(const sw_batch *b, StartsWork &W, DevInputs &d) {
  int rc;
  const int np = b->n_pairs;
  const int64_t nq = b->n_queries, nr = b->n_refs;
  d.qoff = b->query_off;
  d.roff = b->ref_off;
  d.pq = b->pair_query;
  d.pr = b->pair_ref;
  d.q = b->query_res;
  d.r = b->ref_res;
  if (b->device_resident) {
    if (b->stream) {
      hipEvent_t ev;
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      hipError_t e = hipEventRecord(ev, (hipStream_t)b->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(W.st, ev, 0);
      (void)hipEventDestroy(ev);
      HIPCHK(e);
    }
    return SW_OK;
  }
  const int64_t qb = b->query_off[nq], rb = b->ref_off[nr];
  if (qb < 0 || rb < 0) {
    set_error(qb < 0 ? "query offsets not nondecreasing" : "reference offsets not nondecreasing");
    return SW_EINVAL;
  }
  if ((rc = W.tr_qoff.ensure((size_t)(nq + 1) * 8)) || (rc = W.tr_roff.ensure((size_t)(nr + 1) * 8)) ||
      (rc = W.tr_pr.ensure((size_t)np * 4)) || (rc = W.tr_pq.ensure((size_t)np * 4)) ||
      (rc = W.src_q.ensure((size_t)qb + 1)) || (rc = W.src_r.ensure((size_t)rb + 1)))
    return rc;
  if ((rc = stage_up(W, W.tr_qoff.p, b->query_off, (size_t)(nq + 1) * 8)) ||
      (rc = stage_up(W, W.tr_roff.p, b->ref_off, (size_t)(nr + 1) * 8)) ||
      (rc = stage_up(W, W.tr_pr.p, b->pair_ref, (size_t)np * 4)) ||
      (b->pair_query && (rc = stage_up(W, W.tr_pq.p, b->pair_query, (size_t)np * 4))) ||
      (rc = stage_up(W, W.src_q.p, b->query_res, (size_t)qb)) ||
      (rc = stage_up(W, W.src_r.p, b->ref_res, (size_t)rb)))
    return rc;
  d.qoff = W.tr_qoff.as<int64_t>();
  d.roff = W.tr_roff.as<int64_t>();
  d.pr = W.tr_pr.as<int32_t>();
  d.pq = b->pair_query ? W.tr_pq.as<int32_t>() : nullptr;
  d.q = W.src_q.as<uint8_t>();
  d.r = W.src_r.as<uint8_t>();
  return SW_OK;
}

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
  if (cigar_cap < 0 || (cigar_cap > 0 && !cigar)) { set_error("cigar is NULL or its capacity negative"); return SW_EINVAL; }
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_starts.mu);
  StartsWork &W = g_starts;
  HIPCHK(hipSetDevice(g_ctx.device));
  if (!W.st) HIPCHK(hipStreamCreateWithFlags(&W.st, hipStreamNonBlocking));
  if ((rc = stage_begin(W))) return rc;
  DevInputs din;
  if ((rc = device_inputs(b, W, din))) return rc;
  const int64_t nq = b->n_queries, nr = b->n_refs;
  const int64_t *d_qoff = din.qoff, *d_roff = din.roff;
  const int32_t *d_pq = din.pq, *d_pr = din.pr;
  const uint8_t *d_q = din.q, *d_r = din.r;
  constexpr int NC = swk::kTrClasses;
  if ((rc = W.tr_ends.ensure((size_t)np * sizeof(sw_result))) ||
      (rc = W.tr_qs.ensure((size_t)np * 4)) || (rc = W.tr_rs.ensure((size_t)np * 4)) ||
      (rc = W.tr_rect.ensure((size_t)np * sizeof(swk::TracePair))) ||
      (rc = W.tr_cls.ensure((size_t)np)) || (rc = W.tr_hruns.ensure((size_t)np * 8)) ||
      (rc = W.tr_nruns.ensure((size_t)np * 4)) || (rc = W.tr_rstart.ensure((size_t)np * 4)) ||
      (rc = W.tr_qstart.ensure((size_t)np * 4)) ||
      (rc = W.tr_blk.ensure((size_t)swk::kTrBlocks * NC * 4)) ||
      (rc = W.tr_blkcaps.ensure((size_t)swk::kTrBlocks * 8)) ||
      (rc = W.tr_clsmax.ensure((size_t)NC * 16)) || (rc = W.tr_err.ensure(16)) ||
      (rc = W.tr_sum.ensure((size_t)(NC + 2) * 8)) ||
      (rc = W.tr_pairs.ensure((size_t)np * sizeof(swk::TracePair))) ||
      (rc = W.tr_mat.ensure((size_t)S.alpha * S.alpha * sizeof(int32_t))) ||
      (rc = W.tr_off.ensure((size_t)(np + 1) * sizeof(int64_t))) ||
      (rc = W.tr_bsum.ensure((size_t)(np / 4096 + 2) * 8)) ||
      (rc = W.tr_hsum.ensure((size_t)(3 * NC + 8) * 8)))
    return rc;
  if ((rc = stage_up(W, W.tr_ends.p, ends, (size_t)np * sizeof(sw_result)))) return rc;
  if (mode == 0 && ((rc = stage_up(W, W.tr_qs.p, query_start, (size_t)np * 4)) ||
                    (rc = stage_up(W, W.tr_rs.p, ref_start, (size_t)np * 4))))
    return rc;
  HIPCHK(hipMemcpyAsync(W.tr_mat.p, S.M.data(), (size_t)S.alpha * S.alpha * sizeof(int32_t),
                        hipMemcpyHostToDevice, W.st));
  HIPCHK(hipMemsetAsync(W.tr_clsmax.p, 0, (size_t)NC * 16, W.st));
  HIPCHK(hipMemsetAsync(W.tr_err.p, 0xff, 8, W.st));
  int64_t maxabs = 0;
  for (int v : S.M) maxabs = std::max<int64_t>(maxabs, v < 0 ? -(int64_t)v : v);
  // ---- the table: classify, totals, summary to the host
  swk::TrPlanArgs pa;
  pa.np = np;
  pa.nq = (int)nq;
  pa.nr = (int)nr;
  pa.mode = mode;
  pa.alpha = S.alpha;
  pa.go = S.go;
  pa.ge = S.ge;
  pa.max_s = S.max_s;
  pa.maxabs = (int)std::min<int64_t>(maxabs, INT32_MAX);
  pa.qoff = d_qoff;
  pa.roff = d_roff;
  pa.pq = d_pq;
  pa.pr = d_pr;
  pa.ends = W.tr_ends.as<swk::DevResult>();
  pa.qs = W.tr_qs.as<int32_t>();
  pa.rs = W.tr_rs.as<int32_t>();
  pa.rect = W.tr_rect.as<swk::TracePair>();
  pa.cls = W.tr_cls.as<uint8_t>();
  pa.hruns = W.tr_hruns.as<uint32_t>();
  pa.n_runs = W.tr_nruns.as<int32_t>();
  pa.ref_start = W.tr_rstart.as<int32_t>();
  pa.query_start = W.tr_qstart.as<int32_t>();
  pa.blk_count = W.tr_blk.as<int32_t>();
  pa.blk_caps = W.tr_blkcaps.as<int64_t>();
  pa.cls_max = W.tr_clsmax.as<unsigned long long>();
  pa.err = W.tr_err.as<unsigned long long>();
  pa.summary = W.tr_sum.as<int64_t>();
  pa.table = W.tr_pairs.as<swk::TracePair>();
  pa.runs = nullptr;
  HIPCHK(swk::launch_trplan_classify(pa, W.st));
  HIPCHK(swk::launch_trplan_totals(pa, W.st));
  int64_t *hs = W.tr_hsum.as<int64_t>();          // [NC + 2] summary, [2 NC] maxima, error word
  HIPCHK(hipMemcpyAsync(hs, W.tr_sum.p, (size_t)(NC + 2) * 8, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipMemcpyAsync(hs + NC + 2, W.tr_clsmax.p, (size_t)NC * 16, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipMemcpyAsync(hs + 3 * NC + 2, W.tr_err.p, 8, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipStreamSynchronize(W.st));
  const uint64_t err1 = (uint64_t)hs[3 * NC + 2];
  if (err1 != ~0ull)
    return path_error(b, mode, ends, query_start, ref_start, (int)(err1 >> 8), (int)(err1 & 0xff));
  int64_t cstart[NC + 1];
  for (int c = 0; c <= NC; ++c) cstart[c] = hs[c];
  const int64_t region = hs[NC + 1];
  const uint64_t *cmax = (const uint64_t *)(hs + NC + 2);
  const int nt = (int)cstart[NC];
  if ((rc = W.tr_runs.ensure((size_t)std::max<int64_t>(region, 1) * sizeof(uint32_t)))) return rc;
  pa.runs = W.tr_runs.as<uint32_t>();
  HIPCHK(swk::launch_trplan_scatter(pa, W.st));
  // ---- launches: LDS classes (one per variant), device-memory classes
  struct Group { int first, count, waves; int64_t slot_words; int carry_rows; int variant; };
  std::vector<Group> groups;
  constexpr int NS = StartsWork::kTraceStreams;
  int64_t bits_words[NS] = {}, carry_ints[NS] = {};
  for (int c = 3; c < swk::kTrHostClass; ++c) {
    const int64_t cnt = cstart[c + 1] - cstart[c];
    if (!cnt) continue;
    const int64_t slot = (int64_t)cmax[2 * c];
    const int carry_rows = std::max<int>(1, (int)cmax[2 * c + 1]);
    const int64_t per_wave = slot * 2 + 6ll * carry_rows * 4;
    const int waves = launch_waves(cnt, per_wave, mode == 1 ? kTraceGlobalWaves : kTraceMaxWaves);
    const int sk = std::min((int)groups.size(), NS - 1);
    groups.push_back({(int)cstart[c], (int)cnt, waves, slot, carry_rows, (c - 3) % 3});
    bits_words[sk] = std::max<int64_t>(bits_words[sk], slot * waves);
    carry_ints[sk] = std::max<int64_t>(carry_ints[sk], 6ll * carry_rows * waves);
  }
  for (int k = 0; k < NS && k < (int)groups.size(); ++k) {
    if ((rc = W.tr_bits[k].ensure((size_t)std::max<int64_t>(bits_words[k], 1) * sizeof(uint16_t))) ||
        (rc = W.tr_carry[k].ensure((size_t)std::max<int64_t>(carry_ints[k], 1) * sizeof(int32_t))))
      return rc;
    if (!W.tr_st[k]) HIPCHK(hipStreamCreateWithFlags(&W.tr_st[k], hipStreamNonBlocking));
    if (!W.tr_done[k]) HIPCHK(hipEventCreateWithFlags(&W.tr_done[k], hipEventDisableTiming));
  }
  if (!W.tr_ready) HIPCHK(hipEventCreateWithFlags(&W.tr_ready, hipEventDisableTiming));
  swk::TracePair *dp = W.tr_pairs.as<swk::TracePair>();
  swk::TraceArgs ta;
  ta.qres = d_q;
  ta.rres = d_r;
  ta.matrix = W.tr_mat.as<int32_t>();
  ta.alpha = S.alpha;
  ta.go = S.go;
  ta.ge = S.ge;
  ta.cigar = W.tr_runs.as<uint32_t>();
  ta.n_runs = W.tr_nruns.as<int32_t>();
  ta.mode = mode;
  ta.ref_start = W.tr_rstart.as<int32_t>();
  ta.query_start = W.tr_qstart.as<int32_t>();
  ta.slot_words = 0;
  ta.lds_words = 0;
  ta.carry_rows = 0;
  ta.gbits = nullptr;
  ta.gcarry = nullptr;
  const int used = std::min((int)groups.size(), NS);
  if (used) HIPCHK(hipEventRecord(W.tr_ready, W.st));
  for (int k = 0; k < used; ++k) HIPCHK(hipStreamWaitEvent(W.tr_st[k], W.tr_ready, 0));
  static const int kLdsVariant[3] = {swk::kTraceV16x4, swk::kTraceV32, swk::kTraceV16x8};
  for (int c = 0; c < 3; ++c) {
    const int cnt = (int)(cstart[c + 1] - cstart[c]);
    if (!cnt) continue;
    ta.pairs = dp + cstart[c];
    ta.n = cnt;
    // LDS for the class's largest rectangle only (more workgroups per CU)
    ta.lds_words = (int)std::max<uint64_t>(8, (cmax[2 * c] + 7) / 8 * 8);
    ta.carry_rows = (int)cmax[2 * c + 1];   // rows of its rectangles of two or more tiles
    HIPCHK(swk::launch_trace(true, kLdsVariant[c], ta, cnt, W.st));
  }
  for (int g = 0; g < (int)groups.size(); ++g) {
    const Group &gr = groups[g];
    const int k = std::min(g, NS - 1);
    ta.pairs = dp + gr.first;
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
  // ---- run counts checked, offsets by a device prefix sum
  HIPCHK(swk::launch_trplan_check(dp, nt, W.tr_nruns.as<int32_t>(), W.tr_err.as<unsigned long long>(),
                                  W.st));
  HIPCHK(swk::launch_count_scan(W.tr_nruns.as<int32_t>(), np, W.tr_off.as<int64_t>(),
                                W.tr_bsum.as<int64_t>(), W.st));
  HIPCHK(hipMemcpyAsync(hs, W.tr_err.p, 8, hipMemcpyDeviceToHost, W.st));
  if ((rc = stage_down(W, cigar_off, W.tr_off.p, (size_t)(np + 1) * sizeof(int64_t)))) return rc;
  HIPCHK(hipStreamSynchronize(W.st));
  stage_complete(W);
  const uint64_t err2 = (uint64_t)hs[0];
  if (err2 != ~0ull) {
    cigar_off[0] = 0;
    return path_error(b, mode, ends, query_start, ref_start, (int)(err2 >> 8), (int)(err2 & 0xff));
  }
  const int64_t total = cigar_off[np];
  if (total > cigar_cap) {
    set_error("the paths need %lld runs, cigar holds %lld", (long long)total, (long long)cigar_cap);
    return SW_EINVAL;
  }
  if (total > 0) {
    if ((rc = W.tr_packed.ensure((size_t)total * sizeof(uint32_t)))) return rc;
    HIPCHK(swk::launch_pack_runs(dp, nt, W.tr_nruns.as<int32_t>(), W.tr_off.as<int64_t>(),
                                 W.tr_runs.as<uint32_t>(), W.tr_packed.as<uint32_t>(), W.st));
    if ((rc = stage_down(W, cigar, W.tr_packed.p, (size_t)total * sizeof(uint32_t)))) return rc;
  }
  if (mode != 0 && ((rc = stage_down(W, ref_start_out, W.tr_rstart.p, (size_t)np * 4)) ||
                    (rc = stage_down(W, query_start_out, W.tr_qstart.p, (size_t)np * 4))))
    return rc;
  HIPCHK(hipStreamSynchronize(W.st));
  stage_complete(W);
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


// ------------------------------------------------------------------ start cells, tables on the device

namespace {

// Start cells of a batch with one query per pair: the reversed prefixes'
// tables built on the device (startplan_kernel, two prefix sums; each prefix
// cut to the span an alignment of the pair's score can have), the
// prefixes reversed there, one batch call over them (pairs without an
// alignment become empty pairs).  handled = false leaves the batch to the
// host-table path (every aligned pair has the same query).
int starts_device(const sw_batch *b, const sw_scoring *sc, const Scoring &S, StartsWork &W,
                  const sw_result *ends, int32_t *query_start, int32_t *ref_start, bool &handled) {
  handled = true;
  int rc;
  const int np = b->n_pairs;
  HIPCHK(hipSetDevice(g_ctx.device));
  if (!W.st) HIPCHK(hipStreamCreateWithFlags(&W.st, hipStreamNonBlocking));
  if ((rc = stage_begin(W))) return rc;
  DevInputs din;
  if ((rc = device_inputs(b, W, din))) return rc;
  if ((rc = W.tr_ends.ensure((size_t)np * sizeof(sw_result))) ||
      (rc = W.tr_qs.ensure((size_t)np * 4)) || (rc = W.tr_rs.ensure((size_t)np * 4)) ||
      (rc = W.tr_nruns.ensure((size_t)np * 4)) ||
      (rc = W.sp_src.ensure((size_t)(np + 1) * 16)) || (rc = W.sp_dst.ensure((size_t)(np + 1) * 16)) ||
      (rc = W.tr_bsum.ensure((size_t)(np / 4096 + 2) * 8)) || (rc = W.tr_err.ensure(16)) ||
      (rc = W.tr_hsum.ensure(64)))
    return rc;
  if ((rc = stage_up(W, W.tr_ends.p, ends, (size_t)np * sizeof(sw_result)))) return rc;
  static const int32_t kRangeInit[2] = {INT32_MAX, -1};
  HIPCHK(hipMemsetAsync(W.tr_err.p, 0xff, 8, W.st));
  HIPCHK(hipMemcpyAsync((char *)W.tr_err.p + 8, kRangeInit, 8, hipMemcpyHostToDevice, W.st));
  int64_t *qsrc = W.sp_src.as<int64_t>(), *rsrc = qsrc + (np + 1);
  int64_t *qdst = W.sp_dst.as<int64_t>(), *rdst = qdst + (np + 1);
  swk::StartPlanArgs pa;
  pa.np = np;
  pa.nq = b->n_queries;
  pa.nr = b->n_refs;
  pa.go = S.go;
  pa.ge = S.ge;
  pa.max_s = S.max_s;
  pa.ends = W.tr_ends.as<swk::DevResult>();
  pa.qoff = din.qoff;
  pa.roff = din.roff;
  pa.pq = din.pq;
  pa.pr = din.pr;
  pa.qcnt = W.tr_qs.as<int32_t>();
  pa.rcnt = W.tr_rs.as<int32_t>();
  pa.ids = W.tr_nruns.as<int32_t>();
  pa.qsrc = qsrc;
  pa.rsrc = rsrc;
  pa.err = W.tr_err.as<unsigned long long>();
  pa.qrange = (int32_t *)((char *)W.tr_err.p + 8);
  HIPCHK(swk::launch_startplan(pa, W.st));
  HIPCHK(swk::launch_count_scan(pa.qcnt, np, qdst, W.tr_bsum.as<int64_t>(), W.st));
  HIPCHK(swk::launch_count_scan(pa.rcnt, np, rdst, W.tr_bsum.as<int64_t>(), W.st));
  int64_t *hs = W.tr_hsum.as<int64_t>();   // error word, query range, the two totals
  HIPCHK(hipMemcpyAsync(hs, W.tr_err.p, 16, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipMemcpyAsync(hs + 2, qdst + np, 8, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipMemcpyAsync(hs + 3, rdst + np, 8, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipStreamSynchronize(W.st));
  const uint64_t err = (uint64_t)hs[0];
  if (err != ~0ull) {
    const int k = (int)(err >> 8), code = (int)(err & 0xff);
    int64_t m, n;
    pair_lengths(b, k, m, n);
    if (code == swk::kSpErrEnd)
      set_error("pair %d: end cell (%d, %d) outside its %lld x %lld sequences", k, ends[k].query_end,
                ends[k].ref_end, (long long)m, (long long)n);
    else if (code == swk::kTrErrPair)
      set_error("pair %d refers to a query or reference out of range", k);
    else
      set_error(code == swk::kTrErrQoff ? "query offsets not nondecreasing"
                                        : "reference offsets not nondecreasing");
    return SW_EINVAL;
  }
  const int32_t *qr = (const int32_t *)(hs + 1);
  if (qr[1] >= 0 && qr[0] == qr[1]) {   // one query for every aligned pair
    handled = false;
    return SW_OK;
  }
  if (qr[1] < 0) {                        // no alignment at all
    for (int k = 0; k < np; ++k) query_start[k] = ref_start[k] = -1;
    return SW_OK;
  }
  const int64_t qtot = hs[2], rtot = hs[3];
  if ((rc = W.rev_q.ensure((size_t)qtot + 1)) || (rc = W.rev_r.ensure((size_t)rtot + 1))) return rc;
  HIPCHK(swk::launch_reverse_segments(np, din.q, qsrc, qdst, W.rev_q.as<uint8_t>(), W.st));
  HIPCHK(swk::launch_reverse_segments(np, din.r, rsrc, rdst, W.rev_r.as<uint8_t>(), W.st));
  sw_batch nb;
  std::memset(&nb, 0, sizeof(nb));
  nb.n_pairs = np;
  nb.query_res = W.rev_q.as<uint8_t>();
  nb.query_off = qdst;
  nb.n_queries = np;
  nb.ref_res = W.rev_r.as<uint8_t>();
  nb.ref_off = rdst;
  nb.n_refs = np;
  nb.pair_query = pa.ids;
  nb.pair_ref = pa.ids;
  nb.precision = b->precision;
  nb.device_resident = 1;
  nb.stream = W.st;
  // the reversed results in pinned memory (copied back at the bus rate), then
  // the starts on host threads
  if ((rc = W.rev_res.ensure((size_t)np * sizeof(sw_result)))) return rc;
  const sw_result *rev = W.rev_res.as<sw_result>();
  if ((rc = sw_align_batch(&nb, sc, W.rev_res.as<sw_result>()))) return rc;
  const int T = np >= 65536 ? host_threads() : 1;
  std::vector<int> wrong(T, INT_MAX);
  parallel_ranges((size_t)np, T, [&](int t, size_t lo, size_t hi) {
    for (size_t kk = lo; kk < hi; ++kk) {
      const int k = (int)kk;
      const sw_result &e = ends[k];
      if (e.score <= 0) {
        query_start[k] = ref_start[k] = -1;
      } else if (rev[k].score != e.score) {
        wrong[t] = k;
        return;
      } else {
        query_start[k] = e.query_end - rev[k].query_end;
        ref_start[k] = e.ref_end - rev[k].ref_end;
      }
    }
  });
  const int kw = *std::min_element(wrong.begin(), wrong.end());
  if (kw != INT_MAX) {
    for (int u = 0; u < np; ++u) query_start[u] = ref_start[u] = -1;
    set_error("pair %d: score %d is not this pair's optimum at its end cell (%d found)", kw,
              ends[kw].score, rev[kw].score);
    return SW_EINVAL;
  }
  return SW_OK;
}

}  // namespace

// ------------------------------------------------------------------ end-to-end scores
// ------------------------------------------------------------------ end-to-end scores

namespace {

// The message and status of the end-to-end planner's error word for pair k.
int endtoend_error(const sw_batch *b, int k, int code) {
  int64_t m, n;
  pair_lengths(b, k, m, n);
  switch (code) {
    case swk::kTrErrPair:
      set_error("pair %d refers to a query or reference out of range", k);
      return SW_EINVAL;
    case swk::kTrErrQoff:
      set_error("query offsets not nondecreasing");
      return SW_EINVAL;
    case swk::kTrErrRoff:
      set_error("reference offsets not nondecreasing");
      return SW_EINVAL;
    case swk::kTrErrRange:
      set_error("pair %d: %lld x %lld leaves the int32 range of the end-to-end kernel", k,
                (long long)m, (long long)n);
      return SW_EOVERFLOW;
    case swk::kE2eErrScore:
      set_error("pair %d: score below the int32 range", k);
      return SW_EOVERFLOW;
    case swk::kTrErrResidue:
      set_error("pair %d: a residue code is not below alphabet_size", k);
      return SW_EINVAL;
    default:
      set_error("pair %d: internal end-to-end error %d", k, code);
      return SW_EDEVICE;
  }
}

}  // namespace

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
  HIPCHK(hipSetDevice(g_ctx.device));
  if (!W.st) HIPCHK(hipStreamCreateWithFlags(&W.st, hipStreamNonBlocking));
  if ((rc = stage_begin(W))) return rc;
  DevInputs din;
  if ((rc = device_inputs(b, W, din))) return rc;
  int64_t maxabs = 0;
  for (int v : S.M) maxabs = std::max<int64_t>(maxabs, v < 0 ? -(int64_t)v : v);
  constexpr int NC = swk::kE2eClasses;
  if ((rc = W.tr_res.ensure((size_t)np * sizeof(swk::DevResult))) ||
      (rc = W.tr_cls.ensure((size_t)np)) ||
      (rc = W.tr_blk.ensure((size_t)swk::kTrBlocks * NC * 4)) ||
      (rc = W.tr_clsmax.ensure(16)) || (rc = W.tr_err.ensure(16)) ||
      (rc = W.tr_sum.ensure((size_t)(NC + 1) * 8)) ||
      (rc = W.tr_pairs.ensure((size_t)np * sizeof(swk::TracePair))) ||
      (rc = W.tr_mat.ensure((size_t)S.alpha * S.alpha * sizeof(int32_t))) ||
      (rc = W.tr_hsum.ensure((size_t)(NC + 4) * 8)))
    return rc;
  HIPCHK(hipMemcpyAsync(W.tr_mat.p, S.M.data(), (size_t)S.alpha * S.alpha * sizeof(int32_t),
                        hipMemcpyHostToDevice, W.st));
  HIPCHK(hipMemsetAsync(W.tr_clsmax.p, 0, 8, W.st));
  HIPCHK(hipMemsetAsync(W.tr_err.p, 0xff, 8, W.st));
  // ---- the table: classify (empty sides' results written there), totals,
  // summary to the host
  swk::E2ePlanArgs pa;
  pa.np = np;
  pa.nq = b->n_queries;
  pa.nr = b->n_refs;
  pa.mode = mode;
  pa.go = S.go;
  pa.ge = S.ge;
  pa.max_s = S.max_s;
  pa.maxabs = (int)std::min<int64_t>(maxabs, INT32_MAX);
  pa.qoff = din.qoff;
  pa.roff = din.roff;
  pa.pq = din.pq;
  pa.pr = din.pr;
  pa.out = W.tr_res.as<swk::DevResult>();
  pa.cls = W.tr_cls.as<uint8_t>();
  pa.blk_count = W.tr_blk.as<int32_t>();
  pa.rows_max = W.tr_clsmax.as<unsigned long long>();
  pa.err = W.tr_err.as<unsigned long long>();
  pa.summary = W.tr_sum.as<int64_t>();
  pa.table = W.tr_pairs.as<swk::TracePair>();
  HIPCHK(swk::launch_e2eplan_classify(pa, W.st));
  HIPCHK(swk::launch_e2eplan_totals(pa, W.st));
  int64_t *hs = W.tr_hsum.as<int64_t>();   // [NC + 1] summary, rows, error word
  HIPCHK(hipMemcpyAsync(hs, W.tr_sum.p, (size_t)(NC + 1) * 8, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipMemcpyAsync(hs + NC + 1, W.tr_clsmax.p, 8, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipMemcpyAsync(hs + NC + 2, W.tr_err.p, 8, hipMemcpyDeviceToHost, W.st));
  HIPCHK(hipStreamSynchronize(W.st));
  const uint64_t err1 = (uint64_t)hs[NC + 2];
  if (err1 != ~0ull) return endtoend_error(b, (int)(err1 >> 8), (int)(err1 & 0xff));
  const int n1 = (int)(hs[1] - hs[0]), n_one = (int)(hs[2] - hs[1]), nw = (int)(hs[3] - hs[2]);
  const int nm = (int)(hs[4] - hs[3]);
  const int carry_rows = (int)hs[NC + 1];
  if (n1 + n_one + nw + nm > 0) {
    HIPCHK(swk::launch_e2eplan_scatter(pa, W.st));
    const int64_t per_wave = 4ll * carry_rows * (int64_t)sizeof(int32_t);
    const int waves_m = nm == 0 ? 0 : launch_waves(nm, per_wave, kEndMaxWaves);
    if ((rc = W.tr_carry[0].ensure((size_t)std::max<int64_t>(per_wave * waves_m, 4)))) return rc;
    swk::TracePair *dp = W.tr_pairs.as<swk::TracePair>();
    swk::EndArgs ea;
    ea.qres = din.q;
    ea.rres = din.r;
    ea.matrix = W.tr_mat.as<int32_t>();
    ea.alpha = S.alpha;
    ea.go = S.go;
    ea.ge = S.ge;
    ea.gcarry = W.tr_carry[0].as<int32_t>();
    ea.out = W.tr_res.as<swk::DevResult>();
    ea.pairs = dp;
    ea.n = n1;
    ea.carry_rows = 0;
    if (n1 > 2) {
      // couples of equal columns per lane and similar row counts
      if ((rc = W.e2e_sorted.ensure((size_t)n1 * sizeof(swk::TracePair))) ||
          (rc = W.e2e_hist.ensure((size_t)swk::kE2eSortBins * sizeof(int32_t))))
        return rc;
      HIPCHK(hipMemsetAsync(W.e2e_hist.p, 0, (size_t)swk::kE2eSortBins * sizeof(int32_t), W.st));
      HIPCHK(swk::launch_e2e_sort(dp, n1, W.e2e_hist.as<int32_t>(),
                                  W.e2e_sorted.as<swk::TracePair>(), W.st));
      ea.pairs = W.e2e_sorted.as<swk::TracePair>();
    }
    HIPCHK(swk::launch_endtoend2(mode, ea, W.st));   // a workgroup per two pairs
    ea.pairs = dp + n1;
    ea.n = n_one;
    HIPCHK(swk::launch_endtoend(mode, ea, n_one, W.st));        // a workgroup per pair
    ea.pairs = dp + n1 + n_one;
    ea.n = nw;
    HIPCHK(swk::launch_endtoend_wide(mode, ea, nw, W.st));      // a workgroup per pair
    ea.pairs = dp + n1 + n_one + nw;
    ea.n = nm;
    ea.carry_rows = carry_rows;
    HIPCHK(swk::launch_endtoend_wide(mode, ea, waves_m, W.st)); // carries between tiles
    HIPCHK(swk::launch_e2e_check(W.tr_res.as<swk::DevResult>(), np, W.tr_err.as<unsigned long long>(),
                                 W.st));
  }
  // every pair's result (a device result has the API's layout; on success
  // its flags are 0)
  static_assert(sizeof(swk::DevResult) == sizeof(sw_result), "result layouts differ");
  HIPCHK(hipMemcpyAsync(hs, W.tr_err.p, 8, hipMemcpyDeviceToHost, W.st));
  if ((rc = stage_down(W, out, W.tr_res.p, (size_t)np * sizeof(sw_result)))) return rc;
  HIPCHK(hipStreamSynchronize(W.st));
  stage_complete(W);
  const uint64_t err2 = (uint64_t)hs[0];
  if (err2 != ~0ull) return endtoend_error(b, (int)(err2 >> 8), (int)(err2 & 0xff));
  return SW_OK;
}
