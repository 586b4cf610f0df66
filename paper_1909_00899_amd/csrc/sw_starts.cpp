// Start cells of a batch's alignments (include/sw.h, sw_align_batch_starts).
//
// The start of the reported alignment of a pair is the end cell of the same
// local alignment problem on the reversed prefixes q[0..query_end] and
// r[0..ref_end]: every optimal alignment inside the prefixes ends at the
// reported end cell (an alignment ending earlier would precede it in the
// (ref_end, query_end) order the end cell is chosen by), and the smallest end
// of the reversed problem is the largest start of the forward one.  So the
// reversed prefixes are cut out on the device and run through the batch path
// itself (device or host planner, the same kernels, int32 reruns), one query
// per pair.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "sw.h"
#include "sw_internal.h"
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

// Grow-only device buffers and a stream of their own (the batch call takes
// the library context's lock itself); one call at a time.
struct StartsWork {
  std::mutex mu;
  hipStream_t st = nullptr;
  DevBuf src_q, src_r;   // host-resident residue sets, uploaded
  DevBuf rev_q, rev_r;   // reversed prefixes
  DevBuf tab;            // offsets: q src, q dst, r src, r dst (int64), pair ids (int32)
};
StartsWork g_starts;

template <class T>
int read_back(std::vector<T> &dst, const T *src, size_t n, bool device) {
  dst.resize(n);
  if (n == 0) return SW_OK;
  if (device) HIPCHK(hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost));
  else std::memcpy(dst.data(), src, n * sizeof(T));
  return SW_OK;
}

}  // namespace

extern "C" int sw_align_batch_starts(const sw_batch *b, const sw_scoring *sc,
                                     const sw_result *ends, int32_t *query_start,
                                     int32_t *ref_start) {
  if (!b) { set_error("batch is NULL"); return SW_EINVAL; }
  if (b->n_pairs < 0 || b->n_queries < 0 || b->n_refs < 0) { set_error("negative count"); return SW_EINVAL; }
  if (b->precision != SW_PREC_AUTO && b->precision != SW_PREC_I32) { set_error("bad precision"); return SW_EINVAL; }
  Scoring S;
  int rc = prepare_scoring(sc, S);
  if (rc) return rc;
  const int np = b->n_pairs;
  if (np == 0) return SW_OK;
  if (!ends || !query_start || !ref_start) { set_error("ends or an output array is NULL"); return SW_EINVAL; }
  if (!b->query_off || !b->ref_off || !b->pair_ref || b->n_queries < 1 || b->n_refs < 1 ||
      (!b->pair_query && b->n_queries < 1)) {
    set_error("batch arrays are NULL or empty");
    return SW_EINVAL;
  }
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_starts.mu);
  StartsWork &W = g_starts;
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
  // ---- the batch's offsets and pair ids on the host (validated here)
  std::vector<int64_t> qoff, roff;
  std::vector<int32_t> pq, pr;
  if ((rc = read_back(qoff, b->query_off, (size_t)b->n_queries + 1, dev)) ||
      (rc = read_back(roff, b->ref_off, (size_t)b->n_refs + 1, dev)) ||
      (rc = read_back(pr, b->pair_ref, (size_t)np, dev)))
    return rc;
  if (b->pair_query) {
    if ((rc = read_back(pq, b->pair_query, (size_t)np, dev))) return rc;
  } else {
    pq.assign(np, 0);
  }
  for (int k = 0; k < b->n_queries; ++k)
    if (qoff[k] < 0 || qoff[k + 1] < qoff[k]) { set_error("query offsets not nondecreasing"); return SW_EINVAL; }
  for (int k = 0; k < b->n_refs; ++k)
    if (roff[k] < 0 || roff[k + 1] < roff[k]) { set_error("reference offsets not nondecreasing"); return SW_EINVAL; }
  // ---- the reversed prefix of every pair with a positive score
  std::vector<int> live;
  std::vector<int64_t> tab;   // [4][L+1]: q src, q dst, r src, r dst
  std::vector<int64_t> qsrc, qdst{0}, rsrc, rdst{0};
  for (int k = 0; k < np; ++k) {
    const sw_result &e = ends[k];
    query_start[k] = ref_start[k] = -1;
    if (pq[k] < 0 || pq[k] >= b->n_queries || pr[k] < 0 || pr[k] >= b->n_refs) {
      set_error("pair %d refers to a query or reference out of range", k);
      return SW_EINVAL;
    }
    if (e.score <= 0) continue;
    const int64_t m = qoff[pq[k] + 1] - qoff[pq[k]], n = roff[pr[k] + 1] - roff[pr[k]];
    if (e.query_end < 0 || e.query_end >= m || e.ref_end < 0 || e.ref_end >= n) {
      set_error("pair %d: end cell (%d, %d) outside its %lld x %lld sequences", k, e.query_end,
                e.ref_end, (long long)m, (long long)n);
      return SW_EINVAL;
    }
    live.push_back(k);
    qsrc.push_back(qoff[pq[k]]);
    qdst.push_back(qdst.back() + e.query_end + 1);
    rsrc.push_back(roff[pr[k]]);
    rdst.push_back(rdst.back() + e.ref_end + 1);
  }
  const int L = (int)live.size();
  if (L == 0) return SW_OK;
  qsrc.push_back(0);
  rsrc.push_back(0);
  const size_t L1 = (size_t)L + 1;
  const size_t tab_bytes = 4 * L1 * sizeof(int64_t) + (size_t)L * sizeof(int32_t) + 64;
  if ((rc = W.tab.ensure(tab_bytes)) || (rc = W.rev_q.ensure((size_t)qdst.back())) ||
      (rc = W.rev_r.ensure((size_t)rdst.back())))
    return rc;
  int64_t *d_tab = W.tab.as<int64_t>();
  int32_t *d_ids = (int32_t *)(d_tab + 4 * L1);
  std::vector<int32_t> ids(L);
  for (int t = 0; t < L; ++t) ids[t] = t;
  HIPCHK(hipMemcpyAsync(d_tab, qsrc.data(), L1 * sizeof(int64_t), hipMemcpyHostToDevice, W.st));
  HIPCHK(hipMemcpyAsync(d_tab + L1, qdst.data(), L1 * sizeof(int64_t), hipMemcpyHostToDevice, W.st));
  HIPCHK(hipMemcpyAsync(d_tab + 2 * L1, rsrc.data(), L1 * sizeof(int64_t), hipMemcpyHostToDevice, W.st));
  HIPCHK(hipMemcpyAsync(d_tab + 3 * L1, rdst.data(), L1 * sizeof(int64_t), hipMemcpyHostToDevice, W.st));
  HIPCHK(hipMemcpyAsync(d_ids, ids.data(), (size_t)L * sizeof(int32_t), hipMemcpyHostToDevice, W.st));
  // residues on the device
  const uint8_t *d_q = b->query_res, *d_r = b->ref_res;
  if (!dev) {
    const size_t qb = (size_t)qoff[b->n_queries], rb = (size_t)roff[b->n_refs];
    if ((rc = W.src_q.ensure(qb + 1)) || (rc = W.src_r.ensure(rb + 1))) return rc;
    if (qb) HIPCHK(hipMemcpyAsync(W.src_q.p, b->query_res, qb, hipMemcpyHostToDevice, W.st));
    if (rb) HIPCHK(hipMemcpyAsync(W.src_r.p, b->ref_res, rb, hipMemcpyHostToDevice, W.st));
    d_q = W.src_q.as<uint8_t>();
    d_r = W.src_r.as<uint8_t>();
  }
  HIPCHK(swk::launch_reverse_segments(L, d_q, d_tab, d_tab + L1, W.rev_q.as<uint8_t>(), W.st));
  HIPCHK(swk::launch_reverse_segments(L, d_r, d_tab + 2 * L1, d_tab + 3 * L1, W.rev_r.as<uint8_t>(),
                                      W.st));
  HIPCHK(hipStreamSynchronize(W.st));
  // ---- the reversed pairs through the batch path, one query per pair
  sw_batch nb;
  std::memset(&nb, 0, sizeof(nb));
  nb.n_pairs = L;
  nb.query_res = W.rev_q.as<uint8_t>();
  nb.query_off = d_tab + L1;
  nb.n_queries = L;
  nb.ref_res = W.rev_r.as<uint8_t>();
  nb.ref_off = d_tab + 3 * L1;
  nb.n_refs = L;
  nb.pair_query = d_ids;
  nb.pair_ref = d_ids;
  nb.precision = b->precision;
  nb.device_resident = 1;
  nb.stream = W.st;
  std::vector<sw_result> rev(L);
  if ((rc = sw_align_batch(&nb, sc, rev.data()))) return rc;
  for (int t = 0; t < L; ++t) {
    const int k = live[t];
    if (rev[t].score != ends[k].score) {
      for (int u = 0; u < np; ++u) query_start[u] = ref_start[u] = -1;
      set_error("pair %d: score %d is not this pair's optimum at its end cell (%d found)", k,
                ends[k].score, rev[t].score);
      return SW_EINVAL;
    }
    query_start[k] = ends[k].query_end - rev[t].query_end;
    ref_start[k] = ends[k].ref_end - rev[t].ref_end;
  }
  return SW_OK;
}
