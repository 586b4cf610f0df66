// Public C entry points of libswscan.so (include/sw.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "sw.h"
#include "sw_runtime.h"

using namespace swrt;
using swk::PairInfo;

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

constexpr int64_t kI32Limit = 2147483647ll;

bool overflows(int64_t m, int64_t n, int max_s) {
  return std::min(m, n) * (int64_t)max_s >= kI32Limit;
}

}  // namespace

namespace swrt {

// Checks the batch, builds the planner's items and puts PairInfo records,
// sequences and the residue check on the device (context locked by the caller).
int prepare_batch(const sw_batch *b, const Scoring &S, Context &C, ExecInput &in,
                  sw_result *out, int64_t &cells) {
  const int np = b->n_pairs;
  int rc = SW_OK;
  if (!b->query_res || !b->query_off || !b->ref_res || !b->ref_off || !b->pair_ref ||
      b->n_queries < 1 || b->n_refs < 1) {
    set_error("NULL sequence pointer or empty query/reference set");
    return SW_EINVAL;
  }
  hipStream_t st = C.stream;
  if (b->device_resident && b->stream) {
    HIPCHK(hipEventRecord(C.evx, (hipStream_t)b->stream));
    HIPCHK(hipStreamWaitEvent(st, C.evx, 0));
  }
  // host views of offsets and pair lists
  std::vector<int64_t> qoff_v, roff_v;
  std::vector<int32_t> pq_v, pr_v;
  const int64_t *qoff = b->query_off, *roff = b->ref_off;
  const int32_t *pq = b->pair_query, *pr = b->pair_ref;
  if (b->device_resident) {
    qoff_v.resize(b->n_queries + 1);
    roff_v.resize(b->n_refs + 1);
    pr_v.resize(np);
    HIPCHK(hipMemcpyAsync(qoff_v.data(), qoff, qoff_v.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(roff_v.data(), roff, roff_v.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pr_v.data(), pr, pr_v.size() * 4, hipMemcpyDeviceToHost, st));
    if (pq) {
      pq_v.resize(np);
      HIPCHK(hipMemcpyAsync(pq_v.data(), pq, pq_v.size() * 4, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    qoff = qoff_v.data();
    roff = roff_v.data();
    pr = pr_v.data();
    pq = pq ? pq_v.data() : nullptr;
  }
  for (int q = 0; q < b->n_queries; ++q)
    if (qoff[q] < 0 || qoff[q + 1] < qoff[q] || qoff[q + 1] - qoff[q] > kI32Limit) {
      set_error("query offsets not nondecreasing at %d", q);
      return SW_EINVAL;
    }
  for (int r = 0; r < b->n_refs; ++r)
    if (roff[r] < 0 || roff[r + 1] < roff[r] || roff[r + 1] - roff[r] > kI32Limit) {
      set_error("reference offsets not nondecreasing at %d", r);
      return SW_EINVAL;
    }
  in.n_queries = b->n_queries;
  in.q_off_of_query.resize(b->n_queries);
  in.m_of_query.resize(b->n_queries);
  for (int q = 0; q < b->n_queries; ++q) {
    in.q_off_of_query[q] = qoff[q];
    in.m_of_query[q] = (int)(qoff[q + 1] - qoff[q]);
  }
  in.items.reserve(np);
  cells = 0;
  for (int k = 0; k < np; ++k) {
    const int q = pq ? pq[k] : 0;
    const int r = pr[k];
    if (q < 0 || q >= b->n_queries || r < 0 || r >= b->n_refs) {
      set_error("pair %d refers to query %d / reference %d out of range", k, q, r);
      return SW_EINVAL;
    }
    const int m = in.m_of_query[q];
    const int n = (int)(roff[r + 1] - roff[r]);
    if (overflows(m, n, S.max_s)) { set_error("pair %d may overflow int32", k); return SW_EOVERFLOW; }
    out[k] = sw_result{0, -1, -1, 0};
    if (m > 0 && n > 0) {
      in.items.push_back(PlanItem{k, q, m, n});
      cells += (int64_t)m * n;
    }
  }
  // PairInfo records are built on the device from the offsets
  in.n_pairs = np;
  {
    const size_t oq = 0, orr = oq + sizeof(int64_t) * (b->n_queries + 1);
    const size_t opq = orr + sizeof(int64_t) * (b->n_refs + 1);
    const size_t opr = opq + sizeof(int32_t) * np;
    const size_t opairs = (opr + sizeof(int32_t) * np + 15) / 16 * 16;
    const size_t total = opairs + sizeof(PairInfo) * np;
    if ((rc = C.ws.offs.ensure(total))) return rc;
    char *base = C.ws.offs.as<char>();
    const int64_t *d_qoff = b->query_off, *d_roff = b->ref_off;
    const int32_t *d_pq = b->pair_query, *d_pr = b->pair_ref;
    if (!b->device_resident) {
      HIPCHK(hipMemcpyAsync(base + oq, qoff, orr - oq, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(base + orr, roff, opq - orr, hipMemcpyHostToDevice, st));
      if (pq) HIPCHK(hipMemcpyAsync(base + opq, pq, opr - opq, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(base + opr, pr, sizeof(int32_t) * np, hipMemcpyHostToDevice, st));
      d_qoff = (const int64_t *)(base + oq);
      d_roff = (const int64_t *)(base + orr);
      d_pq = pq ? (const int32_t *)(base + opq) : nullptr;
      d_pr = (const int32_t *)(base + opr);
    }
    in.d_pairs = (const PairInfo *)(base + opairs);
    HIPCHK(swk::launch_build_pairs(np, d_qoff, d_roff, d_pq, d_pr, (PairInfo *)(base + opairs), st));
  }
  // sequences on the device
  const int64_t qbytes = qoff[b->n_queries], rbytes = roff[b->n_refs];
  if (b->device_resident) {
    in.d_qres = b->query_res;
    in.d_rres = b->ref_res;
  } else {
    if ((rc = C.qres.ensure(std::max<int64_t>(qbytes, 1))) || (rc = C.rres.ensure(std::max<int64_t>(rbytes, 1))))
      return rc;
    if (qbytes) HIPCHK(hipMemcpyAsync(C.qres.p, b->query_res, qbytes, hipMemcpyHostToDevice, st));
    if (rbytes) HIPCHK(hipMemcpyAsync(C.rres.p, b->ref_res, rbytes, hipMemcpyHostToDevice, st));
    in.d_qres = C.qres.as<uint8_t>();
    in.d_rres = C.rres.as<uint8_t>();
  }
  if ((rc = C.flag.ensure(16))) return rc;
  HIPCHK(hipMemsetAsync(C.flag.p, 0, 16, st));
  HIPCHK(swk::launch_check_residues(in.d_qres, qbytes, S.alpha, C.flag.as<int>(), st));
  HIPCHK(swk::launch_check_residues(in.d_rres, rbytes, S.alpha, C.flag.as<int>(), st));
  return SW_OK;
}

// 1 if the residue check flagged a code >= alphabet_size, 0 if not, -1 on a
// device error.
int residue_flag(Context &C) {
  int bad = 0;
  if (hipMemcpyAsync(&bad, C.flag.p, sizeof(int), hipMemcpyDeviceToHost, C.stream) != hipSuccess ||
      hipStreamSynchronize(C.stream) != hipSuccess) {
    set_error("reading the residue check failed");
    return -1;
  }
  return bad ? 1 : 0;
}

}  // namespace swrt

extern "C" {

const char *sw_strerror(int code) {
  switch (code) {
    case SW_OK: return "ok";
    case SW_PENDING: return "pending";
    case SW_EINVAL: return "invalid argument";
    case SW_ENOMEM: return "out of memory or over the memory budget";
    case SW_EDEVICE: return "HIP device error";
    case SW_EOVERFLOW: return "score could exceed the int32 range";
    case SW_ENOENT: return "unknown ticket";
    case SW_EBUSY: return "queue full";
  }
  return "unknown status";
}

const char *sw_last_error(void) { return g_last_error.c_str(); }

int sw_init(int device) { return ensure_init(device); }

int sw_shutdown(void) {
  std::lock_guard<std::mutex> g(g_ctx.mu);
  g_ctx.shutdown();
  return SW_OK;
}

int sw_align(const uint8_t *query, int32_t query_len, const uint8_t *ref, int32_t ref_len,
             const sw_scoring *sc, sw_result *out) {
  return sw_align_ex(query, query_len, ref, ref_len, sc, out, nullptr);
}

int sw_align_ex(const uint8_t *query, int32_t query_len, const uint8_t *ref, int32_t ref_len,
                const sw_scoring *sc, sw_result *out, sw_stats *stats) {
  const double t0 = now_ms();
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!out || query_len < 0 || ref_len < 0 || (query_len > 0 && !query) ||
      (ref_len > 0 && !ref)) {
    set_error("bad argument to sw_align");
    return SW_EINVAL;
  }
  Scoring S;
  int rc = prepare_scoring(sc, S);
  if (rc) return rc;
  for (int k = 0; k < query_len; ++k)
    if (query[k] >= S.alpha) { set_error("query residue %d out of range", k); return SW_EINVAL; }
  for (int k = 0; k < ref_len; ++k)
    if (ref[k] >= S.alpha) { set_error("reference residue %d out of range", k); return SW_EINVAL; }
  *out = sw_result{0, -1, -1, 0};
  if (query_len == 0 || ref_len == 0) return SW_OK;
  if (overflows(query_len, ref_len, S.max_s)) { set_error("score may overflow int32"); return SW_EOVERFLOW; }
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_ctx.mu);
  Context &C = g_ctx;
  HIPCHK(hipSetDevice(C.device));
  if ((rc = C.qres.ensure(query_len)) || (rc = C.rres.ensure(ref_len))) return rc;
  HIPCHK(hipMemcpyAsync(C.qres.p, query, query_len, hipMemcpyHostToDevice, C.stream));
  HIPCHK(hipMemcpyAsync(C.rres.p, ref, ref_len, hipMemcpyHostToDevice, C.stream));
  ExecInput in;
  in.d_qres = C.qres.as<uint8_t>();
  in.d_rres = C.rres.as<uint8_t>();
  PairInfo p;
  std::memset(&p, 0, sizeof(p));
  p.m = query_len;
  p.n = ref_len;
  in.pairs.push_back(p);
  in.items.push_back(PlanItem{0, 0, query_len, ref_len});
  in.n_queries = 1;
  in.q_off_of_query = {0};
  in.m_of_query = {query_len};
  ExecOptions opt;
  opt.force_kernel = 1;
  opt.force_lanes = 64;
  rc = run_batch(in, S, SW_PREC_I32, opt, C.ws, 1, C.stream, C.ev0, C.ev1, C.num_cus, out,
                 stats);
  if (stats) {
    stats->cells = (int64_t)query_len * ref_len;
    stats->total_ms = now_ms() - t0;
  }
  return rc;
}

int sw_align_batch_ex(const sw_batch *b, const sw_scoring *sc, const sw_options *opt,
                      sw_result *out, sw_stats *stats) {
  const double t0 = now_ms();
  if (!b || !out) { set_error("batch or out is NULL"); return SW_EINVAL; }
  Scoring S;
  int rc = prepare_scoring(sc, S);
  if (rc) return rc;
  ExecOptions eo;
  if (opt) {
    if (opt->algorithm != SW_ALG_SCAN && opt->algorithm != SW_ALG_LAZYF) { set_error("bad algorithm"); return SW_EINVAL; }
    if (opt->force_lanes && opt->force_lanes != 8 && opt->force_lanes != 16 &&
        opt->force_lanes != 32 && opt->force_lanes != 64) {
      set_error("force_lanes must be 0, 8, 16, 32 or 64");
      return SW_EINVAL;
    }
    if (opt->force_seglen < 0 || opt->int16_cap < 0 || opt->int16_cap > 32767 ||
        opt->mixed_layout < 0 || opt->mixed_layout > 2 || opt->use_graph < 0 || opt->use_graph > 1 ||
        opt->force_kernel < 0 || opt->force_kernel > 2 || opt->planner < 0 || opt->planner > 2 ||
        opt->lane_pairing < 0 || opt->lane_pairing > 2 || opt->int32_chains < 0 ||
        opt->int32_chains > 2 || opt->striping < 0 || opt->striping > 2) {
      set_error("bad option value");
      return SW_EINVAL;
    }
    eo.algorithm = opt->algorithm;
    eo.force_lanes = opt->force_lanes;
    eo.force_seglen = opt->force_seglen;
    eo.force_kernel = opt->force_kernel;
    eo.mixed_layout = opt->mixed_layout;
    eo.use_graph = opt->use_graph;
    eo.lane_pairing = opt->lane_pairing;
    eo.int32_chains = opt->int32_chains;
    eo.striping = opt->striping;
    if (opt->int16_cap) eo.int16_cap = opt->int16_cap;
  }
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (b->n_pairs < 0 || b->n_queries < 0 || b->n_refs < 0) { set_error("negative count"); return SW_EINVAL; }
  if (b->precision != SW_PREC_AUTO && b->precision != SW_PREC_I32) { set_error("bad precision"); return SW_EINVAL; }
  const int np = b->n_pairs;
  if (np == 0) return SW_OK;
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_ctx.mu);
  Context &C = g_ctx;
  HIPCHK(hipSetDevice(C.device));
  bool handled = false;
  // swapped striping is planned on the host: unless the caller forces the
  // device planner, it takes the batch
  int planner = opt ? opt->planner : 0;
  if (eo.striping == SW_STRIPE_SHORTER && planner == 0) planner = 1;
  rc = run_device_plan(b, S, eo, planner, C, out, stats, t0, handled);
  if (handled) return rc;
  if (rc) return rc;
  if (eo.force_lanes == 8) {
    set_error("8 lanes per alignment only in the device planner's per-pair kernel (one query "
              "per pair, int16 lanes, scores within int8, queries of at most 152 residues)");
    return SW_EINVAL;
  }
  ExecInput in;
  int64_t cells = 0;
  if ((rc = prepare_batch(b, S, C, in, out, cells))) return rc;
  const double t_prep = now_ms() - t0;
  rc = run_batch(in, S, b->precision, eo, C.ws, np, C.stream, C.ev0, C.ev1, C.num_cus, out, stats);
  int bad = 0;
  if ((rc == SW_OK || rc == SW_EINVAL) && (bad = residue_flag(C)) < 0) return SW_EDEVICE;
  if (bad) {
    for (int k = 0; k < np; ++k) out[k] = sw_result{0, -1, -1, 0};
    set_error("a residue code is >= alphabet_size");
    return SW_EINVAL;
  }
  if (rc) return rc;
  if (stats) {
    stats->cells = cells;
    stats->prep_ms = t_prep;
    stats->total_ms = now_ms() - t0;
  }
  return SW_OK;
}

int sw_align_batch(const sw_batch *b, const sw_scoring *sc, sw_result *out) {
  return sw_align_batch_ex(b, sc, nullptr, out, nullptr);
}

}  // extern "C"
