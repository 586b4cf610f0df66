// Device planner (sw_align_batch): the pairs are validated, counted by
// reference length, ordered longest first and run entirely on the device,
// by the shared-query kernel for a batch with one query, by the per-pair
// kernel when every pair has its own query.  The host reads four offsets
// before the launch (and, for per-pair queries, the longest query length
// once the pairs are counted) and the results after it.
//
// Steps on the device (one stream, capturable as one hipGraph):
//   matrix upload, clearing of the plan words (a fill kernel),
//   residue checks of the query and reference sets,
//   plan_count   PairInfo, reference checks, result initialisation, per-
//                workgroup histograms of ceil(n / 4), sum of the lengths,
//   plan_total   every workgroup's offset inside every bin, bin totals,
//   plan_scatter bin starts (a scan of the totals) and the longest-first
//                order (LDS atomics only), number of runnable pairs,
//   shared_direct_kernel  one persistent launch; task t = entries
//                [t*slots, (t+1)*slots) of the order, residues read from the
//                references.
// The alignment arithmetic is the same column step as every other launch of
// this library (Algorithm 6 with the max-plus scan).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <vector>

#include "sw.h"
#include "sw_internal.h"
#include "sw_menus.h"
#include "sw_runtime.h"

namespace swrt {

using namespace swk;

#define HIPCHK(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                __LINE__);                                                       \
      return SW_EDEVICE;                                                         \
    }                                                                            \
  } while (0)

namespace {

constexpr int kDevPlanMinPairs = 4096;   // smaller batches: the host planner
// LDS of one per-pair wavefront (matrix and profiles): keeps several
// wavefronts per CU
constexpr size_t kPairDirectLds = 24 * 1024;
constexpr int64_t kI32Limit = 2147483647ll;


// The (rows per lane, lanes) shape for query length m: the caller's forced
// shape, else the autotuner's entry, else the smallest compiled shape that
// holds the query in one chunk.  False if none applies.
bool pick_direct_shape(Prec prec, int alpha, int m, const ExecOptions &eo, int &seg, int &lanes) {
  if (eo.force_lanes || eo.force_seglen) {
    for (int k = 0; k < kNumDirectShapes; ++k) {
      const DirectShape d = kDirectShapes[k];
      if ((eo.force_lanes == 0 || d.lanes == eo.force_lanes) &&
          (eo.force_seglen == 0 || d.seg == eo.force_seglen) && d.seg * d.lanes >= m) {
        seg = d.seg;
        lanes = d.lanes;
        return true;
      }
    }
    return false;
  }
  sw_tune_entry te;
  if (eo.use_tuning && tune_lookup(SW_TUNE_SHARED, prec, alpha, m, te) && te.lanes > 0 &&
      shared_direct_has(prec, te.seglen, te.lanes) && te.seglen * te.lanes >= m) {
    seg = te.seglen;
    lanes = te.lanes;
    return true;
  }
  for (int k = 0; k < kNumDirectShapes; ++k) {
    const DirectShape d = kDirectShapes[k];
    if (d.seg * d.lanes >= m) {
      seg = d.seg;
      lanes = d.lanes;
      return true;
    }
  }
  return false;
}

// Rows per virtual lane of the row-pair layout: the forced value, else the
// smallest compiled one that holds the query (32 virtual lanes), within
// 64 KiB of LDS per workgroup.
bool pick_rowpair_seg(int m, int alpha, int force_seg, int &seg) {
  for (int s : {4, 8, 12, 16}) {
    if ((force_seg == 0 || s == force_seg) && 32 * s >= m && shared_rowpair_has(s) &&
        shared_rowpair_lds_bytes(s, alpha) <= 65536) {
      seg = s;
      return true;
    }
  }
  return false;
}

// Shape of the device-planned per-pair kernel for queries of up to max_m
// residues: profile entry bytes (1 where the matrix fits int8), then rows per
// lane for 16-lane sub-groups (the forced value, else the autotuner's 16-lane
// entry, else the smallest compiled one) and for 8-lane sub-groups (int16
// lanes with byte profiles: the smallest compiled one), within the
// per-wavefront LDS budget.  Between the two, forced lanes decide, else the
// smaller modelled VALU work per alignment column: a column costs about 13
// instructions per row (the recurrence's 11, the profile merge and the
// end-cell copy) plus ~22 for the scan, the residue and the record test,
// shared by 8 (16 lanes) or 16 (8 lanes) alignments.
bool pick_pair_shape(Prec prec, const Scoring &S, int max_m, const ExecOptions &eo, int &seg,
                     int &lanes, int &es) {
  es = prec == PREC_I16X2 ? (S.fits_i8 ? 1 : 2) : 4;
  auto fits = [&](int s, int P) {
    return pair_direct_has(s, P) && (int64_t)P * s >= max_m &&
           pair_direct_lds_bytes(prec, s, S.alpha, es) <= kPairDirectLds;
  };
  int s16 = 0, s8 = 0;
  // the autotuner's measured shape for this longest query, when it applies
  sw_tune_entry td;
  if (!eo.force_lanes && !eo.force_seglen && eo.use_tuning &&
      tune_lookup(SW_TUNE_DEVICE_PAIR, prec, S.alpha, max_m, td)) {
    if ((td.lanes == 16 || (td.lanes == 8 && prec == PREC_I16X2 && es == 1)) &&
        fits(td.seglen, td.lanes)) {
      seg = td.seglen;
      lanes = td.lanes;
      return true;
    }
  }
  if (eo.force_lanes != 8) {
    if (eo.force_seglen) {
      if (fits(eo.force_seglen, 16)) s16 = eo.force_seglen;
    } else {
      sw_tune_entry te;
      if (eo.use_tuning && tune_lookup(SW_TUNE_PAIR, prec, S.alpha, max_m, te) && te.lanes == 16 &&
          fits(te.seglen, 16))
        s16 = te.seglen;
      for (int s : kPairSegs)
        if (s16 == 0 && fits(s, 16)) s16 = s;
    }
  }
  if (eo.force_lanes != 16 && prec == PREC_I16X2 && es == 1) {
    for (int s : kPair8Segs)
      if (s8 == 0 && (eo.force_seglen == 0 || s == eo.force_seglen) && fits(s, 8)) s8 = s;
  }
  if (s16 == 0 && s8 == 0) return false;
  bool eight = s16 == 0;
  if (s16 && s8 && !eo.force_seglen) eight = (13.0 * s8 + 22.0) / 16.0 < (13.0 * s16 + 22.0) / 8.0;
  seg = eight ? s8 : s16;
  lanes = eight ? 8 : 16;
  return true;
}

}  // namespace

bool rowpair_shape(int m, int alpha, int &seg) { return pick_rowpair_seg(m, alpha, 0, seg); }
bool rowpair_shape_forced(int m, int alpha, int force_seg, int &seg) {
  return pick_rowpair_seg(m, alpha, force_seg, seg);
}

int run_device_plan(const sw_batch *b, const Scoring &S, const ExecOptions &eo, int planner,
                    Context &C, sw_result *out, sw_stats *stats, double t0, bool &handled,
                    const int32_t *first_row) {
  handled = false;
  const int np = b->n_pairs;
  // ---- does the batch qualify (everything here is host-side)
  if (planner == 1) return SW_OK;
  auto refuse = [&](const char *why) {
    if (planner == 2) {
      handled = true;
      set_error("device planner: %s", why);
      return SW_EINVAL;
    }
    return SW_OK;
  };
  if (eo.algorithm != SW_ALG_SCAN) return refuse("only the scan algorithm is device-planned");
  if (planner == 0 && np < kDevPlanMinPairs && eo.force_lanes != 8) return SW_OK;
  if (!b->query_res || !b->query_off || !b->ref_res || !b->ref_off || !b->pair_ref ||
      b->n_queries < 1 || b->n_refs < 1)
    return SW_OK;   // the host path reports the argument error
  // one query (the shared-query kernel) or one query per pair (the per-pair kernel)
  const bool single = b->pair_query == nullptr || b->n_queries == 1;
  if (single && eo.force_kernel == 2) return refuse("one query runs in the shared-query kernel");
  if (!single && eo.force_kernel == 1) return refuse("several queries run in the per-pair kernel");
  if (!single && eo.lane_pairing == SW_PAIRING_ROWS) return refuse("row pairs need one query");
  if (!single && eo.force_lanes && eo.force_lanes != 16 && eo.force_lanes != 8)
    return refuse("per-pair launches use 8 or 16 lanes");
  if (single && eo.force_lanes == 8) return refuse("8 lanes only for one query per pair");
  hipStream_t st = C.stream;
  Workspace &ws = C.ws;
  // query 0's offsets, the query set's end and the reference set's end
  int64_t hv[4];
  if (b->device_resident) {
    if (b->stream) {
      HIPCHK(hipEventRecord(C.evx, (hipStream_t)b->stream));
      HIPCHK(hipStreamWaitEvent(st, C.evx, 0));
    }
    int rc = ws.staging.ensure(64);
    if (rc) return rc;
    int64_t *pv = ws.staging.as<int64_t>();
    HIPCHK(hipMemcpyAsync(pv, b->query_off, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pv + 2, b->query_off + b->n_queries, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pv + 3, b->ref_off + b->n_refs, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(hv, pv, sizeof(hv));
  } else {
    hv[0] = b->query_off[0];
    hv[1] = b->query_off[1];
    hv[2] = b->query_off[b->n_queries];
    hv[3] = b->ref_off[b->n_refs];
  }
  const int64_t q_off0 = hv[0], qbytes = hv[2], rbytes = hv[3];
  if (q_off0 < 0 || hv[1] < q_off0 || hv[1] > qbytes || hv[1] - q_off0 > kI32Limit || rbytes < 0)
    return SW_OK;   // malformed offsets: the host path reports them
  const int m = single ? (int)(hv[1] - q_off0) : 0;
  if (single && m == 0) return SW_OK;
  if (single && (int64_t)m * S.max_s >= kI32Limit) return refuse("the query may overflow int32");
  const Prec prec = (b->precision == SW_PREC_AUTO && S.fits_i16) ? PREC_I16X2 : PREC_I32;
  int seg = 0, lanes = 16, pes = 0;   // pes: per-pair profile entry bytes
  bool rows = false;   // row pairs: both halves of a lane hold rows of one alignment
  int lrec = eo.lds_records;          // row pairs: end-cell records in LDS
  if (first_row) {
    // start-cell pass: masked row pairs only
    if (!single) return refuse("masked rows need one query");
    if (prec != PREC_I16X2) return refuse("masked rows need int16 lanes");
    if (!pick_rowpair_seg(m, S.alpha, 0, seg)) return refuse("no row-pair shape holds the query");
    rows = true;
    handled = true;
  } else if (single) {
    // the autotuner's measured shape for this query length, when no option
    // forces one
    sw_tune_entry td;
    const bool tuned = eo.use_tuning && !eo.force_lanes && !eo.force_seglen &&
                       eo.lane_pairing == SW_PAIRING_AUTO &&
                       tune_lookup(SW_TUNE_DEVICE_SHARED, prec, S.alpha, m, td);
    if (eo.lane_pairing == SW_PAIRING_ROWS) {
      if (prec != PREC_I16X2) return refuse("row pairs need int16 lanes");
      if (eo.force_lanes && eo.force_lanes != 16) return refuse("row pairs use 16 lanes");
      rows = pick_rowpair_seg(m, S.alpha, eo.force_seglen, seg);
      if (!rows) return refuse("no compiled row-pair shape holds the query");
    } else if (tuned && td.pairing == SW_PAIRING_ROWS && prec == PREC_I16X2 &&
               pick_rowpair_seg(m, S.alpha, td.seglen, seg)) {
      rows = true;
      lrec = td.lds_records;
    } else if (tuned && td.pairing == SW_PAIRING_ALIGNMENTS &&
               shared_direct_has(prec, td.seglen, td.lanes) && td.seglen * td.lanes >= m) {
      seg = td.seglen;
      lanes = td.lanes;
    } else if (eo.lane_pairing == SW_PAIRING_AUTO && prec == PREC_I16X2 && !eo.force_lanes &&
               !eo.force_seglen && pick_rowpair_seg(m, S.alpha, 0, seg)) {
      rows = true;   // the default for int16 lanes: one profile word per row pair
    } else if (!pick_direct_shape(prec, S.alpha, m, eo, seg, lanes)) {
      return refuse("no compiled shape holds the query in one chunk");
    }
    handled = true;
  }

  // ---- buffers
  int rc;
  const size_t mat_bytes = sizeof(int) * S.M.size();
  const size_t plan_words = (size_t)kPlanOrder + np;
  if ((rc = ws.plan.ensure(plan_words * sizeof(int32_t))) ||
      (rc = ws.offs.ensure((size_t)np * sizeof(PairInfo) + 4096)) ||
      (rc = ws.results.ensure((size_t)np * sizeof(DevResult))) ||
      (rc = ws.matrix.ensure(mat_bytes)) ||
      (rc = ws.staging.ensure((mat_bytes + 63) / 64 * 64 + sizeof(int32_t) * (kPlanMeta + kMetaWords))))
    return rc;
  int32_t *plan = ws.plan.as<int32_t>();
  unsigned long long *d_stats = (unsigned long long *)(plan + kPlanStats);
  int32_t *meta = plan + kPlanMeta;
  PairInfo *d_pairs = ws.offs.as<PairInfo>();
  DevResult *d_res = ws.results.as<DevResult>();
  // sequences and offsets on the device
  const uint8_t *d_qres = b->query_res, *d_rres = b->ref_res;
  const int64_t *d_roff = b->ref_off, *d_qoff = b->query_off;
  const int32_t *d_pq = b->pair_query, *d_pr = b->pair_ref;
  if (!b->device_resident) {
    const size_t o_roff = 0, o_qoff = o_roff + sizeof(int64_t) * (b->n_refs + 1);
    const size_t o_pr = o_qoff + sizeof(int64_t) * (b->n_queries + 1);
    const size_t o_pq = o_pr + sizeof(int32_t) * np;
    if ((rc = C.qres.ensure(std::max<int64_t>(qbytes, 1))) ||
        (rc = C.rres.ensure(std::max<int64_t>(rbytes, 1))) ||
        (rc = ws.pairs.ensure(o_pq + sizeof(int32_t) * np + 64)))
      return rc;
    char *base = ws.pairs.as<char>();
    HIPCHK(hipMemcpyAsync(base + o_roff, b->ref_off, o_qoff - o_roff, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + o_qoff, b->query_off, o_pr - o_qoff, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(base + o_pr, b->pair_ref, sizeof(int32_t) * np, hipMemcpyHostToDevice, st));
    if (b->pair_query)
      HIPCHK(hipMemcpyAsync(base + o_pq, b->pair_query, sizeof(int32_t) * np, hipMemcpyHostToDevice, st));
    if (qbytes) HIPCHK(hipMemcpyAsync(C.qres.p, b->query_res, qbytes, hipMemcpyHostToDevice, st));
    if (rbytes) HIPCHK(hipMemcpyAsync(C.rres.p, b->ref_res, rbytes, hipMemcpyHostToDevice, st));
    d_qres = C.qres.as<uint8_t>();
    d_rres = C.rres.as<uint8_t>();
    d_roff = (const int64_t *)(base + o_roff);
    d_qoff = (const int64_t *)(base + o_qoff);
    d_pr = (const int32_t *)(base + o_pr);
    d_pq = b->pair_query ? (const int32_t *)(base + o_pq) : nullptr;
  }
  int *stg = ws.staging.as<int>();
  std::memcpy(stg, S.M.data(), mat_bytes);
  unsigned char *tail = (unsigned char *)ws.staging.p + (mat_bytes + 63) / 64 * 64;

  // ---- the device work: eager, or captured once per parameter signature and
  // replayed (one graph for a single query; for per-pair queries one before
  // and one after the host reads the longest query length)
  int32_t *boff = plan + kPlanOff;
  int32_t *totals = plan + kPlanTotals;
  int32_t *hist = plan + kPlanHist;
  int32_t *order = plan + kPlanOrder;
  const int ni = b->n_refs, nq = b->n_queries;
  const int alpha = S.alpha;
  int32_t *d_mat = ws.matrix.as<int32_t>();
  ExecStats es;
  const std::vector<uint64_t> base_sig = {
      (uint64_t)prec, (uint64_t)np, (uint64_t)(uintptr_t)d_qres, (uint64_t)(uintptr_t)d_rres,
      (uint64_t)(uintptr_t)d_roff, (uint64_t)(uintptr_t)d_qoff, (uint64_t)(uintptr_t)d_pq,
      (uint64_t)(uintptr_t)d_pr, (uint64_t)ni, (uint64_t)nq, (uint64_t)rbytes, (uint64_t)qbytes,
      (uint64_t)m, (uint64_t)q_off0, (uint64_t)alpha, (uint64_t)S.go, (uint64_t)S.ge,
      (uint64_t)eo.int16_cap, (uint64_t)(uintptr_t)plan, (uint64_t)(uintptr_t)d_pairs,
      (uint64_t)(uintptr_t)d_res, (uint64_t)(uintptr_t)d_mat, (uint64_t)(uintptr_t)stg};
  // runs fn eagerly, or as a graph keyed by base_sig + extra; `timed` brackets
  // it with the kernel-time events
  auto run = [&](const std::vector<uint64_t> &extra, const std::function<hipError_t()> &fn,
                 bool timed) -> int {
    if (!eo.use_graph) {
      if (timed) HIPCHK(hipEventRecord(C.ev0, st));
      const hipError_t e = fn();
      if (e != hipSuccess) {
        set_error("device-planned launch: %s", hipGetErrorString(e));
        return SW_EDEVICE;
      }
      if (timed) HIPCHK(hipEventRecord(C.ev1, st));
      return SW_OK;
    }
    std::vector<uint64_t> sv = base_sig;
    sv.insert(sv.end(), extra.begin(), extra.end());
    hipGraphExec_t exec = ws.graphs.find(sv);
    if (exec) {
      es.graph_hits++;
    } else {
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
      const hipError_t e = fn();
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &graph);
      if (e != hipSuccess || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        set_error("device-planned capture: %s", hipGetErrorString(e != hipSuccess ? e : ec));
        return SW_EDEVICE;
      }
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ei));
        return SW_EDEVICE;
      }
      ws.graphs.put(sv, exec);
    }
    if (timed) HIPCHK(hipEventRecord(C.ev0, st));
    HIPCHK(hipGraphLaunch(exec, st));
    if (timed) HIPCHK(hipEventRecord(C.ev1, st));
    return SW_OK;
  };
  auto prep = [=]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(d_mat, stg, mat_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)plan, kPlanCleared, 0u, st);
    if (e == hipSuccess) e = launch_check_residues(d_qres, qbytes, alpha, meta + kMetaErrResidue, st);
    if (e == hipSuccess) e = launch_check_residues(d_rres, rbytes, alpha, meta + kMetaErrResidue, st);
    if (e == hipSuccess)
      e = launch_plan_count(np, single ? nullptr : d_qoff, nq, qbytes, d_roff, d_pq, d_pr, ni,
                            rbytes, m, q_off0, d_pairs, d_res, hist, meta, d_stats, st);
    return e;
  };
  auto place = [=]() -> hipError_t {
    hipError_t e = launch_plan_total(hist, boff, totals, st);
    if (e == hipSuccess) e = launch_plan_scatter(np, d_pairs, totals, boff, order, meta, st);
    return e;
  };
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pairs = d_pairs;
  a.query_res = d_qres;
  a.shared_q_off = q_off0;
  a.shared_m = m;
  a.alpha = S.alpha;
  a.matrix = d_mat;
  a.gap_open = S.go;
  a.gap_extend = S.ge;
  a.last_chunk = 1;
  a.sat_cap = eo.int16_cap;
  a.results = d_res;
  a.stats = d_stats;
  a.order = order;
  a.plan_meta = meta;
  a.ref_res = d_rres;
  a.first_row = first_row;
  const double t_launch0 = now_ms();
  es.plan_ms = t_launch0 - t0;
  int max_m = m;
  if (single) {
    const int slots = rows ? kWave / 16 : (kWave / lanes) * (prec == PREC_I16X2 ? 2 : 1);
    const int ntasks_max = (np + slots - 1) / slots;
    // row pairs: wavefronts wanted (the launcher sizes its workgroups);
    // otherwise workgroups of kWavesPerGroup wavefronts
    const int grid = rows ? std::max(1, std::min(ntasks_max, C.num_cus * 16))
                          : std::max(1, std::min((ntasks_max + kWavesPerGroup - 1) / kWavesPerGroup,
                                                 C.num_cus * 2));
    auto all = [=]() -> hipError_t {
      hipError_t e = prep();
      if (e == hipSuccess) e = place();
      if (e == hipSuccess)
        e = rows ? launch_shared_rowpair(seg, a, grid, st, lrec)
                 : launch_shared_direct(prec, seg, lanes, a, grid, st);
      return e;
    };
    if ((rc = run({0xD1D1, (uint64_t)seg, (uint64_t)lanes, (uint64_t)rows, (uint64_t)grid,
                   (uint64_t)(uintptr_t)first_row, (uint64_t)(int64_t)lrec}, all,
                  true)))
      return rc;
  } else {
    // the longest query decides the rows per lane
    if ((rc = run({0xD2D1}, prep, false))) return rc;
    HIPCHK(hipMemcpyAsync(tail, plan, (size_t)(kPlanMeta + kMetaWords) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int32_t hm0[kMetaWords];
    std::memcpy(hm0, tail + kPlanMeta * sizeof(int32_t), sizeof(hm0));
    max_m = hm0[kMetaMaxM];
    if (!hm0[kMetaErrResidue] && !hm0[kMetaErrPair] && max_m > 0) {
      const bool ok = (int64_t)max_m * S.max_s < kI32Limit &&
                      pick_pair_shape(prec, S, max_m, eo, seg, lanes, pes);
      if (!ok) {
        // nothing was written to `out`: the host planner takes the batch
        if (planner == 2) {
          handled = true;
          set_error("device planner: no per-pair shape holds queries of %d residues", max_m);
          return SW_EINVAL;
        }
        return SW_OK;
      }
      const int slots = (64 / lanes) * (prec == PREC_I16X2 ? 2 : 1);
      const int ntasks_max = (np + slots - 1) / slots;
      const int grid = std::max(1, std::min(ntasks_max, C.num_cus * 16));
      auto rest = [=]() -> hipError_t {
        hipError_t e = place();
        if (e == hipSuccess) e = launch_pair_direct(prec, seg, lanes, pes, a, grid, st);
        return e;
      };
      if ((rc = run({0xD2D2, (uint64_t)seg, (uint64_t)lanes, (uint64_t)pes, (uint64_t)grid}, rest,
                    true)))
        return rc;
    }
    handled = true;
  }
  const double t_fin0 = now_ms();
  es.launch_ms = t_fin0 - t_launch0;
  // ---- results, statistics and the plan's error words
  // staging: [matrix | plan words read back]; results go straight to `out`
  HIPCHK(hipMemcpyAsync(out, d_res, (size_t)np * sizeof(DevResult), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(tail, plan, (size_t)(kPlanMeta + kMetaWords) * sizeof(int32_t),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  unsigned long long hs[8];
  int32_t hm[kMetaWords];
  std::memcpy(hs, tail, sizeof(hs));
  std::memcpy(hm, tail + kPlanMeta * sizeof(int32_t), sizeof(hm));
  float kms = 0;
  if (seg > 0) HIPCHK(hipEventElapsedTime(&kms, C.ev0, C.ev1));
  if (hm[kMetaErrResidue] || hm[kMetaErrPair]) {
    for (int k = 0; k < np; ++k) out[k] = sw_result{0, -1, -1, 0};
    set_error(hm[kMetaErrResidue] ? "a residue code is >= alphabet_size"
                                  : "a pair refers to a query or reference out of range, or "
                                    "offsets that are not nondecreasing");
    return SW_EINVAL;
  }
  // ---- exact int32 rerun of the pairs whose int16 lanes saturated
  std::vector<int> again;
  if (prec == PREC_I16X2 && !first_row)
    for (int k = 0; k < np; ++k)
      if (out[k].flags & kFlagNeedsI32) again.push_back(k);
  if (!again.empty()) {
    std::vector<PairInfo> hp(np);
    HIPCHK(hipMemcpyAsync(hp.data(), d_pairs, (size_t)np * sizeof(PairInfo), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ExecInput in2;
    in2.d_qres = d_qres;
    in2.d_rres = d_rres;
    in2.d_pairs = d_pairs;
    in2.n_pairs = np;
    // one query: query 0 (many reruns share its profile); per-pair queries:
    // every rerun pair as its own query (its PairInfo holds the query offset)
    for (int k : again) {
      const int q = single ? 0 : (int)in2.q_off_of_query.size();
      in2.items.push_back(PlanItem{k, q, hp[k].m, hp[k].n});
      if (!single || in2.q_off_of_query.empty()) {
        in2.q_off_of_query.push_back(hp[k].q_off);
        in2.m_of_query.push_back(hp[k].m);
      }
    }
    in2.n_queries = (int)in2.q_off_of_query.size();
    ExecOptions o2 = eo;
    o2.force_lanes = 0;
    o2.force_seglen = 0;
    o2.lane_pairing = SW_PAIRING_AUTO;   // the int32 rerun has no int16 halves
    o2.force_kernel = 0;
    o2.use_graph = 0;
    ExecStats es2;
    if ((rc = execute(in2, S, PREC_I32, o2, ws, np, st, C.ev0, C.ev1, C.num_cus, es2, false)))
      return rc;
    std::vector<DevResult> hr(np);
    HIPCHK(hipMemcpyAsync(hr.data(), d_res, (size_t)np * sizeof(DevResult), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k : again) {
      out[k].score = hr[k].score;
      out[k].query_end = hr[k].qend;
      out[k].ref_end = hr[k].rend;
      out[k].flags = SW_FLAG_SATURATED;
    }
    es.kernel_ms += es2.kernel_ms;
    es.launches += es2.launches;
  }
  if (stats) {
    stats->kernel_ms = kms + es.kernel_ms;
    stats->total_ms = now_ms() - t0;
    stats->cells = (int64_t)hs[5];
    stats->padded_cells = (int64_t)hs[3];
    stats->n_rerun = (int)again.size();
    stats->n_launches = (seg > 0 ? 1 : 0) + es.launches;
    stats->columns = (int64_t)hs[0];
    stats->record_events = (int64_t)hs[2];
    if (lanes == 8)
      stats->lanes8 = hm[kMetaValid];
    else
      stats->lanes_used[lanes == 16 ? 0 : (lanes == 32 ? 1 : 2)] = hm[kMetaValid];
    stats->seglen_max = seg;
    stats->prep_ms = 0;
    stats->plan_ms = es.plan_ms;
    stats->launch_ms = es.launch_ms;
    stats->finish_ms = now_ms() - t_fin0;
    stats->graph_hits = es.graph_hits;
    stats->planner_used = 2;
    stats->row_pairs = rows ? hm[kMetaValid] : 0;
  }
  return SW_OK;
}

// ---------------------------------------------------------------------------
// The same device plan with every buffer in a caller-given scratch region and
// the results written straight into a device array: no allocation of any kind
// (no device, pinned or heap memory), for callers that cannot allocate.

namespace {

struct NoallocRegions {
  int32_t *plan;
  PairInfo *pairs;
  DevResult *r32;
  int32_t *matrix;
};

NoallocRegions noalloc_regions(unsigned char *scr, int max_pairs) {
  auto up = noalloc_align256;
  NoallocRegions R;
  size_t o = 0;
  R.plan = (int32_t *)(scr + o);
  o += up(((size_t)kPlanOrder + max_pairs) * sizeof(int32_t));
  R.pairs = (PairInfo *)(scr + o);
  o += up((size_t)max_pairs * sizeof(PairInfo) + 4096);
  R.r32 = (DevResult *)(scr + o);
  o += up((size_t)max_pairs * sizeof(DevResult));
  R.matrix = (int32_t *)(scr + o);
  return R;
}

// What one pass reports back (read from the plan words after it).
struct NoallocPass {
  int32_t meta[kMetaWords];
  unsigned long long stats[8];
  float kernel_ms = 0;
  int seg = 0, lanes = 0;
  bool rows = false;
};

#define NA_HIP(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      set_error("no-allocation batch: %s failed: %s", #expr, hipGetErrorString(e_)); \
      return SW_EDEVICE;                                                    \
    }                                                                       \
  } while (0)

// Reads the stats and meta words of the plan into P (synchronous).
int noalloc_read_plan(const int32_t *plan, NoallocPass &P, hipStream_t st) {
  NA_HIP(hipMemcpyAsync(P.stats, plan + kPlanStats, sizeof(P.stats), hipMemcpyDeviceToHost, st));
  NA_HIP(hipMemcpyAsync(P.meta, plan + kPlanMeta, sizeof(P.meta), hipMemcpyDeviceToHost, st));
  NA_HIP(hipStreamSynchronize(st));
  return SW_OK;
}

// One planned pass at precision `prec` whose results go to `res` (n_pairs
// entries).  m > 0: one query of m residues at q_off0; m == 0: a query per
// pair.  check_rerun: before the alignment launch, refuse a per-pair batch
// whose int16 lanes could saturate while no int32 per-pair shape holds its
// longest query (the rerun could not be run).
int noalloc_pass(const sw_batch *b, const Scoring &S, Context &C, const NoallocRegions &R,
                 Prec prec, int m, int64_t q_off0, int64_t qbytes, int64_t rbytes,
                 bool check_rerun, DevResult *res, NoallocPass &P) {
  const hipStream_t st = C.stream;
  const int np = b->n_pairs;
  const bool single = m > 0;
  ExecOptions eo;   // the planner's fixed rule (the tuning table is not consulted)
  eo.use_tuning = false;
  int seg = 0, lanes = 16, pes = 0;
  bool rows = false;
  if (single) {
    if (prec == PREC_I16X2 && pick_rowpair_seg(m, S.alpha, 0, seg)) {
      rows = true;
    } else if (!pick_direct_shape(prec, S.alpha, m, eo, seg, lanes)) {
      set_error("no-allocation batch: no compiled shape holds a query of %d residues", m);
      return SW_EINVAL;
    }
  }
  int32_t *plan = R.plan;
  int32_t *meta = plan + kPlanMeta;
  unsigned long long *d_stats = (unsigned long long *)(plan + kPlanStats);
  const size_t mat_bytes = sizeof(int32_t) * S.M.size();
  NA_HIP(hipMemcpyAsync(R.matrix, S.M.data(), mat_bytes, hipMemcpyHostToDevice, st));
  NA_HIP(launch_fill_u32((uint32_t *)plan, kPlanCleared, 0u, st));
  NA_HIP(launch_check_residues(b->query_res, qbytes, S.alpha, meta + kMetaErrResidue, st));
  NA_HIP(launch_check_residues(b->ref_res, rbytes, S.alpha, meta + kMetaErrResidue, st));
  NA_HIP(launch_plan_count(np, single ? nullptr : b->query_off, b->n_queries, qbytes, b->ref_off,
                           b->pair_query, b->pair_ref, b->n_refs, rbytes, m, q_off0, R.pairs, res,
                           plan + kPlanHist, meta, d_stats, st));
  if (!single) {
    int rc = noalloc_read_plan(plan, P, st);
    if (rc) return rc;
    if (P.meta[kMetaErrResidue] || P.meta[kMetaErrPair] || P.meta[kMetaMaxM] <= 0) return SW_OK;
    const int max_m = P.meta[kMetaMaxM];
    if ((int64_t)max_m * S.max_s >= kI32Limit) {
      set_error("no-allocation batch: a query of %d residues may overflow int32", max_m);
      return SW_EOVERFLOW;
    }
    if (!pick_pair_shape(prec, S, max_m, eo, seg, lanes, pes)) {
      set_error("no-allocation batch: no per-pair shape holds queries of %d residues", max_m);
      return SW_EINVAL;
    }
    int s32 = 0, l32 = 0, e32 = 0;
    if (check_rerun && prec == PREC_I16X2 && (int64_t)max_m * S.max_s >= eo.int16_cap &&
        !pick_pair_shape(PREC_I32, S, max_m, eo, s32, l32, e32)) {
      set_error("no-allocation batch: int16 lanes could saturate on queries of %d residues and "
                "no int32 per-pair shape holds them for the rerun", max_m);
      return SW_EINVAL;
    }
  }
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pairs = R.pairs;
  a.query_res = b->query_res;
  a.shared_q_off = q_off0;
  a.shared_m = m;
  a.alpha = S.alpha;
  a.matrix = R.matrix;
  a.gap_open = S.go;
  a.gap_extend = S.ge;
  a.last_chunk = 1;
  a.sat_cap = eo.int16_cap;
  a.results = res;
  a.stats = d_stats;
  a.order = plan + kPlanOrder;
  a.plan_meta = meta;
  a.ref_res = b->ref_res;
  NA_HIP(launch_plan_total(plan + kPlanHist, plan + kPlanOff, plan + kPlanTotals, st));
  NA_HIP(launch_plan_scatter(np, R.pairs, plan + kPlanTotals, plan + kPlanOff, plan + kPlanOrder,
                             meta, st));
  NA_HIP(hipEventRecord(C.ev0, st));
  if (single) {
    const int slots = rows ? kWave / 16 : (kWave / lanes) * (prec == PREC_I16X2 ? 2 : 1);
    const int ntasks_max = (np + slots - 1) / slots;
    const int grid = rows ? std::max(1, std::min(ntasks_max, C.num_cus * 16))
                          : std::max(1, std::min((ntasks_max + kWavesPerGroup - 1) / kWavesPerGroup,
                                                 C.num_cus * 2));
    NA_HIP(rows ? launch_shared_rowpair(seg, a, grid, st)
                : launch_shared_direct(prec, seg, lanes, a, grid, st));
  } else {
    const int slots = (64 / lanes) * (prec == PREC_I16X2 ? 2 : 1);
    const int ntasks_max = (np + slots - 1) / slots;
    const int grid = std::max(1, std::min(ntasks_max, C.num_cus * 16));
    NA_HIP(launch_pair_direct(prec, seg, lanes, pes, a, grid, st));
  }
  NA_HIP(hipEventRecord(C.ev1, st));
  if (prec == PREC_I16X2) NA_HIP(launch_count_flag(np, res, kFlagNeedsI32, meta + kMetaNeedsI32, st));
  int rc = noalloc_read_plan(plan, P, st);
  if (rc) return rc;
  NA_HIP(hipEventElapsedTime(&P.kernel_ms, C.ev0, C.ev1));
  P.seg = seg;
  P.lanes = rows ? 16 : lanes;
  P.rows = rows;
  return SW_OK;
}

}  // namespace

int run_device_plan_noalloc(const sw_batch *b, const Scoring &S, Context &C, unsigned char *scr,
                            int max_pairs, sw_result *out, sw_stats *stats, double t0) {
  const hipStream_t st = C.stream;
  const int np = b->n_pairs;
  if (b->device_resident && b->stream) {
    NA_HIP(hipEventRecord(C.evx, (hipStream_t)b->stream));
    NA_HIP(hipStreamWaitEvent(st, C.evx, 0));
  }
  const bool single = b->pair_query == nullptr || b->n_queries == 1;
  // query 0's offsets, the query set's end and the reference set's end
  int64_t hv[4];
  NA_HIP(hipMemcpyAsync(hv, b->query_off, 16, hipMemcpyDeviceToHost, st));
  NA_HIP(hipMemcpyAsync(hv + 2, b->query_off + b->n_queries, 8, hipMemcpyDeviceToHost, st));
  NA_HIP(hipMemcpyAsync(hv + 3, b->ref_off + b->n_refs, 8, hipMemcpyDeviceToHost, st));
  NA_HIP(hipStreamSynchronize(st));
  const int64_t q_off0 = hv[0], qbytes = hv[2], rbytes = hv[3];
  if (q_off0 < 0 || hv[1] < q_off0 || hv[1] > qbytes || hv[1] - q_off0 > kI32Limit || rbytes < 0) {
    set_error("no-allocation batch: query or reference offsets are not nondecreasing");
    return SW_EINVAL;
  }
  const int m = single ? (int)(hv[1] - q_off0) : 0;
  const NoallocRegions R = noalloc_regions(scr, max_pairs);
  DevResult *res = (DevResult *)out;
  if (single && m > 0 && (int64_t)m * S.max_s >= kI32Limit) {
    set_error("no-allocation batch: the query may overflow int32");
    return SW_EOVERFLOW;
  }
  if (single && m > 512) {
    set_error("no-allocation batch: one query of %d residues (at most 512)", m);
    return SW_EINVAL;
  }
  const Prec prec = (b->precision == SW_PREC_AUTO && S.fits_i16) ? PREC_I16X2 : PREC_I32;
  NoallocPass P1;
  int rc = SW_OK;
  if (single && m == 0) {
    // no alignment runs; the count pass validates ids and residues and sets
    // every result to {0, -1, -1, 0}
    NA_HIP(launch_fill_u32((uint32_t *)R.plan, kPlanCleared, 0u, st));
    NA_HIP(launch_check_residues(b->query_res, qbytes, S.alpha, R.plan + kPlanMeta + kMetaErrResidue, st));
    NA_HIP(launch_check_residues(b->ref_res, rbytes, S.alpha, R.plan + kPlanMeta + kMetaErrResidue, st));
    NA_HIP(launch_plan_count(np, nullptr, b->n_queries, qbytes, b->ref_off, b->pair_query,
                             b->pair_ref, b->n_refs, rbytes, 0, q_off0, R.pairs, res,
                             R.plan + kPlanHist, R.plan + kPlanMeta,
                             (unsigned long long *)(R.plan + kPlanStats), st));
    if ((rc = noalloc_read_plan(R.plan, P1, st))) return rc;
  } else if ((rc = noalloc_pass(b, S, C, R, prec, m, q_off0, qbytes, rbytes, true, res, P1))) {
    return rc;
  }
  if (P1.meta[kMetaErrResidue] || P1.meta[kMetaErrPair]) {
    NA_HIP(launch_init_results(np, res, st));
    NA_HIP(hipStreamSynchronize(st));
    set_error(P1.meta[kMetaErrResidue] ? "a residue code is >= alphabet_size"
                                       : "a pair refers to a query or reference out of range, or "
                                         "offsets that are not nondecreasing");
    return SW_EINVAL;
  }
  // exact int32 rerun: the whole batch once more in int32 into the scratch
  // results, merged on the device into the pairs whose int16 lanes saturated
  int n_rerun_launches = 0;
  float kms2 = 0;
  if (prec == PREC_I16X2 && P1.meta[kMetaNeedsI32]) {
    NoallocPass P2;
    if ((rc = noalloc_pass(b, S, C, R, PREC_I32, m, q_off0, qbytes, rbytes, false, R.r32, P2)))
      return rc;
    NA_HIP(launch_merge_rerun(np, R.r32, res, st));
    NA_HIP(hipStreamSynchronize(st));
    n_rerun_launches = P2.seg > 0 ? 1 : 0;
    kms2 = P2.kernel_ms;
  }
  if (stats) {
    stats->kernel_ms = (double)P1.kernel_ms + kms2;
    stats->total_ms = now_ms() - t0;
    stats->cells = (int64_t)P1.stats[5];
    stats->padded_cells = (int64_t)P1.stats[3];
    stats->n_launches = (P1.seg > 0 ? 1 : 0) + n_rerun_launches;
    stats->n_rerun = prec == PREC_I16X2 ? P1.meta[kMetaNeedsI32] : 0;
    stats->columns = (int64_t)P1.stats[0];
    stats->record_events = (int64_t)P1.stats[2];
    stats->seglen_max = P1.seg;
    stats->planner_used = 2;
    const int valid = P1.meta[kMetaValid];
    if (P1.rows)
      stats->row_pairs = valid;
    else if (P1.lanes == 8)
      stats->lanes8 = valid;
    else if (P1.seg > 0)
      stats->lanes_used[P1.lanes == 16 ? 0 : (P1.lanes == 32 ? 1 : 2)] = valid;
  }
  return SW_OK;
}

}  // namespace swrt
