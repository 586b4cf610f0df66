// Autotuner of libswscan.so: a process-wide table of measured kernel shapes
// and the search that fills it (include/sw.h, sw_autotune).
//
// The planner's cost model counts VALU instructions of the column step: per
// cell of the inner loop (Algorithm 6) plus, per column, the log2(lanes) steps
// of the max-plus scan and the column set-up, divided by the alignments a
// wavefront carries.  It does not see occupancy, LDS bank conflicts, the
// imbalance of the last wavefronts of a launch or the instruction latency of a
// short inner loop.  The tuner therefore runs the cost model's best few shapes
// on the real batch (or a strided sample of it), times the alignment kernels
// with HIP events and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <vector>

#include "sw.h"
#include "sw_menus.h"
#include "sw_runtime.h"

using namespace swrt;
using namespace swk;

namespace swrt {

namespace {

std::mutex g_tune_mu;
std::vector<sw_tune_entry> g_tune;

int prec_code(Prec p) { return p == PREC_I16X2 ? SW_PREC_AUTO : SW_PREC_I32; }

bool overlaps(const sw_tune_entry &a, const sw_tune_entry &b) {
  return a.kind == b.kind && a.precision == b.precision && a.alphabet_size == b.alphabet_size &&
         a.mixed == b.mixed && a.m_lo <= b.m_hi && b.m_lo <= a.m_hi;
}

// Installs entries, replacing older ones they overlap.
void tune_merge(const std::vector<sw_tune_entry> &add) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto &e : add) {
    g_tune.erase(std::remove_if(g_tune.begin(), g_tune.end(),
                                [&](const sw_tune_entry &o) { return overlaps(o, e); }),
                 g_tune.end());
    g_tune.push_back(e);
  }
}

}  // namespace

int tune_validate(const sw_tune_entry &e) {
  if (e.kind < SW_TUNE_SHARED || e.kind > SW_TUNE_DEVICE_PAIR) return SW_EINVAL;
  if (e.precision != SW_PREC_AUTO && e.precision != SW_PREC_I32) return SW_EINVAL;
  if (e.alphabet_size < 1 || e.alphabet_size > kMaxAlpha) return SW_EINVAL;
  if (e.m_lo < 1 || e.m_hi < e.m_lo) return SW_EINVAL;
  if (e.mixed != 0 && e.mixed != 1) return SW_EINVAL;
  if (e.kind == SW_TUNE_DEVICE_SHARED) {
    if (e.mixed) return SW_EINVAL;
    if (e.pairing == SW_PAIRING_ROWS)
      return e.precision == SW_PREC_AUTO && e.lanes == 16 && shared_rowpair_has(e.seglen) &&
                     (e.lds_records == 0 || e.lds_records == 1)
                 ? SW_OK : SW_EINVAL;
    if (e.pairing == SW_PAIRING_ALIGNMENTS && e.lds_records == 0)
      return shared_direct_has(e.precision == SW_PREC_AUTO ? PREC_I16X2 : PREC_I32, e.seglen,
                               e.lanes) ? SW_OK : SW_EINVAL;
    return SW_EINVAL;
  }
  if (e.kind == SW_TUNE_DEVICE_PAIR) {
    if (e.mixed || e.pairing || e.lds_records) return SW_EINVAL;
    if (e.lanes == 8 && e.precision != SW_PREC_AUTO) return SW_EINVAL;
    return (e.lanes == 8 || e.lanes == 16) && pair_direct_has(e.seglen, e.lanes) ? SW_OK
                                                                                  : SW_EINVAL;
  }
  if (e.pairing || e.lds_records) return SW_EINVAL;
  if (e.kind == SW_TUNE_SHARED) {
    if (e.mixed) return SW_EINVAL;
    if (e.lanes != 0 && e.lanes != 16 && e.lanes != 32 && e.lanes != 64) return SW_EINVAL;
    for (int k = 0; k < shared_menu_count(); ++k) {
      const SharedMenu mm = shared_menu(k);
      const int s = e.lanes == 16 ? mm.seg16 : (e.lanes == 32 ? mm.seg32 : mm.seg64);
      if (s > 0 && s == e.seglen) return SW_OK;
    }
    return SW_EINVAL;
  }
  if (e.lanes != 16 && e.lanes != 32 && e.lanes != 64) return SW_EINVAL;
  return pair_kernel_has(e.precision == SW_PREC_AUTO ? PREC_I16X2 : PREC_I32, e.seglen, e.lanes)
             ? SW_OK : SW_EINVAL;
}

bool tune_lookup(int kind, Prec prec, int alpha, int m, sw_tune_entry &e) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto &t : g_tune)
    if (t.kind == kind && !t.mixed && t.precision == prec_code(prec) && t.alphabet_size == alpha &&
        t.m_lo <= m && m <= t.m_hi) {
      e = t;
      return true;
    }
  return false;
}

bool tune_mixed(Prec prec, int alpha, int m_min, int m_max, sw_tune_entry &e) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto &t : g_tune)
    if (t.kind == SW_TUNE_PAIR && t.mixed && t.precision == prec_code(prec) &&
        t.alphabet_size == alpha && t.m_lo <= m_min && m_max <= t.m_hi) {
      e = t;
      return true;
    }
  return false;
}

}  // namespace swrt

namespace {

// Every k-th item so that the sample holds about `cap` cells (the length mix
// of the group is kept).
std::vector<PlanItem> strided_sample(const std::vector<PlanItem> &items, int64_t cap) {
  int64_t total = 0;
  for (const auto &it : items) total += (int64_t)it.m * it.n;
  if (total <= cap) return items;
  const int64_t stride = (total + cap - 1) / cap;
  std::vector<PlanItem> s;
  for (size_t k = 0; k < items.size(); k += (size_t)stride) s.push_back(items[k]);
  return s;
}

int64_t cells_of(const std::vector<PlanItem> &items) {
  int64_t c = 0;
  for (const auto &it : items) c += (int64_t)it.m * it.n;
  return c;
}

struct Tuner {
  Context &C;
  const Scoring &S;
  ExecInput &in;
  int precision;
  int np;
  std::vector<sw_result> res;

  // Kernel milliseconds of the best of two runs of `items` under `o`.
  int time(std::vector<PlanItem> &items, const ExecOptions &o, double &ms) {
    in.items.swap(items);
    ms = 1e300;
    int rc = SW_OK;
    for (int rep = 0; rep < 2 && rc == SW_OK; ++rep) {
      sw_stats st;
      std::memset(&st, 0, sizeof(st));
      rc = run_batch(in, S, precision, o, C.ws, np, C.stream, C.ev0, C.ev1, C.num_cus,
                     res.data(), &st);
      ms = std::min(ms, st.kernel_ms);
    }
    in.items.swap(items);
    return rc;
  }
};

}  // namespace

extern "C" {

int sw_tune_set(const sw_tune_entry *entries, int32_t n) {
  if (n < 0 || (n > 0 && !entries)) { set_error("bad tuning table"); return SW_EINVAL; }
  for (int k = 0; k < n; ++k)
    if (tune_validate(entries[k])) {
      set_error("tuning entry %d has an unknown kind, precision or shape", k);
      return SW_EINVAL;
    }
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.assign(entries, entries + n);
  return SW_OK;
}

int sw_tune_get(sw_tune_entry *out, int32_t cap, int32_t *n_out) {
  if (cap < 0 || (cap > 0 && !out)) { set_error("bad output buffer"); return SW_EINVAL; }
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (int k = 0; k < cap && k < (int)g_tune.size(); ++k) out[k] = g_tune[k];
  if (n_out) *n_out = (int32_t)g_tune.size();
  return SW_OK;
}

int sw_autotune(const sw_batch *b, const sw_scoring *sc, int64_t sample_cells,
                sw_tune_entry *out, int32_t cap, int32_t *n_out) {
  if (!b || cap < 0 || (cap > 0 && !out) || sample_cells < 0) { set_error("bad argument"); return SW_EINVAL; }
  if (b->n_pairs < 0 || b->n_queries < 0 || b->n_refs < 0) { set_error("negative count"); return SW_EINVAL; }
  if (b->precision != SW_PREC_AUTO && b->precision != SW_PREC_I32) { set_error("bad precision"); return SW_EINVAL; }
  Scoring S;
  int rc = prepare_scoring(sc, S);
  if (rc) return rc;
  if (n_out) *n_out = 0;
  if (b->n_pairs == 0) return SW_OK;
  if ((rc = ensure_init())) return rc;
  std::lock_guard<std::mutex> g(g_ctx.mu);
  Context &C = g_ctx;
  if (hipSetDevice(C.device) != hipSuccess) { set_error("hipSetDevice failed"); return SW_EDEVICE; }
  const int np = b->n_pairs;
  std::vector<sw_result> res(np);
  ExecInput in;
  int64_t cells = 0;
  if ((rc = prepare_batch(b, S, C, in, res.data(), cells))) return rc;
  const int bad = residue_flag(C);
  if (bad < 0) return SW_EDEVICE;
  if (bad) { set_error("a residue code is >= alphabet_size"); return SW_EINVAL; }
  const Prec prec = (b->precision == SW_PREC_AUTO && S.fits_i16) ? PREC_I16X2 : PREC_I32;
  const int pcode = prec == PREC_I16X2 ? SW_PREC_AUTO : SW_PREC_I32;
  const int64_t cap_cells = sample_cells > 0 ? sample_cells : 50000000000ll;
  Tuner T{C, S, in, b->precision, np, std::move(res)};
  std::vector<PlanItem> all;
  all.swap(in.items);

  // groups as the planner forms them: a query with >= 32 pairs runs shared
  std::vector<int> qcount(in.n_queries, 0);
  for (const auto &it : all) qcount[it.query]++;
  std::vector<std::vector<PlanItem>> shared_groups;
  std::vector<int> shared_query;
  std::vector<PlanItem> per_pair;
  {
    std::vector<int> gid(in.n_queries, -1);
    for (const auto &it : all) {
      if (qcount[it.query] >= 32) {
        if (gid[it.query] < 0) {
          gid[it.query] = (int)shared_groups.size();
          shared_groups.emplace_back();
          shared_query.push_back(it.query);
        }
        shared_groups[gid[it.query]].push_back(it);
      } else {
        per_pair.push_back(it);
      }
    }
  }
  std::vector<sw_tune_entry> found;
  auto entry = [&](int kind, int lo, int hi, int lanes, int seg, int mixed, int64_t c, double ms,
                   double model_ms) {
    sw_tune_entry e;
    std::memset(&e, 0, sizeof(e));
    e.kind = kind;
    e.precision = pcode;
    e.alphabet_size = S.alpha;
    e.m_lo = lo;
    e.m_hi = hi;
    e.lanes = lanes;
    e.seglen = seg;
    e.mixed = mixed;
    e.gcups = ms > 0 ? (double)c / ms / 1e6 : 0;
    e.model_gcups = model_ms > 0 ? (double)c / model_ms / 1e6 : 0;
    return e;
  };

  // ---- shared-query groups: rows-per-lane menu x lane policy, the largest
  // eight groups by cells
  std::vector<int> gorder(shared_groups.size());
  for (size_t k = 0; k < gorder.size(); ++k) gorder[k] = (int)k;
  std::sort(gorder.begin(), gorder.end(), [&](int x, int y) {
    return cells_of(shared_groups[x]) > cells_of(shared_groups[y]);
  });
  if (gorder.size() > 8) gorder.resize(8);
  for (int gi : gorder) {
    std::vector<PlanItem> smp = strided_sample(shared_groups[gi], cap_cells);
    const int64_t c = cells_of(smp);
    const int m = in.m_of_query[shared_query[gi]];
    ExecOptions base;
    base.force_kernel = 1;
    base.use_tuning = false;
    double model_ms;
    if ((rc = T.time(smp, base, model_ms))) return rc;
    int min_nch = INT_MAX;
    for (int k = 0; k < shared_menu_count(); ++k) {
      const int rows = 64 * shared_menu(k).seg64;
      min_nch = std::min(min_nch, (m + rows - 1) / rows);
    }
    double best = 1e300;
    int best_l = 0, best_s = 0, best_rows = 0;
    for (int k = 0; k < shared_menu_count(); ++k) {
      const SharedMenu mm = shared_menu(k);
      const int rows = 64 * mm.seg64;
      const int nch = (m + rows - 1) / rows;
      if (nch > std::max(4, min_nch)) continue;
      const int widths = (mm.seg16 > 0) + (mm.seg32 > 0) + (mm.seg64 > 0);
      for (int L : {0, 16, 32, 64}) {
        const int s = L == 0 ? mm.seg64 : (L == 16 ? mm.seg16 : (L == 32 ? mm.seg32 : mm.seg64));
        if (s <= 0 || (L == 0 && widths < 2)) continue;
        ExecOptions o = base;
        o.force_lanes = L;
        o.force_seglen = s;
        double ms;
        if ((rc = T.time(smp, o, ms))) return rc;
        if (ms < best) { best = ms; best_l = L; best_s = s; best_rows = rows; }
      }
    }
    if (best_rows == 0) continue;
    const int nch = (m + best_rows - 1) / best_rows;
    found.push_back(entry(SW_TUNE_SHARED, (nch - 1) * best_rows + 1, nch * best_rows, best_l,
                          best_s, 0, c, best, model_ms));
  }

  // ---- per-pair groups by query-length bucket
  static const int kEdges[] = {1, 33, 65, 97, 129, 161, 193, 257, 321, 385, 513, 769, 1025,
                               1537, 2049, 3073, 4097, 6145, 8193, 12289, 16385, INT_MAX};
  const int nb = (int)(sizeof(kEdges) / sizeof(kEdges[0])) - 1;
  std::vector<std::vector<PlanItem>> buckets(nb);
  for (const auto &it : per_pair) {
    int k = 0;
    while (k + 1 < nb && it.m >= kEdges[k + 1]) ++k;
    buckets[k].push_back(it);
  }
  std::vector<sw_tune_entry> pair_entries;
  int used_buckets = 0;
  for (int k = 0; k < nb; ++k) {
    if (buckets[k].empty()) continue;
    ++used_buckets;
    std::vector<PlanItem> smp = strided_sample(buckets[k], cap_cells);
    const int64_t c = cells_of(smp);
    ExecOptions base;
    base.force_kernel = 2;
    base.use_tuning = false;
    double model_ms;
    if ((rc = T.time(smp, base, model_ms))) return rc;
    double best = 1e300;
    int best_p = 0, best_s = 0;
    for (const auto &cand : pair_candidates(prec, S.alpha, smp.data(), smp.size(), 6)) {
      ExecOptions o = base;
      o.force_lanes = cand.first;
      o.force_seglen = cand.second;
      double ms;
      if ((rc = T.time(smp, o, ms))) return rc;
      if (ms < best) { best = ms; best_p = cand.first; best_s = cand.second; }
    }
    if (best_p == 0) continue;
    const int hi = kEdges[k + 1] == INT_MAX ? INT_MAX : kEdges[k + 1] - 1;
    pair_entries.push_back(entry(SW_TUNE_PAIR, kEdges[k], hi, best_p, best_s, 0, c, best, model_ms));
  }
  tune_merge(pair_entries);
  found.insert(found.end(), pair_entries.begin(), pair_entries.end());

  // ---- mixed layouts for the whole per-pair set, against the tuned buckets
  if (used_buckets >= 2) {
    {
      // re-tuned below: earlier mixed entries must not steer the comparison
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune.erase(std::remove_if(g_tune.begin(), g_tune.end(), [&](const sw_tune_entry &o) {
                     return o.mixed && o.precision == pcode && o.alphabet_size == S.alpha;
                   }), g_tune.end());
    }
    std::vector<PlanItem> smp = strided_sample(per_pair, cap_cells);
    const int64_t c = cells_of(smp);
    int m_min = INT_MAX, m_max = 0;
    for (const auto &it : per_pair) { m_min = std::min(m_min, it.m); m_max = std::max(m_max, it.m); }
    ExecOptions tuned;
    tuned.force_kernel = 2;
    double tuned_ms;
    if ((rc = T.time(smp, tuned, tuned_ms))) return rc;
    double best = 1e300;
    int best_s = 0;
    for (int seg : pair_mixed_candidates(prec, S.alpha, smp.data(), smp.size(), 3)) {
      ExecOptions o = tuned;
      o.use_tuning = false;
      o.mixed_layout = 1;
      o.force_seglen = seg;
      double ms;
      if ((rc = T.time(smp, o, ms))) return rc;
      if (ms < best) { best = ms; best_s = seg; }
    }
    if (best_s && best < 0.97 * tuned_ms) {
      std::vector<sw_tune_entry> mx{entry(SW_TUNE_PAIR, m_min, m_max, 64, best_s, 1, c, best, tuned_ms)};
      tune_merge(mx);
      found.push_back(mx[0]);
    }
  }
  // ---- device-planned batches: every compiled shape that holds the query,
  // timed on the whole batch (the device planner reads it in place)
  {
    std::vector<sw_result> dres(np);
    auto dtime = [&](const ExecOptions &o, double &ms, bool &handled) -> int {
      ms = 1e300;
      handled = false;
      for (int rep = 0; rep < 2; ++rep) {
        sw_stats st;
        std::memset(&st, 0, sizeof(st));
        bool h = false;
        const int r = run_device_plan(b, S, o, 0, C, dres.data(), &st, now_ms(), h);
        if (r) return r;
        if (!h) return SW_OK;
        handled = true;
        ms = std::min(ms, st.kernel_ms);
      }
      return SW_OK;
    };
    ExecOptions fixed;
    fixed.use_tuning = false;
    double model_ms;
    bool handled;
    if ((rc = dtime(fixed, model_ms, handled))) return rc;
    const bool single = b->pair_query == nullptr || b->n_queries == 1;
    if (handled && single) {
      const int m = in.m_of_query[0];
      double best = 1e300;
      int best_seg = 0, best_lanes = 0, best_pair = 0, best_lrec = 0;
      if (prec == PREC_I16X2) {
        for (int s2 : {4, 8, 12, 16}) {
          int seg = 0;
          if (!rowpair_shape_forced(m, S.alpha, s2, seg)) continue;
          for (int lr : {1, 0}) {
            if (lr && !shared_rowpair_lds_records_fit(seg, S.alpha)) continue;
            ExecOptions o = fixed;
            o.lane_pairing = SW_PAIRING_ROWS;
            o.force_seglen = seg;
            o.lds_records = lr;
            double ms;
            bool h;
            if ((rc = dtime(o, ms, h))) return rc;
            if (h && ms < best) { best = ms; best_seg = seg; best_lanes = 16; best_pair = SW_PAIRING_ROWS; best_lrec = lr; }
          }
        }
      }
      for (int k = 0; k < kNumDirectShapes; ++k) {
        const DirectShape d = kDirectShapes[k];
        if (d.seg * d.lanes < m) continue;
        ExecOptions o = fixed;
        o.lane_pairing = SW_PAIRING_ALIGNMENTS;
        o.force_lanes = d.lanes;
        o.force_seglen = d.seg;
        double ms;
        bool h;
        if ((rc = dtime(o, ms, h))) return rc;
        if (h && ms < best) { best = ms; best_seg = d.seg; best_lanes = d.lanes; best_pair = SW_PAIRING_ALIGNMENTS; best_lrec = 0; }
      }
      if (best_seg) {
        sw_tune_entry e = entry(SW_TUNE_DEVICE_SHARED, m, m, best_lanes, best_seg, 0, cells, best,
                                model_ms);
        e.pairing = best_pair;
        e.lds_records = best_lrec;
        found.push_back(e);
      }
    } else if (handled) {
      int max_m = 0;
      for (const auto &it : all) max_m = std::max(max_m, it.m);
      double best = 1e300;
      int best_seg = 0, best_lanes = 0;
      for (int L : {8, 16}) {
        if (L == 8 && !(prec == PREC_I16X2 && S.fits_i8)) continue;
        const int *segs = L == 8 ? kPair8Segs : kPairSegs;
        const int nseg = L == 8 ? kNumPair8Segs : kNumPairSegs;
        for (int k = 0; k < nseg; ++k) {
          if (L * segs[k] < max_m) continue;
          ExecOptions o = fixed;
          o.force_lanes = L;
          o.force_seglen = segs[k];
          double ms;
          bool h;
          if ((rc = dtime(o, ms, h))) return rc;
          if (h && ms < best) { best = ms; best_seg = segs[k]; best_lanes = L; }
        }
      }
      if (best_seg)
        found.push_back(entry(SW_TUNE_DEVICE_PAIR, max_m, max_m, best_lanes, best_seg, 0, cells,
                              best, model_ms));
    }
  }
  tune_merge(found);
  for (int k = 0; k < cap && k < (int)found.size(); ++k) out[k] = found[k];
  if (n_out) *n_out = (int32_t)found.size();
  return SW_OK;
}

}  // extern "C"
