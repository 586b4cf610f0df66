// Host runtime of libswscan.so: argument checks, the work planner, device
// buffers and kernel launches behind the C ABI of include/sw.h.
//
// Readings of the paper that the runtime fixes (Algorithm 6 and the problem
// statement it solves):
//  * a gap of length L costs GapOpen + (L-1)*GapExtend; the method needs
//    GapExtend <= GapOpen, and min(GapExtend, GapOpen) gives identical scores,
//    so the kernels receive the clamped value;
//  * the profile is indexed [query residue][reference residue];
//  * the score is the running maximum of H + profile (taken before the E/F
//    maxima), reported with its lexicographically smallest (ref, query) cell.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <chrono>
#include <map>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <array>
#include <functional>
#include <mutex>
#include <thread>
#include <numeric>
#include <string>
#include <vector>

#include "sw.h"
#include "sw_internal.h"
#include "sw_runtime.h"

namespace swrt {

using namespace swk;

thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

#define HIPCHK(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                __LINE__);                                                       \
      return SW_EDEVICE;                                                         \
    }                                                                            \
  } while (0)

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ buffers

int DevBuf::ensure(size_t bytes) {
  if (bytes <= cap) return SW_OK;
  if (p) {
    if (retired) retired->push_back(p);
    else (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  size_t want = std::max<size_t>(bytes + bytes / 100 * (size_t)grow_pct, 4096);
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    set_error("hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    return SW_ENOMEM;
  }
  cap = want;
  return SW_OK;
}
void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

int HostBuf::ensure(size_t bytes) {
  if (bytes <= cap) return SW_OK;
  if (p) {
    if (retired) retired->push_back(p);
    else (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
  size_t want = std::max<size_t>(bytes + bytes / 100 * (size_t)grow_pct, 4096);
  hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    p = nullptr;
    set_error("hipHostMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    return SW_ENOMEM;
  }
  cap = want;
  return SW_OK;
}
void HostBuf::release() {
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
}

// ------------------------------------------------------------------ graph cache

hipGraphExec_t GraphCache::find(const std::vector<uint64_t> &sig) {
  for (auto &e : entries)
    if (e.sig == sig) { e.stamp = ++clock; return e.exec; }
  return nullptr;
}

void GraphCache::put(const std::vector<uint64_t> &sig, hipGraphExec_t exec) {
  if (entries.size() >= kMaxEntries) {
    auto old = std::min_element(entries.begin(), entries.end(),
                                [](const Entry &x, const Entry &y) { return x.stamp < y.stamp; });
    (void)hipGraphExecDestroy(old->exec);
    entries.erase(old);
  }
  entries.push_back(Entry{sig, exec, ++clock});
}

void GraphCache::clear() {
  for (auto &e : entries) (void)hipGraphExecDestroy(e.exec);
  entries.clear();
}

int Workspace::ensure_side_streams() {
  if (side_ready) return SW_OK;
  for (int k = 0; k < kSideStreams; ++k) {
    // default priority (no priority streams), non-blocking like the main one
    HIPCHK(hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&join[k], hipEventDisableTiming));
  }
  HIPCHK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  side_ready = true;
  return SW_OK;
}

// ------------------------------------------------------------------ device context

Context g_ctx;
std::mutex g_init_mu;

int Context::init(int dev) {
  if (inited) return SW_OK;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    set_error("no HIP device");
    return SW_EDEVICE;
  }
  if (dev < 0) HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipSetDevice(dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error("device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    return SW_EDEVICE;
  }
  device = dev;
  num_cus = prop.multiProcessorCount;
  HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventCreateWithFlags(&evx, hipEventDisableTiming));
  const int rc = noalloc_setup(dev);
  if (rc) return rc;
  inited = true;
  return SW_OK;
}

void Context::shutdown() {
  if (!inited) return;
  (void)hipSetDevice(device);
  (void)hipStreamSynchronize(stream);
  for (DevBuf *b : {&qres, &rres, &flag}) b->release();
  ws.release();
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  (void)hipEventDestroy(evx);
  (void)hipStreamDestroy(stream);
  inited = false;
}

int ensure_init(int dev) {
  std::lock_guard<std::mutex> g(g_init_mu);
  return g_ctx.init(dev);
}

// ------------------------------------------------------------------ scoring

int prepare_scoring(const sw_scoring *sc, Scoring &out) {
  if (!sc || !sc->matrix) { set_error("scoring or matrix is NULL"); return SW_EINVAL; }
  if (sc->alphabet_size < 1 || sc->alphabet_size > kMaxAlpha) {
    set_error("alphabet_size %d outside 1..%d", sc->alphabet_size, kMaxAlpha);
    return SW_EINVAL;
  }
  if (sc->gap_open < 0 || sc->gap_extend < 0) { set_error("negative gap penalty"); return SW_EINVAL; }
  out.alpha = sc->alphabet_size;
  out.M.assign(sc->matrix, sc->matrix + out.alpha * out.alpha);
  out.go = sc->gap_open;
  out.ge = std::min(sc->gap_extend, sc->gap_open);
  int mx = 0;
  bool fits16 = out.go <= 32767, fits8 = true;
  for (int v : out.M) {
    mx = std::max(mx, v);
    if (v < -32767 || v > 32767) fits16 = false;
    if (v < -128 || v > 127) fits8 = false;
  }
  out.max_s = mx;
  out.fits_i16 = fits16;
  out.fits_i8 = fits8;
  return SW_OK;
}

// ------------------------------------------------------------------ planner

void LengthIndex::reset(int max_m) {
  for (int m : ms)
    if (m < (int)dense.size()) dense[m] = 0;
  ms.clear();
  sparse.clear();
  const size_t want = (size_t)std::min(max_m, 1 << 20) + 1;
  if (dense.size() < want) dense.resize(want, 0);
}

int LengthIndex::slot(int m) {
  if (m < (int)dense.size()) {
    int &d = dense[m];
    if (!d) { ms.push_back(m); d = (int)ms.size(); }
    return d - 1;
  }
  auto f = sparse.find(m);
  if (f != sparse.end()) return f->second;
  ms.push_back(m);
  sparse.emplace(m, (int)ms.size() - 1);
  return (int)ms.size() - 1;
}

namespace {

constexpr int64_t kI32Limit = 2147483647ll;
// int32 shared-query launches run one chain per sub-group unless the options
// ask for two: two chains need twice the state registers (about 200 VGPRs at
// 16 rows per lane, two wavefronts per SIMD instead of four), and on the
// long-query workload they ran at 0.48 of the int32 VALU bound against 0.72
// for one chain -- the wavefronts in flight already provide the independent
// instruction streams the interleave would add.
constexpr bool kDualInt32Default = false;


// Approximate VALU instructions per column step of one wavefront.
double step_cost(Prec prec, int P, int seg) {
  const int lg = P == 16 ? 4 : (P == 32 ? 5 : 6);
  const double per_cell = prec == PREC_I16X2 ? 12.0 : 10.0;
  return seg * per_cell + 3.0 * lg + 14.0;
}

int layout_for(int P) { return P == 16 ? 0xF : (P == 32 ? 0x5 : 0x1); }

int round_up(int64_t x, int64_t k) { return (int)(((x + k - 1) / k) * k); }

// Indices of items ordered by reference length, longest first, ties in input
// order (a stable counting sort: the lengths of one batch span a small range).
void sort_by_n_desc(const PlanItem *items, size_t cnt, std::vector<int> &order,
                    std::vector<int> &count) {
  order.resize(cnt);
  if (cnt == 0) return;
  int lo = items[0].n, hi = items[0].n;
  for (size_t k = 0; k < cnt; ++k) { lo = std::min(lo, items[k].n); hi = std::max(hi, items[k].n); }
  const int64_t range = (int64_t)hi - lo + 1;
  if (range > 4 * (int64_t)cnt + 1024) {
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return items[a].n > items[b].n; });
    return;
  }
  count.assign(range + 1, 0);
  for (size_t k = 0; k < cnt; ++k) count[hi - items[k].n + 1]++;
  for (int64_t k = 0; k < range; ++k) count[k + 1] += count[k];
  for (size_t k = 0; k < cnt; ++k) order[count[hi - items[k].n]++] = (int)k;
}

struct LaunchDesc {
  bool shared;
  bool dual;         // shared, int32: two alignments per sub-group
  bool rp;           // per-pair: row pairs (pair_rowpair_kernel)
  int task_begin, task_end;
  int menu;          // shared
  int seg, pmax;     // per-pair
  int nchunks;       // shared: launches; per-pair: inside the kernel
  int query;         // shared
  int grid;
};

}  // namespace

// Builds tasks for one shared-query launch group.
// items: pairs of this query (n > 0, m > 0).  Pairs are ordered by reference
// length (longest first); each pair gets the narrowest lane mode whose task
// stays short next to the average load of a wavefront (long references get
// more lanes so they finish in time); consecutive pairs of one mode share a
// task.  Tasks are emitted longest-first (by estimated cost) across modes.
static void plan_shared(const PlanItem *items, size_t cnt, Prec prec, bool dual, int menu,
                        int num_waves, int force_lanes, HostScratch &hs, std::vector<Task> &tasks,
                        int mode_counts[3]) {
  // alignments per sub-group: two int16 halves, or two int32 chains (dual)
  const int halves = prec == PREC_I16X2 || dual ? 2 : 1;
  auto spw_of = [&](int P) { return halves * (kWave / P); };
  const SharedMenu mm = shared_menu(menu);
  const int segs[3] = {mm.seg16, mm.seg32, mm.seg64};
  const int Ps[3] = {16, 32, 64};
  std::vector<int> &order = hs.order;
  sort_by_n_desc(items, cnt, order, hs.count);
  int narrow = 0;
  for (int k = 0; k < 3; ++k)
    if (segs[k]) { narrow = k; break; }
  double total = 0;
  for (size_t k = 0; k < cnt; ++k) total += (double)items[k].n;
  total *= step_cost(prec, Ps[narrow], segs[narrow]) / spw_of(Ps[narrow]);
  const double per_wave = total / std::max(1, num_waves);
  // mode boundaries in the sorted order: [0, b2) mode 2, [b2, b1) mode 1, rest mode 0
  auto mode_of = [&](int n) {
    if (force_lanes) return force_lanes == 16 ? 0 : (force_lanes == 32 ? 1 : 2);
    int md = narrow;
    while (md < 2 && segs[md + 1] && (double)n * step_cost(prec, Ps[md], segs[md]) > 0.35 * per_wave)
      ++md;
    return md;
  };
  std::vector<int> begin(4, (int)order.size());
  {
    int pos = 0;
    for (int md = 2; md >= 0; --md) {
      begin[md] = pos;
      while (pos < (int)order.size() && mode_of(items[order[pos]].n) == md) ++pos;
    }
    begin[3] = pos;
  }
  std::vector<Task> bym[3];
  for (int md = 2; md >= 0; --md) {
    const int from = begin[md];
    const int to = (md == 0) ? begin[3] : begin[md - 1];
    if (to <= from) continue;
    const int spw = spw_of(Ps[md]);
    mode_counts[md] += to - from;
    bym[md].reserve((to - from + spw - 1) / spw);
    for (int a = from; a < to; a += spw) {
      Task t;
      t.layout = layout_for(Ps[md]);
      t.mode = md;
      t.nchunks = 1;
      t.bnd_off = -1;
      t.stream_off = 0;
      for (int s2 = 0; s2 < kSlots; ++s2) t.pair[s2] = -1;
      int maxn = 1;
      for (int q = 0; q < spw && a + q < to; ++q) {
        const PlanItem &it = items[order[a + q]];
        t.pair[2 * (q / halves) + q % halves] = it.pair;
        maxn = std::max(maxn, it.n);
      }
      t.ncols = round_up(maxn, kBlock);
      bym[md].push_back(t);
    }
  }
  // three lists, each longest-first: merge by estimated cost
  size_t ix[3] = {0, 0, 0};
  auto cost = [&](const Task &t) { return (double)t.ncols * step_cost(prec, Ps[t.mode], segs[t.mode]); };
  tasks.reserve(tasks.size() + bym[0].size() + bym[1].size() + bym[2].size());
  for (;;) {
    int pick = -1;
    double best = -1;
    for (int md = 0; md < 3; ++md)
      if (ix[md] < bym[md].size() && cost(bym[md][ix[md]]) > best) { best = cost(bym[md][ix[md]]); pick = md; }
    if (pick < 0) break;
    tasks.push_back(bym[pick][ix[pick]++]);
  }
}

// Smallest shared menu whose rows per chunk (64*seg64) cover m, or the largest.
static int pick_shared_menu(int m, int force_lanes, int force_seg) {
  const int n = shared_menu_count();
  if (force_seg) {
    for (int k = 0; k < n; ++k) {
      const SharedMenu mm = shared_menu(k);
      const int s = force_lanes == 16 ? mm.seg16 : (force_lanes == 32 ? mm.seg32 : mm.seg64);
      if (s == force_seg) return k;
    }
    return -1;
  }
  // the smallest menu covering m in one chunk that has the forced width, else
  // the largest one that has it (the query is then chunked)
  auto has = [&](const SharedMenu &mm) {
    return force_lanes == 16 ? mm.seg16 > 0 : (force_lanes == 32 ? mm.seg32 > 0 : mm.seg64 > 0);
  };
  int last = -1;
  for (int k = 0; k < n; ++k) {
    const SharedMenu mm = shared_menu(k);
    if (!has(mm)) continue;
    last = k;
    if (64 * mm.seg64 >= m) return k;
  }
  return last;
}


// ------------------------------------------------------------------ per-pair planning

namespace {

struct PairShape {
  int P, seg, nchunks;
  bool rp = false;   // row pairs: one alignment per 16-lane sub-group, 32*seg rows per chunk
};

constexpr int kPairSegs[] = {4, 6, 8, 10, 12, 16};
constexpr size_t kPairLdsBudget = 20 * 1024;   // LDS per wavefront (keeps >= 6 waves per CU)

// LDS bytes of one per-pair wavefront region.
size_t pair_region(Prec prec, int seg, int alpha) {
  return pair_lds_bytes(prec, seg, alpha) - matrix_lds_bytes(alpha);
}

bool pair_seg_allowed(Prec prec, int seg, int alpha, const ExecOptions &opt) {
  if (opt.force_seglen) return seg == opt.force_seglen;
  return seg == 4 || pair_region(prec, seg, alpha) <= kPairLdsBudget;
}

// Modelled VALU cost per reference column of one alignment on P lanes of a
// wavefront whose widest sub-group has pmax lanes (the scan depth).
double pair_cost(Prec prec, int P, int pmax, int seg, int nch) {
  return nch * step_cost(prec, pmax, seg) * P / (64.0 * (prec == PREC_I16X2 ? 2 : 1));
}

// Row pairs: VALU instructions of one wavefront's column step (the recurrence
// and the pair-score table address per row pair, 1 + log2(P) scan steps, two
// virtual-lane moves, records; chunk carries), and per alignment (64/P per
// wavefront).
const int kRpSegs[] = {4, 8, 12, 16};
double rp_step_cost(int P, int seg, int nch) {
  const int lg = P == 16 ? 4 : (P == 32 ? 5 : 6);
  return seg * 13.0 + 3.0 * (lg + 1) + 18.0 + (P > 16 ? 2.0 : 0.0) + (nch > 1 ? 8.0 : 0.0);
}
double rp_cost(int P, int seg, int nch) { return nch * rp_step_cost(P, seg, nch) * P / 64.0; }

// Which lane pairings the options and the batch allow for per-pair launches.
bool rp_allowed(Prec prec, int alpha, const ExecOptions &opt) {
  if (prec != PREC_I16X2 || opt.lane_pairing == SW_PAIRING_ALIGNMENTS) return false;
  if (!pair_rowpair_has(4, alpha)) return false;
  if (opt.lane_pairing == SW_PAIRING_ROWS) return true;
  return !opt.force_lanes && !opt.force_seglen;   // forced shapes keep alignment pairs
}
// Row pairs only: when asked for, or (planner's choice) when the alphabet is
// so large that per-pair profiles would hold just 4 rows per lane: there the
// alignment-pair kernel runs short lanes over many query chunks, and measured
// 1.7x slower on uniform 400 x 400 protein pairs and 1.4x on the serving mix.
bool rows_only(Prec prec, int alpha, const ExecOptions &opt) {
  if (opt.lane_pairing == SW_PAIRING_ROWS) return true;
  if (opt.mixed_layout == 1) return false;   // mixed widths are an alignment-pair layout
  ExecOptions none;
  return rp_allowed(prec, alpha, opt) && !pair_seg_allowed(prec, 6, alpha, none);
}
bool rp_seg_allowed(int seg, int alpha, const ExecOptions &opt) {
  return pair_rowpair_has(seg, alpha) && (!opt.force_seglen || seg == opt.force_seglen);
}

// Modelled cost per reference column of one alignment, and the length of one
// wavefront's chain of column steps per reference column, for a shape.
double shape_cost(Prec prec, const PairShape &ps, int) {
  return ps.rp ? rp_cost(ps.P, ps.seg, ps.nchunks) : pair_cost(prec, ps.P, ps.P, ps.seg, ps.nchunks);
}
double shape_chain(Prec prec, const PairShape &ps) {
  return ps.nchunks * (ps.rp ? rp_step_cost(ps.P, ps.seg, ps.nchunks) : step_cost(prec, ps.P, ps.seg));
}

// Every per-pair shape the options allow for a query of m rows.
template <class F>
void for_each_pair_shape(Prec prec, int m, int alpha, const ExecOptions &opt, F &&f) {
  if (!rows_only(prec, alpha, opt)) {
    for (int P : {16, 32, 64}) {
      if (opt.force_lanes && P != opt.force_lanes) continue;
      for (int seg : kPairSegs) {
        if (!pair_seg_allowed(prec, seg, alpha, opt)) continue;
        f(PairShape{P, seg, (m + P * seg - 1) / (P * seg)});
      }
    }
  }
  if (rp_allowed(prec, alpha, opt)) {
    // unforced: a short menu (16 lanes at 8 or 16 rows, 64 lanes at 16 rows),
    // so that a batch of mixed lengths needs few launches
    const bool forced = opt.force_lanes || opt.force_seglen;
    for (int P : {16, 32, 64}) {
      if (opt.force_lanes && P != opt.force_lanes) continue;
      if (!forced && P == 32) continue;
      for (int seg : kRpSegs) {
        if (!forced && (P == 16 ? (seg != 8 && seg != 16) : seg != 16)) continue;
        if (rp_seg_allowed(seg, alpha, opt))
          f(PairShape{P, seg, (m + 2 * P * seg - 1) / (2 * P * seg), true});
      }
    }
  }
}

// One width per launch: the (lanes, rows per lane) of least modelled cost,
// over alignment pairs and row pairs as the options allow.
PairShape choose_pair_shape(Prec prec, int m, int alpha, const ExecOptions &opt) {
  PairShape best{64, 4, 1 << 30};
  double best_cost = 1e300;
  for_each_pair_shape(prec, m, alpha, opt, [&](const PairShape &ps) {
    const double cost = shape_cost(prec, ps, alpha);
    if (cost < best_cost - 1e-9) { best_cost = cost; best = ps; }
  });
  return best;
}

// Mixed layouts: the narrowest sub-group that holds m rows at `seg` rows per
// lane, else 64 lanes over several query chunks.
PairShape mixed_shape(int m, int seg) {
  for (int P : {16, 32, 64})
    if (P * seg >= m) return PairShape{P, seg, 1};
  return PairShape{64, seg, (m + 64 * seg - 1) / (64 * seg)};
}

}  // namespace

std::vector<std::pair<int, int>> pair_candidates(Prec prec, int alpha, const PlanItem *items,
                                                 size_t cnt, int max_cands) {
  ExecOptions none;
  std::vector<std::pair<double, std::pair<int, int>>> c;
  for (int P : {16, 32, 64})
    for (int seg : kPairSegs) {
      if (!pair_seg_allowed(prec, seg, alpha, none)) continue;
      double cost = 0;
      for (size_t k = 0; k < cnt; ++k) {
        const int nch = (items[k].m + P * seg - 1) / (P * seg);
        cost += (double)items[k].n * pair_cost(prec, P, P, seg, nch);
      }
      c.push_back({cost, {P, seg}});
    }
  std::stable_sort(c.begin(), c.end(),
                   [](const auto &x, const auto &y) { return x.first < y.first; });
  std::vector<std::pair<int, int>> r;
  for (size_t k = 0; k < c.size() && (int)k < max_cands; ++k) r.push_back(c[k].second);
  return r;
}

std::vector<int> pair_mixed_candidates(Prec prec, int alpha, const PlanItem *items, size_t cnt,
                                       int max_cands) {
  ExecOptions none;
  std::vector<std::pair<double, int>> c;
  for (int seg : kPairSegs) {
    if (!pair_seg_allowed(prec, seg, alpha, none)) continue;
    int pm = 16;
    for (size_t k = 0; k < cnt; ++k) {
      const PairShape ps = mixed_shape(items[k].m, seg);
      if (ps.nchunks == 1) pm = std::max(pm, ps.P);
    }
    double cost = 0;
    for (size_t k = 0; k < cnt; ++k) {
      const PairShape ps = mixed_shape(items[k].m, seg);
      cost += (double)items[k].n * pair_cost(prec, ps.P, ps.nchunks == 1 ? pm : 64, seg, ps.nchunks);
    }
    c.push_back({cost, seg});
  }
  std::stable_sort(c.begin(), c.end(),
                   [](const auto &x, const auto &y) { return x.first < y.first; });
  std::vector<int> r;
  for (size_t k = 0; k < c.size() && (int)k < max_cands; ++k) r.push_back(c[k].second);
  return r;
}

// Sub-group widths (in lanes) of a wavefront layout; returns their number.
int layout_groups(int layout, int widths[4]) {
  int n = 0;
  for (int r = 0; r < 4; ++r) {
    if (!((layout >> r) & 1)) continue;
    int e = r + 1;
    while (e < 4 && !((layout >> e) & 1)) ++e;
    widths[n++] = 16 * (e - r);
  }
  return n;
}

// Layouts the kernels support: bit 0 set, 32-lane groups start at row 0 or 2,
// no 48-lane groups, no group wider than pmax.
bool layout_valid(int layout, int pmax) {
  if (layout < 1 || layout > 15 || !(layout & 1)) return false;
  int w[4];
  const int n = layout_groups(layout, w);
  int row = 0;
  for (int g = 0; g < n; ++g) {
    if (w[g] == 48 || w[g] > pmax) return false;
    if (w[g] == 32 && (row & 1)) return false;
    row += w[g] / 16;
  }
  return true;
}

int host_threads() {
  static const int n = std::max(1, std::min(8, (int)std::thread::hardware_concurrency()));
  return n;
}

void parallel_ranges(size_t n, int T, const std::function<void(int, size_t, size_t)> &fn) {
  T = (int)std::max<size_t>(1, std::min<size_t>((size_t)T, n));
  if (T <= 1) { fn(0, 0, n); return; }
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (int t = 1; t < T; ++t) th.emplace_back(fn, t, n * t / T, n * (t + 1) / T);
  fn(0, 0, n / T);
  for (auto &x : th) x.join();
}

namespace {

// Packs sorted pair records into wavefront tasks (appended to `out`).
// A pair takes the next free rows of the open task (32-lane groups start at
// lane 0 or 32); in int16x2 mode the high half of a sub-group takes the next
// pair of the same width if its reference fits the task's columns.
void pack_pairs(const PackRec *rec, int count, int pmax, int halves, std::vector<Task> &out,
                int lanes_used[3]) {
  int ti = -1, rows = 4, nsg = 0, maxn = 1;
  int half_task[3] = {-1, -1, -1}, half_slot[3] = {0, 0, 0};
  auto close = [&]() {
    if (ti < 0) return;
    Task &t = out[ti];
    for (int r = rows; r < 4;) {   // unused rows: empty sub-groups
      t.layout |= 1 << r;
      r += ((r & 1) == 0 && pmax >= 32) ? 2 : 1;
    }
    t.ncols = round_up(maxn, kBlock);
    ti = -1;
  };
  for (int x = 0; x < count; ++x) {
    const PackRec &it = rec[x];
    const int P = it.P;
    const int pc = P == 16 ? 0 : (P == 32 ? 1 : 2);
    lanes_used[pc]++;
    if (halves == 2 && half_task[pc] >= 0) {
      // the second half of a sub-group opened by an earlier pair of this
      // width (as many or more chunks), if its columns cover this reference
      Task &h = out[half_task[pc]];
      if (half_task[pc] == ti || it.n <= h.ncols) {
        h.pair[half_slot[pc]] = it.pair;
        if (half_task[pc] == ti) maxn = std::max(maxn, it.n);
        half_task[pc] = -1;
        continue;
      }
      half_task[pc] = -1;
    }
    int pos = P == 16 ? rows : (P == 32 ? (rows + 1) & ~1 : (rows == 0 ? 0 : 4));
    if (ti < 0 || pos + P / 16 > 4) {
      close();
      Task t;
      std::memset(&t, 0, sizeof(t));
      t.nchunks = it.nch;   // the most of any pair it will hold (sorted)
      t.bnd_off = -1;
      for (int s2 = 0; s2 < kSlots; ++s2) t.pair[s2] = -1;
      out.push_back(t);
      ti = (int)out.size() - 1;
      rows = 0;
      nsg = 0;
      maxn = 1;
      pos = 0;
    }
    Task &t = out[ti];
    for (int r = rows; r < pos; ++r) { t.layout |= 1 << r; ++nsg; }   // skipped row
    t.layout |= 1 << pos;
    t.pair[2 * nsg] = it.pair;
    if (halves == 2) { half_task[pc] = ti; half_slot[pc] = 2 * nsg + 1; }
    ++nsg;
    rows = pos + P / 16;
    maxn = std::max(maxn, it.n);
  }
  close();
}

// Per-pair launches.  Every pair gets a shape (lanes P, rows per lane, query
// chunks); pairs of one launch share rows per lane and chunk count.  With
// mixed layouts one launch also mixes 16-, 32- and 64-lane sub-groups inside
// a wavefront (its kernel is compiled for the widest).  Inside a launch the
// pairs are taken longest reference first; in int16x2 mode the two halves of a
// sub-group hold consecutive pairs of the same width.
int plan_pairs(const PlanItem *items, size_t cnt, Prec prec, int alpha, const ExecOptions &opt,
               int num_cus, HostScratch &hs, std::vector<Task> &tasks,
               std::vector<LaunchDesc> &launches, int64_t &bnd_elems, ExecStats &stats) {
  if (cnt == 0) return SW_OK;
  if (opt.lane_pairing == SW_PAIRING_ROWS &&
      (!rp_allowed(prec, alpha, opt) ||
       (opt.force_seglen && !rp_seg_allowed(opt.force_seglen, alpha, opt)))) {
    set_error("row pairs need int16 lanes, an alphabet of at most 24 letters and 4, 8, 12 "
              "or 16 rows per lane");
    return SW_EINVAL;
  }
  if (opt.force_seglen &&
      std::find(std::begin(kPairSegs), std::end(kPairSegs), opt.force_seglen) == std::end(kPairSegs)) {
    set_error("no compiled per-pair kernel with %d rows per lane", opt.force_seglen);
    return SW_EINVAL;
  }
  if (opt.lane_pairing == SW_PAIRING_ROWS && opt.mixed_layout == 1) {
    set_error("mixed layouts hold alignment pairs, not row pairs");
    return SW_EINVAL;
  }
  // mixed_layout: 0 = planner's choice, 1 = mixed, 2 = one width per launch
  bool mixed = opt.mixed_layout == 1 && !opt.force_lanes;
  int mixed_seg = opt.force_seglen;
  // ---- distinct query lengths
  int max_m = 0, min_m = INT_MAX;
  for (size_t k = 0; k < cnt; ++k) { max_m = std::max(max_m, items[k].m); min_m = std::min(min_m, items[k].m); }
  const bool tunable = opt.use_tuning && !opt.force_lanes && !opt.force_seglen && opt.mixed_layout != 1;
  sw_tune_entry te;
  if (tunable && opt.mixed_layout == 0 && !rows_only(prec, alpha, opt) &&
      tune_mixed(prec, alpha, min_m, max_m, te)) {
    mixed = true;
    mixed_seg = te.seglen;
  }
  LengthIndex &li = hs.lengths;
  li.reset(max_m);
  hs.slot.resize(cnt);
  hs.nsum.clear();
  hs.nmax.clear();
  for (size_t k = 0; k < cnt; ++k) {
    const int s = li.slot(items[k].m);
    if (s >= (int)hs.nsum.size()) { hs.nsum.resize(s + 1, 0.0); hs.nmax.resize(s + 1, 0); }
    hs.nsum[s] += items[k].n;
    hs.nmax[s] = std::max(hs.nmax[s], items[k].n);
    hs.slot[k] = s;
  }
  const int nd = (int)li.ms.size();
  std::vector<PairShape> shape(nd);
  std::vector<char> own(nd, 0);   // mixed batch: a class in a launch of its own shape
  int pmax_mixed = 16;
  double nonmixed_total = 0;
  double bound = 1e300;   // the batch's modelled time on a full GPU (set below)
  if (!mixed) {
    // Least modelled work per pair, unless that leaves one wavefront with a
    // chain of column steps longer than the whole batch needs on a full GPU
    // (small batches of long queries): then the cheapest shape whose chain
    // fits that bound (more lanes, fewer query chunks).
    const double slots = (double)num_cus * 4;   // one full-rate wavefront per SIMD
    double total = 0, lmin = 0;
    for (int s = 0; s < nd; ++s) {
      shape[s] = choose_pair_shape(prec, li.ms[s], alpha, opt);
      total += hs.nsum[s] * shape_cost(prec, shape[s], alpha);
      double best_lat = 1e300;
      for_each_pair_shape(prec, li.ms[s], alpha, opt, [&](const PairShape &ps) {
        best_lat = std::min(best_lat, (double)hs.nmax[s] * shape_chain(prec, ps));
      });
      lmin = std::max(lmin, best_lat);
    }
    bound = std::max(total / slots, lmin);
    nonmixed_total = total;
    for (int s = 0; s < nd; ++s) {
      const int m = li.ms[s];
      if (tunable && !rows_only(prec, alpha, opt) && tune_lookup(SW_TUNE_PAIR, prec, alpha, m, te)) {
        // the tuned alignment-pair shape, unless row pairs model far less work
        const PairShape tuned{te.lanes, te.seglen, (m + te.lanes * te.seglen - 1) / (te.lanes * te.seglen)};
        if (!(shape[s].rp && shape_cost(prec, shape[s], alpha) < 0.7 * shape_cost(prec, tuned, alpha)) &&
            (double)hs.nmax[s] * shape_chain(prec, tuned) <= bound) {
          shape[s] = tuned;
          continue;
        }
      }
      if ((double)hs.nmax[s] * shape_chain(prec, shape[s]) <= bound) continue;
      double best = 1e300;
      for_each_pair_shape(prec, m, alpha, opt, [&](const PairShape &ps) {
        if ((double)hs.nmax[s] * shape_chain(prec, ps) > bound) return;
        const double c = shape_cost(prec, ps, alpha);
        if (c < best - 1e-9) { best = c; shape[s] = ps; }
      });
    }
  }
  // Planner's choice: mixed layouts (one launch for every width, fewer launch
  // tails) unless they model over 15% more work than one width per launch.
  const bool ap = !rows_only(prec, alpha, opt);
  bool try_mixed = mixed && ap;
  if (!mixed && opt.mixed_layout == 0 && !opt.force_lanes && !opt.force_seglen && nd > 0 && ap) {
    bool tuned_any = false;
    for (int s = 0; s < nd && tunable; ++s) tuned_any |= tune_lookup(SW_TUNE_PAIR, prec, alpha, li.ms[s], te);
    try_mixed = !tuned_any;
  }
  if (try_mixed) {
    // one rows-per-lane for the whole batch: the tuned or forced one, else the
    // least modelled total cost
    int best_seg = -1;
    double best = 1e300;
    for (int seg : kPairSegs) {
      if (mixed_seg ? seg != mixed_seg : !pair_seg_allowed(prec, seg, alpha, opt)) continue;
      int pm = 16;
      for (int s = 0; s < nd; ++s) {
        const PairShape ps = mixed_shape(li.ms[s], seg);
        if (ps.nchunks == 1) pm = std::max(pm, ps.P);
      }
      double c = 0;
      for (int s = 0; s < nd; ++s) {
        const PairShape ps = mixed_shape(li.ms[s], seg);
        c += hs.nsum[s] * pair_cost(prec, ps.P, ps.nchunks == 1 ? pm : 64, seg, ps.nchunks);
      }
      if (c < best - 1e-9) { best = c; best_seg = seg; pmax_mixed = pm; }
    }
    if (mixed || best <= 1.15 * nonmixed_total) {
      const bool chosen = !mixed;   // the planner's choice, not forced or tuned
      mixed = true;
      for (int s = 0; s < nd; ++s) shape[s] = mixed_shape(li.ms[s], best_seg);
      // ... keeping the latency bound: a length class whose chain of column
      // steps would outlast the whole batch gets its own launch in the
      // cheapest shape that fits (long queries in a small batch: row pairs
      // halve the chain)
      for (int s = 0; s < nd && chosen; ++s) {
        if ((double)hs.nmax[s] * shape_chain(prec, shape[s]) <= 1.05 * bound) continue;
        double bc = 1e300;
        for_each_pair_shape(prec, li.ms[s], alpha, opt, [&](const PairShape &ps) {
          if ((double)hs.nmax[s] * shape_chain(prec, ps) > bound) return;
          const double c = shape_cost(prec, ps, alpha);
          if (c < bc - 1e-9) { bc = c; shape[s] = ps; own[s] = 1; }
        });
      }
    }
  }
  // ---- launch classes (rows per lane, widest sub-group, chunked or not); a
  // chunked launch holds tasks of any chunk count
  struct Cls { int seg, pmax; bool chunked, rp; };
  std::vector<Cls> cls;
  std::vector<int> cls_of(nd);
  int max_nch = 1;
  for (int s = 0; s < nd; ++s) {
    const PairShape &ps = shape[s];
    // mixed alignment-pair launches share one widest width; a latency-bound
    // class of a mixed batch keeps its own shape and launch
    const int pmax = (mixed && ps.nchunks == 1 && !own[s]) ? pmax_mixed : ps.P;
    const bool chunked = ps.nchunks > 1;
    max_nch = std::max(max_nch, ps.nchunks);
    int c = 0;
    while (c < (int)cls.size() && !(cls[c].seg == ps.seg && cls[c].pmax == pmax &&
                                     cls[c].chunked == chunked && cls[c].rp == ps.rp))
      ++c;
    if (c == (int)cls.size()) {
      if (ps.rp) {
        if (!pair_rowpair_has(ps.seg, alpha)) {
          set_error("no compiled row-pair kernel for %d rows per lane", ps.seg);
          return SW_EINVAL;
        }
        cls.push_back(Cls{ps.seg, ps.P, chunked, true});
        cls_of[s] = c;
        continue;
      }
      if (!pair_kernel_has(prec, ps.seg, pmax)) {
        set_error("no compiled per-pair kernel for %d rows per lane, %d lanes", ps.seg, pmax);
        return SW_EINVAL;
      }
      cls.push_back(Cls{ps.seg, pmax, chunked, false});
    }
    cls_of[s] = c;
  }
  // ---- order: by class, then query chunks and reference length (most work
  // first), stable; one counting sort into compact records so that packing
  // reads sequentially (per-thread histograms for large batches)
  const int ncls = (int)cls.size();
  int nlo = items[0].n, nhi = items[0].n;
  for (size_t k = 0; k < cnt; ++k) { nlo = std::min(nlo, items[k].n); nhi = std::max(nhi, items[k].n); }
  const int64_t range = (int64_t)nhi - nlo + 1;
  const int64_t keys = (int64_t)ncls * max_nch * range;
  std::vector<PackRec> &rec = hs.packed;
  rec.resize(cnt);
  hs.bounds.assign(ncls + 1, 0);
  auto key_of = [&](size_t k) {
    const int s = hs.slot[k];
    return ((cls_of[s] * max_nch) + (max_nch - shape[s].nchunks)) * (int)range + (nhi - items[k].n);
  };
  if (keys <= 65536 && cnt >= 50000) {
    const int T = host_threads();
    std::vector<std::vector<int>> h(T, std::vector<int>((size_t)keys, 0));
    hs.order.resize(cnt);
    parallel_ranges(cnt, T, [&](int t, size_t lo, size_t hi) {
      int *ht = h[t].data();
      for (size_t k = lo; k < hi; ++k) {
        const int key = key_of(k);
        hs.order[k] = key;
        ht[key]++;
      }
    });
    int run = 0;
    for (int64_t key = 0; key < keys; ++key) {
      if (key % (max_nch * range) == 0) hs.bounds[key / (max_nch * range)] = run;
      for (int t = 0; t < T; ++t) { const int c = h[t][key]; h[t][key] = run; run += c; }
    }
    hs.bounds[ncls] = run;
    parallel_ranges(cnt, T, [&](int t, size_t lo, size_t hi) {
      int *ht = h[t].data();
      for (size_t k = lo; k < hi; ++k) {
        const int s = hs.slot[k];
        rec[ht[hs.order[k]]++] = PackRec{items[k].pair, items[k].n, shape[s].P, shape[s].nchunks};
      }
    });
  } else if (keys <= 4 * (int64_t)cnt + 4096) {
    hs.count.assign((size_t)keys + 1, 0);
    hs.order.resize(cnt);   // sort key of each item
    for (size_t k = 0; k < cnt; ++k) {
      const int key = key_of(k);
      hs.order[k] = key;
      hs.count[key + 1]++;
    }
    for (size_t q = 0; q + 1 < hs.count.size(); ++q) hs.count[q + 1] += hs.count[q];
    for (int c = 0; c <= ncls; ++c) hs.bounds[c] = hs.count[(size_t)c * max_nch * range];
    for (size_t k = 0; k < cnt; ++k) {
      const int s = hs.slot[k];
      rec[hs.count[hs.order[k]]++] = PackRec{items[k].pair, items[k].n, shape[s].P, shape[s].nchunks};
    }
  } else {
    hs.order.resize(cnt);
    std::iota(hs.order.begin(), hs.order.end(), 0);
    std::stable_sort(hs.order.begin(), hs.order.end(), [&](int x, int y) {
      const int sx = hs.slot[x], sy = hs.slot[y];
      if (cls_of[sx] != cls_of[sy]) return cls_of[sx] < cls_of[sy];
      if (shape[sx].nchunks != shape[sy].nchunks) return shape[sx].nchunks > shape[sy].nchunks;
      return items[x].n > items[y].n;
    });
    for (size_t x = 0; x < cnt; ++x) {
      const int k = hs.order[x];
      const int s = hs.slot[k];
      rec[x] = PackRec{items[k].pair, items[k].n, shape[s].P, shape[s].nchunks};
      hs.bounds[cls_of[s] + 1]++;
    }
    for (int c = 0; c < ncls; ++c) hs.bounds[c + 1] += hs.bounds[c];
  }
  const int halves_all = prec == PREC_I16X2 ? 2 : 1;
  for (int c = 0; c < ncls; ++c) {
    const int a = hs.bounds[c], b = hs.bounds[c + 1];
    if (a == b) continue;
    const Cls K = cls[c];
    LaunchDesc L{};
    L.shared = false;
    L.seg = K.seg;
    L.pmax = K.pmax;
    L.rp = K.rp;
    L.nchunks = K.chunked ? 2 : 1;   // > 1: the chunked kernel (per-task counts)
    L.task_begin = (int)tasks.size();
    // row pairs: one alignment per sub-group (the even slots)
    const int halves = K.rp ? 1 : halves_all;
    if (b - a >= 50000) {
      // large classes: contiguous sub-ranges packed on several threads, then
      // concatenated in order (each sub-range may end in one partial task)
      const int T = host_threads();
      std::vector<std::vector<Task>> part(T);
      std::vector<std::array<int, 3>> lu(T, std::array<int, 3>{0, 0, 0});
      parallel_ranges((size_t)(b - a), T, [&](int t, size_t lo, size_t hi) {
        pack_pairs(rec.data() + a + lo, (int)(hi - lo), K.pmax, halves, part[t], lu[t].data());
      });
      for (int t = 0; t < T; ++t) {
        tasks.insert(tasks.end(), part[t].begin(), part[t].end());
        for (int q = 0; q < 3; ++q) stats.lanes_used[q] += lu[t][q];
      }
    } else {
      pack_pairs(rec.data() + a, b - a, K.pmax, halves, tasks, stats.lanes_used);
    }
    L.task_end = (int)tasks.size();
    if (K.rp) stats.row_pairs += b - a;
    for (int t = L.task_begin; t < L.task_end; ++t) {
      Task &tk = tasks[t];
      if (K.chunked) { tk.bnd_off = bnd_elems; bnd_elems += 8ll * tk.ncols; }
      int w[4];
      const int ng = layout_groups(tk.layout, w);
      for (int g = 0; g < ng; ++g)
        for (int h = 0; h < halves; ++h)
          if (tk.pair[2 * g + h] >= 0)
            stats.padded_cells += (int64_t)tk.ncols * w[g] * K.seg * tk.nchunks * (K.rp ? 2 : 1);
    }
    stats.seglen_max = std::max(stats.seglen_max, K.seg);
    L.grid = std::max(1, std::min(L.task_end - L.task_begin, num_cus * 16));
    launches.push_back(L);
  }
  return SW_OK;
}

}  // namespace

// ------------------------------------------------------------------ executor

int execute(const ExecInput &in, const Scoring &sc, Prec prec, const ExecOptions &opt,
            Workspace &ws, int n_results, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
            int num_cus, ExecStats &stats, bool reset_results) {
  const double t_plan0 = now_ms();
  HostScratch &hs = ws.host;
  std::vector<Task> &tasks = hs.tasks;
  tasks.clear();
  std::vector<LaunchDesc> launches;
  const bool lazy = opt.algorithm == SW_ALG_LAZYF;
  // ---- split: a query with many pairs runs in the shared-query kernel
  hs.qcount.assign(in.n_queries, 0);
  for (const auto &it : in.items) hs.qcount[it.query]++;
  auto wants_shared = [&](int q) {
    return lazy || opt.force_kernel == 1 || (opt.force_kernel == 0 && hs.qcount[q] >= 32);
  };
  size_t n_shared = 0;
  for (const auto &it : in.items) n_shared += wants_shared(it.query);
  const PlanItem *pp_items = nullptr;   // per-pair items
  size_t pp_cnt = 0;
  const PlanItem *sh_items = nullptr;   // shared items, grouped by query
  hs.qstart.clear();
  int only_query = -1;                  // every item is shared and uses one query
  if (n_shared == 0) {
    pp_items = in.items.data();
    pp_cnt = in.items.size();
  } else if (n_shared == in.items.size() && hs.qcount[in.items[0].query] == (int)in.items.size()) {
    only_query = in.items[0].query;
    sh_items = in.items.data();
  } else {
    hs.per_pair.clear();
    hs.shared_items.resize(n_shared);
    hs.qstart.assign(in.n_queries + 1, 0);
    for (const auto &it : in.items)
      if (wants_shared(it.query)) hs.qstart[it.query + 1]++;
    for (int q = 0; q < in.n_queries; ++q) hs.qstart[q + 1] += hs.qstart[q];
    std::vector<int> pos(hs.qstart.begin(), hs.qstart.end() - 1);
    for (const auto &it : in.items) {
      if (wants_shared(it.query)) hs.shared_items[pos[it.query]++] = it;
      else hs.per_pair.push_back(it);
    }
    sh_items = hs.shared_items.data();
    pp_items = hs.per_pair.data();
    pp_cnt = hs.per_pair.size();
  }
  const int waves_total = num_cus * 16;
  int64_t bnd_elems = 0;
  // ---- shared-query launches
  for (int q = 0; sh_items && q < in.n_queries; ++q) {
    const PlanItem *group;
    size_t gcnt;
    if (only_query >= 0) {
      if (q != only_query) continue;
      group = sh_items;
      gcnt = in.items.size();
    } else {
      if (hs.qstart[q + 1] == hs.qstart[q]) continue;
      group = sh_items + hs.qstart[q];
      gcnt = hs.qstart[q + 1] - hs.qstart[q];
    }
    const int m = in.m_of_query[q];
    int fl = opt.force_lanes, fseg = opt.force_seglen;
    sw_tune_entry te;
    if (opt.use_tuning && !lazy && !fl && !fseg && tune_lookup(SW_TUNE_SHARED, prec, sc.alpha, m, te)) {
      fl = te.lanes;
      fseg = te.seglen;
    }
    const int menu = pick_shared_menu(m, fl ? fl : 64, fseg);
    if (menu < 0) { set_error("no compiled shared kernel with %d rows per lane", opt.force_seglen); return SW_EINVAL; }
    const SharedMenu mm = shared_menu(menu);
    if (fl == 16 && !mm.seg16) { set_error("menu has no 16-lane mode"); return SW_EINVAL; }
    const int rows = 64 * mm.seg64;
    const int nch = (m + rows - 1) / rows;
    LaunchDesc L{};
    L.shared = true;
    // int32 scan launches: two chains per sub-group where the options ask
    // for them (SW_CHAINS_TWO) or leave the choice (the default below)
    L.dual = prec == PREC_I32 && !lazy &&
             (opt.int32_chains == SW_CHAINS_TWO ||
              (opt.int32_chains == SW_CHAINS_AUTO && kDualInt32Default));
    L.menu = menu;
    L.nchunks = nch;
    L.query = q;
    L.task_begin = (int)tasks.size();
    int mc[3] = {0, 0, 0};
    plan_shared(group, gcnt, prec, L.dual, menu, waves_total, fl, hs, tasks, mc);
    L.task_end = (int)tasks.size();
    for (int k = 0; k < 3; ++k) stats.lanes_used[k] += mc[k];
    const int segs[3] = {mm.seg16, mm.seg32, mm.seg64};
    for (int t = L.task_begin; t < L.task_end; ++t) {
      tasks[t].nchunks = nch;
      if (nch > 1) { tasks[t].bnd_off = bnd_elems; bnd_elems += (L.dual ? 16ll : 8ll) * tasks[t].ncols; }
      stats.seglen_max = std::max(stats.seglen_max, segs[tasks[t].mode]);
      const int P = 16 << tasks[t].mode;
      int used = 0;
      for (int s = 0; s < kSlots; ++s) used += tasks[t].pair[s] >= 0;
      stats.padded_cells += (int64_t)used * tasks[t].ncols * P * segs[tasks[t].mode] * nch;
    }
    const int ntask = L.task_end - L.task_begin;
    L.grid = std::max(1, std::min((ntask + kWavesPerGroup - 1) / kWavesPerGroup, num_cus * 2));
    launches.push_back(L);
  }
  // ---- per-pair launches
  int rc = plan_pairs(pp_items, pp_cnt, prec, sc.alpha, opt, num_cus, hs, tasks, launches,
                      bnd_elems, stats);
  if (rc) return rc;
  if (tasks.empty()) return SW_OK;

  // ---- device buffers
  const double t_launch0 = now_ms();
  stats.plan_ms += t_launch0 - t_plan0;
  int64_t stream_bytes = 0;
  for (auto &t : tasks) { t.stream_off = stream_bytes; stream_bytes += (int64_t)t.ncols / kBlock * kStreamBlockBytes; }
  stream_bytes += 4 * kStreamBlockBytes;
  // Every access a kernel makes is derived from these fields: refuse to
  // launch anything the kernels' bounds assumptions do not cover.  (PairInfo
  // index == result index for every path of this library.)
  const int n_pairs_total = in.d_pairs ? in.n_pairs : (int)in.pairs.size();
  std::vector<int> &nlen = hs.nlen;
  std::vector<int> &mlen = hs.mlen;
  nlen.assign(std::max(n_pairs_total, 0), -1);
  mlen.assign(std::max(n_pairs_total, 0), 0);
  for (const auto &it : in.items)
    if (it.pair >= 0 && it.pair < n_pairs_total) { nlen[it.pair] = it.n; mlen[it.pair] = it.m; }
  for (const auto &L : launches) {
    const bool chunked = L.nchunks > 1;
    for (int t = L.task_begin; t < L.task_end; ++t) {
      const Task &tk = tasks[t];
      bool ok = tk.ncols >= kBlock && tk.ncols % kBlock == 0 &&
                layout_valid(tk.layout, L.shared ? 64 : L.pmax) &&
                tk.stream_off + (int64_t)tk.ncols / kBlock * kStreamBlockBytes <= stream_bytes;
      if (chunked) ok = ok && tk.bnd_off >= 0 && tk.bnd_off % 4 == 0 &&
                        tk.bnd_off + (L.dual ? 16ll : 8ll) * tk.ncols <= bnd_elems;
      if (L.shared) ok = ok && tk.mode >= 0 && tk.mode < 3 && tk.layout == layout_for(16 << tk.mode);
      int widths[4];
      const int ngroups = layout_groups(tk.layout, widths);
      for (int s2 = 0; s2 < kSlots; ++s2) {
        const int pid = tk.pair[s2];
        ok = ok && pid >= -1 && pid < n_pairs_total;
        if (pid >= 0) {
          // each planned pair sits in exactly one slot (nlen = -2 once seen)
          const int n = nlen[pid];
          nlen[pid] = -2;
          ok = ok && s2 / 2 < ngroups && n >= 0 && n <= tk.ncols && pid < n_results;
          // per-pair: the task's chunks of this sub-group cover the query
          if (ok && !L.shared)
            ok = tk.nchunks >= 1 && (chunked || tk.nchunks == 1) &&
                 (int64_t)mlen[pid] <= (int64_t)tk.nchunks * widths[s2 / 2] * L.seg * (L.rp ? 2 : 1);
          if ((prec == PREC_I32 && !L.dual) || L.rp) ok = ok && (s2 & 1) == 0;
          if (L.rp) ok = ok && widths[s2 / 2] == L.pmax && prec == PREC_I16X2;
        }
      }
      if (!ok) {
        set_error("internal planner error: task %d of a launch is inconsistent", t);
        return SW_EINVAL;
      }
    }
  }
  for (const auto &it : in.items)
    if (nlen[it.pair] != -2) {
      set_error("internal planner error: pair %d is in no task", it.pair);
      return SW_EINVAL;
    }
  const size_t n_launch_total = [&] { size_t c = 0; for (auto &L : launches) c += L.shared ? L.nchunks : 1; return c; }();
  const size_t misc_bytes = 32 + 4 * n_launch_total + 16;   // stats (3 x u64, padded) + counters
  if ((rc = ws.tasks.ensure(tasks.size() * sizeof(Task))) ||
      (rc = ws.pairs.ensure(std::max<size_t>(1, in.pairs.size()) * sizeof(PairInfo))) ||
      (rc = ws.streams.ensure(stream_bytes)) ||
      (rc = ws.results.ensure(std::max(1, n_results) * sizeof(DevResult))) ||
      (rc = ws.misc.ensure(misc_bytes)) ||
      (rc = ws.matrix.ensure(sizeof(int) * sc.M.size())))
    return rc;
  const int64_t bnd_half = bnd_elems + 64;
  if (bnd_elems > 0 && (rc = ws.bnd.ensure(2 * bnd_half * sizeof(uint32_t)))) return rc;

  // one staging upload: tasks | pairs | matrix | misc zeros
  const size_t o_tasks = 0;
  const size_t o_pairs = o_tasks + tasks.size() * sizeof(Task);
  const size_t o_mat = o_pairs + in.pairs.size() * sizeof(PairInfo);
  const size_t o_misc = o_mat + sizeof(int) * sc.M.size();
  const size_t staging_bytes = o_misc + misc_bytes;
  if ((rc = ws.staging.ensure(staging_bytes))) return rc;
  unsigned char *stg = ws.staging.as<unsigned char>();
  std::memcpy(stg + o_tasks, tasks.data(), tasks.size() * sizeof(Task));
  std::memcpy(stg + o_pairs, in.pairs.data(), in.pairs.size() * sizeof(PairInfo));
  std::memcpy(stg + o_mat, sc.M.data(), sizeof(int) * sc.M.size());
  std::memset(stg + o_misc, 0, misc_bytes);

  // The device work of this execution as a list of operations, so that it can
  // run eagerly or be captured once into a hipGraph and replayed.  `sig`
  // collects every parameter of every operation: equal signatures mean an
  // identical graph (the staging contents are read when the graph runs).
  std::vector<std::function<hipError_t()>> ops;
  std::vector<uint64_t> sig;
  auto note = [&](const void *p, size_t n) {
    const size_t w = sig.size();
    sig.resize(w + (n + 7) / 8, 0);
    std::memcpy(sig.data() + w, p, n);
  };
  auto copy_op = [&](void *dst, const void *src, size_t bytes) {
    const uint64_t v[4] = {1, (uint64_t)(uintptr_t)dst, (uint64_t)(uintptr_t)src, bytes};
    note(v, sizeof(v));
    ops.push_back([=]() { return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st); });
  };
  copy_op(ws.tasks.p, stg + o_tasks, o_pairs - o_tasks);
  if (!in.pairs.empty()) copy_op(ws.pairs.p, stg + o_pairs, o_mat - o_pairs);
  copy_op(ws.matrix.p, stg + o_mat, o_misc - o_mat);
  copy_op(ws.misc.p, stg + o_misc, misc_bytes);
  if (reset_results) {
    DevResult *r = ws.results.as<DevResult>();
    const uint64_t v[3] = {2, (uint64_t)(uintptr_t)r, (uint64_t)n_results};
    note(v, sizeof(v));
    ops.push_back([=]() { return launch_init_results(n_results, r, st); });
  }
  uint32_t *bndA = ws.bnd.as<uint32_t>();
  uint32_t *bndB = bndA ? bndA + bnd_half : nullptr;
  if (bnd_elems > 0) {
    // the first query chunk reads zero boundaries (a fill kernel, not a memset
    // node: the sequence may be captured into a graph)
    const uint64_t v[3] = {3, (uint64_t)(uintptr_t)bndA, (uint64_t)bnd_half};
    note(v, sizeof(v));
    ops.push_back([=]() { return launch_fill_u32(bndA, bnd_half, 0u, st); });
  }
  {
    const Task *dt = ws.tasks.as<Task>();
    const int nt = (int)tasks.size();
    const PairInfo *dp = in.d_pairs ? in.d_pairs : ws.pairs.as<PairInfo>();
    const uint8_t *rr = in.d_rres;
    uint8_t *ds = ws.streams.as<uint8_t>();
    const int sent = sc.alpha;
    const uint64_t v[7] = {4, (uint64_t)(uintptr_t)dt, (uint64_t)nt, (uint64_t)(uintptr_t)dp,
                           (uint64_t)(uintptr_t)rr, (uint64_t)(uintptr_t)ds, (uint64_t)sent};
    note(v, sizeof(v));
    ops.push_back([=]() { return launch_build_streams(dt, nt, dp, rr, ds, sent, st); });
  }
  const size_t first_kernel_op = ops.size();
  unsigned long long *d_stats = (unsigned long long *)ws.misc.p;
  int *d_counters = (int *)((char *)ws.misc.p + 32);
  // Per-pair launches are independent of each other and of the shared-query
  // launches: they run concurrently on the workspace's side streams (fork and
  // join through events, which a graph capture turns into dependencies).  The
  // chunk launches of one shared query stay in order on the main stream.
  bool any_shared = false;
  int n_pair_launches = 0;
  for (const auto &L : launches) { any_shared |= L.shared; n_pair_launches += !L.shared; }
  const int side_wanted = std::min(kSideStreams, any_shared ? n_pair_launches : n_pair_launches - 1);
  if (side_wanted > 0 && (rc = ws.ensure_side_streams())) return rc;
  hipStream_t lane_stream[kSideStreams + 1] = {st};
  for (int k = 0; k < side_wanted; ++k) lane_stream[k + 1] = ws.side[k];
  if (side_wanted > 0) {
    hipEvent_t fork = ws.fork;
    std::vector<hipStream_t> sides(lane_stream + 1, lane_stream + 1 + side_wanted);
    const uint64_t v[2] = {7, (uint64_t)side_wanted};
    note(v, sizeof(v));
    ops.push_back([=]() {
      hipError_t e = hipEventRecord(fork, st);
      for (hipStream_t x : sides)
        if (e == hipSuccess) e = hipStreamWaitEvent(x, fork, 0);
      return e;
    });
  }
  int pair_ordinal = 0;
  int ci = 0;
  for (const auto &L : launches) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tasks = ws.tasks.as<Task>() + L.task_begin;
    a.ntasks = L.task_end - L.task_begin;
    a.pairs = in.d_pairs ? in.d_pairs : ws.pairs.as<PairInfo>();
    a.streams = ws.streams.as<uint8_t>();
    a.query_res = in.d_qres;
    a.alpha = sc.alpha;
    a.matrix = ws.matrix.as<int32_t>();
    a.gap_open = sc.go;
    a.gap_extend = sc.ge;
    a.sat_cap = opt.int16_cap;
    a.results = ws.results.as<DevResult>();
    a.stats = d_stats;
    const Alg alg = lazy ? ALG_LAZYF : ALG_SCAN;
    if (L.shared) {
      a.shared_q_off = in.q_off_of_query[L.query];
      a.shared_m = in.m_of_query[L.query];
      for (int c = 0; c < L.nchunks; ++c) {
        a.chunk = c;
        a.last_chunk = c + 1 == L.nchunks;
        a.task_counter = d_counters + ci++;
        a.bnd_in = (c & 1) ? bndB : bndA;
        a.bnd_out = (c & 1) ? bndA : bndB;
        const int menu = L.menu, grid = L.grid;
        const bool chunked = L.nchunks > 1, dual = L.dual;
        const uint64_t v[7] = {5, (uint64_t)prec, (uint64_t)alg, (uint64_t)menu, (uint64_t)chunked,
                               (uint64_t)grid, (uint64_t)dual};
        note(v, sizeof(v));
        note(&a, sizeof(a));
        ops.push_back([=]() { return launch_shared(prec, alg, menu, chunked, dual, a, grid, st); });
        stats.launches++;
      }
    } else {
      a.task_counter = d_counters + ci++;
      a.bnd = bndA;
      a.bnd_half = bnd_half;
      a.bnd_in = bndA;
      const int seg = L.seg, pmax = L.pmax, grid = L.grid;
      const bool chunked = L.nchunks > 1, rp = L.rp;
      // lane 0 is the main stream when no shared launch occupies it
      const int lane = side_wanted == 0 ? 0
                       : (any_shared ? 1 + pair_ordinal % side_wanted
                                     : pair_ordinal % (side_wanted + 1));
      ++pair_ordinal;
      hipStream_t ls = lane_stream[lane];
      const uint64_t v[8] = {6, (uint64_t)prec, (uint64_t)seg, (uint64_t)pmax, (uint64_t)chunked,
                             (uint64_t)grid, (uint64_t)lane, (uint64_t)rp};
      note(v, sizeof(v));
      note(&a, sizeof(a));
      ops.push_back([=]() {
        return rp ? launch_pair_rowpair(seg, pmax, chunked, a, grid, ls)
                  : launch_pair(prec, seg, pmax, chunked, a, grid, ls);
      });
      stats.launches++;
    }
  }
  if (side_wanted > 0) {
    std::vector<hipStream_t> sides(lane_stream + 1, lane_stream + 1 + side_wanted);
    std::vector<hipEvent_t> joins(ws.join, ws.join + side_wanted);
    ops.push_back([=]() {
      hipError_t e = hipSuccess;
      for (size_t k = 0; k < sides.size() && e == hipSuccess; ++k) {
        e = hipEventRecord(joins[k], sides[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, joins[k], 0);
      }
      return e;
    });
  }
  auto run_ops = [&](size_t from, size_t to) -> int {
    for (size_t k = from; k < to; ++k) {
      const hipError_t e = ops[k]();
      if (e != hipSuccess) {
        set_error("device operation %zu failed: %s", k, hipGetErrorString(e));
        return SW_EDEVICE;
      }
    }
    return SW_OK;
  };
  if (!opt.use_graph) {
    if ((rc = run_ops(0, first_kernel_op))) return rc;
    HIPCHK(hipEventRecord(e0, st));
    if ((rc = run_ops(first_kernel_op, ops.size()))) return rc;
    HIPCHK(hipEventRecord(e1, st));
  } else {
    hipGraphExec_t exec = ws.graphs.find(sig);
    if (exec) {
      stats.graph_hits++;
    } else {
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
      rc = run_ops(0, ops.size());
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ec));
        return SW_EDEVICE;
      }
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ei));
        return SW_EDEVICE;
      }
      ws.graphs.put(sig, exec);
    }
    // with a graph the timed span also covers the uploads and stream building
    HIPCHK(hipEventRecord(e0, st));
    HIPCHK(hipGraphLaunch(exec, st));
    HIPCHK(hipEventRecord(e1, st));
  }
  const double t_fin0 = now_ms();
  stats.launch_ms += t_fin0 - t_launch0;
  unsigned long long hstats[3];
  HIPCHK(hipMemcpyAsync(hstats, d_stats, sizeof(hstats), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  stats.kernel_ms += ms;
  stats.dev_stats[0] += hstats[0];
  stats.dev_stats[1] += hstats[1];
  stats.dev_stats[2] += hstats[2];
  stats.finish_ms += now_ms() - t_fin0;
  return SW_OK;
}

// Pairs in the swapped layout (reference striped over one wavefront, query
// streamed; int32): grouped by rows per lane (the fewest that hold the
// reference), each group one persistent launch, the groups spread over the
// main stream and the side streams.  Results go to ws.results (n_results
// entries, all initialised first when init_all).  Synchronous.
static int run_swapped(const ExecInput &in, const std::vector<PlanItem> &items, const Scoring &sc,
                       Workspace &ws, int n_results, bool init_all, hipStream_t st,
                       hipEvent_t e0, hipEvent_t e1, int num_cus, ExecStats &es) {
  int rc;
  constexpr int kNumSeg = (int)(sizeof(kSwapSegs) / sizeof(kSwapSegs[0]));
  std::vector<std::vector<const PlanItem *>> by(kNumSeg);
  for (const auto &it : items) {
    int g = 0;
    while (g < kNumSeg && 64 * kSwapSegs[g] < it.n) ++g;
    if (g == kNumSeg) { set_error("internal planner error: swapped pair beyond %d rows", kSwapMaxRows); return SW_EINVAL; }
    by[g].push_back(&it);
  }
  std::vector<Task> tasks;
  tasks.reserve(items.size());
  struct Group { int seg, begin, end; double work; };
  std::vector<Group> groups;
  for (int g = 0; g < kNumSeg; ++g) {
    if (by[g].empty()) continue;
    // longest queries first inside a group (one wavefront per pair)
    std::stable_sort(by[g].begin(), by[g].end(),
                     [](const PlanItem *x, const PlanItem *y) { return x->m > y->m; });
    Group G{kSwapSegs[g], (int)tasks.size(), 0, 0.0};
    for (const PlanItem *it : by[g]) {
      Task t;
      std::memset(&t, 0, sizeof(t));
      t.layout = 1;
      t.mode = 0;
      t.nchunks = 1;
      t.bnd_off = -1;
      for (int k = 0; k < kSlots; ++k) t.pair[k] = -1;
      t.pair[0] = it->pair;
      t.ncols = round_up(std::max(it->m, 1), kBlock);
      G.work += (double)t.ncols * kSwapSegs[g];
      tasks.push_back(t);
    }
    G.end = (int)tasks.size();
    groups.push_back(G);
  }
  if (tasks.empty()) return SW_OK;
  const PairInfo *d_pairs = in.d_pairs;
  const size_t task_bytes = tasks.size() * sizeof(Task);
  const size_t misc_bytes = 64 + 4 * groups.size();
  if ((rc = ws.results.ensure((size_t)std::max(1, n_results) * sizeof(DevResult))) ||
      (rc = ws.matrix.ensure(sizeof(int32_t) * sc.M.size())) ||
      (rc = ws.tasks.ensure(task_bytes)) || (rc = ws.misc.ensure(misc_bytes)) ||
      (rc = ws.staging.ensure(task_bytes + sizeof(int32_t) * sc.M.size() + 64)))
    return rc;
  if (!d_pairs) {
    if ((rc = ws.pairs.ensure(std::max<size_t>(1, in.pairs.size()) * sizeof(PairInfo)))) return rc;
    HIPCHK(hipMemcpyAsync(ws.pairs.p, in.pairs.data(), in.pairs.size() * sizeof(PairInfo),
                          hipMemcpyHostToDevice, st));
    d_pairs = ws.pairs.as<PairInfo>();
  }
  char *stg = ws.staging.as<char>();
  std::memcpy(stg, tasks.data(), task_bytes);
  std::memcpy(stg + task_bytes, sc.M.data(), sizeof(int32_t) * sc.M.size());
  HIPCHK(hipMemcpyAsync(ws.tasks.p, stg, task_bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws.matrix.p, stg + task_bytes, sizeof(int32_t) * sc.M.size(),
                        hipMemcpyHostToDevice, st));
  uint32_t *misc = ws.misc.as<uint32_t>();
  unsigned long long *d_stats = (unsigned long long *)misc;   // 3 x u64, then counters
  HIPCHK(launch_fill_u32(misc, (int64_t)(misc_bytes / 4), 0u, st));
  if (init_all) HIPCHK(launch_init_results(n_results, ws.results.as<DevResult>(), st));
  // the largest groups first, round robin over the streams
  std::vector<int> order(groups.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return groups[x].work > groups[y].work; });
  const int nside = std::min<int>(kSideStreams, (int)groups.size() - 1);
  if (nside > 0 && (rc = ws.ensure_side_streams())) return rc;
  HIPCHK(hipEventRecord(e0, st));
  if (nside > 0) {
    HIPCHK(hipEventRecord(ws.fork, st));
    for (int k = 0; k < nside; ++k) HIPCHK(hipStreamWaitEvent(ws.side[k], ws.fork, 0));
  }
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const Group &G = groups[order[oi]];
    const int lane = nside > 0 ? (int)(oi % (nside + 1)) : 0;
    hipStream_t ls = lane == 0 ? st : ws.side[lane - 1];
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tasks = ws.tasks.as<Task>() + G.begin;
    a.ntasks = G.end - G.begin;
    a.task_counter = (int32_t *)(misc + 16) + order[oi];
    a.pairs = d_pairs;
    a.query_res = in.d_qres;
    a.ref_res = in.d_rres;
    a.alpha = sc.alpha;
    a.matrix = ws.matrix.as<int32_t>();
    a.gap_open = sc.go;
    a.gap_extend = sc.ge;
    a.results = ws.results.as<DevResult>();
    a.stats = d_stats;
    a.sat_cap = 32767;
    const int grid = std::max(1, std::min(a.ntasks, num_cus * 24));
    HIPCHK(launch_swap(G.seg, a, grid, ls));
    es.launches++;
    es.seglen_max = std::max(es.seglen_max, G.seg);
  }
  for (int k = 0; k < nside; ++k) {
    HIPCHK(hipEventRecord(ws.join[k], ws.side[k]));
    HIPCHK(hipStreamWaitEvent(st, ws.join[k], 0));
  }
  HIPCHK(hipEventRecord(e1, st));
  unsigned long long hs[3];
  HIPCHK(hipMemcpyAsync(hs, d_stats, sizeof(hs), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  es.kernel_ms += ms;
  for (int k = 0; k < 3; ++k) es.dev_stats[k] += hs[k];
  for (const Group &G : groups)
    for (int t = G.begin; t < G.end; ++t) es.padded_cells += (int64_t)tasks[t].ncols * 64 * G.seg;
  return SW_OK;
}

int run_batch(const ExecInput &in, const Scoring &sc, int precision, const ExecOptions &opt,
              Workspace &ws, int n_pairs, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
              int num_cus, sw_result *out, sw_stats *stats) {
  Prec prec = (precision == SW_PREC_AUTO && sc.fits_i16 && opt.algorithm == SW_ALG_SCAN)
                  ? PREC_I16X2 : PREC_I32;
  ExecStats es;
  // swapped striping: pairs whose reference fits one wavefront's rows and is
  // shorter than the query run with the reference striped (scan only)
  std::vector<PlanItem> swapped;
  ExecInput rest_in;
  const ExecInput *main_in = &in;
  if (opt.striping == SW_STRIPE_SHORTER && opt.algorithm == SW_ALG_SCAN) {
    rest_in.d_qres = in.d_qres;
    rest_in.d_rres = in.d_rres;
    rest_in.d_pairs = in.d_pairs;
    rest_in.pairs = in.pairs;
    rest_in.n_pairs = in.n_pairs;
    rest_in.n_queries = in.n_queries;
    rest_in.q_off_of_query = in.q_off_of_query;
    rest_in.m_of_query = in.m_of_query;
    for (const auto &it : in.items) {
      if (it.n <= kSwapMaxRows && it.n < it.m) swapped.push_back(it);
      else rest_in.items.push_back(it);
    }
    main_in = &rest_in;
  }
  int rc = execute(*main_in, sc, prec, opt, ws, n_pairs, st, e0, e1, num_cus, es, true);
  if (rc) return rc;
  if (!swapped.empty()) {
    rc = run_swapped(in, swapped, sc, ws, n_pairs, main_in->items.empty(), st, e0, e1, num_cus,
                     es);
    if (rc) return rc;
  }
  const double t_res0 = now_ms();
  int rerun = 0;
  static_assert(sizeof(DevResult) == sizeof(sw_result), "result layout");
  if (!in.items.empty()) {
    // device results have the sw_result layout: copy straight into out
    HIPCHK(hipMemcpyAsync(out, ws.results.p, (size_t)n_pairs * sizeof(DevResult),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<PlanItem> again;
    if (prec == PREC_I16X2) {
      for (const auto &it : in.items)
        if (out[it.pair].flags & kFlagNeedsI32) again.push_back(it);
    }
    if (!again.empty()) {
      rerun = (int)again.size();
      ExecInput in2;
      in2.d_qres = in.d_qres;
      in2.d_rres = in.d_rres;
      in2.d_pairs = in.d_pairs ? in.d_pairs : ws.pairs.as<PairInfo>();
      in2.n_pairs = in.d_pairs ? in.n_pairs : (int)in.pairs.size();
      in2.items = again;
      in2.n_queries = in.n_queries;
      in2.q_off_of_query = in.q_off_of_query;
      in2.m_of_query = in.m_of_query;
      ExecOptions o2 = opt;
      o2.force_lanes = 0;
      o2.force_seglen = 0;
      o2.lane_pairing = SW_PAIRING_AUTO;   // the int32 rerun has no int16 halves
      rc = execute(in2, sc, PREC_I32, o2, ws, n_pairs, st, e0, e1, num_cus, es, false);
      if (rc) return rc;
      if ((rc = ws.staging.ensure((size_t)n_pairs * sizeof(DevResult)))) return rc;
      DevResult *hr = ws.staging.as<DevResult>();
      HIPCHK(hipMemcpyAsync(hr, ws.results.p, (size_t)n_pairs * sizeof(DevResult),
                            hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (const auto &it : again) {
        const DevResult &r = hr[it.pair];
        out[it.pair].score = r.score;
        out[it.pair].query_end = r.qend;
        out[it.pair].ref_end = r.rend;
        out[it.pair].flags = SW_FLAG_SATURATED;
      }
    }
  }
  es.finish_ms += now_ms() - t_res0;
  if (stats) {
    stats->kernel_ms = es.kernel_ms;
    stats->plan_ms = es.plan_ms;
    stats->launch_ms = es.launch_ms;
    stats->finish_ms = es.finish_ms;
    stats->padded_cells = es.padded_cells;
    stats->n_rerun = rerun;
    stats->n_launches = es.launches;
    stats->lazyf_steps = (int64_t)es.dev_stats[1];
    stats->columns = (int64_t)es.dev_stats[0];
    stats->record_events = (int64_t)es.dev_stats[2];
    stats->graph_hits = es.graph_hits;
    stats->planner_used = 1;
    stats->row_pairs = es.row_pairs;
    for (int k = 0; k < 3; ++k) stats->lanes_used[k] = es.lanes_used[k];
    stats->seglen_max = es.seglen_max;
  }
  return SW_OK;
}

}  // namespace swrt
