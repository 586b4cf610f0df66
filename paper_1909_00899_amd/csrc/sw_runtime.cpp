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
#include <chrono>
#include <map>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
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
  if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
  size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
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
  if (p) { (void)hipHostFree(p); p = nullptr; cap = 0; }
  size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
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
  bool fits16 = out.go <= 32767;
  for (int v : out.M) {
    mx = std::max(mx, v);
    if (v < -32767 || v > 32767) fits16 = false;
  }
  out.max_s = mx;
  out.fits_i16 = fits16;
  return SW_OK;
}

// ------------------------------------------------------------------ planner

namespace {

constexpr int64_t kI32Limit = 2147483647ll;

int slots_per_wave(Prec prec, int P) { return (prec == PREC_I16X2 ? 2 : 1) * (kWave / P); }

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
void sort_by_n_desc(const std::vector<PlanItem> &items, std::vector<int> &order) {
  order.resize(items.size());
  if (items.empty()) return;
  int lo = items[0].n, hi = items[0].n;
  for (const auto &it : items) { lo = std::min(lo, it.n); hi = std::max(hi, it.n); }
  const int64_t range = (int64_t)hi - lo + 1;
  if (range > 4 * (int64_t)items.size() + 1024) {
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return items[a].n > items[b].n; });
    return;
  }
  std::vector<int> start(range + 1, 0);
  for (const auto &it : items) start[hi - it.n + 1]++;
  for (int64_t k = 0; k < range; ++k) start[k + 1] += start[k];
  for (size_t k = 0; k < items.size(); ++k) order[start[hi - items[k].n]++] = (int)k;
}

}  // namespace

// Builds tasks for one shared-query launch group.
// items: pairs of this query (n > 0, m > 0).  Pairs are ordered by reference
// length (longest first); each pair gets the narrowest lane mode whose task
// stays short next to the average load of a wavefront (long references get
// more lanes so they finish in time); consecutive pairs of one mode share a
// task.  Tasks are emitted longest-first (by estimated cost) across modes.
static void plan_shared(const std::vector<PlanItem> &items, Prec prec, int menu, int num_waves,
                        int force_lanes, std::vector<Task> &tasks, int mode_counts[3]) {
  const SharedMenu mm = shared_menu(menu);
  const int segs[3] = {mm.seg16, mm.seg32, mm.seg64};
  const int Ps[3] = {16, 32, 64};
  std::vector<int> order;
  sort_by_n_desc(items, order);
  int narrow = 0;
  for (int k = 0; k < 3; ++k)
    if (segs[k]) { narrow = k; break; }
  double total = 0;
  for (const auto &it : items) total += (double)it.n;
  total *= step_cost(prec, Ps[narrow], segs[narrow]) / slots_per_wave(prec, Ps[narrow]);
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
  const int halves = prec == PREC_I16X2 ? 2 : 1;
  std::vector<Task> bym[3];
  for (int md = 2; md >= 0; --md) {
    const int from = begin[md];
    const int to = (md == 0) ? begin[3] : begin[md - 1];
    if (to <= from) continue;
    const int spw = slots_per_wave(prec, Ps[md]);
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
};

// LDS bytes of one per-pair wavefront region.
size_t pair_region(Prec prec, int seg, int alpha) {
  return pair_lds_bytes(prec, seg, alpha) - matrix_lds_bytes(alpha);
}

PairShape choose_pair_shape(Prec prec, int m, int alpha, const ExecOptions &opt) {
  static const int kSegs[] = {4, 6, 8, 10, 12, 16};
  const size_t budget = 20 * 1024;   // LDS per wavefront (keeps >= 6 waves per CU)
  PairShape best{64, 4, 1 << 30};
  double best_cost = 1e300;
  for (int P : {16, 32, 64}) {
    if (opt.force_lanes && P != opt.force_lanes) continue;
    for (int seg : kSegs) {
      if (opt.force_seglen && seg != opt.force_seglen) continue;
      if (!opt.force_seglen && pair_region(prec, seg, alpha) > budget && seg != 4) continue;
      const int rows = P * seg;
      const int nch = (m + rows - 1) / rows;
      // cost per reference column, normalised per alignment slot
      const double cost = (double)nch * step_cost(prec, P, seg) / slots_per_wave(prec, P);
      if (cost < best_cost - 1e-9) { best_cost = cost; best = PairShape{P, seg, nch}; }
    }
  }
  return best;
}

}  // namespace

// ------------------------------------------------------------------ executor

namespace {

struct LaunchDesc {
  bool shared;
  int task_begin, task_end;
  int menu;          // shared
  int seg, pmax;     // per-pair
  int nchunks;       // shared: launches; per-pair: inside the kernel
  int query;         // shared
  int grid;
};

}  // namespace

int execute(const ExecInput &in, const Scoring &sc, Prec prec, const ExecOptions &opt,
            Workspace &ws, int n_results, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
            int num_cus, ExecStats &stats, bool reset_results) {
  const double t_plan0 = now_ms();
  std::vector<Task> tasks;
  std::vector<LaunchDesc> launches;
  const bool lazy = opt.algorithm == SW_ALG_LAZYF;
  // ---- group by query
  std::vector<int> count(in.n_queries, 0);
  for (const auto &it : in.items) count[it.query]++;
  std::vector<std::vector<PlanItem>> by_query(in.n_queries);
  std::vector<PlanItem> per_pair;
  auto wants_shared = [&](int q) {
    return lazy || opt.force_kernel == 1 || (opt.force_kernel == 0 && count[q] >= 32);
  };
  int only_query = -1;   // every item uses one query that runs shared: no copy
  if (!in.items.empty() && count[in.items[0].query] == (int)in.items.size() &&
      wants_shared(in.items[0].query))
    only_query = in.items[0].query;
  if (only_query < 0) {
    for (const auto &it : in.items) {
      if (wants_shared(it.query)) by_query[it.query].push_back(it);
      else per_pair.push_back(it);
    }
  }
  const int waves_total = num_cus * 16;
  int64_t bnd_elems = 0;
  // ---- shared-query launches
  for (int q = 0; q < in.n_queries; ++q) {
    if (q != only_query && by_query[q].empty()) continue;
    const std::vector<PlanItem> &group = q == only_query ? in.items : by_query[q];
    const int m = in.m_of_query[q];
    int fl = opt.force_lanes;
    const int menu = pick_shared_menu(m, fl ? fl : 64, opt.force_seglen);
    if (menu < 0) { set_error("no compiled shared kernel with %d rows per lane", opt.force_seglen); return SW_EINVAL; }
    const SharedMenu mm = shared_menu(menu);
    if (fl == 16 && !mm.seg16) { set_error("menu has no 16-lane mode"); return SW_EINVAL; }
    const int rows = 64 * mm.seg64;
    const int nch = (m + rows - 1) / rows;
    LaunchDesc L{};
    L.shared = true;
    L.menu = menu;
    L.nchunks = nch;
    L.query = q;
    L.task_begin = (int)tasks.size();
    int mc[3] = {0, 0, 0};
    plan_shared(group, prec, menu, waves_total, fl, tasks, mc);
    L.task_end = (int)tasks.size();
    for (int k = 0; k < 3; ++k) stats.lanes_used[k] += mc[k];
    const int segs[3] = {mm.seg16, mm.seg32, mm.seg64};
    for (int t = L.task_begin; t < L.task_end; ++t) {
      tasks[t].nchunks = nch;
      if (nch > 1) { tasks[t].bnd_off = bnd_elems; bnd_elems += 8ll * tasks[t].ncols; }
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
  // ---- per-pair launches, grouped by (seg, P, chunks)
  if (!per_pair.empty()) {
    struct Key { int seg, P, nch; bool operator<(const Key &o) const {
      return std::tie(seg, P, nch) < std::tie(o.seg, o.P, o.nch); } };
    // shapes depend on the query length only: decide once per distinct length
    std::map<int, PairShape> shape_of_m;
    std::map<Key, std::vector<PlanItem>> groups;
    for (const auto &it : per_pair) {
      auto f = shape_of_m.find(it.m);
      if (f == shape_of_m.end())
        f = shape_of_m.emplace(it.m, choose_pair_shape(prec, it.m, sc.alpha, opt)).first;
      const PairShape &ps = f->second;
      groups[Key{ps.seg, ps.P, ps.nchunks}].push_back(it);
    }
    std::vector<std::pair<Key, PlanItem>> keyed;
    keyed.reserve(per_pair.size());
    std::vector<int> ord;
    for (auto &g : groups) {
      sort_by_n_desc(g.second, ord);
      for (int k : ord) keyed.push_back({g.first, g.second[k]});
    }
    size_t a = 0;
    while (a < keyed.size()) {
      size_t b = a;
      while (b < keyed.size() && !(keyed[a].first < keyed[b].first) && !(keyed[b].first < keyed[a].first)) ++b;
      const Key k = keyed[a].first;
      LaunchDesc L{};
      L.shared = false;
      L.seg = k.seg;
      L.pmax = k.P;
      L.nchunks = k.nch;
      L.task_begin = (int)tasks.size();
      const int halves = prec == PREC_I16X2 ? 2 : 1;
      const int spw = slots_per_wave(prec, k.P);
      for (size_t x = a; x < b; x += spw) {
        Task t;
        std::memset(&t, 0, sizeof(t));
        t.layout = layout_for(k.P);
        t.nchunks = k.nch;
        t.bnd_off = -1;
        for (int s = 0; s < kSlots; ++s) t.pair[s] = -1;
        int maxn = 1;
        for (int q = 0; q < spw && x + q < b; ++q) {
          const int sg = q / halves, h = q % halves;
          t.pair[2 * sg + h] = keyed[x + q].second.pair;
          maxn = std::max(maxn, keyed[x + q].second.n);
        }
        t.ncols = round_up(maxn, kBlock);
        if (k.nch > 1) { t.bnd_off = bnd_elems; bnd_elems += 8ll * t.ncols; }
        stats.padded_cells += (int64_t)std::min<size_t>(spw, b - x) * t.ncols * k.P * k.seg * k.nch;
        tasks.push_back(t);
      }
      L.task_end = (int)tasks.size();
      stats.lanes_used[k.P == 16 ? 0 : (k.P == 32 ? 1 : 2)] += (int)(b - a);
      stats.seglen_max = std::max(stats.seglen_max, k.seg);
      L.grid = std::max(1, std::min(L.task_end - L.task_begin, num_cus * 16));
      launches.push_back(L);
      a = b;
    }
  }
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
  std::vector<int> nlen(std::max(n_pairs_total, 0), -1);
  for (const auto &it : in.items)
    if (it.pair >= 0 && it.pair < n_pairs_total) nlen[it.pair] = it.n;
  for (const auto &L : launches) {
    const bool chunked = L.nchunks > 1;
    for (int t = L.task_begin; t < L.task_end; ++t) {
      const Task &tk = tasks[t];
      bool ok = tk.ncols >= kBlock && tk.ncols % kBlock == 0 && (tk.layout & 1) &&
                tk.stream_off + (int64_t)tk.ncols / kBlock * kStreamBlockBytes <= stream_bytes;
      if (chunked) ok = ok && tk.bnd_off >= 0 && tk.bnd_off % 4 == 0 &&
                        tk.bnd_off + 8ll * tk.ncols <= bnd_elems;
      if (L.shared) ok = ok && tk.mode >= 0 && tk.mode < 3 && tk.layout == layout_for(16 << tk.mode);
      for (int s2 = 0; s2 < kSlots; ++s2) {
        const int pid = tk.pair[s2];
        ok = ok && pid >= -1 && pid < n_pairs_total;
        if (pid >= 0) {
          ok = ok && nlen[pid] >= 0 && nlen[pid] <= tk.ncols && pid < n_results;
          if (prec == PREC_I32) ok = ok && (s2 & 1) == 0;
        }
      }
      if (!ok) {
        set_error("internal planner error: task %d of a launch is inconsistent", t);
        return SW_EINVAL;
      }
    }
  }
  int rc;
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
  unsigned char *hs = ws.staging.as<unsigned char>();
  std::memcpy(hs + o_tasks, tasks.data(), tasks.size() * sizeof(Task));
  std::memcpy(hs + o_pairs, in.pairs.data(), in.pairs.size() * sizeof(PairInfo));
  std::memcpy(hs + o_mat, sc.M.data(), sizeof(int) * sc.M.size());
  std::memset(hs + o_misc, 0, misc_bytes);
  HIPCHK(hipMemcpyAsync(ws.tasks.p, hs + o_tasks, o_pairs - o_tasks, hipMemcpyHostToDevice, st));
  if (!in.pairs.empty())
    HIPCHK(hipMemcpyAsync(ws.pairs.p, hs + o_pairs, o_mat - o_pairs, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws.matrix.p, hs + o_mat, o_misc - o_mat, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws.misc.p, hs + o_misc, misc_bytes, hipMemcpyHostToDevice, st));
  if (reset_results) HIPCHK(launch_init_results(n_results, ws.results.as<DevResult>(), st));
  if (bnd_elems > 0) HIPCHK(hipMemsetAsync(ws.bnd.p, 0, bnd_half * sizeof(uint32_t), st));
  const int sent = sc.alpha;
  HIPCHK(launch_build_streams(ws.tasks.as<Task>(), (int)tasks.size(),
                              in.d_pairs ? in.d_pairs : ws.pairs.as<PairInfo>(),
                              in.d_rres, ws.streams.as<uint8_t>(), sent, st));
  unsigned long long *d_stats = (unsigned long long *)ws.misc.p;
  int *d_counters = (int *)((char *)ws.misc.p + 32);
  uint32_t *bndA = ws.bnd.as<uint32_t>();
  uint32_t *bndB = bndA ? bndA + bnd_half : nullptr;

  HIPCHK(hipEventRecord(e0, st));
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
    if (L.shared) {
      a.shared_q_off = in.q_off_of_query[L.query];
      a.shared_m = in.m_of_query[L.query];
      for (int c = 0; c < L.nchunks; ++c) {
        a.chunk = c;
        a.last_chunk = c + 1 == L.nchunks;
        a.task_counter = d_counters + ci++;
        a.bnd_in = (c & 1) ? bndB : bndA;
        a.bnd_out = (c & 1) ? bndA : bndB;
        HIPCHK(launch_shared(prec, lazy ? ALG_LAZYF : ALG_SCAN, L.menu, L.nchunks > 1, a,
                             L.grid, st));
        stats.launches++;
      }
    } else {
      a.task_counter = d_counters + ci++;
      a.bnd = bndA;
      a.bnd_half = bnd_half;
      a.bnd_in = bndA;
      HIPCHK(launch_pair(prec, L.seg, L.pmax, L.nchunks > 1, a, L.grid, st));
      stats.launches++;
    }
  }
  HIPCHK(hipEventRecord(e1, st));
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

int run_batch(const ExecInput &in, const Scoring &sc, int precision, const ExecOptions &opt,
              Workspace &ws, int n_pairs, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
              int num_cus, sw_result *out, sw_stats *stats) {
  Prec prec = (precision == SW_PREC_AUTO && sc.fits_i16 && opt.algorithm == SW_ALG_SCAN)
                  ? PREC_I16X2 : PREC_I32;
  ExecStats es;
  int rc = execute(in, sc, prec, opt, ws, n_pairs, st, e0, e1, num_cus, es, true);
  if (rc) return rc;
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
    for (int k = 0; k < 3; ++k) stats->lanes_used[k] = es.lanes_used[k];
    stats->seglen_max = es.seglen_max;
  }
  return SW_OK;
}

}  // namespace swrt
