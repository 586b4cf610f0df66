// Continuous-batching request server (include/sw.h, "Serving").
//
// Requests (one query against one resident database reference) enter the
// FIFO of their class (scoring scheme and size).  n_streams worker threads
// each own a HIP stream and a device workspace; an idle worker takes, under
// the server lock, the longest prefix of the FIFO that holds the oldest
// waiting request that fits the remaining memory budget (at most max_batch),
// marks them admitted, releases the lock and runs them as one batch (the batch planner re-buckets them by
// length into per-pair kernel launches).  Requests that arrive meanwhile wait
// for the next idle worker, so their kernels overlap with the batches already
// on the device.  Each result is the batch path's result for that pair.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sw.h"
#include "sw_runtime.h"

using namespace swrt;
using swk::PairInfo;

namespace {

// A request is long when its query needs chunks in the per-pair kernels or
// its matrix is large: such pairs bound a batch's time (one wavefront runs
// one alignment's column chain), so they are batched apart from short ones.
constexpr int kLongQuery = 1024;
constexpr int64_t kLongCells = 1 << 20;
bool is_long(int64_t m, int64_t n) { return m > kLongQuery || m * n > kLongCells; }

int64_t mono_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket;
  const uint8_t *query = nullptr;   // the residues: `own`, or the replay caller's buffer
  int32_t qlen = 0;
  std::vector<uint8_t> own;
  int32_t ref_id, scoring_id;
  int32_t klass;             // batch class: scoring and size (see kLongCells)
  size_t bytes;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
  sw_result res{0, -1, -1, 0};
  int status = SW_PENDING;   // SW_PENDING until finished, then SW_OK or an error
  bool done = false;
};

}  // namespace

struct sw_server {
  int device = 0;
  int num_cus = 256;
  size_t budget = 0, in_flight = 0;
  int max_queued = 0, max_batch = 0;
  std::vector<Scoring> scorings;
  DevBuf db;                         // resident reference residues
  std::vector<int64_t> db_off;
  std::vector<uint8_t> db_max_code;  // largest residue code of each reference (0 if empty)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  // One FIFO per batch class (two per scoring: short and long requests): a
  // worker takes the class of the oldest waiting request and pops from the
  // front of that FIFO only, so admission costs the batch, not the depth of
  // the backlog (a scan of one shared queue, erasing from its middle, held
  // the lock for milliseconds once it was deep and stalled every submit)
  std::vector<std::deque<Request *>> queues;
  int64_t queued = 0;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> table;
  uint64_t next_ticket = 1;
  int outstanding = 0;               // accepted and not yet finished
  int idle_workers = 0;              // workers waiting for requests (a submit wakes
                                     // one only then: a wake-up is a system call)
  int running = 0;                   // batches on the device
  bool stop = false;
  // While a replay runs, workers append the tickets of each finished batch
  // here, so that its collector takes only finished requests (one lock per
  // batch) instead of polling every outstanding ticket in turn.
  std::vector<uint64_t> *done_sink = nullptr;
  std::vector<std::thread> workers;

  size_t request_bytes(int m, int n) const {
    // query + residue stream (8 bytes per column per slot-half, rounded) +
    // chunk boundaries (two buffers of 8 u32 per column per task) + result
    return (size_t)m + 16 * (size_t)(n + 8) + 64 * (size_t)(n + 8) + 64;
  }

  void worker_main();
};

void sw_server::worker_main() {
  hipSetDevice(device);
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  Workspace ws;
  DevBuf qbuf;
  HostBuf qstage;
  // batches grow with the load: buffers double on growth, and an outgrown
  // one is kept until the worker exits (freeing it would wait for the whole
  // device, stalling every other worker's batch); at most the final size
  // again is held that way
  std::vector<void *> dev_old, host_old;
  ws.set_growth(100, &dev_old, &host_old);
  qbuf.grow_pct = 100;
  qbuf.retired = &dev_old;
  qstage.grow_pct = 100;
  qstage.retired = &host_old;
  std::vector<Request *> batch;
  std::vector<sw_result> out;
  for (;;) {
    batch.clear();
    size_t bytes = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (!stop && queued == 0) {
        ++idle_workers;
        cv_work.wait(lk, [&] { return stop || queued > 0; });
        --idle_workers;
      }
      if (stop && queued == 0) break;
      // admission: the class (scoring and size) of the oldest waiting
      // request, in FIFO order, within the budget; a batch lasts as long as
      // its longest pair, so short requests do not wait behind long ones of
      // the same scoring
      int klass = -1;
      for (int c = 0; c < (int)queues.size(); ++c)
        if (!queues[c].empty() &&
            (klass < 0 || queues[c].front()->ticket < queues[klass].front()->ticket))
          klass = c;
      std::deque<Request *> &q = queues[klass];
      while (!q.empty() && (int)batch.size() < max_batch) {
        Request *r = q.front();
        if (in_flight + bytes + r->bytes > budget && !(batch.empty() && in_flight == 0)) break;
        bytes += r->bytes;
        batch.push_back(r);
        q.pop_front();
      }
      queued -= (int64_t)batch.size();
      if (batch.empty()) {
        // the head does not fit next to what is running: wait for a finish
        cv_done.wait(lk, [&] { return stop || in_flight == 0 || queued == 0; });
        continue;
      }
      in_flight += bytes;
      ++running;
      const int64_t t = mono_ns();
      for (Request *r : batch) r->t_admit = t;
    }
    // ---- run the batch (outside the lock)
    const Scoring &sc = scorings[batch[0]->scoring_id];
    int64_t qtotal = 0;
    for (Request *r : batch) qtotal += (int64_t)r->qlen;
    int rc = qstage.ensure(std::max<int64_t>(qtotal, 1));
    if (!rc) rc = qbuf.ensure(std::max<int64_t>(qtotal, 1));
    ExecInput in;
    if (!rc) {
      unsigned char *h = qstage.as<unsigned char>();
      int64_t off = 0;
      in.n_queries = (int)batch.size();
      in.pairs.resize(batch.size());
      in.q_off_of_query.resize(batch.size());
      in.m_of_query.resize(batch.size());
      for (size_t k = 0; k < batch.size(); ++k) {
        Request *r = batch[k];
        if (r->qlen) std::memcpy(h + off, r->query, (size_t)r->qlen);
        PairInfo &p = in.pairs[k];
        std::memset(&p, 0, sizeof(p));
        p.q_off = off;
        p.r_off = db_off[r->ref_id];
        p.m = (int)r->qlen;
        p.n = (int)(db_off[r->ref_id + 1] - db_off[r->ref_id]);
        p.out = (int)k;
        in.q_off_of_query[k] = off;
        in.m_of_query[k] = p.m;
        if (p.m > 0 && p.n > 0) in.items.push_back(PlanItem{(int)k, (int)k, p.m, p.n});
        off += (int64_t)r->qlen;
      }
      if (qtotal && hipMemcpyAsync(qbuf.p, h, qtotal, hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("server: query upload failed");
        rc = SW_EDEVICE;
      }
      in.d_qres = qbuf.as<uint8_t>();
      in.d_rres = db.as<uint8_t>();
    }
    out.assign(batch.size(), sw_result{0, -1, -1, 0});
    if (!rc) {
      ExecOptions opt;
      rc = run_batch(in, sc, SW_PREC_AUTO, opt, ws, (int)batch.size(), st, e0, e1, num_cus,
                     out.data(), nullptr);
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      const int64_t t = mono_ns();
      for (size_t k = 0; k < batch.size(); ++k) {
        Request *r = batch[k];
        r->res = out[k];
        r->status = rc ? rc : SW_OK;
        r->t_done = t;
        r->done = true;
      }
      if (done_sink)
        for (Request *r : batch) done_sink->push_back(r->ticket);
      in_flight -= bytes;
      --running;
      outstanding -= (int)batch.size();
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
  ws.release();
  qbuf.release();
  qstage.release();
  for (void *p : dev_old) (void)hipFree(p);
  for (void *p : host_old) (void)hipHostFree(p);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamDestroy(st);
}

extern "C" {

int sw_server_create(const sw_server_config *cfg, sw_server **out) {
  if (!cfg || !out || cfg->n_db < 1 || !cfg->db_res || !cfg->db_off || !cfg->scorings ||
      cfg->n_scorings < 1 || cfg->max_queued < 0 || cfg->max_batch < 0 || cfg->n_streams < 0) {
    set_error("bad server config");
    return SW_EINVAL;
  }
  int rc = ensure_init();
  if (rc) return rc;
  std::unique_ptr<sw_server> s(new sw_server());
  s->device = g_ctx.device;
  s->num_cus = g_ctx.num_cus;
  s->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : ((size_t)1 << 32);
  s->max_queued = cfg->max_queued ? cfg->max_queued : 1 << 20;
  s->max_batch = cfg->max_batch ? cfg->max_batch : 16384;
  const int nst = cfg->n_streams ? cfg->n_streams : 4;
  for (int k = 0; k < cfg->n_scorings; ++k) {
    Scoring sc;
    if ((rc = prepare_scoring(&cfg->scorings[k], sc))) return rc;
    s->scorings.push_back(sc);
  }
  s->db_off.assign(cfg->db_off, cfg->db_off + cfg->n_db + 1);
  if (s->db_off[0] != 0) { set_error("bad db offsets"); return SW_EINVAL; }
  for (int r = 0; r < cfg->n_db; ++r)
    if (s->db_off[r] < 0 || s->db_off[r + 1] < s->db_off[r]) { set_error("bad db offsets"); return SW_EINVAL; }
  const int64_t nbytes = s->db_off[cfg->n_db];
  // A reference is only scored under schemes whose alphabet holds all of its
  // residues (a larger code would index past the scheme's profile); submit
  // checks this against the largest code recorded here.
  s->db_max_code.assign(cfg->n_db, 0);
  for (int r = 0; r < cfg->n_db; ++r) {
    uint8_t mx = 0;
    for (int64_t k = s->db_off[r]; k < s->db_off[r + 1]; ++k) mx = std::max(mx, cfg->db_res[k]);
    s->db_max_code[r] = mx;
  }
  if ((rc = s->db.ensure(std::max<int64_t>(nbytes, 1)))) return rc;
  if (hipSetDevice(s->device) != hipSuccess ||
      (nbytes && hipMemcpy(s->db.p, cfg->db_res, nbytes, hipMemcpyHostToDevice) != hipSuccess)) {
    set_error("server: database upload failed");
    return SW_EDEVICE;
  }
  s->queues.resize(2 * s->scorings.size());
  for (int k = 0; k < nst; ++k) s->workers.emplace_back(&sw_server::worker_main, s.get());
  *out = s.release();
  return SW_OK;
}

}  // extern "C"

namespace {

// sw_server_submit; with copy == false the request reads the caller's
// residues in place (the replay, whose buffer outlives all its requests).
int submit_impl(sw_server *s, const uint8_t *query, int32_t query_len, int32_t ref_id,
                int32_t scoring_id, uint64_t *ticket, bool copy) {
  if (!s || !ticket || query_len < 0 || (query_len > 0 && !query)) { set_error("bad submit"); return SW_EINVAL; }
  if (ref_id < 0 || ref_id + 1 >= (int64_t)s->db_off.size() || scoring_id < 0 ||
      scoring_id >= (int)s->scorings.size()) {
    set_error("ref_id or scoring_id out of range");
    return SW_EINVAL;
  }
  const Scoring &sc = s->scorings[scoring_id];
  uint8_t qmax = 0;
  for (int k = 0; k < query_len; ++k) qmax = std::max(qmax, query[k]);
  if (query_len > 0 && qmax >= sc.alpha) {
    int k = 0;
    while (query[k] < sc.alpha) ++k;
    set_error("query residue %d out of range", k);
    return SW_EINVAL;
  }
  const int64_t n = s->db_off[ref_id + 1] - s->db_off[ref_id];
  if (n > 0 && s->db_max_code[ref_id] >= sc.alpha) {
    set_error("reference %d holds residue code %d, not below scoring %d's alphabet size %d",
              ref_id, (int)s->db_max_code[ref_id], scoring_id, sc.alpha);
    return SW_EINVAL;
  }
  if (std::min<int64_t>(query_len, n) * (int64_t)sc.max_s >= 2147483647ll) {
    set_error("score may overflow int32");
    return SW_EOVERFLOW;
  }
  std::unique_ptr<Request> r(new Request());
  if (copy) {
    r->own.assign(query, query + query_len);
    r->query = r->own.data();
  } else {
    r->query = query;
  }
  r->qlen = query_len;
  r->ref_id = ref_id;
  r->scoring_id = scoring_id;
  r->klass = 2 * scoring_id + (is_long(query_len, n) ? 1 : 0);
  r->bytes = s->request_bytes(query_len, (int)n);
  if (r->bytes > s->budget) { set_error("request needs %zu bytes, budget %zu", r->bytes, s->budget); return SW_ENOMEM; }
  r->t_submit = mono_ns();
  bool wake = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) { set_error("server stopping"); return SW_EINVAL; }
    if ((int)s->table.size() >= s->max_queued) return SW_EBUSY;
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queues[r->klass].push_back(r.get());
    s->queued++;
    s->outstanding++;
    s->table.emplace(r->ticket, std::move(r));
    wake = s->idle_workers > 0;
  }
  if (wake) s->cv_work.notify_one();
  return SW_OK;
}

}  // namespace

extern "C" {

int sw_server_submit(sw_server *s, const uint8_t *query, int32_t query_len, int32_t ref_id,
                     int32_t scoring_id, uint64_t *ticket) {
  return submit_impl(s, query, query_len, ref_id, scoring_id, ticket, true);
}

int sw_server_poll(sw_server *s, uint64_t ticket, sw_result *out, int64_t *ts) {
  if (!s || !out) { set_error("bad poll"); return SW_EINVAL; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->table.find(ticket);
  if (it == s->table.end()) return SW_ENOENT;
  Request *r = it->second.get();
  if (!r->done) return SW_PENDING;
  const int st = r->status;
  *out = r->res;
  if (ts) { ts[0] = r->t_submit; ts[1] = r->t_admit; ts[2] = r->t_done; }
  s->table.erase(it);
  return st;
}

int sw_server_drain(sw_server *s) {
  if (!s) return SW_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  return SW_OK;
}

int sw_server_destroy(sw_server *s) {
  if (!s) return SW_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto &q : s->queues) q.clear();
    s->queued = 0;
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  for (auto &t : s->workers) t.join();
  hipSetDevice(s->device);
  s->db.release();
  delete s;
  return SW_OK;
}

int sw_server_replay(sw_server *s, int32_t n, const uint8_t *qres, const int64_t *qoff,
                     const int32_t *ref_id, const int32_t *scoring_id, const int64_t *arrival_ns,
                     sw_result *out, int64_t *times_ns) {
  if (!s || n < 0 || (n > 0 && (!qres || !qoff || !ref_id || !scoring_id || !arrival_ns || !out || !times_ns))) {
    set_error("bad replay arguments");
    return SW_EINVAL;
  }
  // The collector below takes the tickets of finished batches from the
  // server (one lock per wake-up) instead of polling every outstanding
  // ticket in turn; one replay at a time can collect them.
  std::vector<uint64_t> sink, work;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->done_sink) {
      set_error("another replay is running on this server");
      return SW_EBUSY;
    }
    s->done_sink = &sink;
    s->table.reserve(s->table.size() + (size_t)n);
  }
  std::vector<uint64_t> tickets(n, 0);
  std::vector<int64_t> first_try(n, 0);
  std::atomic<int> submitted{0};
  std::atomic<int> err{SW_OK};
  const int64_t t0 = mono_ns();
  std::thread producer([&] {
    for (int k = 0; k < n; ++k) {
      const int64_t due = t0 + arrival_ns[k];
      int64_t now;
      while ((now = mono_ns()) < due) {
        if (due - now > 200000) std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
      first_try[k] = mono_ns();
      int rc;
      uint64_t tk = 0;
      while ((rc = submit_impl(s, qres + qoff[k], (int32_t)(qoff[k + 1] - qoff[k]), ref_id[k],
                               scoring_id[k], &tk, false)) == SW_EBUSY)
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      if (rc != SW_OK) { err = rc; tickets[k] = 0; }
      else tickets[k] = tk;
      submitted.store(k + 1, std::memory_order_release);
    }
  });
  // Collector: matches finished tickets to request indices as the producer
  // publishes its tickets, and fetches each result with one poll.
  std::unordered_map<uint64_t, int> index;
  index.reserve((size_t)n);
  std::vector<std::pair<uint64_t, int>> matched;
  std::vector<std::unique_ptr<Request>> freed;
  int remaining = n, indexed = 0;
  while (remaining > 0) {
    const int upto = submitted.load(std::memory_order_acquire);
    for (; indexed < upto; ++indexed) {
      if (tickets[indexed] == 0) {       // rejected at submit
        out[indexed] = sw_result{0, -1, -1, 0};
        times_ns[3 * indexed + 0] = times_ns[3 * indexed + 1] = times_ns[3 * indexed + 2] =
            first_try[indexed] - t0;
        --remaining;
      } else {
        index.emplace(tickets[indexed], indexed);
      }
    }
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (sink.empty())
        s->cv_done.wait_for(lk, std::chrono::microseconds(work.empty() ? 500 : 20),
                            [&] { return !sink.empty(); });
      work.insert(work.end(), sink.begin(), sink.end());
      sink.clear();
    }
    size_t keep = 0;
    matched.clear();
    for (const uint64_t tk : work) {
      auto it = index.find(tk);
      if (it == index.end()) { work[keep++] = tk; continue; }   // submit not yet returned
      matched.emplace_back(tk, it->second);
      index.erase(it);
    }
    work.resize(keep);
    if (matched.empty()) continue;
    {
      // the finished requests of these batches, taken under one lock (their
      // records are freed after it is released)
      std::lock_guard<std::mutex> lk(s->mu);
      for (const auto &tk_k : matched) {
        auto it = s->table.find(tk_k.first);
        const int k = tk_k.second;
        times_ns[3 * k + 0] = first_try[k] - t0;
        if (it == s->table.end()) {
          err = SW_ENOENT;
          out[k] = sw_result{0, -1, -1, 0};
          times_ns[3 * k + 1] = times_ns[3 * k + 2] = times_ns[3 * k + 0];
          continue;
        }
        const Request *r = it->second.get();
        if (r->status != SW_OK) err = r->status;
        out[k] = r->res;
        times_ns[3 * k + 1] = r->t_admit - t0;
        times_ns[3 * k + 2] = r->t_done - t0;
        freed.push_back(std::move(it->second));
        s->table.erase(it);
      }
    }
    freed.clear();
    remaining -= (int)matched.size();
  }
  producer.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->done_sink = nullptr;
  }
  return err.load();
}

}  // extern "C"
