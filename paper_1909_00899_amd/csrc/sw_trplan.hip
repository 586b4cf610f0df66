// Path tables on the device (include/sw.h, sw_align_batch_cigar and
// sw_align_batch_global_cigar), and the end-to-end score tables
// (sw_align_batch_global) at the end: each pair's rectangle, its kernel variant and
// size class, the planner-made runs of end-to-end alignments with an empty
// side, the table ordered by class with a run region per entry, and after the
// path kernels the run-count check and the prefix sum of the counts.  The
// host reads two small summaries (class starts and sizes; the error word and
// the run total) instead of building the table itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "sw_internal.h"
#include "sw_trace.h"

namespace swk {
namespace dev {
namespace {

constexpr uint8_t kSkip = 0xff;
constexpr int kThreads = 256;

__device__ __forceinline__ void set_err(unsigned long long *err, int k, int code) {
  atomicMin(err, ((unsigned long long)(unsigned)k << 8) | (unsigned)code);
}

__device__ __forceinline__ int64_t gap_cost(int go, int ge, int64_t L) {
  return L <= 0 ? 0 : go + (L - 1) * (int64_t)ge;
}
__device__ __forceinline__ int64_t gap_cost(const TrPlanArgs &a, int64_t L) {
  return gap_cost(a.go, a.ge, L);
}

// Pair k's class (or kSkip) and rectangle, or a negative error code.  The
// rules are the API's (include/sw.h): mode 0 takes the rectangle between the
// start cell and the end cell of a positive score; modes 1-4 take
// r[0..ref_end] x q[0..query_end] and need the end cell of that mode.
__device__ int classify(const TrPlanArgs &a, int k, TracePair &tp) {
  const bool col_free = a.mode == 2 || a.mode == 4, row_free = a.mode == 3 || a.mode == 4;
  const DevResult e = a.ends[k];
  const int q = a.pq ? a.pq[k] : 0, r = a.pr[k];
  if (q < 0 || q >= a.nq || r < 0 || r >= a.nr) return -kTrErrPair;
  const int64_t q0 = a.qoff[q], q1 = a.qoff[q + 1], r0 = a.roff[r], r1 = a.roff[r + 1];
  // within the residue arrays too (they hold qoff[nq] and roff[nr] bytes)
  if (q0 < 0 || q1 < q0 || q1 > a.qoff[a.nq]) return -kTrErrQoff;
  if (r0 < 0 || r1 < r0 || r1 > a.roff[a.nr]) return -kTrErrRoff;
  const int64_t m = q1 - q0, n = r1 - r0;
  int qs = 0, rs = 0;
  if (a.mode == 0) {
    if (e.score <= 0) return kSkip;
    qs = a.qs[k];
    rs = a.rs[k];
    if (qs < 0 || qs > e.qend || e.qend >= m || rs < 0 || rs > e.rend || e.rend >= n)
      return -kTrErrRect;
  } else {
    const bool in = e.rend >= -1 && e.rend < n && e.qend >= -1 && e.qend < m;
    const bool on_q = e.qend == m - 1, on_r = e.rend == n - 1;
    const bool ok = a.mode == 1 ? on_q && on_r : a.mode == 2 ? on_q : a.mode == 3 ? on_r
                                                                                   : on_q || on_r;
    if (!in || !ok) return -kTrErrEnd;
    if (e.qend < 0 || e.rend < 0) {
      // nothing to pair: runs from the best virtual start element -- the
      // largest (ref, query) one -- to the end cell
      const int64_t A0 = e.rend + 1, B0 = e.qend + 1;
      int64_t best = INT64_MIN, bx = 0, by = 0;
      auto consider = [&](int64_t x, int64_t y) {
        const int64_t v = -gap_cost(a, A0 - 1 - x) - gap_cost(a, B0 - 1 - y);
        if (v > best || (v == best && (x > bx || (x == bx && y > by)))) {
          best = v;
          bx = x;
          by = y;
        }
      };
      consider(-1, -1);
      for (int64_t x = 0; col_free && x < A0; ++x) consider(x, -1);
      for (int64_t y = 0; row_free && y < B0; ++y) consider(-1, y);
      if (e.score != best) return -kTrErrOptimum;
      int nrun = 0;
      uint32_t run[2] = {0, 0};
      if (A0 - 1 - bx) run[nrun++] = (uint32_t)(A0 - 1 - bx) << 4 | kCigarD;
      if (B0 - 1 - by) run[nrun++] = (uint32_t)(B0 - 1 - by) << 4 | kCigarI;
      a.hruns[2 * (int64_t)k] = run[0];
      a.hruns[2 * (int64_t)k + 1] = run[1];
      a.ref_start[k] = (int32_t)(bx + 1);
      a.query_start[k] = (int32_t)(by + 1);
      tp.q = tp.r = tp.out = 0;
      tp.A = tp.B = 0;
      tp.score = e.score;
      tp.cap = 2;
      tp.id = k;
      tp.pad = nrun;   // planner-made entries: the run count
      return kTrHostClass;
    }
  }
  const int64_t A = e.rend - rs + 1, Bq = e.qend - qs + 1;
  // every reachable value stays above -2^28 and every row term below 2^30,
  // so unreachable values (near -2^30) never meet reachable ones
  const int64_t maxabs = a.maxabs;
  const int64_t lo = 2 * (maxabs + a.go) + (A + Bq + 2 * kTraceTileCols) * (a.ge + 1);
  const int64_t hi = (A < Bq ? A : Bq) * (int64_t)a.max_s + (Bq + kTraceTileCols) * a.ge;
  if (lo >= (1ll << 27) || hi >= (1ll << 30)) return -kTrErrRange;
  tp.q = q0 + qs;
  tp.r = r0 + rs;
  tp.out = 0;
  tp.A = (int32_t)A;
  tp.B = (int32_t)Bq;
  tp.score = e.score;
  // end-to-end: k <= min(A, B) pairs, k M runs and two gap runs in each of
  // the k + 1 gaps (start, between pairs, end)
  const int64_t mn = A < Bq ? A : Bq;
  tp.cap = (int32_t)(a.mode == 0 ? trace_run_bound(A, Bq)
                                 : (A + Bq + 2 < 3 * mn + 2 ? A + Bq + 2 : 3 * mn + 2));
  tp.id = k;
  // columns per lane: the fewest that hold a one-tile query (4 beyond)
  tp.pad = (int32_t)((Bq + 63) / 64 < 4 ? (Bq + 63) / 64 : 4);
  // 16-bit values (4 or 8 columns per lane) when the rectangle's range
  // provably fits: every reachable value -- a pair and two gap runs from the
  // start or a boundary, plus a gap opening, or a scan term with its tile
  // offset -- stays above every value derived from an unreachable edge
  // (-32768 plus a score, a tile's scan offsets and an opening), and the
  // largest chain score with its tile offset stays below 32767
  if (Bq > 64) {
    const int64_t tc = Bq <= 256 ? 256 : 512;
    const int64_t span = 5 * (maxabs + a.go) + (A + Bq + 3 + tc) * (int64_t)a.ge + 256;
    const int64_t top = mn * (int64_t)a.max_s + tc * a.ge + maxabs + 256;
    if (span < 32768 && top < 32767) tp.pad = kTracePad16 | (int32_t)(tc / 64);
  }
  const int64_t slot = trace_slot_words(tp);
  const int variant = trace_variant(tp.pad);
  if (slot <= (int64_t)kTraceLdsRowTiles * 64)
    return variant == kTraceV16x4 ? 0 : variant == kTraceV32 ? 1 : 2;
  if (slot * 2 > (2ll << 30)) return -kTrErrScratch;
  return trace_size_class(slot, variant);
}

// Workgroup w's pairs: a contiguous range, the same in classify and scatter.
__device__ __forceinline__ void block_range(int np, int w, int nw, int &lo, int &hi) {
  lo = (int)((int64_t)np * w / nw);
  hi = (int)((int64_t)np * (w + 1) / nw);
}

__global__ __launch_bounds__(kThreads) void trplan_classify_kernel(TrPlanArgs a) {
  // per class: count, largest slot and most rows, reduced in LDS first (most
  // pairs of a batch share a few classes: one global atomic per workgroup
  // and class instead of one per pair)
  __shared__ int cnt[kTrClasses];
  __shared__ unsigned long long mx[2 * kTrClasses];
  __shared__ unsigned long long caps;
  for (int c = threadIdx.x; c < kTrClasses; c += kThreads) {
    cnt[c] = 0;
    mx[2 * c] = mx[2 * c + 1] = 0;
  }
  if (threadIdx.x == 0) caps = 0;
  __syncthreads();
  int lo, hi;
  block_range(a.np, blockIdx.x, gridDim.x, lo, hi);
  unsigned long long mycaps = 0;
  for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
    if (a.mode != 0) {
      a.ref_start[k] = 0;
      a.query_start[k] = 0;
    }
    TracePair tp;
    const int c = classify(a, k, tp);
    if (c < 0) {
      set_err(a.err, k, -c);
      a.cls[k] = kSkip;
      a.n_runs[k] = 0;
      continue;
    }
    a.cls[k] = (uint8_t)c;
    a.n_runs[k] = 0;
    if (c == kSkip) continue;
    a.rect[k] = tp;
    atomicAdd(&cnt[c], 1);
    mycaps += (unsigned long long)tp.cap;
    if (c != kTrHostClass) {
      atomicMax(&mx[2 * c], (unsigned long long)trace_slot_words(tp));
      // rows that need carries: an LDS class's rectangles of two or more
      // tiles only (a device-memory class sizes its slots by every row)
      const bool one_tile = tp.B <= trace_tile_cols(tp.pad);
      atomicMax(&mx[2 * c + 1], (unsigned long long)(c < 3 && one_tile ? 0 : tp.A));
    }
  }
  atomicAdd(&caps, mycaps);
  __syncthreads();
  for (int c = threadIdx.x; c < kTrClasses; c += kThreads) {
    a.blk_count[(size_t)blockIdx.x * kTrClasses + c] = cnt[c];
    if (cnt[c]) {
      atomicMax(&a.cls_max[2 * c], mx[2 * c]);
      atomicMax(&a.cls_max[2 * c + 1], mx[2 * c + 1]);
    }
  }
  if (threadIdx.x == 0) a.blk_caps[blockIdx.x] = (int64_t)caps;
}

// One workgroup: per class the workgroups' first positions (turned into
// absolute table positions), the class starts, and per workgroup the first
// word of its run regions.
__global__ __launch_bounds__(kThreads) void trplan_totals_kernel(TrPlanArgs a) {
  __shared__ int64_t total[kTrClasses];
  const int nb = kTrBlocks;
  for (int c = threadIdx.x; c < kTrClasses; c += kThreads) {
    int64_t run = 0;
    for (int b = 0; b < nb; ++b) {
      const int v = a.blk_count[(size_t)b * kTrClasses + c];
      a.blk_count[(size_t)b * kTrClasses + c] = (int)run;
      run += v;
    }
    total[c] = run;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int c = 0; c < kTrClasses; ++c) {
      a.summary[c] = s;
      s += total[c];
    }
    a.summary[kTrClasses] = s;   // entries; the region total follows
    int64_t reg = 0;
    for (int b = 0; b < nb; ++b) {
      const int64_t v = a.blk_caps[b];
      a.blk_caps[b] = reg;
      reg += v;
    }
    a.summary[kTrClasses + 1] = reg;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kTrClasses; c += kThreads) {
    const int64_t base = a.summary[c];
    for (int b = 0; b < nb; ++b) a.blk_count[(size_t)b * kTrClasses + c] += (int)base;
  }
}

// Each workgroup places its pairs (the classify ranges) with LDS cursors: a
// table position per class, a run region from the workgroup's base.  Order
// inside a class is free (each entry's work is independent).  Planner-made
// runs go straight to the end of their region.
__global__ __launch_bounds__(kThreads) void trplan_scatter_kernel(TrPlanArgs a) {
  __shared__ int cur[kTrClasses];
  __shared__ unsigned long long reg;
  for (int c = threadIdx.x; c < kTrClasses; c += kThreads)
    cur[c] = a.blk_count[(size_t)blockIdx.x * kTrClasses + c];
  if (threadIdx.x == 0) reg = (unsigned long long)a.blk_caps[blockIdx.x];
  __syncthreads();
  int lo, hi;
  block_range(a.np, blockIdx.x, gridDim.x, lo, hi);
  for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
    const int c = a.cls[k];
    if (c == kSkip) continue;
    TracePair tp = a.rect[k];
    const int pos = atomicAdd(&cur[c], 1);
    tp.out = (int64_t)atomicAdd(&reg, (unsigned long long)tp.cap);
    a.table[pos] = tp;
    if (c == kTrHostClass) {
      const int n = tp.pad;
      for (int j = 0; j < n; ++j) a.runs[tp.out + tp.cap - n + j] = a.hruns[2 * (int64_t)k + j];
      a.n_runs[k] = n;
    }
  }
}

__global__ __launch_bounds__(kThreads) void trplan_check_kernel(const TracePair *table, int nt,
                                                                const int32_t *n_runs,
                                                                unsigned long long *err) {
  for (int t = blockIdx.x * kThreads + threadIdx.x; t < nt; t += gridDim.x * kThreads) {
    const TracePair P = table[t];
    if (P.A == 0) continue;   // planner-made runs
    const int c = n_runs[P.id];
    if (c == kTraceBadResidue) set_err(err, P.id, kTrErrResidue);
    else if (c == kTraceInconsistent) set_err(err, P.id, kTrErrInconsistent);
    else if (c < 1 || c > P.cap) set_err(err, P.id, kTrErrCount);
  }
}

// Exclusive prefix sum of per-pair counts in three passes: 4096-entry chunk
// sums, their prefix (one workgroup), then every chunk again from its base.
constexpr int kScanChunk = 4096;
constexpr int kScanPer = kScanChunk / kThreads;   // 16 entries per thread

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *lds, int64_t &total) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int d = 1; d < kThreads; d <<= 1) {
    const int64_t x = t >= d ? lds[t - d] : 0;
    __syncthreads();
    lds[t] += x;
    __syncthreads();
  }
  total = lds[kThreads - 1];
  const int64_t incl = lds[t];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kThreads) void scan_sums_kernel(const int32_t *counts, int np,
                                                             int64_t *bsum) {
  __shared__ int64_t lds[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int64_t s = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t k = base + j;
    if (k < np) s += counts[k] > 0 ? counts[k] : 0;
  }
  int64_t total;
  (void)block_excl_scan(s, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void scan_bases_kernel(int64_t *bsum, int nb) {
  __shared__ int64_t lds[kThreads];
  int64_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kThreads) {
    const int b = b0 + threadIdx.x;
    const int64_t v = b < nb ? bsum[b] : 0;
    int64_t total;
    const int64_t ex = block_excl_scan(v, lds, total);
    if (b < nb) bsum[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kThreads) void scan_write_kernel(const int32_t *counts, int np,
                                                              const int64_t *bsum, int64_t *off) {
  __shared__ int64_t lds[kThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int64_t s = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t k = base + j;
    if (k < np) s += counts[k] > 0 ? counts[k] : 0;
  }
  int64_t total;
  int64_t run = bsum[blockIdx.x] + block_excl_scan(s, lds, total);
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t k = base + j;
    if (k < np) {
      run += counts[k] > 0 ? counts[k] : 0;
      off[k + 1] = run;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[0] = 0;
}

// ---------------------------------------------------------------- start-cell tables

__global__ __launch_bounds__(kThreads) void startplan_kernel(StartPlanArgs a) {
  const int stride = gridDim.x * kThreads;
  int qmin = INT_MAX, qmax = -1;
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < a.np; k += stride) {
    const DevResult e = a.ends[k];
    int qc = 0, rc = 0;
    int64_t qs = 0, rs = 0;
    a.ids[k] = k;
    if (e.score > 0) {
      const int q = a.pq[k], r = a.pr[k];
      if (q < 0 || q >= a.nq || r < 0 || r >= a.nr) {
        set_err(a.err, k, kTrErrPair);
      } else {
        const int64_t q0 = a.qoff[q], q1 = a.qoff[q + 1], r0 = a.roff[r], r1 = a.roff[r + 1];
        if (q0 < 0 || q1 < q0 || q1 > a.qoff[a.nq]) {
          set_err(a.err, k, kTrErrQoff);
        } else if (r0 < 0 || r1 < r0 || r1 > a.roff[a.nr]) {
          set_err(a.err, k, kTrErrRoff);
        } else if (e.qend < 0 || e.qend >= q1 - q0 || e.rend < 0 || e.rend >= r1 - r0) {
          set_err(a.err, k, kSpErrEnd);
        } else {
          // the spans an alignment of this score can have (P <= the other
          // prefix's length pairs; rounding toward zero only widens them)
          const int64_t Lq = e.qend + 1, Lr = e.rend + 1;
          int64_t Qb = Lq, Rb = Lr;
          if (a.ge > 0) {
            const int64_t sr = Lq + 1 + (Lq * a.max_s - a.go - e.score) / a.ge;
            const int64_t sq = Lr + 1 + (Lr * a.max_s - a.go - e.score) / a.ge;
            Rb = min(Lr, max(Lq, sr));
            Qb = min(Lq, max(Lr, sq));
          }
          qc = (int)Qb;
          rc = (int)Rb;
          qs = q0 + (Lq - Qb);   // the prefixes' last Qb and Rb residues
          rs = r0 + (Lr - Rb);
          qmin = min(qmin, q);
          qmax = max(qmax, q);
        }
      }
    }
    a.qcnt[k] = qc;
    a.rcnt[k] = rc;
    a.qsrc[k] = qs;
    a.rsrc[k] = rs;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.qsrc[a.np] = 0;
    a.rsrc[a.np] = 0;
  }
  // one atomic pair per wavefront
  for (int d = 1; d < 64; d <<= 1) {
    qmin = min(qmin, __shfl_xor(qmin, d));
    qmax = max(qmax, __shfl_xor(qmax, d));
  }
  if ((threadIdx.x & 63) == 0 && qmax >= 0) {
    atomicMin(&a.qrange[0], qmin);
    atomicMax(&a.qrange[1], qmax);
  }
}

// ---------------------------------------------------------------- end-to-end score tables

constexpr int kE2eMulti = 3;

// Pair k's class (0 couples, 1 one 256 tile, 2 one 512 tile, 3 longer; kSkip
// with an empty side,
// whose result is written here) and table entry, or a negative error code.
// The rules are the API's (include/sw.h, sw_align_batch_global).
__device__ int e2e_classify(const E2ePlanArgs &a, int k, TracePair &tp) {
  const int q = a.pq ? a.pq[k] : 0, r = a.pr[k];
  if (q < 0 || q >= a.nq || r < 0 || r >= a.nr) return -kTrErrPair;
  const int64_t q0 = a.qoff[q], q1 = a.qoff[q + 1], r0 = a.roff[r], r1 = a.roff[r + 1];
  if (q0 < 0 || q1 < q0 || q1 > a.qoff[a.nq]) return -kTrErrQoff;
  if (r0 < 0 || r1 < r0 || r1 > a.roff[a.nr]) return -kTrErrRoff;
  const int64_t m = q1 - q0, n = r1 - r0;
  if (m == 0 || n == 0) {
    // one gap run per charged side (or none); the ends where the charged
    // sides are used up
    const bool qc = a.mode == 0 || a.mode == 1, rc = a.mode == 0 || a.mode == 2;
    const int64_t s = -(qc ? gap_cost(a.go, a.ge, m) : 0) - (rc ? gap_cost(a.go, a.ge, n) : 0);
    if (s < INT32_MIN) return -kE2eErrScore;
    DevResult res;
    res.score = (int32_t)s;
    res.qend = qc ? (int32_t)(m - 1) : -1;
    res.rend = rc ? (int32_t)(n - 1) : -1;
    res.flags = 0;
    a.out[k] = res;
    return kSkip;
  }
  // the 32-bit range of the end-to-end kernels (their unreachable values
  // near -2^30 stay below every reachable one; a tile's padding columns
  // carry scan terms too)
  const int64_t lo = 2 * ((int64_t)a.maxabs + a.go) + (m + n + 2 * kE2eWideCols) * (a.ge + 1);
  const int64_t hi = (m < n ? m : n) * (int64_t)a.max_s + (m + kE2eWideCols) * a.ge;
  if (lo >= (1ll << 27) || hi >= (1ll << 30)) return -kTrErrRange;
  tp.q = q0;
  tp.r = r0;
  tp.out = 0;
  tp.A = (int32_t)n;
  tp.B = (int32_t)m;
  tp.score = 0;
  tp.cap = 0;
  tp.id = k;
  // query columns per lane: 32 lanes per pair up to kE2eDualCols columns
  // (two pairs per wavefront), 64 lanes up to one tile of 256 or of
  // kE2eWideCols, tiles of kE2eWideCols beyond
  if (m <= kE2eDualCols) {
    tp.pad = (int32_t)((m + 31) / 32);
    return 0;
  }
  if (m <= kE2eWideCols) {
    tp.pad = (int32_t)((m + 63) / 64);
    return m <= kTraceTileCols ? 1 : 2;
  }
  // as many tiles as kE2eWideCols-column tiles would need, each as narrow as
  // covers the query (5-8 columns per lane: 640 columns for 600 residues
  // instead of 1024)
  const int64_t tiles = (m + kE2eWideCols - 1) / kE2eWideCols;
  tp.pad = (int32_t)((m + 64 * tiles - 1) / (64 * tiles));
  return kE2eMulti;
}

__global__ __launch_bounds__(kThreads) void e2eplan_classify_kernel(E2ePlanArgs a) {
  __shared__ int cnt[kE2eClasses];
  __shared__ unsigned long long rows;
  if (threadIdx.x < kE2eClasses) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) rows = 0;
  __syncthreads();
  int lo, hi;
  block_range(a.np, blockIdx.x, gridDim.x, lo, hi);
  for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
    TracePair tp;
    const int c = e2e_classify(a, k, tp);
    if (c < 0) {
      set_err(a.err, k, -c);
      a.cls[k] = kSkip;
      continue;
    }
    a.cls[k] = (uint8_t)c;
    if (c == kSkip) continue;
    atomicAdd(&cnt[c], 1);
    if (c == kE2eMulti) atomicMax(&rows, (unsigned long long)tp.A);
  }
  __syncthreads();
  if (threadIdx.x < kE2eClasses)
    a.blk_count[(size_t)blockIdx.x * kE2eClasses + threadIdx.x] = cnt[threadIdx.x];
  if (threadIdx.x == 0 && rows) atomicMax(a.rows_max, rows);
}

// One workgroup: per class the workgroups' first table positions, and the
// class starts.
__global__ __launch_bounds__(kThreads) void e2eplan_totals_kernel(E2ePlanArgs a) {
  __shared__ int64_t total[kE2eClasses];
  const int c = threadIdx.x;
  if (c < kE2eClasses) {
    int64_t run = 0;
    for (int b = 0; b < kTrBlocks; ++b) {
      const int v = a.blk_count[(size_t)b * kE2eClasses + c];
      a.blk_count[(size_t)b * kE2eClasses + c] = (int)run;
      run += v;
    }
    total[c] = run;
  }
  __syncthreads();
  if (c == 0) {
    int64_t s = 0;
    for (int k = 0; k < kE2eClasses; ++k) {
      a.summary[k] = s;
      s += total[k];
    }
    a.summary[kE2eClasses] = s;
  }
  __syncthreads();
  if (c < kE2eClasses)
    for (int b = 0; b < kTrBlocks; ++b) a.blk_count[(size_t)b * kE2eClasses + c] += (int)a.summary[c];
}

// Each workgroup places its pairs (the classify ranges) with LDS cursors;
// order inside a class is free.
__global__ __launch_bounds__(kThreads) void e2eplan_scatter_kernel(E2ePlanArgs a) {
  __shared__ int cur[kE2eClasses];
  if (threadIdx.x < kE2eClasses)
    cur[threadIdx.x] = a.blk_count[(size_t)blockIdx.x * kE2eClasses + threadIdx.x];
  __syncthreads();
  int lo, hi;
  block_range(a.np, blockIdx.x, gridDim.x, lo, hi);
  for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
    const int c = a.cls[k];
    if (c == kSkip) continue;
    TracePair tp;
    (void)e2e_classify(a, k, tp);   // a non-empty pair: only the entry is rebuilt
    a.table[atomicAdd(&cur[c], 1)] = tp;
  }
}

// Bucket of a two-pairs-per-wavefront entry: more columns per lane first,
// then more rows.
__device__ __forceinline__ int e2e_sort_key(const TracePair &tp) {
  const int pc = tp.pad < 1 ? 1 : tp.pad > 5 ? 5 : tp.pad;
  const int rows = tp.A < 0 ? 0 : tp.A < kE2eSortRows - 1 ? tp.A : kE2eSortRows - 1;
  return (5 - pc) * kE2eSortRows + (kE2eSortRows - 1 - rows);
}

// Bucket sizes: a workgroup histogram in LDS, added into hist.
__global__ __launch_bounds__(kThreads) void e2esort_count_kernel(const TracePair *in, int n,
                                                                 int32_t *hist) {
  __shared__ int cnt[kE2eSortBins];
  for (int b = threadIdx.x; b < kE2eSortBins; b += kThreads) cnt[b] = 0;
  __syncthreads();
  int lo, hi;
  block_range(n, blockIdx.x, gridDim.x, lo, hi);
  for (int k = lo + threadIdx.x; k < hi; k += kThreads) atomicAdd(&cnt[e2e_sort_key(in[k])], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kE2eSortBins; b += kThreads)
    if (cnt[b]) atomicAdd(&hist[b], cnt[b]);
}

// One workgroup: the bucket sizes turned into bucket starts, in place.
__global__ __launch_bounds__(kThreads) void e2esort_scan_kernel(int32_t *hist) {
  static_assert(kE2eSortBins % kThreads == 0, "buckets per thread");
  constexpr int kPer = kE2eSortBins / kThreads;
  __shared__ int part[kThreads];
  const int b0 = threadIdx.x * kPer;
  int s = 0;
  for (int j = 0; j < kPer; ++j) s += hist[b0 + j];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < kThreads; ++t) {
      const int v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int j = 0; j < kPer; ++j) {
    const int v = hist[b0 + j];
    hist[b0 + j] = run;
    run += v;
  }
}

// Each workgroup reserves its share of every bucket with one atomic and
// places its entries there with LDS cursors.
__global__ __launch_bounds__(kThreads) void e2esort_scatter_kernel(const TracePair *in, int n,
                                                                   int32_t *start,
                                                                   TracePair *out) {
  __shared__ int cur[kE2eSortBins];
  for (int b = threadIdx.x; b < kE2eSortBins; b += kThreads) cur[b] = 0;
  __syncthreads();
  int lo, hi;
  block_range(n, blockIdx.x, gridDim.x, lo, hi);
  for (int k = lo + threadIdx.x; k < hi; k += kThreads) atomicAdd(&cur[e2e_sort_key(in[k])], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kE2eSortBins; b += kThreads)
    if (cur[b]) cur[b] = atomicAdd(&start[b], cur[b]);
  __syncthreads();
  for (int k = lo + threadIdx.x; k < hi; k += kThreads) {
    const TracePair tp = in[k];
    out[atomicAdd(&cur[e2e_sort_key(tp)], 1)] = tp;
  }
}

__global__ __launch_bounds__(kThreads) void e2e_check_kernel(const DevResult *res, int np,
                                                             unsigned long long *err) {
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < np; k += gridDim.x * kThreads)
    if (res[k].flags & kFlagBadResidue) set_err(err, k, kTrErrResidue);
}

}  // namespace
}  // namespace dev

hipError_t launch_startplan(const StartPlanArgs &a, hipStream_t st) {
  if (a.np <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(((int64_t)a.np + dev::kThreads - 1) / dev::kThreads, 2048);
  hipLaunchKernelGGL(dev::startplan_kernel, dim3(grid), dim3(dev::kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_e2eplan_classify(const E2ePlanArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(dev::e2eplan_classify_kernel, dim3(kTrBlocks), dim3(dev::kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_e2eplan_totals(const E2ePlanArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(dev::e2eplan_totals_kernel, dim3(1), dim3(dev::kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_e2eplan_scatter(const E2ePlanArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(dev::e2eplan_scatter_kernel, dim3(kTrBlocks), dim3(dev::kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_e2e_sort(const TracePair *in, int n, int32_t *hist, TracePair *out,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(kTrBlocks, ((int64_t)n + 2047) / 2048);
  hipLaunchKernelGGL(dev::e2esort_count_kernel, dim3(grid), dim3(dev::kThreads), 0, st, in, n,
                     hist);
  hipLaunchKernelGGL(dev::e2esort_scan_kernel, dim3(1), dim3(dev::kThreads), 0, st, hist);
  hipLaunchKernelGGL(dev::e2esort_scatter_kernel, dim3(grid), dim3(dev::kThreads), 0, st, in, n,
                     hist, out);
  return hipGetLastError();
}

hipError_t launch_e2e_check(const DevResult *res, int np, unsigned long long *err,
                            hipStream_t st) {
  if (np <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(((int64_t)np + dev::kThreads - 1) / dev::kThreads, 4096);
  hipLaunchKernelGGL(dev::e2e_check_kernel, dim3(grid), dim3(dev::kThreads), 0, st, res, np, err);
  return hipGetLastError();
}

hipError_t launch_trplan_classify(const TrPlanArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(dev::trplan_classify_kernel, dim3(kTrBlocks), dim3(dev::kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_trplan_totals(const TrPlanArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(dev::trplan_totals_kernel, dim3(1), dim3(dev::kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_trplan_scatter(const TrPlanArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(dev::trplan_scatter_kernel, dim3(kTrBlocks), dim3(dev::kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_trplan_check(const TracePair *table, int nt, const int32_t *n_runs,
                               unsigned long long *err, hipStream_t st) {
  if (nt <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(((int64_t)nt + dev::kThreads - 1) / dev::kThreads, 4096);
  hipLaunchKernelGGL(dev::trplan_check_kernel, dim3(grid), dim3(dev::kThreads), 0, st, table, nt,
                     n_runs, err);
  return hipGetLastError();
}

hipError_t launch_count_scan(const int32_t *counts, int np, int64_t *off, int64_t *bsum,
                             hipStream_t st) {
  if (np <= 0) return hipSuccess;
  const int nb = (int)(((int64_t)np + dev::kScanChunk - 1) / dev::kScanChunk);
  hipLaunchKernelGGL(dev::scan_sums_kernel, dim3(nb), dim3(dev::kThreads), 0, st, counts, np, bsum);
  hipLaunchKernelGGL(dev::scan_bases_kernel, dim3(1), dim3(dev::kThreads), 0, st, bsum, nb);
  hipLaunchKernelGGL(dev::scan_write_kernel, dim3(nb), dim3(dev::kThreads), 0, st, counts, np,
                     bsum, off);
  return hipGetLastError();
}

}  // namespace swk
