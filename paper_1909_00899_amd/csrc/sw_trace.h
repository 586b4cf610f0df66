// Paths and end-to-end scores (sw_trace.hip): shared between the kernels
// and the host code that plans their launches (sw_starts.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_internal.h"

namespace swk {

constexpr int kTraceTileCols = 256;      // query columns per tile at 4 columns per lane
constexpr int kTraceLdsRowTiles = 160;   // rows x tiles of 2-byte decision words that fit in LDS
constexpr int kTraceLdsCarryRows = 80;   // a rectangle of two or more tiles in LDS has <= 80 rows
constexpr int kCigarM = 0, kCigarI = 1, kCigarD = 2;
constexpr int kTraceInconsistent = -2;   // no alignment of the given score from start to end
constexpr int kTraceBadResidue = -3;     // a residue code >= alphabet size in the rectangle

// One rectangle: query residues qres[q .. q + B), reference residues
// rres[r .. r + A); its runs are written backward from cigar[out + cap - 1]
// (first run of the path last); the count goes to n_runs[id], or
// kTraceInconsistent / kTraceBadResidue.
// pad: query columns per lane in the low bits, 1-4 (a tile of 64 * pad
// columns), 32-bit values; with kTracePad16 set, 4 or 8 columns per lane
// whose values fit 16 bits (two adjacent columns per register; the host
// checks the rectangle's value range).
constexpr int kTracePad16 = 16;
__host__ __device__ constexpr int trace_cols(int pad) { return pad & (kTracePad16 - 1); }
__host__ __device__ constexpr int trace_tile_cols(int pad) { return 64 * trace_cols(pad); }
// bytes of one lane's decision word per row (4 bits per column)
__host__ __device__ constexpr int trace_word_bytes(int pad) { return trace_cols(pad) > 4 ? 4 : 2; }
// kernel variants: every pair of one launch has the same one
constexpr int kTraceV32 = 0, kTraceV16x4 = 1, kTraceV16x8 = 2;
__host__ __device__ constexpr int trace_variant(int pad) {
  return (pad & kTracePad16) ? (trace_cols(pad) == 8 ? kTraceV16x8 : kTraceV16x4) : kTraceV32;
}
struct TracePair {
  int64_t q, r, out;
  int32_t A, B, score, cap, id, pad;
};

// Runs a local path can have between start and end: every run but the first
// is preceded by a change of operation, M runs alternate with one or two gap
// runs, and a rectangle of A x B cells holds at most min(A, B) pairs.
__host__ __device__ inline int64_t trace_run_bound(int64_t A, int64_t B) {
  return A + B - 1 < 3 * (A < B ? A : B) - 2 ? A + B - 1 : 3 * (A < B ? A : B) - 2;
}
// Lanes per row of a rectangle's decision words: a one-tile rectangle keeps
// only the lanes that hold its columns (rounded up to 8, so a row is a whole
// number of 16-byte units), a longer one all 64.
__host__ __device__ inline int trace_lane_stride(int B, int C) {
  if (B > 64 * C) return 64;
  const int nl = (B > 0 ? B + C - 1 : C) / C;
  const int r = (nl + 7) / 8 * 8;
  return r < 64 ? r : 64;
}
// 2-byte units of a rectangle's decision words: rows x tiles x its lane
// stride x the word width of its variant (constant divisors)
__host__ __device__ inline int64_t trace_slot_words(const TracePair &P) {
  int64_t tiles;
  switch (trace_cols(P.pad)) {
    case 1: tiles = (P.B + 63) / 64; break;
    case 2: tiles = (P.B + 127) / 128; break;
    case 3: tiles = (P.B + 191) / 192; break;
    case 8: tiles = (P.B + 511) / 512; break;
    default: tiles = (P.B + 255) / 256; break;
  }
  return (int64_t)P.A * tiles * trace_lane_stride(P.B, trace_cols(P.pad)) *
         (trace_word_bytes(P.pad) / 2);
}

// ---- path tables on the device (sw_trplan.hip)
//
// Every pair is classified once: no path (a local alignment of score <= 0),
// runs made by the planner itself (an end-to-end alignment with an empty
// side: at most a D and an I run from the best virtual start element), or a
// rectangle of one of the classes below; a pair that breaks the API's rules
// sets an error word (the smallest pair index wins).  Classes: the three LDS
// variants (16-bit x4, 32-bit, 16-bit x8: one launch each), then device-
// memory rectangles by variant and power of two below their slot, largest
// first (any member needs more than half its class's largest slot: one
// launch group per class), then the planner-made runs.
constexpr int kTrBuckets = 40;                         // slots below 2^40 words
constexpr int kTrClasses = 3 + 3 * kTrBuckets + 1;
constexpr int kTrHostClass = kTrClasses - 1;
constexpr int kTrBlocks = 256;                         // classify / scatter workgroups
__host__ __device__ inline int trace_size_class(int64_t slot, int variant) {
  int b = 0;
  for (int64_t s = slot; s > 1 && b + 1 < kTrBuckets; s >>= 1) ++b;
  return 3 + (kTrBuckets - 1 - b) * 3 + variant;
}
// error codes of the planner's error word (pair index << 8 | code)
enum : int {
  kTrErrRect = 1,        // mode 0: start and end are not a rectangle of the pair
  kTrErrEnd = 2,         // modes 1-4: not an end cell of that mode
  kTrErrOptimum = 3,     // modes 1-4, empty side: the score is not the optimum
  kTrErrRange = 4,       // the rectangle leaves the 32-bit range of the path kernel
  kTrErrScratch = 5,     // more than 2 GiB of decision bits
  kTrErrPair = 6,        // pair index out of range
  kTrErrQoff = 7,        // the pair's query offsets decrease or are negative
  kTrErrRoff = 8,        // the pair's reference offsets decrease or are negative
  kTrErrResidue = 9,     // after the path kernels: a residue code >= alphabet size
  kTrErrInconsistent = 10,
  kTrErrCount = 11,      // a run count outside 1..cap
};
struct TrPlanArgs {
  int np, nq, nr, mode, alpha, go, ge, max_s, maxabs;
  const int64_t *qoff, *roff;        // device
  const int32_t *pq, *pr;            // device; pq may be null (query 0)
  const DevResult *ends;             // device copy of the caller's results
  const int32_t *qs, *rs;            // device copies of the start cells (mode 0)
  TracePair *rect;                   // per pair: its rectangle (scratch)
  uint8_t *cls;                      // per pair: its class, or 0xff (no path)
  uint32_t *hruns;                   // per pair: planner-made runs (2 words)
  int32_t *n_runs;                   // per pair: run count (0 without a path)
  int32_t *ref_start, *query_start;  // modes 1-4: start element + 1 per pair
  int32_t *blk_count;                // [kTrBlocks][kTrClasses]
  int64_t *blk_caps;                 // [kTrBlocks] run capacity per workgroup
  unsigned long long *cls_max;       // [kTrClasses][2]: largest slot, most rows
  unsigned long long *err;           // error word (initialised to ~0)
  int64_t *summary;                  // [kTrClasses + 2]: class starts, entries, region total
  TracePair *table;                  // the entries by class, with run regions
  uint32_t *runs;                    // run regions (planner-made runs written here)
};
// classify + workgroup histograms; totals (class starts, workgroup cursors,
// region bases); scatter.  The host reads the summary between totals and
// scatter (it sizes the run regions and the launches).
hipError_t launch_trplan_classify(const TrPlanArgs &a, hipStream_t st);
hipError_t launch_trplan_totals(const TrPlanArgs &a, hipStream_t st);
hipError_t launch_trplan_scatter(const TrPlanArgs &a, hipStream_t st);
// after the path kernels: every rectangle's run count checked (error word),
// and off[0..np] = the exclusive prefix sum of the per-pair counts
// (negative ones as 0); off[np] is the total; bsum: (np + 4095) / 4096 + 1
// scratch entries
hipError_t launch_trplan_check(const TracePair *table, int nt, const int32_t *n_runs,
                               unsigned long long *err, hipStream_t st);
hipError_t launch_count_scan(const int32_t *counts, int np, int64_t *off, int64_t *bsum,
                             hipStream_t st);

// Start-cell tables on the device for one query per pair
// (sw_align_batch_starts): per pair k the lengths of the reversed prefixes it
// aligns (0 without an alignment) and their sources, the identity index, the
// first error (indices, offsets, an end cell outside the pair) and the
// smallest and largest query id of a pair with an alignment.  A prefix is cut
// to the span an alignment of the pair's score can have: every alignment of
// that score inside the prefixes ends at the end cell (the first maximum), so
// reversed it starts at the origin, and with P pairs it spans at most
// P + 1 + (P max_s - go - score) / ge residues of either sequence.
enum : int { kSpErrEnd = 13 };
struct StartPlanArgs {
  int np, nq, nr;
  int go, ge, max_s;                     // ge = min(gap_extend, gap_open); max_s >= 0
  const DevResult *ends;                 // device copy of the caller's results
  const int64_t *qoff, *roff;
  const int32_t *pq, *pr;
  int32_t *qcnt, *rcnt, *ids;            // [np]
  int64_t *qsrc, *rsrc;                  // [np + 1]
  unsigned long long *err;               // error word (initialised to ~0)
  int32_t *qrange;                       // {min, max} (initialised to {INT_MAX, -1})
};
hipError_t launch_startplan(const StartPlanArgs &a, hipStream_t st);

// End-to-end score tables on the device (sw_align_batch_global): each pair
// checked and put in a class -- couples of queries up to kE2eDualCols
// residues, queries of one 256-column tile, of one kE2eWideCols tile, longer
// ones in tiles of kE2eWideCols -- or, with an empty side, its
// result written at once; workgroup histograms, class starts, the table.
constexpr int kE2eClasses = 4;        // couples, one 256 tile, one 512 tile, 512 tiles
constexpr int kE2eDualCols = 160;
constexpr int kE2eWideCols = 512;
enum : int { kE2eErrScore = 12 };   // an empty side's score below the int32 range
struct E2ePlanArgs {
  int np, nq, nr, mode, go, ge, max_s, maxabs;   // mode: the API's (0-3)
  const int64_t *qoff, *roff;                    // device
  const int32_t *pq, *pr;                        // device; pq may be null (query 0)
  DevResult *out;                                // per pair; empty sides written here
  uint8_t *cls;                                  // per pair: its class or 0xff
  int32_t *blk_count;                            // [kTrBlocks][kE2eClasses]
  unsigned long long *rows_max;                  // most rows of a longer-query pair
  unsigned long long *err;                       // error word (initialised to ~0)
  int64_t *summary;                              // [kE2eClasses + 1]: class starts, entries
  TracePair *table;
};
// classify + histograms; totals; scatter (the host reads the summary and the
// error word between totals and scatter)
hipError_t launch_e2eplan_classify(const E2ePlanArgs &a, hipStream_t st);
hipError_t launch_e2eplan_totals(const E2ePlanArgs &a, hipStream_t st);
hipError_t launch_e2eplan_scatter(const E2ePlanArgs &a, hipStream_t st);
// The two-pairs-per-wavefront class reordered so that a wavefront's two
// pairs have the same columns per lane and similar row counts (a couple runs
// its longer pair's rows at its wider pair's columns), most columns and rows
// first: a counting sort of in[0 .. n) into out over (pad, rows) buckets,
// rows from kE2eSortRows - 1 on sharing one; hist holds kE2eSortBins
// counters that the caller zeroes; the order inside a bucket is free.
constexpr int kE2eSortRows = 1024;
constexpr int kE2eSortBins = 5 * kE2eSortRows;   // pad 1-5
hipError_t launch_e2e_sort(const TracePair *in, int n, int32_t *hist, TracePair *out,
                           hipStream_t st);
// after the kernels: the first pair whose result has kFlagBadResidue
hipError_t launch_e2e_check(const DevResult *res, int np, unsigned long long *err,
                            hipStream_t st);

struct TraceArgs {
  const TracePair *pairs;
  int n;
  const uint8_t *qres, *rres;
  const int32_t *matrix;   // alpha x alpha, [query code][ref code], device
  int alpha, go, ge;       // ge <= go
  uint16_t *gbits;         // device-memory variant: slot_words 2-byte units per workgroup
  int64_t slot_words;
  int lds_words;           // LDS variant: 2-byte units of LDS for decision words, a
                           // multiple of 8 and >= every pair's trace_slot_words
  int32_t *gcarry;         // device-memory variant: 6 * carry_rows per workgroup
  int carry_rows;          // rows of carries (LDS variant: in LDS, 0 when every
                           // rectangle of the launch is one tile)
  uint32_t *cigar;         // device
  int32_t *n_runs;         // device, indexed by TracePair::id
  int mode;                // 0 local rectangle; 1-4 the end-to-end mode + 1 (global,
                           // semi-global query fitted, semi-global reference fitted,
                           // overlap)
  int32_t *ref_start;      // modes 1-4: the start element's coordinates + 1, device,
  int32_t *query_start;    // indexed by TracePair::id
};

// LDS bytes of a workgroup (the matrix sized for the alphabet); with
// lds_bits the decision bits and tile carries live in LDS, else in gbits /
// gcarry (grid-stride over the pairs).
size_t trace_lds_bytes(bool lds_bits, int alpha, int lds_words, int carry_rows);
// every pair of a.pairs[0 .. a.n) must have trace_variant(pad) == variant
hipError_t launch_trace(bool lds_bits, int variant, const TraceArgs &a, int grid, hipStream_t st);
// End-to-end scores (sw_trace.hip): TracePair with A = n, B = m (both >= 1);
// results to out[id] (flags kFlagBadResidue for a residue >= alphabet size).
constexpr int kFlagBadResidue = 1 << 20;
struct EndArgs {
  const TracePair *pairs;
  int n;
  const uint8_t *qres, *rres;
  const int32_t *matrix;
  int alpha, go, ge;
  int32_t *gcarry;         // 4 * carry_rows per workgroup (pairs of two or more tiles)
  int carry_rows;
  DevResult *out;
};
size_t endtoend_lds_bytes(int alpha);
hipError_t launch_endtoend(int mode, const EndArgs &a, int grid, hipStream_t st);
// Pairs with m <= 160, two per wavefront; pad = ceil(m / 32).
hipError_t launch_endtoend2(int mode, const EndArgs &a, hipStream_t st);
// Pairs with m > 256: pad = 5-8 query columns per lane (tiles of 64 pad
// columns: one up to 512 residues, beyond that ceil(m / 512) tiles).
hipError_t launch_endtoend_wide(int mode, const EndArgs &a, int grid, hipStream_t st);

// Runs of every pair (n_runs[id] of them, ending at out + cap) to
// dst[dst_off[id] ..]; every count must be <= its pair's cap.
hipError_t launch_pack_runs(const TracePair *pairs, int n, const int32_t *n_runs,
                            const int64_t *dst_off, const uint32_t *src, uint32_t *dst,
                            hipStream_t st);

}  // namespace swk
