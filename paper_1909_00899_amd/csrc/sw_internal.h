// Internal structures shared by the host runtime and the gfx950 kernels of
// libswscan.so.  Not part of the public ABI (include/sw.h is).
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace swk {

constexpr int kWave = 64;          // gfx950 wavefront width
constexpr int kMaxAlpha = 32;      // largest supported alphabet
constexpr int kSlots = 8;          // slot-halves per task: 4 sub-groups x 2 int16 halves
constexpr int kBlock = 4;          // reference columns per unrolled block
constexpr int kStreamBlockBytes = kSlots * kBlock;  // residue-stream bytes per block

// A task is the unit a wavefront pops from the queue: up to four sub-groups
// (16/32/64 lanes each), each holding one alignment per int16 half (or one
// int32 alignment), all stepping through the same number of reference
// columns in lockstep.
struct Task {
  int32_t ncols;        // reference columns to run (multiple of kBlock)
  int32_t layout;       // bit r set <=> a sub-group starts at lane 16*r
  int64_t stream_off;   // byte offset of the task's residue stream
  int32_t pair[kSlots]; // PairInfo index of slot-half 2*sub_group + half, or -1
  int64_t bnd_off;      // element offset of this task's chunk boundary arrays
  int32_t mode;         // shared-query kernel: index of the lane-width mode
  int32_t nchunks;      // per-pair kernel: query chunks (same for every slot)
};
static_assert(sizeof(Task) == 64, "task layout");

struct PairInfo {
  int64_t q_off;        // query residue offset (per-pair kernel)
  int64_t r_off;        // reference residue offset
  int32_t m;            // query length
  int32_t n;            // reference length
  int32_t out;          // index of the result slot
  int32_t pad;
};
static_assert(sizeof(PairInfo) == 32, "pair layout");

struct DevResult {
  int32_t score;
  int32_t qend;
  int32_t rend;
  uint32_t flags;
};

enum : uint32_t { kFlagSaturated = 1u, kFlagNeedsI32 = 2u };

// Kernel arguments (passed by value).
struct KArgs {
  const Task *tasks;
  int32_t ntasks;
  int32_t chunk;              // shared-query kernel: query chunk of this launch
  int32_t *task_counter;      // one int, zeroed before the launch
  const PairInfo *pairs;
  const uint8_t *streams;     // residue streams ([ncols/4][8 slot-halves][4] bytes per task)
  const uint8_t *query_res;   // residues of every query (device)
  int64_t shared_q_off;       // shared-query kernel: the query
  int32_t shared_m;
  int32_t alpha;
  const int32_t *matrix;      // alpha*alpha, [query code][ref code] (device)
  int32_t gap_open;
  int32_t gap_extend;         // already min(gap_extend, gap_open)
  int32_t last_chunk;         // shared-query kernel: 1 if no chunk follows
  int32_t sat_cap;            // int16 saturation threshold (<= 32767)
  uint32_t *bnd_in;           // chunk boundaries read (shared-query kernel)
  uint32_t *bnd_out;          // chunk boundaries written
  uint32_t *bnd;              // per-pair kernel: double-buffered boundaries
  int64_t bnd_half;           // per-pair kernel: element distance between the two buffers
  DevResult *results;
  unsigned long long *stats;  // [0] column steps, [1] lazy-F inner steps, [2] record branches,
                              // [3] padded cells (device-planned launches)
  // device-planned shared-query launches (tasks are implicit, residues are
  // read from the references directly)
  const int32_t *order;       // valid pairs, longest reference first
  int32_t *plan_meta;         // kMeta* words
  const uint8_t *ref_res;     // residues of every reference (device)
  // masked shared row-pair launches (start cells): per pair (PairInfo index)
  // the number of leading rows of the shared query outside its alignment,
  // whose profile scores are capped at 0; nullptr otherwise
  const int32_t *first_row;
};

// Device planner of a single-query batch: words of the plan_meta array.
enum : int {
  kMetaValid = 0,       // pairs with m > 0 and n > 0 (entries of `order`)
  kMetaCounter = 1,     // task counter of the alignment kernel
  kMetaErrResidue = 2,  // set if a residue code is >= alpha
  kMetaErrPair = 3,     // set if a pair's query / reference id or offsets are invalid
  kMetaMaxM = 4,        // largest query length of the runnable pairs
  kMetaNeedsI32 = 5,    // int16 results that ask for the int32 rerun
  kMetaWords = 16
};
// Length bins of the planner's counting sort: bin = ceil(n / kBlock), the
// last bin also takes every longer reference.
constexpr int kPlanBins = 4096;
constexpr int kPlanBlocks = 32;   // workgroups of the planner's count and place passes

// Layout of the device planner's plan buffer, in int32 words.
constexpr int kPlanStats = 0;                                     // 8 x u64: stats words
constexpr int kPlanMeta = 16;                                     // kMetaWords
constexpr int kPlanHist = kPlanMeta + kMetaWords;                 // kPlanBlocks x kPlanBins
constexpr int kPlanOff = kPlanHist + kPlanBlocks * kPlanBins;     // kPlanBlocks x kPlanBins
constexpr int kPlanTotals = kPlanOff + kPlanBlocks * kPlanBins;   // kPlanBins
constexpr int kPlanOrder = kPlanTotals + kPlanBins;               // n_pairs
constexpr int kPlanCleared = kPlanMeta + kMetaWords;              // words cleared per call

// Host-side launchers (defined in sw_kernels.hip).
enum Prec { PREC_I16X2 = 0, PREC_I32 = 1 };
enum Alg { ALG_SCAN = 0, ALG_LAZYF = 1 };

// Shared-query kernel: every task uses the launch's query (one chunk of it).
// The menu index `menu` selects the rows-per-lane triple compiled into one
// kernel; task.mode picks 16 (seg16), 32 (seg32) or 64 (seg64) lanes.
struct SharedMenu { int seg16, seg32, seg64; };
int shared_menu_count();
SharedMenu shared_menu(int idx);
size_t shared_lds_bytes(Prec prec, int menu, int alpha);
// dual: int32 lanes (scan algorithm) with two alignments per sub-group,
// the task's even and odd slots, each with its own chunk boundaries
// ([8 slots][ncols] H words, then F words).
hipError_t launch_shared(Prec prec, Alg alg, int menu, bool chunked, bool dual, const KArgs &a,
                         int grid, hipStream_t st);

// Per-pair kernel: each slot-half has its own query; profiles live in each
// wavefront's own LDS region.  seg = rows per lane, pmax = widest sub-group.
bool pair_kernel_has(Prec prec, int seg, int pmax);
size_t pair_lds_bytes(Prec prec, int seg, int alpha);
hipError_t launch_pair(Prec prec, int seg, int pmax, bool chunked, const KArgs &a,
                       int grid, hipStream_t st);

// Residue streams for a list of tasks (SENT-padded, 4-aligned).
hipError_t launch_build_streams(const Task *tasks, int ntasks, const PairInfo *pairs,
                                const uint8_t *ref_res, uint8_t *streams, int sent_code,
                                hipStream_t st);

// p[0..n) = v.
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);

// Device planner, run by kPlanBlocks workgroups that each take a contiguous
// range of the pairs.  qoff == nullptr: one query (id 0) of length m at
// q_off0; else every pair's own query (pq, query offsets, query bytes).
// plan_count: PairInfo of every pair with its query and reference checked
// (ids in range, 0 <= off[id] <= off[id+1] <= bytes; otherwise
// meta[kMetaErrPair] is set and the pair gets m = n = 0), results set to
// {0, -1, -1, 0}, block_hist[w][bin] = the workgroup's pairs with m, n > 0 per
// length bin, stats[4] += sum of their n, stats[5] += sum of m*n,
// meta[kMetaMaxM] = their largest m.
hipError_t launch_plan_count(int n_pairs, const int64_t *qoff, int n_queries, int64_t qbytes,
                             const int64_t *roff, const int32_t *pq, const int32_t *pr, int n_refs,
                             int64_t ref_bytes, int m, int64_t q_off0, PairInfo *pairs,
                             DevResult *results, int32_t *block_hist, int32_t *meta,
                             unsigned long long *stats, hipStream_t st);
// plan_total: block_off[w][bin] = workgroup w's first position inside the
// bin, totals[bin] = pairs of the bin.
hipError_t launch_plan_total(const int32_t *block_hist, int32_t *block_off, int32_t *totals,
                             hipStream_t st);
// plan_scatter: order[...] = every pair with m, n > 0, longest reference first
// (pairs of one bin in any order); meta[kMetaValid] = number of entries,
// meta[kMetaCounter] = 0.
hipError_t launch_plan_scatter(int n_pairs, const PairInfo *pairs, const int32_t *totals,
                               const int32_t *block_off, int32_t *order, int32_t *meta,
                               hipStream_t st);
// Device-planned shared-query kernel: rows per lane `seg`, `lanes` lanes per
// alignment; a.order / a.plan_meta / a.ref_res describe the work.
bool shared_direct_has(Prec prec, int seg, int lanes);
size_t shared_direct_lds_bytes(Prec prec, int seg, int lanes, int alpha);
hipError_t launch_shared_direct(Prec prec, int seg, int lanes, const KArgs &a, int grid,
                                hipStream_t st);

// Device-planned shared-query kernel in the row-pair layout (int16 only):
// 16 lanes per alignment, each lane's two halves holding two row segments of
// `seg` rows (32*seg query rows).  grid: wavefronts wanted.
bool shared_rowpair_has(int seg);
size_t shared_rowpair_lds_bytes(int seg, int alpha);
// lrec: end-cell records in LDS (1, when they fit, else in registers), in
// registers (0), or in LDS when they fit (-1).
hipError_t launch_shared_rowpair(int seg, const KArgs &a, int grid, hipStream_t st, int lrec = -1);
bool shared_rowpair_lds_records_fit(int seg, int alpha);

// Device-planned per-pair kernel: four 16-lane sub-groups per wavefront,
// `seg` rows per lane (16*seg query rows at most), profiles per task.
// lanes 8: eight sub-groups of eight lanes (int16 lanes and byte profiles
// only).  es: profile entry bytes, 1 (scores within int8) or the lane type's.
bool pair_direct_has(int seg, int lanes);
size_t pair_direct_lds_bytes(Prec prec, int seg, int alpha, int es);
hipError_t launch_pair_direct(Prec prec, int seg, int lanes, int es, const KArgs &a, int grid,
                              hipStream_t st);

// Host-planned per-pair kernel in the row-pair layout (int16 only): one
// alignment per sub-group of `lanes` (16, 32, 64) lanes (task slot
// 2*sub_group), `seg` rows per virtual lane (2*lanes*seg query rows per
// chunk), a pair-score table of (alpha+1)^3 words in LDS instead of per-pair
// profiles (alphabets up to 24).  grid = wavefronts.
bool pair_rowpair_has(int seg, int alpha);
size_t pair_rowpair_lds_bytes(int alpha);
hipError_t launch_pair_rowpair(int seg, int lanes, bool chunked, const KArgs &a, int grid,
                               hipStream_t st);

// Swapped striping (int32): task t = pair tasks[t].pair[0] with its query
// streamed over tasks[t].ncols columns and its reference (at most 64*seg
// rows) striped over one wavefront; results to results[pairs[pid].out].
constexpr int kSwapSegs[] = {4, 8, 12, 16, 20, 24, 28, 32};
constexpr int kSwapMaxRows = 64 * 32;
bool swap_has(int seg);
size_t swap_lds_bytes(int alpha, int seg);
hipError_t launch_swap(int seg, const KArgs &a, int grid, hipStream_t st);

// Sets every result to {0, -1, -1, 0}.
hipError_t launch_init_results(int n, DevResult *r, hipStream_t st);
// *count += the entries of r[0..n) with a flag bit of `mask`.
hipError_t launch_count_flag(int n, const DevResult *r, uint32_t mask, int32_t *count,
                             hipStream_t st);
// out[k] = r32[k] with flags kFlagSaturated for every k whose out[k] has
// kFlagNeedsI32 (the int32 rerun's results merged on the device).
hipError_t launch_merge_rerun(int n, const DevResult *r32, DevResult *out, hipStream_t st);

// dst segment t = the dst_off[t+1] - dst_off[t] bytes of src from src_off[t]
// on, reversed (offsets validated by the host; n segments).
hipError_t launch_reverse_segments(int n, const uint8_t *src, const int64_t *src_off,
                                   const int64_t *dst_off, uint8_t *dst, hipStream_t st);

// PairInfo of every pair from device-resident CSR offsets (indices already
// validated by the host).
hipError_t launch_build_pairs(int n_pairs, const int64_t *qoff, const int64_t *roff,
                              const int32_t *pq, const int32_t *pr, PairInfo *out,
                              hipStream_t st);

// Sets *flag to 1 if any residue in p[0..n) is >= alpha.
hipError_t launch_check_residues(const uint8_t *p, int64_t n, int alpha, int *flag,
                                 hipStream_t st);

constexpr int kWavesPerGroup = 8;   // shared-query kernel: threads per workgroup = 512

// LDS bytes of the staged substitution matrix (alpha^2 int32, 16-byte aligned).
__host__ __device__ constexpr uint32_t matrix_lds_bytes(int alpha) {
  return (uint32_t)(((alpha * alpha * 4) + 15) / 16 * 16);
}

}  // namespace swk
