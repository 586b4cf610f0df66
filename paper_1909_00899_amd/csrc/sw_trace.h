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

struct TraceArgs {
  const TracePair *pairs;
  int n;
  const uint8_t *qres, *rres;
  const int32_t *matrix;   // alpha x alpha, [query code][ref code], device
  int alpha, go, ge;       // ge <= go
  uint16_t *gbits;         // device-memory variant: slot_words 2-byte units per workgroup
  int64_t slot_words;
  int32_t *gcarry;         // device-memory variant: 6 * carry_rows per workgroup
  int carry_rows;
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
size_t trace_lds_bytes(bool lds_bits, int alpha);
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

// Runs of every pair (n_runs[id] of them, ending at out + cap) to
// dst[dst_off[id] ..]; every count must be <= its pair's cap.
hipError_t launch_pack_runs(const TracePair *pairs, int n, const int32_t *n_runs,
                            const int64_t *dst_off, const uint32_t *src, uint32_t *dst,
                            hipStream_t st);

}  // namespace swk
