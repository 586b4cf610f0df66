// Alignment paths (include/sw.h, sw_align_batch_cigar).
//
// The paper's kernels return only the maximum (Algorithm 6 keeps Max); the
// path of the reported alignment is this library's extension.  With its start
// and end cell known, the path lies in the rectangle between them and every
// cell of it is scored relative to the start pair (no zero floor).  Writing
// a = reference index and b = query index inside the rectangle, s(a, b) the
// substitution score and g(k) = go + (k - 1) ge the cost of a k-gap run:
//
//   M(a, b)  = s(a, b) + V(a-1, b-1)        (M(0, 0) = s(0, 0); other edge pairs unreachable)
//   Eg(a, b) = max(M(a, b-1) - go, Eg(a, b-1) - ge)      query residues skipped along row a
//   G(a, b)  = max(M(a, b), Eg(a, b))                    best "pair, then query gap" in row a
//   Fv(a, b) = max(G(a-1, b) - go, Fv(a-1, b) - ge)      reference residues skipped down column b
//   V(a, b)  = max(G(a, b), Fv(a, b))
//
// V(a, b) is the best score of a chain from the start whose last pair (x, y)
// satisfies x <= a, y <= b, counting the gaps to (a, b): exactly Gotoh's H
// anchored at the start, with the two gap states ordered so that a walk back
// from V meets the reference gap first and the query gap second.  Preferring
// G over Fv and an opening over an extension therefore picks, before each
// aligned pair, the predecessor pair with the largest reference index, then
// the largest query index: the path rule of the library (sw.h).
//
// Layout: one wavefront per pair; the query span is cut into tiles of 256
// columns, four consecutive columns per lane.  A row of a tile costs one
// four-column pass per lane plus one max-plus scan over the 64 lanes for Eg
// (Eg(a, b) = max_{y<b} (M(a, y) + y ge) - go - (b - 1) ge, the scan of the
// paper's Fscan turned along the row) and DPP moves for the diagonal.  Four
// decision bits per cell are kept -- in LDS when the rectangle fits, in a
// per-wavefront slot of device memory otherwise -- and the wavefront then
// walks them back from the end cell, writing CIGAR runs.
//
// End-to-end scores (sw_align_batch_global) reuse the row step without the
// decision bits: the same recurrences over the whole pair with the boundary of
// a global alignment (row -1 and column -1 priced as gap runs from a virtual
// pair at (-1, -1)) or of a semi-global one (column -1 free: a virtual pair at
// every (a, -1)), and the score read at the last column.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sw_internal.h"
#include "sw_trace.h"

namespace swk {
namespace dev {
namespace {

constexpr int kNeg = -(1 << 30);     // unreachable edge; every reachable value stays above -2^28
constexpr int kWalkRows = 64;        // rows of one tile in the walk window (8 KiB)

__device__ __forceinline__ int dpp_wave_shr1(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, 0x138, 0xf, 0xf, false);
}
// lanes without a source (and rows the mask leaves out) read INT_MIN, the
// identity of max, so each step fuses into one v_max_i32 with a DPP operand
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_move(int x) {
  return __builtin_amdgcn_update_dpp((int)0x80000000, x, CTRL, ROWMASK, 0xf, false);
}

// inclusive max over lanes 0..lane
__device__ __forceinline__ int wave_max_scan(int x) {
  x = max(x, dpp_move<0x111, 0xf>(x));   // row_shr:1
  x = max(x, dpp_move<0x112, 0xf>(x));   // row_shr:2
  x = max(x, dpp_move<0x114, 0xf>(x));   // row_shr:4
  x = max(x, dpp_move<0x118, 0xf>(x));   // row_shr:8
  x = max(x, dpp_move<0x142, 0xa>(x));   // row_bcast:15 into rows 1 and 3
  x = max(x, dpp_move<0x143, 0xc>(x));   // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ int readlane(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

// LDS words of the staged matrix: alpha^2, rounded up to 16 bytes
__host__ __device__ constexpr int mat_words(int alpha) { return (alpha * alpha + 3) / 4 * 4; }

// One pair at C query columns per lane (a tile of 64 C columns).  MODE 0:
// the rectangle between a local alignment's start and end pair, anchored at
// the start pair; MODE 1-4: a whole end-to-end alignment in the API's mode
// MODE - 1 (global, semi-global either way, overlap: the boundaries of
// endtoend_kernel) over r[0..ref_end] x q[0..query_end], walked back from
// its end cell to a virtual start element.
template <bool LB, int C, int MODE>
__device__ __forceinline__ void trace_one(const TraceArgs &a, const TracePair &P, const int *smat,
                                          uint16_t *lbits, int *lcarry, uint16_t *lwin) {
  // row -1 free: virtual pairs (-1, j) (query prefix free); column -1 free:
  // virtual pairs (i, -1) (reference prefix free)
  constexpr bool kRowFree = MODE == 3 || MODE == 4, kColFree = MODE == 2 || MODE == 4;
  constexpr int TC = 64 * C;
  const int L = threadIdx.x;
  const int alpha = a.alpha, go = a.go, ge = a.ge;
  const int A = P.A, B = P.B, T = (B + TC - 1) / TC;
  uint16_t *bits = LB ? lbits : a.gbits + (size_t)blockIdx.x * a.slot_words;
  int *carry = LB ? lcarry : a.gcarry + (size_t)blockIdx.x * 6 * a.carry_rows;
  const int crow = LB ? kTraceLdsCarryRows : a.carry_rows;
  bool bad = false, ok = false;

  for (int t = 0; t < T; ++t) {
    const int base = t * TC, jc0 = base + C * L;
    const int *cr = carry + ((t + 1) & 1) * 3 * crow;   // written by tile t - 1
    int *cw = carry + (t & 1) * 3 * crow;                // read by tile t + 1
    int qb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int code = jc0 + c < B ? (int)a.qres[P.q + jc0 + c] : 0;
      bad |= code >= alpha;
      qb[c] = min(code, alpha - 1) * alpha;
    }
    int Vp[C], Gp[C], Fp[C], wj[C], ej[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      // row -1: nothing (MODE 0), the gap run of the first j + 1 query
      // residues, or a free query prefix (a virtual pair at (-1, j))
      Vp[c] = Gp[c] = MODE == 0 ? kNeg : kRowFree ? 0 : -(go + (jc0 + c) * ge);
      Fp[c] = kNeg;
      wj[c] = (jc0 + c) * ge;              // scan term offset of column j
      ej[c] = go + (jc0 + c - 1) * ge;     // Eg(., j) = prefix max - go - (j - 1) ge
    }
    // V(-1, base - 1)
    int cv_prev = MODE == 0 ? kNeg : base == 0 || kRowFree ? 0 : -(go + (base - 1) * ge);
    int rreg = 0, crv = kNeg, crm = kNeg, crp = kNeg;
    for (int i = 0; i < A; ++i) {
      if ((i & 63) == 0) {                   // 64 rows of residues (and carries) at a time
        const int row = i + L;
        rreg = row < A ? (int)a.rres[P.r + row] : 0;
        if (t == 0) bad |= rreg >= alpha;
        if (t > 0 && row < A) {
          crv = cr[3 * row];
          crm = cr[3 * row + 1];
          crp = cr[3 * row + 2];
        }
      }
      const int rc = min(readlane(rreg, i & 63), alpha - 1);
      // column -1 (tile 0): V(i, -1), M(i, -1) and its scan term: nothing in
      // MODE 0; the reference gap run from the virtual start (-1, -1); or a
      // virtual start pair at (i, -1) (free reference prefix)
      const int cv_in = t ? readlane(crv, i & 63) : MODE == 0 ? kNeg : kColFree ? 0 : -(go + i * ge);
      const int cm_in = t ? readlane(crm, i & 63) : kColFree ? 0 : kNeg;
      const int cp_in = t ? readlane(crp, i & 63) : kColFree ? -ge : kNeg;
      int Mv[C];
      // no clamps below: every cell off row 0 and column 0 is reachable
      // (gaps from the start), so unreachable values only arise next to
      // the kNeg edges and never drift (the host bounds the rest)
      const int d0 = dpp_wave_shr1(cv_prev, Vp[C - 1]);
#pragma unroll
      for (int c = 0; c < C; ++c) Mv[c] = smat[qb[c] + rc] + (c ? Vp[c - 1] : d0);
      if (MODE == 0 && i == 0 && jc0 == 0) Mv[0] = smat[qb[0] + rc];   // the start pair
      int w[C], lp[C];
#pragma unroll
      for (int c = 0; c < C; ++c) w[c] = Mv[c] + wj[c];
      lp[0] = kNeg;
#pragma unroll
      for (int c = 1; c < C; ++c) lp[c] = c == 1 ? w[0] : max(lp[c - 1], w[c - 1]);
      const int agg = C == 1 ? w[0] : max(lp[C - 1], w[C - 1]);
      const int exc = max(dpp_wave_shr1(kNeg, wave_max_scan(agg)), cp_in);
      const int m_left = dpp_wave_shr1(cm_in, Mv[C - 1]);      // M(i, jc0 - 1)
      uint32_t word = 0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int eg = max(exc, lp[c]) - ej[c];
        const int mprev = c ? Mv[c - 1] : m_left;
        const int g = max(Mv[c], eg);
        const int fo = Gp[c] - go, fe = Fp[c] - ge;
        const int f = max(fo, fe);
        const int v = max(g, f);
        const uint32_t nib = (uint32_t)(g >= f) | (uint32_t)(fo >= fe) << 1 |
                             (uint32_t)(Mv[c] >= eg) << 2 | (uint32_t)(mprev - go == eg) << 3;
        word |= nib << (4 * c);
        Vp[c] = v;
        Gp[c] = g;
        Fp[c] = f;
      }
      bits[((size_t)t * A + i) * 64 + L] = (uint16_t)word;
      if (t + 1 < T && L == 63) {
        cw[3 * i] = Vp[C - 1];
        cw[3 * i + 1] = Mv[C - 1];
        cw[3 * i + 2] = max(exc, agg);
      }
      cv_prev = cv_in;
      if (t == T - 1 && i == A - 1) {
        // the end pair's M (MODE 0) or the end cell's V reaches the score
        const int jb = B - 1 - jc0;
        int mend = MODE == 0 ? Mv[0] : Vp[0];
#pragma unroll
        for (int c = 1; c < C; ++c)
          if (jb == c) mend = MODE == 0 ? Mv[c] : Vp[c];
        ok = __ballot(jb >= 0 && jb < C && mend == P.score) != 0;
      }
    }
    // carries and bits are read back by this same wavefront: a workgroup-
    // scope fence (wait for its own stores) is enough; an agent-scope one
    // would write back the L2 of the XCD on every tile
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
  bad = __ballot(bad) != 0;

  // ---- walk back from the end pair; runs written backward from the end of
  // the pair's region (the last run of the path at out + cap - 1)
  int nrun = 0;
  bool fail = !ok || bad;
  const int64_t end = P.out + P.cap;
  auto emit = [&](uint32_t v) {
    if (nrun < P.cap && L == 0) a.cigar[end - 1 - nrun] = v;
    ++nrun;
  };
  // device-memory bits are read through an LDS window of kWalkRows rows of
  // one tile (the walk only moves up and left): one coalesced copy per
  // window instead of a dependent device-memory load per step
  int w_tile = -1, w_lo = 0;
  auto nib_at = [&](int i, int j) -> int {
    const int t = j / TC, col = (j % TC) / C;
    uint32_t wd;
    if (LB) {
      wd = bits[((size_t)t * A + i) * 64 + col];
    } else {
      if (t != w_tile || i < w_lo || i >= w_lo + kWalkRows) {
        w_tile = t;
        w_lo = max(0, i - kWalkRows + 1);
        const int rows = min(kWalkRows, A - w_lo);
        const uint4 *src = (const uint4 *)(bits + ((size_t)t * A + w_lo) * 64);
        uint4 *dst = (uint4 *)lwin;
        for (int k = L; k < rows * 8; k += 64) dst[k] = src[k];
      }
      wd = lwin[(i - w_lo) * 64 + col];
    }
    return (int)(wd >> (4 * (j % C))) & 15;
  };
  // Runs of plain diagonal steps (a pair whose predecessor is the pair just
  // up-left: V = G = M, bits 0 and 2 of the nibble) are found 64 cells at a
  // time: lane k reads the nibble of (i - k, j - k), and the run is the
  // number of consecutive plain cells from lane 0 on (one LDS read per lane
  // instead of a dependent read per step).  A cell outside the rectangle,
  // or (device-memory bits) outside the window the caller loaded for (i, j),
  // ends the run; the step-by-step walk continues from there.
  auto diag_run = [&](int i, int j) -> int {
    const int ii = i - L, jj = j - L;
    bool in = ii >= 0 && jj >= 0;
    if (!LB) in = in && jj / TC == w_tile && ii >= w_lo;
    int nib = 0;
    if (in) {
      const int t = jj / TC, col = (jj % TC) / C;
      const uint32_t wd = LB ? (uint32_t)bits[((size_t)t * A + ii) * 64 + col]
                             : (uint32_t)lwin[(ii - w_lo) * 64 + col];
      nib = (int)(wd >> (4 * (jj % C))) & 15;
    }
    const uint64_t plain = __ballot(in && (nib & 5) == 5);
    return plain == ~0ull ? 64 : __builtin_ctzll(~plain);
  };
  // the virtual start element: (vstart, -1) or (-1, qvstart)
  int vstart = -1, qvstart = -1;
  if (!fail && MODE != 0) {
    // from the end cell (state V); pairs are counted into M runs, the gaps
    // between two elements (the end, pairs, the virtual start) into one D
    // and one I run; reaching row -1 or column -1 ends the walk
    int i = A - 1, j = B - 1, mrun = 0, guard = A + B + 2;
    for (;;) {
      if (--guard < 0) { fail = true; break; }
      while (i >= 0 && j >= 0) {            // pairs of a diagonal run
        if (!LB) (void)nib_at(i, j);         // the window holds (i, j)
        const int n = diag_run(i, j);
        mrun += n;
        i -= n;
        j -= n;
        if (n < 64) break;
      }
      int nd = 0, ni = 0;
      bool start = false;
      if (i < 0 || j < 0) {                  // on the boundary: to the virtual start
        if (i >= 0 && kColFree) vstart = i;           // V(i, -1) = 0: a free reference prefix
        else if (i >= 0) nd = i + 1;                  // the reference gap run from (-1, -1)
        else if (kRowFree) qvstart = j;               // V(-1, j) = 0: a free query prefix
        else ni = j + 1;                              // row -1: the query gap run
        start = true;
      } else {
        int nib = nib_at(i, j);
        if (!(nib & 1)) {                    // a reference gap ends at (i, j)
          for (;;) {
            ++nd;
            const bool open = nib & 2;
            if (--i < 0) {                   // G(-1, j): row -1 (a run, or a virtual pair)
              if (!open) fail = true;
              if (kRowFree) qvstart = j;
              else ni = j + 1;
              start = true;
              break;
            }
            nib = nib_at(i, j);
            if (open) break;
          }
        }
        if (!fail && !start && !(nib & 4)) { // a query gap ends at (i, j)
          for (;;) {
            ++ni;
            const bool open = nib & 8;
            if (--j < 0) {                   // M(i, -1): a virtual start pair
              if (!open || !kColFree) fail = true;
              vstart = i;
              start = true;
              break;
            }
            nib = nib_at(i, j);
            if (open) break;
          }
        }
      }
      if (fail) break;
      if (nd | ni) {
        if (mrun) emit((uint32_t)mrun << 4 | kCigarM);
        if (ni) emit((uint32_t)ni << 4 | kCigarI);
        if (nd) emit((uint32_t)nd << 4 | kCigarD);
        mrun = 0;
      }
      if (start) break;
      ++mrun;                                // the pair (i, j)
      --i;
      --j;
    }
    if (!fail && mrun) emit((uint32_t)mrun << 4 | kCigarM);
  }
  if (!fail && MODE == 0) {
    int ra = A - 1, qb_ = B - 1, mrun = 1, guard = A + B + 2;
    while ((ra | qb_) != 0) {
      while (ra > 0 && qb_ > 0) {           // predecessors along a diagonal run
        if (!LB) (void)nib_at(ra - 1, qb_ - 1);   // the window holds (ra-1, qb_-1)
        const int n = diag_run(ra - 1, qb_ - 1);
        mrun += n;
        ra -= n;
        qb_ -= n;
        if (n < 64) break;
      }
      if ((ra | qb_) == 0) break;
      if (ra == 0 || qb_ == 0 || --guard < 0) { fail = true; break; }
      int i = ra - 1, j = qb_ - 1, nd = 0, ni = 0;
      int nib = nib_at(i, j);
      if (!(nib & 1)) {                      // a reference gap ends at (i, j)
        for (;;) {
          ++nd;
          const bool open = nib & 2;
          if (--i < 0) { fail = true; break; }
          nib = nib_at(i, j);
          if (open) break;
        }
        if (fail) break;
      }
      if (!(nib & 4)) {                      // a query gap ends at (i, j)
        for (;;) {
          ++ni;
          const bool open = nib & 8;
          if (--j < 0) { fail = true; break; }
          nib = nib_at(i, j);
          if (open) break;
        }
        if (fail) break;
      }
      if (nd | ni) {
        emit((uint32_t)mrun << 4 | kCigarM);
        if (ni) emit((uint32_t)ni << 4 | kCigarI);
        if (nd) emit((uint32_t)nd << 4 | kCigarD);
        mrun = 0;
      }
      ++mrun;
      ra = i;
      qb_ = j;
    }
    if (!fail) emit((uint32_t)mrun << 4 | kCigarM);
  }
  if (L == 0) {
    a.n_runs[P.id] = bad ? kTraceBadResidue : fail ? kTraceInconsistent : nrun;
    if (MODE != 0) {
      a.ref_start[P.id] = vstart + 1;
      a.query_start[P.id] = qvstart + 1;
    }
  }
}

template <bool LB, int MODE>
__device__ __forceinline__ void trace_mode(const TraceArgs &a, const TracePair &P, const int *smat,
                                           uint16_t *lbits, int *lcarry, uint16_t *lwin) {
  switch (P.pad) {
    case 1: trace_one<LB, 1, MODE>(a, P, smat, lbits, lcarry, lwin); break;
    case 2: trace_one<LB, 2, MODE>(a, P, smat, lbits, lcarry, lwin); break;
    case 3: trace_one<LB, 3, MODE>(a, P, smat, lbits, lcarry, lwin); break;
    default: trace_one<LB, 4, MODE>(a, P, smat, lbits, lcarry, lwin); break;
  }
}

// C per pair from TracePair::pad: the fewest columns per lane that cover a
// one-tile query, so short queries leave few lanes idle.
template <bool LB>
__global__ __launch_bounds__(64) void trace_kernel(TraceArgs a) {
  extern __shared__ int smem[];
  int *smat = smem;                                            // [query code][ref code]
  // the matrix takes alpha^2 words (16-byte aligned), the bits follow
  uint16_t *lbits = (uint16_t *)(smem + mat_words(a.alpha));
  int *lcarry = (int *)(lbits + kTraceLdsRowTiles * 64);
  uint16_t *lwin = lbits;                                      // walk window (device-memory bits)
  for (int k = threadIdx.x; k < a.alpha * a.alpha; k += 64) smat[k] = a.matrix[k];
  __syncthreads();
  for (int p = blockIdx.x; p < a.n; p += gridDim.x) {
    const TracePair P = a.pairs[p];
    switch (a.mode) {
      case 0: trace_mode<LB, 0>(a, P, smat, lbits, lcarry, lwin); break;
      case 1: trace_mode<LB, 1>(a, P, smat, lbits, lcarry, lwin); break;
      case 2: trace_mode<LB, 2>(a, P, smat, lbits, lcarry, lwin); break;
      case 3: trace_mode<LB, 3>(a, P, smat, lbits, lcarry, lwin); break;
      default: trace_mode<LB, 4>(a, P, smat, lbits, lcarry, lwin); break;
    }
  }
}

// End-to-end modes (the API's): 0 global, 1 semi-global with the query end
// to end (column -1 free: a virtual pair at every (i, -1)), 2 semi-global
// with the reference end to end (row -1 free: a virtual pair at every
// (-1, j), entering the column gap), 3 overlap (both free).
template <int MODE> struct EndMode {
  static constexpr bool kRowFree = MODE == 2 || MODE == 3;   // query prefix free
  static constexpr bool kColFree = MODE == 1 || MODE == 3;   // reference prefix free
  static constexpr bool kEndCol = MODE == 1 || MODE == 3;    // ends on the query's last column
  static constexpr bool kEndRow = MODE == 2 || MODE == 3;    // ends on the reference's last row
};

// (v, col) of the larger value, the smaller column on ties: the end cells of
// the last row in (ref_end, query_end) order.  Lanes xor-paired within `width`.
template <int WIDTH>
__device__ __forceinline__ void argmax_first(int &v, int &col) {
#pragma unroll
  for (int d = 1; d < WIDTH; d <<= 1) {
    const int ov = __shfl_xor(v, d), oc = __shfl_xor(col, d);
    if (ov > v || (ov == v && oc < col)) {
      v = ov;
      col = oc;
    }
  }
}

// End-to-end score of each pair (modes of EndMode); one wavefront per pair,
// the query in tiles of 256 columns as in trace_kernel, V and the scan total
// of each tile's last column carried per row in the wavefront's slot of
// gcarry.
template <int MODE, int C>
__device__ __forceinline__ void endtoend_one(const EndArgs &a, const TracePair &P,
                                             const int *smat) {
  using EM = EndMode<MODE>;
  constexpr int TC = 64 * C;
  const int L = threadIdx.x;
  const int alpha = a.alpha, go = a.go, ge = a.ge;
  const int A = P.A, B = P.B, T = (B + TC - 1) / TC;
  int *carry = a.gcarry + (size_t)blockIdx.x * 4 * a.carry_rows;
  bool bad = false;
  // end cells on the last column: the best V(a, B-1) over a = -1 .. A-1
  // (overlap: .. A-2, the last row's cells follow), the first one on ties
  int best = EM::kRowFree ? 0 : -(go + (B - 1) * ge), best_row = -1, score = 0;
  // end cells on the last row: V(A-1, b) over b = -1 .. B-1 (this lane's columns)
  int rbest = EM::kColFree ? 0 : -(go + (A - 1) * ge), rcol = -1;
  for (int t = 0; t < T; ++t) {
    const int base = t * TC, jc0 = base + C * L;
    const int *cr = carry + ((t + 1) & 1) * 2 * a.carry_rows;
    int *cw = carry + (t & 1) * 2 * a.carry_rows;
    int qb[C], Vp[C], Gp[C], Fp[C], wj[C], ej[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int code = jc0 + c < B ? (int)a.qres[P.q + jc0 + c] : 0;
      bad |= code >= alpha;
      qb[c] = min(code, alpha - 1) * alpha;
      // row -1: the first j + 1 query residues skipped, or a free prefix
      Vp[c] = Gp[c] = EM::kRowFree ? 0 : -(go + (jc0 + c) * ge);
      Fp[c] = kNeg;
      wj[c] = (jc0 + c) * ge;
      ej[c] = go + (jc0 + c - 1) * ge;
    }
    // V(-1, base - 1): the virtual pair, or the row -1 gap run
    int cv_prev = base == 0 || EM::kRowFree ? 0 : -(go + (base - 1) * ge);
    int rreg = 0, crv = kNeg, crp = kNeg;
    for (int i = 0; i < A; ++i) {
      if ((i & 63) == 0) {
        const int row = i + L;
        rreg = row < A ? (int)a.rres[P.r + row] : 0;
        if (t == 0) bad |= rreg >= alpha;
        if (t > 0 && row < A) {
          crv = cr[2 * row];
          crp = cr[2 * row + 1];
        }
      }
      const int rc = min(readlane(rreg, i & 63), alpha - 1);
      // column -1: V(i, -1) and the scan term of M(i, -1)
      const int cv_in = t ? readlane(crv, i & 63) : (EM::kColFree ? 0 : -(go + i * ge));
      const int cp_in = t ? readlane(crp, i & 63) : (EM::kColFree ? -ge : kNeg);
      int Mv[C];
      const int d0 = dpp_wave_shr1(cv_prev, Vp[C - 1]);
#pragma unroll
      for (int c = 0; c < C; ++c) Mv[c] = smat[qb[c] + rc] + (c ? Vp[c - 1] : d0);
      int w[C], lp[C];
#pragma unroll
      for (int c = 0; c < C; ++c) w[c] = Mv[c] + wj[c];
      lp[0] = kNeg;
#pragma unroll
      for (int c = 1; c < C; ++c) lp[c] = c == 1 ? w[0] : max(lp[c - 1], w[c - 1]);
      const int agg = C == 1 ? w[0] : max(lp[C - 1], w[C - 1]);
      const int exc = max(dpp_wave_shr1(kNeg, wave_max_scan(agg)), cp_in);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int g = max(Mv[c], max(exc, lp[c]) - ej[c]);
        const int f = max(Gp[c] - go, Fp[c] - ge);
        Vp[c] = max(g, f);
        Gp[c] = g;
        Fp[c] = f;
      }
      if (t + 1 < T && L == 63) {
        cw[2 * i] = Vp[C - 1];
        cw[2 * i + 1] = max(exc, agg);
      }
      cv_prev = cv_in;
      if (t == T - 1) {
        const int jb = B - 1 - jc0;
        int v = Vp[0];
#pragma unroll
        for (int c = 1; c < C; ++c)
          if (jb == c) v = Vp[c];
        if (EM::kEndCol && (MODE == 1 || i < A - 1) && v > best) {
          best = v;
          best_row = i;
        }
        score = v;
      }
      if (EM::kEndRow && i == A - 1) {
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (jc0 + c < B && Vp[c] > rbest) {
            rbest = Vp[c];
            rcol = jc0 + c;
          }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");   // carries before tile t + 1
  }
  bad = __ballot(bad) != 0;
  if (EM::kEndRow) argmax_first<64>(rbest, rcol);
  const int jb = B - 1 - (T - 1) * TC - C * L;
  if (jb >= 0 && jb < C) {
    DevResult r;
    r.score = MODE == 0 ? score : MODE == 1 ? best : MODE == 2 ? rbest : max(best, rbest);
    // overlap: a last-column end precedes every last-row end in (ref, query) order
    const bool on_col = MODE == 0 || MODE == 1 || (MODE == 3 && best >= rbest);
    r.qend = on_col ? B - 1 : rcol;
    r.rend = MODE == 0 ? A - 1 : on_col ? best_row : A - 1;
    r.flags = bad ? kFlagBadResidue : 0;
    a.out[P.id] = r;
  }
}

// inclusive max over the lanes 0..l of each 32-lane half
__device__ __forceinline__ int half_max_scan(int x) {
  x = max(x, dpp_move<0x111, 0xf>(x));   // row_shr:1
  x = max(x, dpp_move<0x112, 0xf>(x));   // row_shr:2
  x = max(x, dpp_move<0x114, 0xf>(x));   // row_shr:4
  x = max(x, dpp_move<0x118, 0xf>(x));   // row_shr:8
  x = max(x, dpp_move<0x142, 0xa>(x));   // row_bcast:15 into rows 1 and 3
  return x;
}

// Two one-tile pairs per wavefront, 32 lanes each (lanes 0-31 the first,
// 32-63 the second), C query columns per lane: the row's scan and bookkeeping
// serve both pairs, which halves their share per pair.  The wavefront runs
// the longer pair's rows; the other half's extra rows change nothing it
// reports.  Boundaries and results as in endtoend_one.
template <int MODE, int C>
__device__ __forceinline__ void endtoend_two(const EndArgs &a, const TracePair &P0,
                                             const TracePair &P1, bool has1, const int *smat) {
  using EM = EndMode<MODE>;
  const int L = threadIdx.x, l = L & 31;
  const bool h = L >= 32;
  const int alpha = a.alpha, go = a.go, ge = a.ge;
  // this half's pair, field by field
  const int A = h ? (has1 ? P1.A : 0) : P0.A;
  const int B = h ? P1.B : P0.B;
  const int64_t pq = h ? P1.q : P0.q;
  const int64_t pr = h ? P1.r : P0.r;
  const int pid = h ? P1.id : P0.id;
  const int Amax = max(P0.A, has1 ? P1.A : 0);
  const int jc0 = C * l;
  bool bad = false;
  int qb[C], Vp[C], Gp[C], Fp[C], wj[C], ej[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int code = jc0 + c < B ? (int)a.qres[pq + jc0 + c] : 0;
    bad |= code >= alpha;
    qb[c] = min(code, alpha - 1) * alpha;
    Vp[c] = Gp[c] = EM::kRowFree ? 0 : -(go + (jc0 + c) * ge);
    Fp[c] = kNeg;
    wj[c] = (jc0 + c) * ge;
    ej[c] = go + (jc0 + c - 1) * ge;
  }
  int best = EM::kRowFree ? 0 : -(go + (B - 1) * ge), best_row = -1, score = 0;
  int rbest = EM::kColFree ? 0 : -(go + (A - 1) * ge), rcol = -1;
  int cv_prev = 0, rreg = 0;
  for (int i = 0; i < Amax; ++i) {
    if ((i & 31) == 0) {                     // 32 rows of each pair's residues at a time
      const int row = i + l;
      rreg = row < A ? (int)a.rres[pr + row] : 0;
      bad |= rreg >= alpha;
    }
    const int r0 = readlane(rreg, i & 31), r1 = readlane(rreg, 32 + (i & 31));
    const int rc = min(h ? r1 : r0, alpha - 1);
    const int cv_in = EM::kColFree ? 0 : -(go + i * ge);
    const int cp_in = EM::kColFree ? -ge : kNeg;
    const int dsh = dpp_wave_shr1(cv_prev, Vp[C - 1]);
    const int d0 = l == 0 ? cv_prev : dsh;
    int Mv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Mv[c] = smat[qb[c] + rc] + (c ? Vp[c - 1] : d0);
    int w[C], lp[C];
#pragma unroll
    for (int c = 0; c < C; ++c) w[c] = Mv[c] + wj[c];
    lp[0] = kNeg;
#pragma unroll
    for (int c = 1; c < C; ++c) lp[c] = c == 1 ? w[0] : max(lp[c - 1], w[c - 1]);
    const int agg = C == 1 ? w[0] : max(lp[C - 1], w[C - 1]);
    const int sh = dpp_wave_shr1(kNeg, half_max_scan(agg));
    const int exc = max(l == 0 ? kNeg : sh, cp_in);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int g = max(Mv[c], max(exc, lp[c]) - ej[c]);
      const int f = max(Gp[c] - go, Fp[c] - ge);
      Vp[c] = max(g, f);
      Gp[c] = g;
      Fp[c] = f;
    }
    cv_prev = cv_in;
    const int jb = B - 1 - jc0;
    int v = Vp[0];
#pragma unroll
    for (int c = 1; c < C; ++c)
      if (jb == c) v = Vp[c];
    if (i < A) {
      if (EM::kEndCol && (MODE == 1 || i < A - 1) && v > best) {
        best = v;
        best_row = i;
      }
      score = v;
    }
    if (EM::kEndRow && i == A - 1) {
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (jc0 + c < B && Vp[c] > rbest) {
          rbest = Vp[c];
          rcol = jc0 + c;
        }
    }
  }
  const uint64_t bb = __ballot(bad);
  const bool bad_h = h ? (bb >> 32) != 0 : (bb & 0xffffffffull) != 0;
  if (EM::kEndRow) argmax_first<32>(rbest, rcol);   // within each 32-lane half
  const int jb = B - 1 - jc0;
  if (jb >= 0 && jb < C && (!h || has1)) {
    DevResult r;
    r.score = MODE == 0 ? score : MODE == 1 ? best : MODE == 2 ? rbest : max(best, rbest);
    const bool on_col = MODE == 0 || MODE == 1 || (MODE == 3 && best >= rbest);
    r.qend = on_col ? B - 1 : rcol;
    r.rend = MODE == 0 ? A - 1 : on_col ? best_row : A - 1;
    r.flags = bad_h ? kFlagBadResidue : 0;
    a.out[pid] = r;
  }
}

// Couples of pairs with m <= 160 (pairs[2p], pairs[2p + 1]); TracePair::pad
// holds ceil(m / 32) and a couple runs at the larger of its two (at most 5
// columns per lane keeps the kernel's registers at several wavefronts per SIMD).
template <int MODE>
__global__ __launch_bounds__(64) void endtoend2_kernel(EndArgs a) {
  extern __shared__ int smem[];
  int *smat = smem;
  for (int k = threadIdx.x; k < a.alpha * a.alpha; k += 64) smat[k] = a.matrix[k];
  __syncthreads();
  for (int p = blockIdx.x; 2 * p < a.n; p += gridDim.x) {
    const TracePair P0 = a.pairs[2 * p];
    const bool has1 = 2 * p + 1 < a.n;
    const TracePair P1 = a.pairs[has1 ? 2 * p + 1 : 2 * p];
    switch (max(P0.pad, P1.pad)) {
      case 1: endtoend_two<MODE, 1>(a, P0, P1, has1, smat); break;
      case 2: endtoend_two<MODE, 2>(a, P0, P1, has1, smat); break;
      case 3: endtoend_two<MODE, 3>(a, P0, P1, has1, smat); break;
      case 4: endtoend_two<MODE, 4>(a, P0, P1, has1, smat); break;
      default: endtoend_two<MODE, 5>(a, P0, P1, has1, smat); break;
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(64) void endtoend_kernel(EndArgs a) {
  extern __shared__ int smem[];
  int *smat = smem;
  for (int k = threadIdx.x; k < a.alpha * a.alpha; k += 64) smat[k] = a.matrix[k];
  __syncthreads();
  for (int p = blockIdx.x; p < a.n; p += gridDim.x) {
    const TracePair P = a.pairs[p];
    switch (P.pad) {   // query columns per lane
      case 1: endtoend_one<MODE, 1>(a, P, smat); break;
      case 2: endtoend_one<MODE, 2>(a, P, smat); break;
      case 3: endtoend_one<MODE, 3>(a, P, smat); break;
      default: endtoend_one<MODE, 4>(a, P, smat); break;
    }
  }
}

// Pair t's runs (the last n_runs[id] entries of its region) to
// cigar_dst[dst_off[id] ..]; a workgroup per pair, grid-stride.
__global__ __launch_bounds__(256) void pack_runs_kernel(const TracePair *pairs, int n,
                                                        const int32_t *n_runs,
                                                        const int64_t *dst_off,
                                                        const uint32_t *src, uint32_t *dst) {
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const TracePair P = pairs[t];
    const int cnt = min(n_runs[P.id], P.cap);   // the host checked every count already
    const int64_t s0 = P.out + P.cap - cnt, d0 = dst_off[P.id];
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) dst[d0 + k] = src[s0 + k];
  }
}

}  // namespace
}  // namespace dev

size_t trace_lds_bytes(bool lds_bits, int alpha) {
  size_t b = (size_t)dev::mat_words(alpha) * sizeof(int);
  if (lds_bits) b += (size_t)kTraceLdsRowTiles * 64 * sizeof(uint16_t) + 6 * kTraceLdsCarryRows * sizeof(int);
  else b += (size_t)dev::kWalkRows * 64 * sizeof(uint16_t);
  return b;
}

size_t endtoend_lds_bytes(int alpha) { return (size_t)dev::mat_words(alpha) * sizeof(int); }

hipError_t launch_endtoend2(int mode, const EndArgs &a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(((int64_t)a.n + 1) / 2, 1 << 30);
  const size_t lds = endtoend_lds_bytes(a.alpha);
  switch (mode) {
    case 0: hipLaunchKernelGGL(dev::endtoend2_kernel<0>, dim3(grid), dim3(64), lds, st, a); break;
    case 1: hipLaunchKernelGGL(dev::endtoend2_kernel<1>, dim3(grid), dim3(64), lds, st, a); break;
    case 2: hipLaunchKernelGGL(dev::endtoend2_kernel<2>, dim3(grid), dim3(64), lds, st, a); break;
    case 3: hipLaunchKernelGGL(dev::endtoend2_kernel<3>, dim3(grid), dim3(64), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_endtoend(int mode, const EndArgs &a, int grid, hipStream_t st) {
  if (a.n <= 0 || grid <= 0) return hipSuccess;
  const size_t lds = endtoend_lds_bytes(a.alpha);
  switch (mode) {
    case 0: hipLaunchKernelGGL(dev::endtoend_kernel<0>, dim3(grid), dim3(64), lds, st, a); break;
    case 1: hipLaunchKernelGGL(dev::endtoend_kernel<1>, dim3(grid), dim3(64), lds, st, a); break;
    case 2: hipLaunchKernelGGL(dev::endtoend_kernel<2>, dim3(grid), dim3(64), lds, st, a); break;
    case 3: hipLaunchKernelGGL(dev::endtoend_kernel<3>, dim3(grid), dim3(64), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pack_runs(const TracePair *pairs, int n, const int32_t *n_runs,
                            const int64_t *dst_off, const uint32_t *src, uint32_t *dst,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::pack_runs_kernel, dim3(std::min(n, 65535)), dim3(256), 0, st, pairs, n,
                     n_runs, dst_off, src, dst);
  return hipGetLastError();
}

hipError_t launch_trace(bool lds_bits, const TraceArgs &a, int grid, hipStream_t st) {
  if (a.n <= 0 || grid <= 0) return hipSuccess;
  if (lds_bits)
    hipLaunchKernelGGL(dev::trace_kernel<true>, dim3(grid), dim3(64), trace_lds_bytes(true, a.alpha),
                       st, a);
  else
    hipLaunchKernelGGL(dev::trace_kernel<false>, dim3(grid), dim3(64),
                       trace_lds_bytes(false, a.alpha), st, a);
  return hipGetLastError();
}

}  // namespace swk
