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
#include <type_traits>

#include "sw_internal.h"
#include "sw_trace.h"

namespace swk {
namespace dev {
namespace {

constexpr int kNeg = -(1 << 30);     // unreachable edge; every reachable value stays above -2^28

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
// the same matrix as 16-bit entries, after it (alpha^2 shorts, 16-byte rounded)
__host__ __device__ constexpr int mat16_words(int alpha) { return (alpha * alpha + 7) / 8 * 4; }
constexpr int kWalkWindowBytes = 8192;  // LDS window of the walk over device-memory bits

// ---------------------------------------------------------------- 16-bit fill
//
// Rectangles whose values provably fit 16 bits (the host checks the range)
// keep two adjacent columns per 32-bit register, the even column in the low
// half, and run the row step on packed saturating 16-bit operations: half the
// VALU instructions of the 32-bit step per cell.  The lane scan stays a
// fused 32-bit DPP scan of one value per lane.  A decision bit is the sign of
// a packed difference (x - y < 0 exactly when x >= y fails; saturation keeps
// the sign); one v_perm_b32 with sign-replicating selectors gathers the four
// signs of two registers into four bytes, and one and-or places them, so a
// row's decision word costs two instructions per decision and register pair.
constexpr int kNeg16 = -32768;          // unreachable; reachable values stay far above

typedef short tr16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t padd(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(__builtin_bit_cast(tr16x2, a),
                                                                    __builtin_bit_cast(tr16x2, b)));
}
__device__ __forceinline__ uint32_t psub(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(tr16x2, a),
                                                                    __builtin_bit_cast(tr16x2, b)));
}
__device__ __forceinline__ uint32_t pmax(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(tr16x2, a),
                                                                __builtin_bit_cast(tr16x2, b)));
}
__device__ __forceinline__ uint32_t ppack(int lo, int hi) {
  return ((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16);
}
__device__ __forceinline__ uint32_t psplat(int v) { return ((uint32_t)v & 0xffffu) * 0x10001u; }
__device__ __forceinline__ int plo(uint32_t x) { return (int)(short)(x & 0xffffu); }
__device__ __forceinline__ int phi(uint32_t x) { return (int)x >> 16; }
// (x.hi, x.hi)
__device__ __forceinline__ uint32_t phi2(uint32_t x) { return __builtin_amdgcn_perm(x, x, 0x03020302u); }
// (lo.hi, hi.lo): for each of hi's two columns, the column before it
__device__ __forceinline__ uint32_t pshift(uint32_t hi, uint32_t lo) {
  return __builtin_amdgcn_alignbit(hi, lo, 16);
}
// bytes 0-3 = 0xff where the sign bit of (x.lo, x.hi, y.lo, y.hi) is set
__device__ __forceinline__ uint32_t psigns(uint32_t x, uint32_t y) {
  return __builtin_amdgcn_perm(x, y, 0x09080B0Au);
}
__device__ __forceinline__ uint32_t dpp_shr1_u(uint32_t old, uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, 0x138, 0xf, 0xf, false);
}

// Nibble of column c (of the lane's C) in its decision word: 4c for 32-bit
// values; with 16-bit values the order the byte gather leaves.
template <int C, bool W16>
__device__ __forceinline__ int nib_shift(int c) {
  if constexpr (!W16) return 4 * c;
  else if constexpr (C == 4) return 8 * (c & 1) + 4 * (c >> 1);
  else return 8 * (c & 3) + 4 * (c >> 2);
}

// Fills the decision words of rectangle P at C = 4 or 8 columns per lane in
// 16-bit values (the recurrences of the 32-bit fill in trace_one, in the same
// notation).  The Eg scan runs per tile in the tile's frame: the term of
// column j is M(a, j) + (j - base) ge, so every term stays in 16 bits;
// a tile passes V, M and the scan total (already in the next tile's frame)
// of its last column per row.
template <int C, int MODE, bool FIRST, bool NEXT, class Word>
__device__ __forceinline__ void fill16_tile(const TraceArgs &a, const TracePair &P,
                                            const short *smat16, Word *bits, int LS, const int *cr,
                                            int *cw, int t, bool &bad, bool &ok) {
  constexpr bool kRowFree = MODE == 3 || MODE == 4, kColFree = MODE == 2 || MODE == 4;
  constexpr int NP = C / 2, TC = 64 * C;
  const int L = threadIdx.x;
  const int alpha = a.alpha, go = a.go, ge = a.ge;
  const int A = P.A, B = P.B;
  const bool last_tile = !NEXT;
  const int base = t * TC, jr0 = C * L, jc0 = base + jr0;
  const uint32_t go2 = psplat(go), ge2 = psplat(ge), negw = 0x80008000u;
  int qoff[C];   // [query code][.] row of the 16-bit matrix for each column
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int code = jc0 + c < B ? (int)a.qres[P.q + jc0 + c] : 0;
    bad |= code >= alpha;
    qoff[c] = min(code, alpha - 1) * alpha;
  }
  uint32_t Vp[NP], Gp[NP], Fp[NP], wj[NP], ej[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int j0 = jc0 + 2 * p;
    // row -1: nothing (MODE 0), the query gap run, or a free query prefix
    const int v0 = MODE == 0 ? kNeg16 : kRowFree ? 0 : -(go + j0 * ge);
    const int v1 = MODE == 0 ? kNeg16 : kRowFree ? 0 : -(go + (j0 + 1) * ge);
    Vp[p] = Gp[p] = ppack(v0, v1);
    Fp[p] = psplat(kNeg16);
    wj[p] = ppack((jr0 + 2 * p) * ge, (jr0 + 2 * p + 1) * ge);
    ej[p] = ppack(go + (jr0 + 2 * p - 1) * ge, go + (jr0 + 2 * p) * ge);
  }
  // V(-1, base - 1); in MODE 0 the first tile's V(-1, -1) = 0 makes the
  // start pair's M its own score
  int cv_prev = MODE == 0 ? (FIRST ? 0 : kNeg16) : (FIRST || kRowFree) ? 0 : -(go + (base - 1) * ge);
  Word *brow = bits + (size_t)t * A * LS + L;   // lanes past LS hold no column
  for (int blk = 0; blk < A; blk += 64) {
    const int row = blk + L;
    int rreg = row < A ? (int)a.rres[P.r + row] : 0;
    if (FIRST) bad |= rreg >= alpha;
    rreg = min(rreg, alpha - 1);
    // column -1 of the tile for the block's rows: the previous tile's carry,
    // or the boundary (nothing in MODE 0, the reference gap run from the
    // virtual start, or a free reference prefix)
    int crv, crm, crp;
    if (FIRST) {
      crv = MODE == 0 ? kNeg16 : kColFree ? 0 : -(go + row * ge);
      crm = kColFree ? 0 : kNeg16;
      crp = kColFree ? -ge : kNeg16;
    } else {
      crv = row < A ? cr[3 * row] : kNeg16;
      crm = row < A ? cr[3 * row + 1] : kNeg16;
      crp = row < A ? cr[3 * row + 2] : kNeg16;
    }
    const int nr = min(64, A - blk);
    for (int ii = 0; ii < nr; ++ii) {
      const int i = blk + ii;
      const int rc = readlane(rreg, ii);
      const int cv_in = readlane(crv, ii), cm_in = readlane(crm, ii);
      const int cp_in = readlane(crp, ii);
      uint32_t s2[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p)
        s2[p] = ppack(smat16[qoff[2 * p] + rc], smat16[qoff[2 * p + 1] + rc]);
      // the diagonal: V(i-1, j-1), the left lane's last column (or the
      // carry) for the lane's first one
      const uint32_t vleft = dpp_shr1_u((uint32_t)cv_prev << 16, Vp[NP - 1]);
      uint32_t Mv[NP], w[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        Mv[p] = padd(s2[p], pshift(Vp[p], p ? Vp[p - 1] : vleft));
        w[p] = padd(Mv[p], wj[p]);
      }
      // exclusive prefix maxima of the scan terms inside the lane
      uint32_t I[NP], lp[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const uint32_t r = pmax(w[p], pshift(w[p], negw));
        I[p] = p ? pmax(r, phi2(I[p - 1])) : r;
        lp[p] = pshift(I[p], p ? I[p - 1] : negw);
      }
      const int agg = phi(I[NP - 1]);
      const int exc = max(dpp_wave_shr1(kNeg16, wave_max_scan(agg)), cp_in);
      const uint32_t exc2 = psplat(exc);
      // the scan term of the column before the lane's first: the left lane's
      // last, or M(i, base - 1) - ge from the carry
      const int wl_in = max(cm_in - ge, kNeg16);
      const uint32_t wleft = dpp_shr1_u((uint32_t)wl_in << 16, w[NP - 1]);
      uint32_t D0[NP], D1[NP], D2[NP], D3[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const uint32_t mx = pmax(exc2, lp[p]);
        const uint32_t eg = psub(mx, ej[p]);
        const uint32_t g = pmax(Mv[p], eg);
        const uint32_t fo = psub(Gp[p], go2), fe = psub(Fp[p], ge2);
        const uint32_t f = pmax(fo, fe);
        const uint32_t wprev = pshift(w[p], p ? w[p - 1] : wleft);
        // sign set = the decision fails: V = G?, Fv opened?, G = M?, Eg
        // opened (the previous column's term is the prefix maximum)?
        D0[p] = psub(g, f);
        D1[p] = psub(fo, fe);
        D2[p] = psub(Mv[p], eg);
        D3[p] = psub(wprev, mx);
        Vp[p] = pmax(g, f);
        Gp[p] = g;
        Fp[p] = f;
      }
      uint32_t word;
      if constexpr (NP == 2) {
        uint32_t acc = psigns(D0[0], D0[1]) & 0x10100101u;
        acc |= psigns(D1[0], D1[1]) & 0x20200202u;
        acc |= psigns(D2[0], D2[1]) & 0x40400404u;
        acc |= psigns(D3[0], D3[1]) & 0x80800808u;
        word = ~(acc | (acc >> 16)) & 0xffffu;
      } else {
        uint32_t acc = (psigns(D0[0], D0[1]) & 0x01010101u) | (psigns(D0[2], D0[3]) & 0x10101010u);
        acc |= (psigns(D1[0], D1[1]) & 0x02020202u) | (psigns(D1[2], D1[3]) & 0x20202020u);
        acc |= (psigns(D2[0], D2[1]) & 0x04040404u) | (psigns(D2[2], D2[3]) & 0x40404040u);
        acc |= (psigns(D3[0], D3[1]) & 0x08080808u) | (psigns(D3[2], D3[3]) & 0x80808080u);
        word = ~acc;
      }
      if (L < LS) brow[(size_t)i * LS] = (Word)word;
      if (NEXT && L == 63) {
        cw[3 * i] = phi(Vp[NP - 1]);
        cw[3 * i + 1] = phi(Mv[NP - 1]);
        cw[3 * i + 2] = max(max(exc, agg) - TC * ge, kNeg16);
      }
      cv_prev = cv_in;
      if (last_tile && i == A - 1) {
        // the end pair's M (MODE 0) or the end cell's V reaches the score
        const int jb = B - 1 - jc0;
        int mend = 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const uint32_t x = MODE == 0 ? Mv[c / 2] : Vp[c / 2];
          if (jb == c) mend = (c & 1) ? phi(x) : plo(x);
        }
        ok = __ballot(jb >= 0 && jb < C && mend == P.score) != 0;
      }
    }
  }
}

template <bool LB, int C, int MODE, class Word>
__device__ __forceinline__ void fill16(const TraceArgs &a, const TracePair &P, const short *smat16,
                                       Word *bits, int LS, int *carry, int crow, bool &bad,
                                       bool &ok) {
  const int T = (P.B + 64 * C - 1) / (64 * C);
  for (int t = 0; t < T; ++t) {
    const int *cr = carry + ((t + 1) & 1) * 3 * crow;   // written by tile t - 1
    int *cw = carry + (t & 1) * 3 * crow;                // read by tile t + 1
    const bool next = t + 1 < T;
    if (t == 0) {
      if (next) fill16_tile<C, MODE, true, true>(a, P, smat16, bits, LS, cr, cw, t, bad, ok);
      else fill16_tile<C, MODE, true, false>(a, P, smat16, bits, LS, cr, cw, t, bad, ok);
    } else {
      if (next) fill16_tile<C, MODE, false, true>(a, P, smat16, bits, LS, cr, cw, t, bad, ok);
      else fill16_tile<C, MODE, false, false>(a, P, smat16, bits, LS, cr, cw, t, bad, ok);
    }
    // carries and bits are read back by this same wavefront (see trace_one)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
}

// One pair at C query columns per lane (a tile of 64 C columns).  MODE 0:
// the rectangle between a local alignment's start and end pair, anchored at
// the start pair; MODE 1-4: a whole end-to-end alignment in the API's mode
// MODE - 1 (global, semi-global either way, overlap: the boundaries of
// endtoend_kernel) over r[0..ref_end] x q[0..query_end], walked back from
// its end cell to a virtual start element.
template <bool LB, int C, int MODE, bool W16>
__device__ __forceinline__ void trace_one(const TraceArgs &a, const TracePair &P, const int *smat,
                                          const short *smat16, uint16_t *lbits, int *lcarry,
                                          uint16_t *lwin16) {
  // row -1 free: virtual pairs (-1, j) (query prefix free); column -1 free:
  // virtual pairs (i, -1) (reference prefix free)
  constexpr bool kRowFree = MODE == 3 || MODE == 4, kColFree = MODE == 2 || MODE == 4;
  constexpr int TC = 64 * C;
  // one lane's decision word per row: 4 bits per column
  using Word = typename std::conditional<(C > 4), uint32_t, uint16_t>::type;
  constexpr int kWinRows = kWalkWindowBytes / (64 * (int)sizeof(Word));
  const int L = threadIdx.x;
  const int alpha = a.alpha, go = a.go, ge = a.ge;
  const int A = P.A, B = P.B, T = (B + TC - 1) / TC;
  const int LS = trace_lane_stride(B, C);   // lanes per row of decision words
  Word *bits = (Word *)(LB ? lbits : a.gbits + (size_t)blockIdx.x * a.slot_words);
  Word *lwin = (Word *)lwin16;
  int *carry = LB ? lcarry : a.gcarry + (size_t)blockIdx.x * 6 * a.carry_rows;
  const int crow = a.carry_rows;   // LDS: <= kTraceLdsCarryRows, 0 if every rectangle is one tile
  bool bad = false, ok = false;

  if constexpr (W16) fill16<LB, C, MODE, Word>(a, P, smat16, bits, LS, carry, crow, bad, ok);
  else for (int t = 0; t < T; ++t) {
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
      if (L < LS) bits[((size_t)t * A + i) * LS + L] = (Word)word;
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
  // device-memory bits are read through an LDS window of kWinRows rows of
  // one tile (the walk only moves up and left): one coalesced copy per
  // window instead of a dependent device-memory load per step
  int w_tile = -1, w_lo = 0;
  auto nib_at = [&](int i, int j) -> int {
    const int t = j / TC, col = (j % TC) / C;
    uint32_t wd;
    if (LB) {
      wd = bits[((size_t)t * A + i) * LS + col];
    } else {
      if (t != w_tile || i < w_lo || i >= w_lo + kWinRows) {
        w_tile = t;
        w_lo = max(0, i - kWinRows + 1);
        const int rows = min(kWinRows, A - w_lo);
        // rows of LS words: LS * sizeof(Word) / 16 units of 16 bytes each
        const uint4 *src = (const uint4 *)(bits + ((size_t)t * A + w_lo) * LS);
        uint4 *dst = (uint4 *)lwin;
        const int units = rows * LS * (int)sizeof(Word) / 16;
        for (int k = L; k < units; k += 64) dst[k] = src[k];
      }
      wd = lwin[(i - w_lo) * LS + col];
    }
    return (int)(wd >> nib_shift<C, W16>(j % C)) & 15;
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
      const uint32_t wd = LB ? (uint32_t)bits[((size_t)t * A + ii) * LS + col]
                             : (uint32_t)lwin[(ii - w_lo) * LS + col];
      nib = (int)(wd >> nib_shift<C, W16>(jj % C)) & 15;
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

// V: the variant of every pair of the launch (kTraceV32: C from
// TracePair::pad, the fewest columns per lane that cover a one-tile query, so
// short queries leave few lanes idle; kTraceV16x4 / kTraceV16x8: 16-bit
// values at 4 / 8 columns per lane).  One kernel per variant, so that each
// keeps its own register budget and occupancy.
template <bool LB, int MODE, int V>
__device__ __forceinline__ void trace_mode(const TraceArgs &a, const TracePair &P, const int *smat,
                                           const short *smat16, uint16_t *lbits, int *lcarry,
                                           uint16_t *lwin) {
  if constexpr (V == kTraceV16x4) {
    trace_one<LB, 4, MODE, true>(a, P, smat, smat16, lbits, lcarry, lwin);
  } else if constexpr (V == kTraceV16x8) {
    trace_one<LB, 8, MODE, true>(a, P, smat, smat16, lbits, lcarry, lwin);
  } else {
    switch (P.pad) {
      case 1: trace_one<LB, 1, MODE, false>(a, P, smat, smat16, lbits, lcarry, lwin); break;
      case 2: trace_one<LB, 2, MODE, false>(a, P, smat, smat16, lbits, lcarry, lwin); break;
      case 3: trace_one<LB, 3, MODE, false>(a, P, smat, smat16, lbits, lcarry, lwin); break;
      default: trace_one<LB, 4, MODE, false>(a, P, smat, smat16, lbits, lcarry, lwin); break;
    }
  }
}

template <bool LB, int V>
__global__ __launch_bounds__(64) void trace_kernel(TraceArgs a) {
  extern __shared__ int smem[];
  int *smat = smem;                                            // [query code][ref code]
  short *smat16 = (short *)(smem + mat_words(a.alpha));        // the same, 16-bit entries
  // the matrices take alpha^2 words and shorts (16-byte aligned), the bits follow
  uint16_t *lbits = (uint16_t *)(smem + mat_words(a.alpha) + mat16_words(a.alpha));
  int *lcarry = (int *)(lbits + a.lds_words);                  // LDS variant: after the bits
  uint16_t *lwin = lbits;                                      // walk window (device-memory bits)
  for (int k = threadIdx.x; k < a.alpha * a.alpha; k += 64) {
    smat[k] = a.matrix[k];
    smat16[k] = (short)a.matrix[k];
  }
  __syncthreads();
  for (int p = blockIdx.x; p < a.n; p += gridDim.x) {
    const TracePair P = a.pairs[p];
    switch (a.mode) {
      case 0: trace_mode<LB, 0, V>(a, P, smat, smat16, lbits, lcarry, lwin); break;
      case 1: trace_mode<LB, 1, V>(a, P, smat, smat16, lbits, lcarry, lwin); break;
      case 2: trace_mode<LB, 2, V>(a, P, smat, smat16, lbits, lcarry, lwin); break;
      case 3: trace_mode<LB, 3, V>(a, P, smat, smat16, lbits, lcarry, lwin); break;
      default: trace_mode<LB, 4, V>(a, P, smat, smat16, lbits, lcarry, lwin); break;
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

// endtoend_kernel for queries beyond 256 residues: 5-8 columns per lane, one
// tile up to 512 residues, beyond that as many tiles as 512-column ones would
// need (a kernel of its own, so that the wider lanes' registers do not lower
// the narrow kernel's occupancy).
template <int MODE>
__global__ __launch_bounds__(64) void endtoend_wide_kernel(EndArgs a) {
  extern __shared__ int smem[];
  int *smat = smem;
  for (int k = threadIdx.x; k < a.alpha * a.alpha; k += 64) smat[k] = a.matrix[k];
  __syncthreads();
  for (int p = blockIdx.x; p < a.n; p += gridDim.x) {
    const TracePair P = a.pairs[p];
    switch (P.pad) {   // query columns per lane
      case 5: endtoend_one<MODE, 5>(a, P, smat); break;
      case 6: endtoend_one<MODE, 6>(a, P, smat); break;
      case 7: endtoend_one<MODE, 7>(a, P, smat); break;
      default: endtoend_one<MODE, 8>(a, P, smat); break;
    }
  }
}

// Pair t's runs (the last n_runs[id] entries of its region) to
// cigar_dst[dst_off[id] ..]; a wavefront per pair (most paths have a few
// runs), four per workgroup, grid-stride.
__global__ __launch_bounds__(256) void pack_runs_kernel(const TracePair *pairs, int n,
                                                        const int32_t *n_runs,
                                                        const int64_t *dst_off,
                                                        const uint32_t *src, uint32_t *dst) {
  const int lane = threadIdx.x & 63;
  const int per_block = blockDim.x / 64;
  const int stride = gridDim.x * per_block;
  for (int t = blockIdx.x * per_block + threadIdx.x / 64; t < n; t += stride) {
    const TracePair P = pairs[t];
    const int cnt = min(n_runs[P.id], P.cap);   // the host checked every count already
    const int64_t s0 = P.out + P.cap - cnt, d0 = dst_off[P.id];
    for (int k = lane; k < cnt; k += 64) dst[d0 + k] = src[s0 + k];
  }
}

}  // namespace
}  // namespace dev

size_t trace_lds_bytes(bool lds_bits, int alpha, int lds_words, int carry_rows) {
  size_t b = (size_t)(dev::mat_words(alpha) + dev::mat16_words(alpha)) * sizeof(int);
  if (lds_bits) b += (size_t)lds_words * sizeof(uint16_t) + 6 * (size_t)carry_rows * sizeof(int);
  else b += (size_t)dev::kWalkWindowBytes;
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

hipError_t launch_endtoend_wide(int mode, const EndArgs &a, int grid, hipStream_t st) {
  if (a.n <= 0 || grid <= 0) return hipSuccess;
  const size_t lds = endtoend_lds_bytes(a.alpha);
  switch (mode) {
    case 0: hipLaunchKernelGGL(dev::endtoend_wide_kernel<0>, dim3(grid), dim3(64), lds, st, a); break;
    case 1: hipLaunchKernelGGL(dev::endtoend_wide_kernel<1>, dim3(grid), dim3(64), lds, st, a); break;
    case 2: hipLaunchKernelGGL(dev::endtoend_wide_kernel<2>, dim3(grid), dim3(64), lds, st, a); break;
    case 3: hipLaunchKernelGGL(dev::endtoend_wide_kernel<3>, dim3(grid), dim3(64), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pack_runs(const TracePair *pairs, int n, const int32_t *n_runs,
                            const int64_t *dst_off, const uint32_t *src, uint32_t *dst,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::pack_runs_kernel, dim3(std::min((n + 3) / 4, 65535)), dim3(256), 0, st,
                     pairs, n, n_runs, dst_off, src, dst);
  return hipGetLastError();
}

template <bool LB>
static void launch_trace_v(int variant, const TraceArgs &a, int grid, hipStream_t st) {
  const size_t lds = trace_lds_bytes(LB, a.alpha, a.lds_words, a.carry_rows);
  switch (variant) {
    case kTraceV16x4: hipLaunchKernelGGL((dev::trace_kernel<LB, kTraceV16x4>), dim3(grid), dim3(64), lds, st, a); break;
    case kTraceV16x8: hipLaunchKernelGGL((dev::trace_kernel<LB, kTraceV16x8>), dim3(grid), dim3(64), lds, st, a); break;
    default: hipLaunchKernelGGL((dev::trace_kernel<LB, kTraceV32>), dim3(grid), dim3(64), lds, st, a); break;
  }
}

hipError_t launch_trace(bool lds_bits, int variant, const TraceArgs &a, int grid, hipStream_t st) {
  if (a.n <= 0 || grid <= 0) return hipSuccess;
  if (variant != kTraceV32 && variant != kTraceV16x4 && variant != kTraceV16x8)
    return hipErrorInvalidValue;
  if (lds_bits && (a.lds_words < 8 || a.lds_words % 8 || a.lds_words > kTraceLdsRowTiles * 64 ||
                   a.carry_rows < 0 || a.carry_rows > kTraceLdsCarryRows))
    return hipErrorInvalidValue;
  if (lds_bits) launch_trace_v<true>(variant, a, grid, st);
  else launch_trace_v<false>(variant, a, grid, st);
  return hipGetLastError();
}

}  // namespace swk
