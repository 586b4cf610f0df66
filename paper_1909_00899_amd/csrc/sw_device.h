// gfx950 kernels for the striped Smith-Waterman scan (paper: Algorithm 6).
//
// Layout (paper: striped layout of Algorithm 1/6).  One alignment runs on a
// sub-group of P = 16, 32 or 64 lanes of a wavefront.  Lane l holds query rows
// l*SEG + j, j < SEG, of the current query chunk, with H[j] and E[j] in VGPRs.
// In packed int16 mode every 32-bit lane value carries two independent
// alignments (low and high half), so a wavefront of four 16-lane sub-groups
// runs eight alignments; the cross-lane data movement is identical for both
// halves.  One reference residue = one column step for every sub-group of the
// wavefront, in lockstep.
//
// Column step for reference residue r_i (paper: Algorithm 6, with the readings
// spelled out in the host runtime's documentation):
//   top       H_last = max(H[SEG-1], Fscan - (SEG-1)*ge)   corrected last row of
//             the previous column; moved one lane down (lane 0 of a sub-group
//             gets 0, or the previous query chunk's boundary value).
//   inner     hd = Hin + prof[r_i][j];  Max = max(Max, hd)
//             h = max(hd, E[j], F);     t = h - go (saturating at 0)
//             E[j] = max(E[j] - ge, t); F = max(F - ge, t)
//             Hin = max(H_old[j], Fscan - j*ge)   (deferred "lazier" H fix-up)
//   scan      G = F;  G = max(G, G[l-d] - d*SEG*ge) for d = 1, 2, 4, ...
//             (inclusive max-plus scan over the sub-group; Hillis-Steele form
//             of the scan loop of Algorithm 6), then Fscan = G shifted one lane
//             down: the vertical-gap value entering each lane's first row.
// Subtraction saturates at 0 (the paper's "-" never goes negative), so E, F and
// every scan value stay >= 0 and a lane shifted in as 0 is neutral.
//
// Cross-lane moves are DPP: row_shr:1/2/4/8 inside 16-lane rows, row_bcast:15
// and row_bcast:31 to cross rows, wave_shr:1 for the one-lane shift.  Weights
// of the broadcast steps are per lane, so a wavefront may mix 32- and 16-lane
// sub-groups (a lane that must not receive gets an infinite weight).
#pragma once
#include <type_traits>

#include "sw_internal.h"

namespace swk {
namespace dev {

template <class T, class F>
__device__ __forceinline__ T bc(F x) { return __builtin_bit_cast(T, x); }

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- lane arithmetic

struct OpsI32 {
  static constexpr int kHalves = 1;
  static constexpr int kES = 4;                       // profile entry bytes
  static constexpr uint32_t kWeightCap = 0x7fffffffu;
  __device__ static uint32_t hadd(uint32_t a, uint32_t b) {
    return (uint32_t)__builtin_elementwise_add_sat((int)a, (int)b);
  }
  __device__ static uint32_t vmax(uint32_t a, uint32_t b) { return (uint32_t)max((int)a, (int)b); }
  __device__ static uint32_t usub(uint32_t a, uint32_t b) { return __builtin_elementwise_sub_sat(a, b); }
  __device__ static int get(uint32_t x, int) { return (int)x; }
  __device__ static uint32_t set(uint32_t, int, int v) { return (uint32_t)v; }
  __device__ static uint32_t splat(uint32_t v) { return v; }
};

struct OpsI16 {
  static constexpr int kHalves = 2;
  static constexpr int kES = 2;
  static constexpr uint32_t kWeightCap = 0xffffu;
  __device__ static uint32_t hadd(uint32_t a, uint32_t b) {
    return bc<uint32_t>(__builtin_elementwise_add_sat(bc<s16x2>(a), bc<s16x2>(b)));
  }
  __device__ static uint32_t vmax(uint32_t a, uint32_t b) {
    return bc<uint32_t>(__builtin_elementwise_max(bc<s16x2>(a), bc<s16x2>(b)));
  }
  __device__ static uint32_t vmin(uint32_t a, uint32_t b) {
    return bc<uint32_t>(__builtin_elementwise_min(bc<s16x2>(a), bc<s16x2>(b)));
  }
  __device__ static uint32_t usub(uint32_t a, uint32_t b) {
    return bc<uint32_t>(__builtin_elementwise_sub_sat(bc<u16x2>(a), bc<u16x2>(b)));
  }
  __device__ static int get(uint32_t x, int h) { return (int)(short)(h ? (x >> 16) : (x & 0xffffu)); }
  __device__ static uint32_t set(uint32_t x, int h, int v) {
    return h ? ((x & 0xffffu) | ((uint32_t)v << 16)) : ((x & 0xffff0000u) | ((uint32_t)v & 0xffffu));
  }
  __device__ static uint32_t splat(uint32_t v) { return (v & 0xffffu) * 0x10001u; }
};

// Weight k*unit capped to the lane type's "infinite" (subtracting it from any
// valid value saturates to 0), splatted to both halves in int16 mode.
template <class O>
__device__ __forceinline__ uint32_t weight(uint64_t k, uint64_t unit) {
  uint64_t w = k * unit;
  return O::splat((uint32_t)(w > O::kWeightCap ? O::kWeightCap : w));
}

// Capped per-half weights lo_k*unit (low half) and hi_k*unit (high half).
__device__ __forceinline__ uint32_t weight2(uint64_t lo_k, uint64_t hi_k, uint64_t unit) {
  using O = OpsI16;
  return (weight<O>(lo_k, unit) & 0xffffu) | (weight<O>(hi_k, unit) & 0xffff0000u);
}

// ---------------------------------------------------------------- DPP

template <int CTRL, int ROWMASK = 0xf, bool BOUND = true>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xf, BOUND);
}
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kWaveShr1 = 0x138, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
// quad_perm [1,0,3,2] and [2,3,0,1] (lane xor 1, xor 2), the mirror of each
// eight-lane half of a row (lane xor 7 inside the half) and of the whole row
// (lane xor 15)
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kRowHalfMirror = 0x141, kRowMirror = 0x140;

// ---------------------------------------------------------------- lane layout

struct LaneCtx {
  int lane;      // 0..63
  int sg;        // sub-group ordinal in the wavefront
  int P;         // sub-group width (16, 32, 64)
  int l;         // lane index inside the sub-group
  bool start;    // first lane of its sub-group
  bool last;     // last lane of its sub-group
  uint32_t w16;  // weight of the row_bcast:15 scan step for this lane
  uint32_t w32;  // weight of the row_bcast:31 scan step
  uint32_t wcarry;  // weight applied to a chunk carry entering this lane's G
  uint32_t rx16;    // all ones if this lane takes the row_bcast:15 value (same sub-group)
  uint32_t rx32;    // all ones if this lane takes the row_bcast:31 value
  int glast;        // wavefront lane index of the last lane of this sub-group
  // eight-lane sub-groups only: scan weights of the row_shr:1/2/4 steps
  // (infinite where the source lane lies in the previous sub-group) and the
  // mask that clears what a one-lane move brings across the boundary
  uint32_t v1, v2, v4;
  uint32_t keep;
};

// layout: bit r set <=> a sub-group starts at lane 16*r (bit 0 always set).
template <class O>
__device__ __forceinline__ LaneCtx make_lane(int layout, int seg, uint32_t ge) {
  LaneCtx L;
  L.lane = (int)(threadIdx.x & 63);
  const int row = L.lane >> 4;
  int s0 = row;
  while (s0 > 0 && !((layout >> s0) & 1)) --s0;
  int e0 = row + 1;
  while (e0 < 4 && !((layout >> e0) & 1)) ++e0;
  L.P = (e0 - s0) * 16;
  L.l = L.lane - s0 * 16;
  L.sg = __builtin_popcount(layout & ((2 << s0) - 1)) - 1;
  L.start = L.l == 0;
  L.last = L.l == L.P - 1;
  const uint64_t unit = (uint64_t)seg * ge;
  const uint32_t inf = O::splat(O::kWeightCap);
  // row_bcast:15 writes rows 1 and 3 with the last lane of rows 0 and 2.
  const bool r15 = (row & 1) && s0 < row;
  L.w16 = r15 ? weight<O>((uint64_t)(L.lane & 15) + 1, unit) : inf;
  // row_bcast:31 writes rows 2 and 3 with lane 31.
  const bool r31 = row >= 2 && s0 == 0;
  L.w32 = r31 ? weight<O>((uint64_t)(L.lane & 31) + 1, unit) : inf;
  L.wcarry = L.start ? weight<O>(1, unit) : inf;
  L.rx16 = r15 ? 0xffffffffu : 0u;
  L.rx32 = r31 ? 0xffffffffu : 0u;
  L.glast = s0 * 16 + L.P - 1;
  L.v1 = L.v2 = L.v4 = inf;
  L.keep = 0xffffffffu;
  return L;
}

// Eight sub-groups of eight lanes (per-pair kernels for short queries):
// sub-group g is wavefront lanes 8g..8g+7.  Two sub-groups share each 16-lane
// DPP row, so a row shift by d brings lanes of the previous sub-group into the
// first d lanes of the upper one: their scan weight is infinite and the
// one-lane moves are masked there.
template <class O>
__device__ __forceinline__ LaneCtx make_lane8(int seg, uint32_t ge) {
  LaneCtx L;
  L.lane = (int)(threadIdx.x & 63);
  L.P = 8;
  L.l = L.lane & 7;
  L.sg = L.lane >> 3;
  L.start = L.l == 0;
  L.last = L.l == 7;
  const uint64_t unit = (uint64_t)seg * ge;
  const uint32_t inf = O::splat(O::kWeightCap);
  L.v1 = L.l >= 1 ? weight<O>(unit, 1) : inf;
  L.v2 = L.l >= 2 ? weight<O>(2 * unit, 1) : inf;
  L.v4 = L.l >= 4 ? weight<O>(4 * unit, 1) : inf;
  L.keep = L.start ? 0u : 0xffffffffu;
  L.w16 = L.w32 = L.wcarry = inf;
  L.rx16 = L.rx32 = 0u;
  L.glast = L.lane | 7;
  return L;
}

// Move x one lane down inside each sub-group; the first lane of a sub-group
// receives `carry`.
template <int PMAX, bool CARRY>
__device__ __forceinline__ uint32_t shift1(uint32_t x, const LaneCtx &L, uint32_t carry) {
  if constexpr (PMAX == 8) {
    static_assert(!CARRY, "eight-lane sub-groups hold the whole query");
    return dpp<kRowShr1>(x) & L.keep;
  } else if constexpr (PMAX == 16) {
    uint32_t s = dpp<kRowShr1>(x);
    if constexpr (CARRY) s = L.start ? carry : s;
    return s;
  } else {
    uint32_t s = dpp<kWaveShr1>(x);
    return L.start ? (CARRY ? carry : 0u) : s;
  }
}

// ---------------------------------------------------------------- per-lane state

// End cell.  Each lane keeps a record threshold G (per half) and, whenever
// the column maximum of H_diag in one of its halves exceeds it, the column
// index, that maximum (S) and a copy of the column's new H values (before
// any cross-lane correction).  At the end the row is the first row of the copy
// whose H reaches S.  Every few columns G is raised to the largest threshold
// among the lanes before it in the sub-group (all thresholds are values of
// cells in earlier columns), so that only lanes that beat the alignment's
// best so far record.
//
// Why this is exact for the cell that matters: let X be the lexicographically
// smallest (column, row) cell holding the overall maximum, in lane l and
// column c.  Every cell of an earlier column scores below it (else it would
// precede X), so lane l's threshold is below it at column c, lane l records
// column c, and no later column exceeds what it recorded.  Every E and F
// entering lane l's rows in column c comes from cells of earlier columns (all
// below the maximum) or from rows of lane l above X (all below it) minus a
// non-negative gap cost, so the first row whose new H reaches the maximum is
// X's row.  Other lanes' records may point at a wrong row, but they score below
// the maximum, or equal it in a later column or in a later lane of the same
// column, so they never win the final (score, column, row) reduction.
template <int SEG>
struct State {
  uint32_t H[SEG];    // H of the previous column, before the cross-lane fix-up
  uint32_t E[SEG];
  uint32_t snap[SEG]; // H of the column where this lane last improved (per half)
  uint32_t Fscan;     // vertical-gap value entering this lane's first row
  uint32_t G;         // record threshold (per half)
  uint32_t S;         // column maximum of H_diag at the last record (per half)
  int rc[2];          // column of the last improvement (per half), or INT_MAX
  uint32_t events;    // improvement branches taken (statistics)
};

template <int SEG>
__device__ __forceinline__ void state_reset(State<SEG> &st, uint32_t g0) {
#pragma unroll
  for (int j = 0; j < SEG; ++j) { st.H[j] = 0; st.E[j] = 0; st.snap[j] = 0; }
  st.Fscan = 0;
  st.G = g0;
  st.S = 0;
  st.rc[0] = st.rc[1] = 0x7fffffff;
  st.events = 0;
}

struct Params {
  uint32_t go, ge;            // splatted gap penalties
  uint32_t w1, w2, w4, w8;    // scan weights d*SEG*ge
  uint32_t wlast;             // (SEG-1)*ge
};

template <class O, int SEG>
__device__ __forceinline__ Params make_params(uint32_t go, uint32_t ge) {
  Params p;
  p.go = O::splat(go);
  p.ge = O::splat(ge);
  p.w1 = weight<O>(1ull * SEG, ge);
  p.w2 = weight<O>(2ull * SEG, ge);
  p.w4 = weight<O>(4ull * SEG, ge);
  p.w8 = weight<O>(8ull * SEG, ge);
  p.wlast = weight<O>((uint64_t)(SEG - 1), ge);
  return p;
}

// ---------------------------------------------------------------- profile access

extern __shared__ __align__(16) unsigned char smem[];

// Loads the profile entry of row j for the low-half residue (base lo) and the
// high-half residue (base hi); JSTRIDE = bytes between consecutive j.
template <class O, int JSTRIDE>
struct ProfLds {
  __device__ __forceinline__ uint32_t load(uint32_t lo, uint32_t hi, int j) const {
    if constexpr (O::kHalves == 2) {
      uint32_t a = *(const unsigned short *)(smem + lo + j * JSTRIDE);
      uint32_t b = *(const unsigned short *)(smem + hi + j * JSTRIDE);
      return a | (b << 16);
    } else {
      return *(const uint32_t *)(smem + lo + j * JSTRIDE);
    }
  }
};

// Byte profile entries (matrices whose scores fit in int8), sign-extended to
// the lane type; otherwise as ProfLds.
template <class O, int JSTRIDE>
struct ProfLds8 {
  __device__ __forceinline__ uint32_t load(uint32_t lo, uint32_t hi, int j) const {
    if constexpr (O::kHalves == 2) {
      // two byte loads merged by one permute: the d16 loads that would write
      // each byte into its half directly zero the register's other half on
      // this chip (SRAM ECC), so they cannot build the pair
      s16x2 v;
      v.x = (short)*(const signed char *)(smem + lo + j * JSTRIDE);
      v.y = (short)*(const signed char *)(smem + hi + j * JSTRIDE);
      return bc<uint32_t>(v);
    } else {
      return (uint32_t)(int)*(const signed char *)(smem + lo + j * JSTRIDE);
    }
  }
};

// Per-half mask where nb > g, given nb >= g: 0xffff in each 16-bit half
// (packed: the sign of g - nb, which cannot overflow for values in
// [0, 32767], spread over the half), or all ones (int32).
template <class O>
__device__ __forceinline__ uint32_t gain_mask(uint32_t nb, uint32_t g) {
  if constexpr (O::kHalves == 2) {
    return bc<uint32_t>((bc<s16x2>(g) - bc<s16x2>(nb)) >> (short)15);
  } else {
    return nb != g ? 0xffffffffu : 0u;
  }
}

// Column end: lanes whose running maximum improves copy this column's H.
template <class O, int SEG>
__device__ __forceinline__ void record(State<SEG> &st, uint32_t cmax, int i) {
  const uint32_t nb = O::vmax(st.G, cmax);
  if (__any(nb != st.G)) {
    ++st.events;
    uint32_t m = gain_mask<O>(nb, st.G);
    // keep the copies below as one bit-select per register (an empty asm
    // hides where the mask came from, so it is not split into per-half selects)
    asm("" : "+v"(m));
#pragma unroll
    for (int j = 0; j < SEG; ++j) st.snap[j] = (st.H[j] & m) | (st.snap[j] & ~m);
    if constexpr (O::kHalves == 2) {
      // 32-bit masks of the two halves: sign-extended low half, high half
      const uint32_t mlo = (uint32_t)((int)(m << 16) >> 16);
      const uint32_t mhi = (uint32_t)((int)m >> 16);
      st.rc[0] = (int)(((uint32_t)i & mlo) | ((uint32_t)st.rc[0] & ~mlo));
      st.rc[1] = (int)(((uint32_t)i & mhi) | ((uint32_t)st.rc[1] & ~mhi));
    } else {
      if (m) st.rc[0] = i;
    }
    st.G = nb;
    st.S = (nb & m) | (st.S & ~m);
  }
}

// record() for int16 lanes with the end-cell record in LDS instead of VGPRs:
// a lane whose low (high) half improves stores the low (high) halves of the
// column's H with 16-bit LDS stores (row j at snap + 256*j), the column index
// (row SEG for the low half, SEG+1 for the high half) and the column maximum
// (row SEG+2, 16 bits per half).  The stores take LDS issue slots instead of
// a VALU select per row and the per-half column and maximum selects.
constexpr int kRecRows = 3;   // rows after the copy: column (low, high), maximum

template <int SEG>
__device__ __forceinline__ void record_lds(State<SEG> &st, uint32_t cmax, int i, uint32_t snap) {
  using O = OpsI16;
  const uint32_t nb = O::vmax(st.G, cmax);
  if (__any(nb != st.G)) {
    ++st.events;
    const uint32_t g = st.G;
    st.G = nb;
    if ((unsigned short)nb != (unsigned short)g) {
#pragma unroll
      for (int j = 0; j < SEG; ++j) *(unsigned short *)(smem + snap + 256 * j) = (unsigned short)st.H[j];
      *(int *)(smem + snap + 256 * SEG) = i;
      *(unsigned short *)(smem + snap + 256 * (SEG + 2)) = (unsigned short)nb;
    }
    if ((nb >> 16) != (g >> 16)) {
#pragma unroll
      for (int j = 0; j < SEG; ++j)
        *(unsigned short *)(smem + snap + 256 * j + 2) = (unsigned short)(st.H[j] >> 16);
      *(int *)(smem + snap + 256 * (SEG + 1)) = i;
      *(unsigned short *)(smem + snap + 256 * (SEG + 2) + 2) = (unsigned short)(nb >> 16);
    }
  }
}

// No record yet: columns INT_MAX, maxima 0 (this lane's words only).
template <int SEG>
__device__ __forceinline__ void record_lds_reset(uint32_t snap) {
  *(int *)(smem + snap + 256 * SEG) = 0x7fffffff;
  *(int *)(smem + snap + 256 * (SEG + 1)) = 0x7fffffff;
  *(uint32_t *)(smem + snap + 256 * (SEG + 2)) = 0u;
}

// Raises every lane's record threshold to the largest threshold of its
// sub-group: an inclusive prefix maximum over the sub-group (thresholds are
// non-negative, so the zeros shifted in are neutral), then the last lane's
// value read back for every lane of the sub-group.
template <class O, int SEG, int PMAX>
__device__ __forceinline__ void share_threshold(State<SEG> &st, const LaneCtx &L) {
  if constexpr (PMAX <= 16) {
    // butterfly over the eight or sixteen lanes: every lane ends with the maximum
    uint32_t T = st.G;
    T = O::vmax(T, dpp<kQuadXor1>(T));
    T = O::vmax(T, dpp<kQuadXor2>(T));
    T = O::vmax(T, dpp<kRowHalfMirror>(T));
    if constexpr (PMAX == 16) T = O::vmax(T, dpp<kRowMirror>(T));
    st.G = T;
    return;
  }
  uint32_t T = st.G;
  T = O::vmax(T, dpp<kRowShr1>(T));
  T = O::vmax(T, dpp<kRowShr2>(T));
  T = O::vmax(T, dpp<kRowShr4>(T));
  T = O::vmax(T, dpp<kRowShr8>(T));
  if constexpr (PMAX >= 32) T = O::vmax(T, dpp<kRowBcast15, 0xa, false>(T) & L.rx16);
  if constexpr (PMAX >= 64) T = O::vmax(T, dpp<kRowBcast31, 0xc, false>(T) & L.rx32);
  const uint32_t t15 = (uint32_t)__builtin_amdgcn_readlane((int)T, 15);
  const uint32_t t31 = (uint32_t)__builtin_amdgcn_readlane((int)T, 31);
  const uint32_t t47 = (uint32_t)__builtin_amdgcn_readlane((int)T, 47);
  const uint32_t t63 = (uint32_t)__builtin_amdgcn_readlane((int)T, 63);
  st.G = L.glast == 15 ? t15 : (L.glast == 31 ? t31 : (L.glast == 47 ? t47 : t63));
}

// Record rule of the swapped layout (the reference striped over the lanes,
// the query streamed as columns): the end cell is still the smallest
// (ref_end, query_end) among the cells holding the maximum, which here is the
// smallest (row, column) instead of (column, row).  A lane records when its
// column maximum rises above its threshold as record() does, and also when
// it ties the threshold with a row smaller than the recorded one.  For the
// cell X that matters (the smallest row, then column, holding the overall
// maximum S): no cell of a smaller row holds S, so no H of such a row reaches
// S either (E and F come from cells of smaller or equal rows minus a gap
// cost), so in X's column the first row of X's lane whose H reaches S is X's
// row, and every earlier record of S in that lane lies in a larger row: the
// lane ends with X recorded.  Records of other lanes score below S or lie in
// larger rows.
template <class P> struct SwapRecord { static constexpr bool value = false; };

// ---------------------------------------------------------------- one column

template <class O, int SEG, int PMAX, bool CHUNKED, bool LAZY, class Prof>
__device__ __forceinline__ void column(State<SEG> &st, const LaneCtx &L, const Params &pr,
                                       const Prof &pf, uint32_t blo, uint32_t bhi,
                                       uint32_t hb_in, uint32_t fb_in, uint32_t &hb_out,
                                       uint32_t &fb_out, int i, uint32_t &lazy_steps) {
  uint32_t cmax;
  if constexpr (!LAZY) {
    uint32_t Fj = st.Fscan;
    const uint32_t hlast = O::vmax(st.H[SEG - 1], O::usub(Fj, pr.wlast));
    hb_out = hlast;
    uint32_t Hin = shift1<PMAX, CHUNKED>(hlast, L, hb_in);
    uint32_t F = 0;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const uint32_t p = pf.load(blo, bhi, j);
      const uint32_t hd = O::hadd(Hin, p);
      cmax = j == 0 ? hd : O::vmax(cmax, hd);
      const uint32_t h = O::vmax(O::vmax(hd, st.E[j]), F);
      const uint32_t hold = st.H[j];
      st.H[j] = h;
      const uint32_t t = O::usub(h, pr.go);
      st.E[j] = O::vmax(O::usub(st.E[j], pr.ge), t);
      F = O::vmax(O::usub(F, pr.ge), t);
      if (j + 1 < SEG) {
        Hin = O::vmax(hold, Fj);
        Fj = O::usub(Fj, pr.ge);
      }
    }
    // max-plus scan of the per-lane vertical-gap outputs
    uint32_t G = F;
    if constexpr (CHUNKED) G = O::vmax(G, O::usub(fb_in, L.wcarry));
    if constexpr (PMAX == 8) {
      G = O::vmax(G, O::usub(dpp<kRowShr1>(G), L.v1));
      G = O::vmax(G, O::usub(dpp<kRowShr2>(G), L.v2));
      G = O::vmax(G, O::usub(dpp<kRowShr4>(G), L.v4));
    } else {
      G = O::vmax(G, O::usub(dpp<kRowShr1>(G), pr.w1));
      G = O::vmax(G, O::usub(dpp<kRowShr2>(G), pr.w2));
      G = O::vmax(G, O::usub(dpp<kRowShr4>(G), pr.w4));
      G = O::vmax(G, O::usub(dpp<kRowShr8>(G), pr.w8));
    }
    if constexpr (PMAX >= 32) G = O::vmax(G, O::usub(dpp<kRowBcast15, 0xa, false>(G), L.w16));
    if constexpr (PMAX >= 64) G = O::vmax(G, O::usub(dpp<kRowBcast31, 0xc, false>(G), L.w32));
    fb_out = G;
    st.Fscan = shift1<PMAX, CHUNKED>(G, L, fb_in);
    if constexpr (SwapRecord<Prof>::value) pf.record(st, cmax, i);
    else record<O, SEG>(st, cmax, i);
  } else {
    // Algorithm 1: H[] already holds corrected values.
    hb_out = st.H[SEG - 1];
    uint32_t Hin = shift1<PMAX, CHUNKED>(st.H[SEG - 1], L, hb_in);
    uint32_t F = 0;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const uint32_t p = pf.load(blo, bhi, j);
      const uint32_t hd = O::hadd(Hin, p);
      cmax = j == 0 ? hd : O::vmax(cmax, hd);
      const uint32_t h = O::vmax(O::vmax(hd, st.E[j]), F);
      Hin = st.H[j];
      st.H[j] = h;
      const uint32_t t = O::usub(h, pr.go);
      st.E[j] = O::vmax(O::usub(st.E[j], pr.ge), t);
      F = O::vmax(O::usub(F, pr.ge), t);
    }
    record<O, SEG>(st, cmax, i);
    // Lazy-F loop: propagate the vertical gap across lanes until, in every
    // lane at once, the propagated value can no longer exceed what the first
    // pass already derived (F <= max(H_before - go, 0)); then stop.
    uint32_t Fexit = F;
    uint32_t Fp = shift1<PMAX, CHUNKED>(F, L, fb_in);
    bool done = false;
    for (int k = 0; k < PMAX && !done; ++k) {
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const uint32_t hb = st.H[j];
        st.H[j] = O::vmax(hb, Fp);
        Fp = O::usub(Fp, pr.ge);
        const uint32_t lim = O::usub(hb, pr.go);
        ++lazy_steps;
        if (__all(O::vmax(Fp, lim) == lim)) { done = true; break; }
      }
      if (!done) {
        Fexit = O::vmax(Fexit, Fp);
        Fp = shift1<PMAX, false>(Fp, L, 0u);
      }
    }
    fb_out = Fexit;
  }
}

// ---------------------------------------------------------------- column loop

// Runs `ncols` reference columns for every sub-group of the wavefront.
// stream: this task's residue stream; bnd_*: the task's chunk-boundary arrays
// (HB then FB, [4 sub-groups][ncols] each) or nullptr.
// Reference residues, four columns per 32-bit word (column 4b+k in byte k),
// for the low and the high half of this lane's sub-group.
//
// StreamSrc reads a task's residue stream ([ncols/4][8 slot-halves][4]
// bytes, sentinel-padded by the stream builder; the stream buffer ends with
// spare blocks, so reading two blocks past the task's end stays inside it).
struct StreamSrc {
  const uint2 *sp;   // this sub-group's (low, high) word of block 0
  __device__ __forceinline__ uint2 get(int b) const { return sp[b * 4]; }
};

// DirectSrc reads the references themselves: a full word where all four
// columns lie inside the reference (an unaligned 4-byte load), single bytes
// in the last partial word, and the sentinel code at and past the end (no
// memory access there).
struct DirectSrc {
  const uint8_t *plo, *phi;   // first residue of the low / high half's reference
  int nlo, nhi;               // their lengths (0 for an empty slot)
  uint32_t sentw;             // sentinel code in all four bytes
  __device__ __forceinline__ static uint32_t word(const uint8_t *p, int n, int b, uint32_t sentw) {
    const int i = b * kBlock;
    if (i + kBlock <= n) {
      uint32_t w;
      __builtin_memcpy(&w, p + i, 4);
      return w;
    }
    uint32_t w = sentw;
    if (i < n) {
#pragma unroll
      for (int q = 0; q < kBlock - 1; ++q)
        if (i + q < n) w = (w & ~(0xffu << (8 * q))) | ((uint32_t)p[i + q] << (8 * q));
    }
    return w;
  }
  __device__ __forceinline__ uint2 get(int b) const {
    return make_uint2(word(plo, nlo, b, sentw), word(phi, nhi, b, sentw));
  }
};

template <class O, int SEG, int PMAX, bool CHUNKED, bool LAZY, class ProfMap, class Src>
__device__ __forceinline__ void run_columns(State<SEG> &st, const LaneCtx &L, const Params &pr,
                                            const ProfMap &pm, const Src &src, int ncols,
                                            const uint32_t *hb_in, const uint32_t *fb_in,
                                            uint32_t *hb_out, uint32_t *fb_out,
                                            uint32_t &lazy_steps) {
  const int nblk = ncols / kBlock;
  uint32_t ev_shared = st.events;
  // residue words of this sub-group (low half, high half), two blocks ahead
  uint2 rc = src.get(0);
  uint2 rn = src.get(1);
  uint4 hbc, hbn, fbc, fbn;
  if constexpr (CHUNKED) {
    hbc = ((const uint4 *)hb_in)[0];
    hbn = ((const uint4 *)hb_in)[1];
    fbc = ((const uint4 *)fb_in)[0];
    fbn = ((const uint4 *)fb_in)[1];
  }
  for (int b = 0; b < nblk; ++b) {
    const uint2 r = rc;
    rc = rn;
    rn = src.get(b + 2);
    uint4 hbv = make_uint4(0, 0, 0, 0), fbv = make_uint4(0, 0, 0, 0);
    if constexpr (CHUNKED) {
      hbv = hbc; hbc = hbn; hbn = ((const uint4 *)hb_in)[b + 2];
      fbv = fbc; fbc = fbn; fbn = ((const uint4 *)fb_in)[b + 2];
    }
    uint32_t ho[kBlock], fo[kBlock];
    const uint32_t hin[kBlock] = {hbv.x, hbv.y, hbv.z, hbv.w};
    const uint32_t fin[kBlock] = {fbv.x, fbv.y, fbv.z, fbv.w};
#pragma unroll
    for (int k = 0; k < kBlock; ++k) {
      const uint32_t clo = (r.x >> (8 * k)) & 0xffu;
      const uint32_t chi = (r.y >> (8 * k)) & 0xffu;
      column<O, SEG, PMAX, CHUNKED, LAZY>(st, L, pr, pm.prof, pm.base_lo(clo), pm.base_hi(chi),
                                          hin[k], fin[k], ho[k], fo[k], b * kBlock + k,
                                          lazy_steps);
    }
    if (hb_out != nullptr && L.last) {
      ((uint4 *)hb_out)[b] = make_uint4(ho[0], ho[1], ho[2], ho[3]);
      ((uint4 *)fb_out)[b] = make_uint4(fo[0], fo[1], fo[2], fo[3]);
    }
    // share thresholds after blocks in which some lane recorded
    if (st.events != ev_shared) {
      share_threshold<O, SEG, PMAX>(st, L);
      ev_shared = st.events;
    }
  }
}

// ---------------------------------------------------------------- results

__device__ __forceinline__ bool better(int s, int c, int r, int s2, int c2, int r2) {
  return s > s2 || (s == s2 && (c < c2 || (c == c2 && r < r2)));
}

// Reduces each slot-half's recorded cells over its sub-group, merges with
// the result of the previous query chunks (prev_*, identical in every lane of
// the sub-group, updated in place) and writes the merged result.
struct Prev {
  int s[2], c[2], r[2];
  uint32_t f[2];
};

__device__ __forceinline__ void prev_reset(Prev &p) {
  p.s[0] = p.s[1] = 0;
  p.c[0] = p.c[1] = p.r[0] = p.r[1] = 0x7fffffff;
  p.f[0] = p.f[1] = 0;
}

// Loads the previous chunks' merged results of this lane's slot-halves.
template <class O>
__device__ __forceinline__ void prev_load(Prev &p, const LaneCtx &L, const Task *tp,
                                          const PairInfo *pairs, const DevResult *results) {
  prev_reset(p);
#pragma unroll
  for (int h = 0; h < O::kHalves; ++h) {
    const int pid = tp->pair[2 * L.sg + h];
    if (pid >= 0) {
      const DevResult r = results[pairs[pid].out];
      if (r.score > 0) { p.s[h] = r.score; p.c[h] = r.rend; p.r[h] = r.qend; }
      p.f[h] = r.flags;
    }
  }
}

// Initial record G: ties with a previous chunk's best must still be seen (a
// tie in an earlier column wins), so start one below it.
template <class O>
__device__ __forceinline__ uint32_t prev_g0(const Prev &p) {
  uint32_t g = 0;
#pragma unroll
  for (int h = 0; h < O::kHalves; ++h) g = O::set(g, h, p.s[h] > 0 ? p.s[h] - 1 : 0);
  return g;
}

// pid[h]: PairInfo index of this lane's sub-group in half h, or -1.
template <class O, int SEG>
__device__ __forceinline__ void finish(const State<SEG> &st, const LaneCtx &L, const int pid[2],
                                       const PairInfo *pairs, DevResult *results, int row_base,
                                       Prev &prev, int sat_cap) {
#pragma unroll
  for (int h = 0; h < O::kHalves; ++h) {
    int s = st.rc[h] != 0x7fffffff ? O::get(st.S, h) : 0;
    int c = 0x7fffffff, r = 0x7fffffff;
    if (s > 0) {
      int jj = SEG - 1;
#pragma unroll
      for (int j = SEG - 1; j >= 0; --j)
        if (O::get(st.snap[j], h) >= s) jj = j;
      c = st.rc[h];
      r = L.l * SEG + jj + row_base;
    } else {
      s = 0;
    }
    for (int d = 1; d < kWave; d <<= 1) {
      const int s2 = __shfl_xor(s, d), c2 = __shfl_xor(c, d), r2 = __shfl_xor(r, d);
      if (d < L.P && better(s2, c2, r2, s, c, r)) { s = s2; c = c2; r = r2; }
    }
    uint32_t flags = prev.f[h];
    if (O::kHalves == 2 && s >= sat_cap) flags |= kFlagNeedsI32;
    if (prev.s[h] > 0 && (s <= 0 || better(prev.s[h], prev.c[h], prev.r[h], s, c, r))) {
      s = prev.s[h]; c = prev.c[h]; r = prev.r[h];
    }
    if (s <= 0) { s = 0; c = 0x7fffffff; r = 0x7fffffff; }
    prev.s[h] = s; prev.c[h] = c; prev.r[h] = r; prev.f[h] = flags;
    if (L.start && pid[h] >= 0) {
      DevResult res;
      res.score = s;
      res.qend = s > 0 ? r : -1;
      res.rend = s > 0 ? c : -1;
      res.flags = flags;
      results[pairs[pid[h]].out] = res;
    }
  }
}

__device__ __forceinline__ int pop_task(int *counter) {
  int t = 0;
  if ((threadIdx.x & 63) == 0) t = atomicAdd(counter, 1);
  return __builtin_amdgcn_readfirstlane(t);
}

__device__ __forceinline__ void stage_matrix(const KArgs &a) {
  int32_t *M = (int32_t *)smem;
  for (int k = threadIdx.x; k < a.alpha * a.alpha; k += blockDim.x) M[k] = a.matrix[k];
}

// ================================================================ shared-query kernel

// LDS: [matrix][profile of mode 0][mode 1][mode 2]; each profile is
// [alpha+1][SEG][P] entries with the residue stride padded so that the four
// 16-lane sub-groups reading different residues spread over the banks.
__host__ __device__ constexpr uint32_t shared_cstride(int seg, int P, int es) {
  return (uint32_t)(((seg * P * es + 127) / 128) * 128 + 32);
}

template <class O, int SEG, int P>
struct SharedMap {
  ProfLds<O, P * O::kES> prof;
  uint32_t lane_base;   // bytes: profile base + l * ES
  __device__ __forceinline__ uint32_t base_lo(uint32_t c) const {
    return lane_base + c * shared_cstride(SEG, P, O::kES);
  }
  __device__ __forceinline__ uint32_t base_hi(uint32_t c) const { return base_lo(c); }
};

template <class O, int SEG, int P>
__device__ void build_shared_profile(const KArgs &a, uint32_t off) {
  const int32_t *M = (const int32_t *)smem;
  const int nrow = a.alpha + 1;
  const int total = nrow * SEG * P;
  const int64_t row0 = (int64_t)a.chunk * (P * SEG);
  for (int k = threadIdx.x; k < total; k += blockDim.x) {
    const int l = k % P;
    const int j = (k / P) % SEG;
    const int c = k / (P * SEG);
    const int64_t row = row0 + l * SEG + j;
    int v;
    const int qc = (row < a.shared_m) ? (int)a.query_res[a.shared_q_off + row] : a.alpha;
    if (c < a.alpha && qc < a.alpha) {
      v = M[qc * a.alpha + c];
    } else {
      v = O::kES == 2 ? -32768 : (int)0x80000000;
    }
    unsigned char *dst = smem + off + c * shared_cstride(SEG, P, O::kES) + (j * P + l) * O::kES;
    if constexpr (O::kES == 2) *(short *)dst = (short)v;
    else *(int *)dst = v;
  }
}

template <class O, int SEG, int P, bool CHUNKED, bool LAZY>
__device__ __forceinline__ void shared_task(const KArgs &a, const Task &t, const Task *tp,
                                            uint32_t prof_off,
                                            uint32_t &lazy_steps, unsigned long long &cols,
                                            unsigned long long &events) {
  const LaneCtx L = make_lane<O>(t.layout, SEG, (uint32_t)a.gap_extend);
  const Params pr = make_params<O, SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
  SharedMap<O, SEG, P> pm;
  pm.lane_base = prof_off + L.l * O::kES;
  Prev prev;
  prev_reset(prev);
  if (CHUNKED && a.chunk > 0) prev_load<O>(prev, L, tp, a.pairs, a.results);
  State<SEG> st;
  state_reset(st, prev_g0<O>(prev));
  const uint32_t *hb_in = nullptr, *fb_in = nullptr;
  uint32_t *hb_out = nullptr, *fb_out = nullptr;
  if constexpr (CHUNKED) {
    const int64_t base = t.bnd_off + (int64_t)L.sg * t.ncols;
    const int64_t fofs = 4ll * t.ncols;
    hb_in = a.bnd_in + base;
    fb_in = a.bnd_in + base + fofs;
    if (!a.last_chunk) {
      hb_out = a.bnd_out + base;
      fb_out = a.bnd_out + base + fofs;
    }
  }
  const StreamSrc src{(const uint2 *)(a.streams + t.stream_off) + L.sg};
  run_columns<O, SEG, P, CHUNKED, LAZY>(st, L, pr, pm, src, t.ncols, hb_in, fb_in, hb_out,
                                        fb_out, lazy_steps);
  cols += (unsigned long long)t.ncols;
  events += st.events;
  const int pid[2] = {tp->pair[2 * L.sg], tp->pair[2 * L.sg + 1]};
  finish<O, SEG>(st, L, pid, a.pairs, a.results, a.chunk * P * SEG, prev, a.sat_cap);
}

template <class O, int S16, int S32, int S64, bool CHUNKED, bool LAZY>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
void shared_kernel(KArgs a, uint32_t mode_mask) {
  stage_matrix(a);
  __syncthreads();
  uint32_t off0 = 0, off1 = 0, off2 = 0;
  uint32_t cur = matrix_lds_bytes(a.alpha);
  const int nrow = a.alpha + 1;
  if constexpr (S16 > 0) {
    if (mode_mask & 1u) {
      off0 = cur;
      build_shared_profile<O, S16, 16>(a, cur);
      cur += nrow * shared_cstride(S16, 16, O::kES);
    }
  }
  if constexpr (S32 > 0) {
    if (mode_mask & 2u) {
      off1 = cur;
      build_shared_profile<O, S32, 32>(a, cur);
      cur += nrow * shared_cstride(S32, 32, O::kES);
    }
  }
  if constexpr (S64 > 0) {
    if (mode_mask & 4u) {
      off2 = cur;
      build_shared_profile<O, S64, 64>(a, cur);
      cur += nrow * shared_cstride(S64, 64, O::kES);
    }
  }
  __syncthreads();
  uint32_t lazy_steps = 0;
  unsigned long long cols = 0, events = 0;
  for (;;) {
    const int ti = pop_task(a.task_counter);
    if (ti >= a.ntasks) break;
    const Task t = a.tasks[ti];
    if constexpr (S16 > 0) {
      if (t.mode == 0) { shared_task<O, S16, 16, CHUNKED, LAZY>(a, t, a.tasks + ti, off0, lazy_steps, cols, events); continue; }
    }
    if constexpr (S32 > 0) {
      if (t.mode == 1) { shared_task<O, S32, 32, CHUNKED, LAZY>(a, t, a.tasks + ti, off1, lazy_steps, cols, events); continue; }
    }
    if constexpr (S64 > 0) {
      if (t.mode == 2) { shared_task<O, S64, 64, CHUNKED, LAZY>(a, t, a.tasks + ti, off2, lazy_steps, cols, events); continue; }
    }
  }
  if ((threadIdx.x & 63) == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (lazy_steps) atomicAdd(&a.stats[1], (unsigned long long)lazy_steps);
    if (events) atomicAdd(&a.stats[2], events);
  }
}

// ================================================================ two chains per sub-group (int32)

// int32 lanes carry one alignment each, so a sub-group's column step is one
// dependent chain (profile reads, the inner loop's F and Hin carries, the
// scan's DPP steps).  Two alignments per sub-group -- the task's even and odd
// slot, each with its own state, residue and chunk boundaries -- give every
// step an independent twin the compiler interleaves with it, and share the
// per-column work that does not depend on the alignment (residue words, loop
// control, the record test): the explicit interleave of two Smith-Waterman
// executions that the paper's closing remarks propose, where int16 lanes get
// it from their two halves.

// Record of both chains under one branch: a lane whose maximum improves in a
// chain copies that chain's H (as record()).
template <int SEG>
__device__ __forceinline__ void record_dual(State<SEG> &s0, State<SEG> &s1, uint32_t c0,
                                            uint32_t c1, int i) {
  using O = OpsI32;
  const uint32_t n0 = O::vmax(s0.G, c0), n1 = O::vmax(s1.G, c1);
  if (__any(n0 != s0.G || n1 != s1.G)) {
    ++s0.events;
    const uint32_t m0 = n0 != s0.G ? 0xffffffffu : 0u;
    const uint32_t m1 = n1 != s1.G ? 0xffffffffu : 0u;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      s0.snap[j] = (s0.H[j] & m0) | (s0.snap[j] & ~m0);
      s1.snap[j] = (s1.H[j] & m1) | (s1.snap[j] & ~m1);
    }
    if (m0) s0.rc[0] = i;
    if (m1) s1.rc[0] = i;
    s0.S = (n0 & m0) | (s0.S & ~m0);
    s1.S = (n1 & m1) | (s1.S & ~m1);
    s0.G = n0;
    s1.G = n1;
  }
}

// One column step (Algorithm 6, as column()) of two independent alignments of
// the sub-group: chain 0 against the residue at profile base b0, chain 1 at b1.
template <int SEG, int PMAX, bool CHUNKED, class Prof>
__device__ __forceinline__ void column_dual(State<SEG> &s0, State<SEG> &s1, const LaneCtx &L,
                                            const Params &pr, const Prof &pf, uint32_t b0,
                                            uint32_t b1, uint32_t hin0, uint32_t fin0,
                                            uint32_t hin1, uint32_t fin1, uint32_t &ho0,
                                            uint32_t &fo0, uint32_t &ho1, uint32_t &fo1, int i) {
  using O = OpsI32;
  uint32_t Fj0 = s0.Fscan, Fj1 = s1.Fscan;
  const uint32_t hl0 = O::vmax(s0.H[SEG - 1], O::usub(Fj0, pr.wlast));
  const uint32_t hl1 = O::vmax(s1.H[SEG - 1], O::usub(Fj1, pr.wlast));
  ho0 = hl0;
  ho1 = hl1;
  uint32_t Hin0 = shift1<PMAX, CHUNKED>(hl0, L, hin0);
  uint32_t Hin1 = shift1<PMAX, CHUNKED>(hl1, L, hin1);
  uint32_t F0 = 0, F1 = 0, c0 = 0, c1 = 0;
#pragma unroll
  for (int j = 0; j < SEG; ++j) {
    const uint32_t p0 = pf.load(b0, b0, j), p1 = pf.load(b1, b1, j);
    const uint32_t hd0 = O::hadd(Hin0, p0), hd1 = O::hadd(Hin1, p1);
    c0 = j == 0 ? hd0 : O::vmax(c0, hd0);
    c1 = j == 0 ? hd1 : O::vmax(c1, hd1);
    const uint32_t h0 = O::vmax(O::vmax(hd0, s0.E[j]), F0);
    const uint32_t h1 = O::vmax(O::vmax(hd1, s1.E[j]), F1);
    const uint32_t o0 = s0.H[j], o1 = s1.H[j];
    s0.H[j] = h0;
    s1.H[j] = h1;
    const uint32_t t0 = O::usub(h0, pr.go), t1 = O::usub(h1, pr.go);
    s0.E[j] = O::vmax(O::usub(s0.E[j], pr.ge), t0);
    s1.E[j] = O::vmax(O::usub(s1.E[j], pr.ge), t1);
    F0 = O::vmax(O::usub(F0, pr.ge), t0);
    F1 = O::vmax(O::usub(F1, pr.ge), t1);
    if (j + 1 < SEG) {
      Hin0 = O::vmax(o0, Fj0);
      Hin1 = O::vmax(o1, Fj1);
      Fj0 = O::usub(Fj0, pr.ge);
      Fj1 = O::usub(Fj1, pr.ge);
    }
  }
  // the two max-plus scans, step by step side by side
  uint32_t G0 = F0, G1 = F1;
  if constexpr (CHUNKED) {
    G0 = O::vmax(G0, O::usub(fin0, L.wcarry));
    G1 = O::vmax(G1, O::usub(fin1, L.wcarry));
  }
  G0 = O::vmax(G0, O::usub(dpp<kRowShr1>(G0), pr.w1));
  G1 = O::vmax(G1, O::usub(dpp<kRowShr1>(G1), pr.w1));
  G0 = O::vmax(G0, O::usub(dpp<kRowShr2>(G0), pr.w2));
  G1 = O::vmax(G1, O::usub(dpp<kRowShr2>(G1), pr.w2));
  G0 = O::vmax(G0, O::usub(dpp<kRowShr4>(G0), pr.w4));
  G1 = O::vmax(G1, O::usub(dpp<kRowShr4>(G1), pr.w4));
  G0 = O::vmax(G0, O::usub(dpp<kRowShr8>(G0), pr.w8));
  G1 = O::vmax(G1, O::usub(dpp<kRowShr8>(G1), pr.w8));
  if constexpr (PMAX >= 32) {
    G0 = O::vmax(G0, O::usub(dpp<kRowBcast15, 0xa, false>(G0), L.w16));
    G1 = O::vmax(G1, O::usub(dpp<kRowBcast15, 0xa, false>(G1), L.w16));
  }
  if constexpr (PMAX >= 64) {
    G0 = O::vmax(G0, O::usub(dpp<kRowBcast31, 0xc, false>(G0), L.w32));
    G1 = O::vmax(G1, O::usub(dpp<kRowBcast31, 0xc, false>(G1), L.w32));
  }
  fo0 = G0;
  fo1 = G1;
  s0.Fscan = shift1<PMAX, CHUNKED>(G0, L, fin0);
  s1.Fscan = shift1<PMAX, CHUNKED>(G1, L, fin1);
  record_dual<SEG>(s0, s1, c0, c1, i);
}

// run_columns() for two chains: chain h reads residue word half h (the
// task's slot 2*sg + h) and, when chunked, its own boundary arrays.
template <int SEG, int PMAX, bool CHUNKED, class ProfMap, class Src>
__device__ __forceinline__ void run_columns_dual(State<SEG> &s0, State<SEG> &s1, const LaneCtx &L,
                                                 const Params &pr, const ProfMap &pm,
                                                 const Src &src, int ncols,
                                                 const uint32_t *const hb_in[2],
                                                 const uint32_t *const fb_in[2],
                                                 uint32_t *const hb_out[2],
                                                 uint32_t *const fb_out[2]) {
  using O = OpsI32;
  const int nblk = ncols / kBlock;
  uint32_t ev_shared = s0.events;
  uint2 rc = src.get(0);
  uint2 rn = src.get(1);
  for (int b = 0; b < nblk; ++b) {
    const uint2 r = rc;
    rc = rn;
    rn = src.get(b + 2);
    uint4 h0 = make_uint4(0, 0, 0, 0), f0 = h0, h1 = h0, f1 = h0;
    if constexpr (CHUNKED) {
      h0 = ((const uint4 *)hb_in[0])[b];
      f0 = ((const uint4 *)fb_in[0])[b];
      h1 = ((const uint4 *)hb_in[1])[b];
      f1 = ((const uint4 *)fb_in[1])[b];
    }
    const uint32_t hi0[kBlock] = {h0.x, h0.y, h0.z, h0.w}, fi0[kBlock] = {f0.x, f0.y, f0.z, f0.w};
    const uint32_t hi1[kBlock] = {h1.x, h1.y, h1.z, h1.w}, fi1[kBlock] = {f1.x, f1.y, f1.z, f1.w};
    uint32_t ho0[kBlock], fo0[kBlock], ho1[kBlock], fo1[kBlock];
#pragma unroll
    for (int k = 0; k < kBlock; ++k) {
      const uint32_t c0 = (r.x >> (8 * k)) & 0xffu;
      const uint32_t c1 = (r.y >> (8 * k)) & 0xffu;
      column_dual<SEG, PMAX, CHUNKED>(s0, s1, L, pr, pm.prof, pm.base_lo(c0), pm.base_hi(c1),
                                      hi0[k], fi0[k], hi1[k], fi1[k], ho0[k], fo0[k], ho1[k],
                                      fo1[k], b * kBlock + k);
    }
    if (hb_out[0] != nullptr && L.last) {
      ((uint4 *)hb_out[0])[b] = make_uint4(ho0[0], ho0[1], ho0[2], ho0[3]);
      ((uint4 *)fb_out[0])[b] = make_uint4(fo0[0], fo0[1], fo0[2], fo0[3]);
      ((uint4 *)hb_out[1])[b] = make_uint4(ho1[0], ho1[1], ho1[2], ho1[3]);
      ((uint4 *)fb_out[1])[b] = make_uint4(fo1[0], fo1[1], fo1[2], fo1[3]);
    }
    if (s0.events != ev_shared) {
      share_threshold<O, SEG, PMAX>(s0, L);
      share_threshold<O, SEG, PMAX>(s1, L);
      ev_shared = s0.events;
    }
  }
}

// Previous query chunks' merged result of one slot (int32: one half).
__device__ __forceinline__ void prev_load_slot(Prev &p, int pid, const PairInfo *pairs,
                                               const DevResult *results) {
  prev_reset(p);
  if (pid >= 0) {
    const DevResult r = results[pairs[pid].out];
    if (r.score > 0) { p.s[0] = r.score; p.c[0] = r.rend; p.r[0] = r.qend; }
    p.f[0] = r.flags;
  }
}

// One task of the shared-query kernel with two int32 chains per sub-group.
// Chunk boundaries: [8 slots][ncols] H words, then [8 slots][ncols] F words.
template <int SEG, int P, bool CHUNKED>
__device__ __forceinline__ void shared_task_dual(const KArgs &a, const Task &t, const Task *tp,
                                                 uint32_t prof_off, unsigned long long &cols,
                                                 unsigned long long &events) {
  using O = OpsI32;
  const LaneCtx L = make_lane<O>(t.layout, SEG, (uint32_t)a.gap_extend);
  const Params pr = make_params<O, SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
  SharedMap<O, SEG, P> pm;
  pm.lane_base = prof_off + L.l * O::kES;
  const int pid0 = tp->pair[2 * L.sg], pid1 = tp->pair[2 * L.sg + 1];
  Prev prev0, prev1;
  prev_reset(prev0);
  prev_reset(prev1);
  if (CHUNKED && a.chunk > 0) {
    prev_load_slot(prev0, pid0, a.pairs, a.results);
    prev_load_slot(prev1, pid1, a.pairs, a.results);
  }
  State<SEG> s0, s1;
  state_reset(s0, prev_g0<O>(prev0));
  state_reset(s1, prev_g0<O>(prev1));
  const uint32_t *hb_in[2] = {nullptr, nullptr}, *fb_in[2] = {nullptr, nullptr};
  uint32_t *hb_out[2] = {nullptr, nullptr}, *fb_out[2] = {nullptr, nullptr};
  if constexpr (CHUNKED) {
    const int64_t fofs = 8ll * t.ncols;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t base = t.bnd_off + (int64_t)(2 * L.sg + h) * t.ncols;
      hb_in[h] = a.bnd_in + base;
      fb_in[h] = a.bnd_in + base + fofs;
      if (!a.last_chunk) {
        hb_out[h] = a.bnd_out + base;
        fb_out[h] = a.bnd_out + base + fofs;
      }
    }
  }
  const StreamSrc src{(const uint2 *)(a.streams + t.stream_off) + L.sg};
  run_columns_dual<SEG, P, CHUNKED>(s0, s1, L, pr, pm, src, t.ncols, hb_in, fb_in, hb_out,
                                    fb_out);
  cols += (unsigned long long)t.ncols;
  events += s0.events;
  const int p0[2] = {pid0, -1}, p1[2] = {pid1, -1};
  finish<O, SEG>(s0, L, p0, a.pairs, a.results, a.chunk * P * SEG, prev0, a.sat_cap);
  finish<O, SEG>(s1, L, p1, a.pairs, a.results, a.chunk * P * SEG, prev1, a.sat_cap);
}

// shared_kernel for int32 with two chains per sub-group (scan algorithm).
// Two chains need twice the state registers: up to 16 rows per lane that is
// more than 128 VGPRs, so the kernel is built for two wavefronts per SIMD (each
// with the work of two).
template <int S16, int S32, int S64, bool CHUNKED>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void shared_dual_kernel(KArgs a, uint32_t mode_mask) {
  using O = OpsI32;
  stage_matrix(a);
  __syncthreads();
  uint32_t off0 = 0, off1 = 0, off2 = 0;
  uint32_t cur = matrix_lds_bytes(a.alpha);
  const int nrow = a.alpha + 1;
  if constexpr (S16 > 0) {
    if (mode_mask & 1u) {
      off0 = cur;
      build_shared_profile<O, S16, 16>(a, cur);
      cur += nrow * shared_cstride(S16, 16, O::kES);
    }
  }
  if constexpr (S32 > 0) {
    if (mode_mask & 2u) {
      off1 = cur;
      build_shared_profile<O, S32, 32>(a, cur);
      cur += nrow * shared_cstride(S32, 32, O::kES);
    }
  }
  if constexpr (S64 > 0) {
    if (mode_mask & 4u) {
      off2 = cur;
      build_shared_profile<O, S64, 64>(a, cur);
      cur += nrow * shared_cstride(S64, 64, O::kES);
    }
  }
  __syncthreads();
  unsigned long long cols = 0, events = 0;
  for (;;) {
    const int ti = pop_task(a.task_counter);
    if (ti >= a.ntasks) break;
    const Task t = a.tasks[ti];
    if constexpr (S16 > 0) {
      if (t.mode == 0) { shared_task_dual<S16, 16, CHUNKED>(a, t, a.tasks + ti, off0, cols, events); continue; }
    }
    if constexpr (S32 > 0) {
      if (t.mode == 1) { shared_task_dual<S32, 32, CHUNKED>(a, t, a.tasks + ti, off1, cols, events); continue; }
    }
    if constexpr (S64 > 0) {
      if (t.mode == 2) { shared_task_dual<S64, 64, CHUNKED>(a, t, a.tasks + ti, off2, cols, events); continue; }
    }
  }
  if ((threadIdx.x & 63) == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (events) atomicAdd(&a.stats[2], events);
  }
}

// ================================================================ device-planned shared-query kernel

// One query (one chunk), one sub-group width.  Task t is entries
// [t*slots, (t+1)*slots) of the planner's longest-first order, entry
// t*slots + s going to sub-group s / halves, half s % halves; the task runs
// as many columns as its longest reference (rounded up to a block).  Residues
// come from the references themselves.  Nothing runs when the planner or the
// residue check flagged the batch (the host then reports the error).
template <class O, int SEG, int P>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
void shared_direct_kernel(KArgs a) {
  if (a.plan_meta[kMetaErrResidue] | a.plan_meta[kMetaErrPair]) return;
  stage_matrix(a);
  __syncthreads();
  const uint32_t off = matrix_lds_bytes(a.alpha);
  build_shared_profile<O, SEG, P>(a, off);
  __syncthreads();
  constexpr int kSlotsPerTask = (kWave / P) * O::kHalves;
  const int nvalid = a.plan_meta[kMetaValid];
  const int ntasks = (nvalid + kSlotsPerTask - 1) / kSlotsPerTask;
  const LaneCtx L = make_lane<O>(P == 16 ? 0xF : (P == 32 ? 0x5 : 0x1), SEG,
                                 (uint32_t)a.gap_extend);
  const Params pr = make_params<O, SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
  SharedMap<O, SEG, P> pm;
  pm.lane_base = off + L.l * O::kES;
  const uint32_t sentw = (uint32_t)a.alpha * 0x01010101u;
  uint32_t lazy_steps = 0;
  unsigned long long cols = 0, events = 0, padded = 0;
  for (;;) {
    const int ti = pop_task(a.plan_meta + kMetaCounter);
    if (ti >= ntasks) break;
    int pid[2] = {-1, -1};
    int64_t roff[2] = {0, 0};
    int n[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < O::kHalves; ++h) {
      const int e = ti * kSlotsPerTask + L.sg * O::kHalves + h;
      if (e < nvalid) {
        pid[h] = a.order[e];
        const PairInfo p = a.pairs[pid[h]];
        roff[h] = p.r_off;
        n[h] = p.n;
      }
    }
    int nmax = max(n[0], n[1]);
    for (int d = 1; d < kWave; d <<= 1) nmax = max(nmax, __shfl_xor(nmax, d));
    const int ncols = (nmax + kBlock - 1) / kBlock * kBlock;
    Prev prev;
    prev_reset(prev);
    State<SEG> st;
    state_reset(st, 0u);
    const DirectSrc src{a.ref_res + roff[0], a.ref_res + roff[1], n[0], n[1], sentw};
    run_columns<O, SEG, P, false, false>(st, L, pr, pm, src, ncols, nullptr, nullptr, nullptr,
                                         nullptr, lazy_steps);
    cols += (unsigned long long)ncols;
    events += st.events;
    padded += (unsigned long long)min(kSlotsPerTask, nvalid - ti * kSlotsPerTask) * ncols * P * SEG;
    finish<O, SEG>(st, L, pid, a.pairs, a.results, 0, prev, a.sat_cap);
  }
  if ((threadIdx.x & 63) == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (events) atomicAdd(&a.stats[2], events);
    if (padded) atomicAdd(&a.stats[3], padded);
  }
}

// ================================================================ row-pair layout

// int16 lanes may also carry two row segments of ONE alignment instead of two
// alignments: in a 16-lane sub-group, lane l holds virtual lanes 2l (low half)
// and 2l+1 (high half), and virtual lane v holds rows v*SEG + j.  Both halves
// read the same reference residue, so one 32-bit LDS word holds the profile
// entries of rows (2l)*SEG + j and (2l+1)*SEG + j: a single ds_read_b32 per
// row pair and no half-merging instruction.  Cross-lane moves gain one step:
// moving a value one virtual lane down takes the high half of the lane
// before and the own low half (row_shr:1 and an align of the two words).

// One virtual lane down inside each 16-lane sub-group (a DPP row); virtual
// lane 0 receives 0.
__device__ __forceinline__ uint32_t rp_vshift(uint32_t x) {
  const uint32_t y = dpp<kRowShr1>(x);
  return __builtin_amdgcn_alignbit(x, y, 16);
}

// One virtual lane down inside sub-groups of P lanes; virtual lane 0 of each
// sub-group receives 0.  P = 16: DPP rows; wider: a wave shift with the
// sub-group's first lane cleared (`keep` is zero there).
template <int P>
__device__ __forceinline__ uint32_t rp_vshift_p(uint32_t x, uint32_t keep) {
  if constexpr (P == 16) {
    return rp_vshift(x);
  } else {
    uint32_t y = dpp<kWaveShr1>(x);
    if constexpr (P == 32) y &= keep;
    return __builtin_amdgcn_alignbit(x, y, 16);
  }
}

// Per-lane constants of the row-pair layout with P lanes per alignment.
struct RpLane {
  int lane, sg, l;        // wavefront lane, sub-group, lane inside the sub-group
  uint32_t keep;          // 0 in the first lane of a sub-group, else all ones
  uint32_t w16, w32;      // weights of the row_bcast:15 / :31 scan steps (inf: no input)
  uint32_t rx16, rx32;    // all ones where the broadcast value belongs to the sub-group
};

template <int P, int SEG>
__device__ __forceinline__ RpLane make_rp_lane(uint32_t ge) {
  using O = OpsI16;
  RpLane L;
  L.lane = (int)(threadIdx.x & 63);
  L.sg = L.lane / P;
  L.l = L.lane % P;
  L.keep = L.l == 0 ? 0u : 0xffffffffu;
  const int row = L.lane >> 4;
  const uint64_t unit = (uint64_t)SEG * ge;   // one virtual lane
  const uint32_t inf = O::splat(O::kWeightCap);
  const bool r15 = P >= 32 && (row & 1);
  const bool r31 = P >= 64 && row >= 2;
  // the broadcast lane's total reaches this lane e lanes further down
  const uint64_t e15 = (uint64_t)(L.lane & 15) + 1, e31 = (uint64_t)(L.lane & 31) + 1;
  L.w16 = r15 ? weight2(2 * e15 - 1, 2 * e15, unit) : inf;
  L.w32 = r31 ? weight2(2 * e31 - 1, 2 * e31, unit) : inf;
  L.rx16 = r15 ? 0xffffffffu : 0u;
  L.rx32 = r31 ? 0xffffffffu : 0u;
  return L;
}

// Largest value of both halves, in both halves.
__device__ __forceinline__ uint32_t rp_both(uint32_t x) {
  return OpsI16::vmax(x, __builtin_amdgcn_alignbit(x, x, 16));
}

struct RpParams {
  uint32_t go, ge;            // splatted gap penalties
  uint32_t wv;                // SEG*ge: one virtual lane
  // lane steps of the scan: the total of the lane d lanes up (its high half,
  // virtual lane 2(l-d)+1) reaches this lane's low half over 2d-1 virtual lanes
  // and its high half over 2d: weights (2d-1)*SEG*ge | 2d*SEG*ge << 16
  uint32_t w1, w2, w4, w8;
  uint32_t wlast;             // (SEG-1)*ge
  // 16-lane sub-groups (lane l = threadIdx.x % 16): the 32-bit scan's offset
  // l*2*SEG*ge, the lane before's max(l-1, 0)*2*SEG*ge, and 0 | SEG*ge << 16
  int tn;
  uint32_t tc, w0h;
};

template <int SEG>
__device__ __forceinline__ RpParams make_rp_params(uint32_t go, uint32_t ge) {
  using O = OpsI16;
  RpParams p;
  p.go = O::splat(go);
  p.ge = O::splat(ge);
  p.wv = weight<O>(1ull * SEG, ge);
  p.w1 = weight2(1, 2, (uint64_t)SEG * ge);
  p.w2 = weight2(3, 4, (uint64_t)SEG * ge);
  p.w4 = weight2(7, 8, (uint64_t)SEG * ge);
  p.w8 = weight2(15, 16, (uint64_t)SEG * ge);
  p.wlast = weight<O>((uint64_t)(SEG - 1), ge);
  const int l = (int)(threadIdx.x & 15);
  const uint64_t u2 = 2ull * SEG * ge;   // at most 2*16*32767: fits easily in int32
  p.tn = (int)(l * u2);
  p.tc = (uint32_t)((l > 0 ? l - 1 : 0) * u2);
  p.w0h = weight2(0, 1, (uint64_t)SEG * ge);
  return p;
}

// x's high half in both halves (a packed operand select, not an instruction).
__device__ __forceinline__ uint32_t rp_hi2(uint32_t x) {
  const u16x2 v = bc<u16x2>(x);
  return bc<uint32_t>(__builtin_shufflevector(v, v, 1, 1));
}
// x's low half in both halves.
__device__ __forceinline__ uint32_t rp_lo2(uint32_t x) {
  const u16x2 v = bc<u16x2>(x);
  return bc<uint32_t>(__builtin_shufflevector(v, v, 0, 0));
}

// LDS profile of the row-pair layout: [alpha+1][SEG][16 lanes] words, the
// residue stride a multiple of 256 bytes.  Two copies, the second shifted by
// 16 banks: even sub-groups read the first, odd ones the second, so the two
// sub-groups of a half-wave never share a bank whatever residues they read.
__host__ __device__ constexpr uint32_t rp_cstride(int seg) {
  return (uint32_t)((seg * 16 * 4 + 255) / 256 * 256);
}
__host__ __device__ constexpr uint32_t rp_copy_bytes(int seg, int alpha) {
  return (uint32_t)(alpha + 1) * rp_cstride(seg) + 64;
}

template <int SEG>
__device__ void build_rowpair_profile(const KArgs &a, uint32_t off) {
  const int32_t *M = (const int32_t *)smem;
  const int nrow = a.alpha + 1;
  const int total = nrow * SEG * 16;
  for (int k = threadIdx.x; k < total; k += blockDim.x) {
    const int l = k % 16;
    const int j = (k / 16) % SEG;
    const int c = k / (16 * SEG);
    uint32_t w = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t row = (int64_t)(2 * l + h) * SEG + j;
      const int qc = row < a.shared_m ? (int)a.query_res[a.shared_q_off + row] : a.alpha;
      const int v = (c < a.alpha && qc < a.alpha) ? M[qc * a.alpha + c] : -32768;
      w |= ((uint32_t)v & 0xffffu) << (16 * h);
    }
    const uint32_t at = c * rp_cstride(SEG) + (j * 16 + l) * 4;
    *(uint32_t *)(smem + off + at) = w;
    *(uint32_t *)(smem + off + rp_copy_bytes(SEG, a.alpha) + at) = w;
  }
}

// Profile words of one column in the row-pair layout: word j holds the scores
// of rows (2l)*SEG + j (low half) and (2l+1)*SEG + j (high half) against the
// column's reference residue.
// RpShared: the query profile of a shared query, base = this lane's word of row
// 0 for the residue (rows 64 bytes apart).
struct RpShared {
  uint32_t base;
  __device__ __forceinline__ uint32_t operator()(int j) const {
    return *(const uint32_t *)(smem + base + j * 64);
  }
};
// RpWords: words already read into registers (the next column's profile is
// read during the current column, before its end-cell record stores, which
// the compiler cannot move loads across).
template <int SEG>
struct RpWords {
  const uint32_t (&w)[SEG];
  __device__ __forceinline__ uint32_t operator()(int j) const { return w[j]; }
};
// RpPairs: the pair-score table (word (qa*(alpha+1) + qb)*(alpha+1) + r holds
// S(qa, r) and S(qb, r)); qq[j] = byte address of this lane's row pair j,
// c4 = 4 * the column's residue.
template <int SEG>
struct RpPairs {
  const uint32_t (&qq)[SEG];
  uint32_t c4;
  __device__ __forceinline__ uint32_t operator()(int j) const {
    return *(const uint32_t *)(smem + qq[j] + c4);
  }
};

// One column of the row-pair layout (the same column step as column(), with
// virtual-lane moves).  CHUNKED: cin_h / cin_f are the previous query chunk's
// corrected last-row H and vertical-gap carry at this column, already placed
// in the low half of the sub-group's first lane (zero elsewhere); hb_out /
// fb_out receive this chunk's (in the low 16 bits, meaningful in the last lane).
template <int SEG, bool CHUNKED, class Prof, int P = 16, bool LREC = false>
__device__ __forceinline__ void rp_column(State<SEG> &st, const RpParams &pr, const Prof &pf,
                                          int i, uint32_t cin_h, uint32_t cin_f,
                                          uint32_t &hb_out, uint32_t &fb_out,
                                          const RpLane *lp = nullptr, uint32_t snap = 0) {
  using O = OpsI16;
  const uint32_t keep = P == 32 ? lp->keep : 0u;
  uint32_t Fj = st.Fscan;
  const uint32_t hlast = O::vmax(st.H[SEG - 1], O::usub(Fj, pr.wlast));
  uint32_t Hin = rp_vshift_p<P>(hlast, keep);
  if constexpr (CHUNKED) {
    Hin |= cin_h;
    hb_out = hlast >> 16;
  }
  uint32_t F = 0, cmax;
#pragma unroll
  for (int j = 0; j < SEG; ++j) {
    const uint32_t p = pf(j);
    const uint32_t hd = O::hadd(Hin, p);
    cmax = j == 0 ? hd : O::vmax(cmax, hd);
    const uint32_t h = O::vmax(O::vmax(hd, st.E[j]), F);
    const uint32_t hold = st.H[j];
    st.H[j] = h;
    const uint32_t t = O::usub(h, pr.go);
    st.E[j] = O::vmax(O::usub(st.E[j], pr.ge), t);
    F = O::vmax(O::usub(F, pr.ge), t);
    if (j + 1 < SEG) {
      Hin = O::vmax(hold, Fj);
      Fj = O::usub(Fj, pr.ge);
    }
  }
  // inclusive max-plus scan over the 32 virtual lanes (a carry from the
  // previous chunk enters as virtual lane -1), then one virtual lane down
  // (first inside the lane: high half from low half; then Hillis-Steele over
  // the lanes on their totals, the high halves, with per-half weights)
  uint32_t G = F;
  if constexpr (CHUNKED) G = O::vmax(G, O::usub(cin_f, pr.wv));
  G = O::vmax(G, O::usub(rp_lo2(G), pr.wv));
  if constexpr (P == 16) {
    // 16 lanes: the lane totals (high halves) as 32-bit values plus l*2*SEG*ge,
    // so that the scan over the lanes is a plain prefix maximum (one max with
    // a DPP operand per step; lanes past the row's start read 0, which is
    // neutral for these non-negative values), then without the offset again.
    int Tn = (int)(G >> 16) + pr.tn;
    Tn = max(Tn, (int)dpp<kRowShr1>((uint32_t)Tn));
    Tn = max(Tn, (int)dpp<kRowShr2>((uint32_t)Tn));
    Tn = max(Tn, (int)dpp<kRowShr4>((uint32_t)Tn));
    Tn = max(Tn, (int)dpp<kRowShr8>((uint32_t)Tn));
    // scan value of virtual lane 2l-1 (the lane before's total; 0 in lane 0)
    const uint32_t X = dpp<kRowShr1>((uint32_t)Tn) - pr.tc;
    // entering virtual lane 2l: X; entering 2l+1: max(own low half, X - SEG*ge)
    st.Fscan = O::vmax(O::usub(rp_lo2(X), pr.w0h), G << 16);
    if constexpr (CHUNKED) {
      st.Fscan |= cin_f;
      fb_out = (uint32_t)(Tn - pr.tn);
    }
  } else {
    G = O::vmax(G, O::usub(rp_hi2(dpp<kRowShr1>(G)), pr.w1));
    G = O::vmax(G, O::usub(rp_hi2(dpp<kRowShr2>(G)), pr.w2));
    G = O::vmax(G, O::usub(rp_hi2(dpp<kRowShr4>(G)), pr.w4));
    G = O::vmax(G, O::usub(rp_hi2(dpp<kRowShr8>(G)), pr.w8));
    if constexpr (P >= 32) G = O::vmax(G, O::usub(rp_hi2(dpp<kRowBcast15, 0xa, false>(G)), lp->w16));
    if constexpr (P >= 64) G = O::vmax(G, O::usub(rp_hi2(dpp<kRowBcast31, 0xc, false>(G)), lp->w32));
    st.Fscan = rp_vshift_p<P>(G, keep);
    if constexpr (CHUNKED) {
      st.Fscan |= cin_f;
      fb_out = G >> 16;
    }
  }
  if constexpr (LREC) record_lds<SEG>(st, cmax, i, snap);
  else record<O, SEG>(st, cmax, i);
}

// Record thresholds raised to the largest of the sub-group (both halves):
// a butterfly over the 16 lanes, every lane ends with the maximum.
template <int SEG>
__device__ __forceinline__ void rp_share_threshold(State<SEG> &st, int) {
  using O = OpsI16;
  uint32_t T = rp_both(st.G);
  T = O::vmax(T, dpp<kQuadXor1>(T));
  T = O::vmax(T, dpp<kQuadXor2>(T));
  T = O::vmax(T, dpp<kRowHalfMirror>(T));
  st.G = O::vmax(T, dpp<kRowMirror>(T));
}

// Record thresholds raised to the largest of the P-lane sub-group (both halves).
template <int SEG, int P>
__device__ __forceinline__ void rp_share_threshold_p(State<SEG> &st, const RpLane &L) {
  if constexpr (P == 16) {
    rp_share_threshold<SEG>(st, L.lane);
  } else {
    using O = OpsI16;
    uint32_t T = rp_both(st.G);
    T = O::vmax(T, dpp<kRowShr1>(T));
    T = O::vmax(T, dpp<kRowShr2>(T));
    T = O::vmax(T, dpp<kRowShr4>(T));
    T = O::vmax(T, dpp<kRowShr8>(T));
    T = O::vmax(T, dpp<kRowBcast15, 0xa, false>(T) & L.rx16);
    if constexpr (P >= 64) T = O::vmax(T, dpp<kRowBcast31, 0xc, false>(T) & L.rx32);
    const uint32_t t63 = (uint32_t)__builtin_amdgcn_readlane((int)T, 63);
    if constexpr (P == 64) {
      st.G = t63;
    } else {
      const uint32_t t31 = (uint32_t)__builtin_amdgcn_readlane((int)T, 31);
      st.G = L.sg == 0 ? t31 : t63;
    }
  }
}

// MASKED: cap[j] caps the profile words of row pair j (0 in a half whose row
// lies before the alignment's first row, 32767 otherwise).
template <int SEG, bool LREC, bool MASKED, class Src>
__device__ __forceinline__ void rp_run_columns(State<SEG> &st, int lane, const RpParams &pr,
                                               uint32_t lane_base, const Src &src, int ncols,
                                               uint32_t snap, const uint32_t (&cap)[SEG]) {
  const int nblk = ncols / kBlock;
  uint32_t ev_shared = st.events;
  uint32_t rc = src.get(0).x;
  uint32_t rn = src.get(1).x;
  // byte k of a residue word alone (a byte permute; written as shifts and
  // masks the compiler spends two instructions on it), then one shift-add
  auto base = [&](uint32_t r, int k) {
    return lane_base + __builtin_amdgcn_perm(0u, r, 0x0c0c0c00u | (uint32_t)k) * rp_cstride(SEG);
  };
  // profile words of the current column, read one column ahead
  uint32_t pw[SEG];
  {
    const RpShared p0{base(rc, 0)};
#pragma unroll
    for (int j = 0; j < SEG; ++j) pw[j] = MASKED ? OpsI16::vmin(p0(j), cap[j]) : p0(j);
  }
  for (int b = 0; b < nblk; ++b) {
    const uint32_t r = rc;
    rc = rn;
    rn = src.get(b + 2).x;
#pragma unroll
    for (int k = 0; k < kBlock; ++k) {
      // the next column's residue: this word's next byte, or the next word's
      // first (past the last column: a sentinel or padding code, still a
      // valid profile row)
      const RpShared pn{k + 1 < kBlock ? base(r, k + 1) : base(rc, 0)};
      uint32_t nw[SEG];
#pragma unroll
      for (int j = 0; j < SEG; ++j) nw[j] = pn(j);
      // keep the reads here, a whole column ahead of their use (the
      // scheduler would otherwise sink them to the end of the column)
      __builtin_amdgcn_sched_barrier(0);
      uint32_t ho, fo;
      rp_column<SEG, false, RpWords<SEG>, 16, LREC>(st, pr, RpWords<SEG>{pw}, b * kBlock + k, 0u, 0u,
                                                   ho, fo, nullptr, snap);
#pragma unroll
      for (int j = 0; j < SEG; ++j) pw[j] = MASKED ? OpsI16::vmin(nw[j], cap[j]) : nw[j];
    }
    if (st.events != ev_shared) {
      rp_share_threshold<SEG>(st, lane);
      ev_shared = st.events;
    }
  }
}

// Result of the alignment of this lane's sub-group: the best recorded cell of
// each half (virtual lane 2l + h), then the best over the 16 lanes.
template <int SEG, bool LREC>
__device__ __forceinline__ void rp_finish(const State<SEG> &st, int lane, int pid,
                                          const PairInfo *pairs, DevResult *results,
                                          int sat_cap, uint32_t snap) {
  using O = OpsI16;
  const int l = lane & 15;
  int s = 0, c = 0x7fffffff, r = 0x7fffffff;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int rch, sh;
    if constexpr (LREC) {
      rch = *(const int *)(smem + snap + 256 * (SEG + h));
      sh = (int)*(const short *)(smem + snap + 256 * (SEG + 2) + 2 * h);
    } else {
      rch = st.rc[h];
      sh = O::get(st.S, h);
    }
    if (rch == 0x7fffffff) sh = 0;
    if (sh > 0) {
      int jj = SEG - 1;
#pragma unroll
      for (int j = SEG - 1; j >= 0; --j) {
        int v;
        if constexpr (LREC) v = (int)*(const short *)(smem + snap + 256 * j + 2 * h);
        else v = O::get(st.snap[j], h);
        if (v >= sh) jj = j;
      }
      const int ch = rch, rh = (2 * l + h) * SEG + jj;
      if (s <= 0 || better(sh, ch, rh, s, c, r)) { s = sh; c = ch; r = rh; }
    }
  }
  for (int d = 1; d < 16; d <<= 1) {
    const int s2 = __shfl_xor(s, d), c2 = __shfl_xor(c, d), r2 = __shfl_xor(r, d);
    if (s2 > 0 && (s <= 0 || better(s2, c2, r2, s, c, r))) { s = s2; c = c2; r = r2; }
  }
  if (l == 0 && pid >= 0) {
    DevResult res;
    res.score = s > 0 ? s : 0;
    res.qend = s > 0 ? r : -1;
    res.rend = s > 0 ? c : -1;
    res.flags = s >= sat_cap ? kFlagNeedsI32 : 0u;
    results[pairs[pid].out] = res;
  }
}

// Device-planned shared-query kernel in the row-pair layout: four
// alignments per wavefront (one per 16-lane sub-group); task t is entries
// [4t, 4t+4) of the longest-first order.
// LREC: end-cell records in LDS ([16 wavefronts][SEG + kRecRows][64 lanes]
// words after the two profile copies) instead of VGPRs, one workgroup of 16
// wavefronts per CU sharing one profile; else 8 wavefronts per workgroup.
// MASKED (start cells): pair p aligns only the query rows from
// a.first_row[p] on (the reversed prefix ending at its end cell is a suffix of
// the reversed query); the rows before get profile scores capped at 0, so their
// H, E and F stay 0 and the first real row starts as after a zero row, exactly
// as in the alignment of that suffix alone.  Reported rows count from row 0.
__host__ __device__ constexpr int rowpair_waves_per_group(bool lrec) { return lrec ? 16 : 8; }

template <int SEG, bool LREC, bool MASKED = false>
__global__ __launch_bounds__(rowpair_waves_per_group(LREC) * 64) __attribute__((amdgpu_waves_per_eu(4)))
void shared_rowpair_kernel(KArgs a) {
  if (a.plan_meta[kMetaErrResidue] | a.plan_meta[kMetaErrPair]) return;
  stage_matrix(a);
  __syncthreads();
  const uint32_t off = (matrix_lds_bytes(a.alpha) + 255) / 256 * 256;
  build_rowpair_profile<SEG>(a, off);
  __syncthreads();
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t snap = off + 2 * rp_copy_bytes(SEG, a.alpha) +
                        (uint32_t)(threadIdx.x >> 6) * ((SEG + kRecRows) * 256) + (uint32_t)lane * 4;
  const int sg = lane >> 4;
  const int nvalid = a.plan_meta[kMetaValid];
  const int ntasks = (nvalid + 3) / 4;
  const RpParams pr = make_rp_params<SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
  const uint32_t lane_base = off + (sg & 1) * rp_copy_bytes(SEG, a.alpha) + (lane & 15) * 4;
  const uint32_t sentw = (uint32_t)a.alpha * 0x01010101u;
  unsigned long long cols = 0, events = 0, padded = 0;
  for (;;) {
    const int ti = pop_task(a.plan_meta + kMetaCounter);
    if (ti >= ntasks) break;
    const int e = ti * 4 + sg;
    int pid = -1, n = 0;
    int64_t roff = 0;
    if (e < nvalid) {
      pid = a.order[e];
      const PairInfo p = a.pairs[pid];
      roff = p.r_off;
      n = p.n;
    }
    int nmax = n;
    for (int d = 16; d < kWave; d <<= 1) nmax = max(nmax, __shfl_xor(nmax, d));
    const int ncols = (nmax + kBlock - 1) / kBlock * kBlock;
    State<SEG> st;
    state_reset(st, 0u);
    if constexpr (LREC) record_lds_reset<SEG>(snap);
    const DirectSrc src{a.ref_res + roff, a.ref_res + roff, n, 0, sentw};
    uint32_t cap[SEG];
    if constexpr (MASKED) {
      const int r0 = pid >= 0 ? a.first_row[pid] : 0;
      const int lo0 = 2 * (lane & 15) * SEG;
#pragma unroll
      for (int j = 0; j < SEG; ++j)
        cap[j] = (lo0 + j < r0 ? 0u : 0x7fffu) | (lo0 + SEG + j < r0 ? 0u : 0x7fff0000u);
    }
    rp_run_columns<SEG, LREC, MASKED>(st, lane, pr, lane_base, src, ncols, snap, cap);
    cols += (unsigned long long)ncols;
    events += st.events;
    padded += (unsigned long long)min(4, nvalid - ti * 4) * ncols * 32 * SEG;
    rp_finish<SEG, LREC>(st, lane, pid, a.pairs, a.results, a.sat_cap, snap);
  }
  if (lane == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (events) atomicAdd(&a.stats[2], events);
    if (padded) atomicAdd(&a.stats[3], padded);
  }
}

// ================================================================ swapped striping

// The paper stripes the query over the lanes and streams the reference.  For
// a long query against short references the roles can swap: the reference
// is striped (lane l holds reference rows l*SEG + j) and the query streamed
// one residue per column, so a query of any length needs no chunks and its
// residues are the same for every lane (one word per four columns).  A
// per-reference profile would take (alpha+1) x rows bytes of LDS per
// alignment (40 KB for 2000 protein rows); instead every cell reads the
// substitution matrix itself, staged in LDS as [query code][ref code] with a
// sentinel row and column of -2^30: lane-constant byte offsets of its rows'
// reference codes plus the column's row offset (one address add per cell).
// One 64-lane alignment per wavefront, int32 lanes, the swapped record rule.
template <int SEG>
struct SwapProf {
  uint32_t roff[SEG];   // bytes: reference code of row l*SEG + j, times 4
  uint32_t snap;        // LDS bytes of this lane's end-cell copy (row j at + 256*j)
  __device__ __forceinline__ uint32_t load(uint32_t lo, uint32_t, int j) const {
    return *(const uint32_t *)(smem + lo + roff[j]);
  }
  __device__ __forceinline__ uint32_t snap_at(int j) const {
    return *(const uint32_t *)(smem + snap + 256 * j);
  }
  // The swapped record rule, with the copy of H in LDS (a wavefront's SEG x
  // 64 words) instead of SEG registers: a lane records when its column
  // maximum rises above its threshold, or ties it (above 0) in a row smaller
  // than the recorded one (rows of a record of a smaller value never block).
  __device__ __forceinline__ void record(State<SEG> &st, uint32_t cmax, int i) const {
    const int g = (int)st.G, cm = (int)cmax;
    const bool up = cm > g, tie = cm == g && g > 0;
    if (__any(up || tie)) {
      ++st.events;
      bool take = up;
      if (tie) {
        int rn = SEG, ro = SEG;
        const bool held = (int)st.S == g;
#pragma unroll
        for (int j = SEG - 1; j >= 0; --j) {
          if ((int)st.H[j] >= g) rn = j;
          if (held && (int)snap_at(j) >= g) ro = j;
        }
        take = rn < ro;
      }
      if (take) {
#pragma unroll
        for (int j = 0; j < SEG; ++j) *(uint32_t *)(smem + snap + 256 * j) = st.H[j];
        st.rc[0] = i;
        st.S = cmax;
      }
      st.G = (uint32_t)max(g, cm);
    }
  }
};
template <int SEG> struct SwapRecord<SwapProf<SEG>> { static constexpr bool value = true; };

template <int SEG>
struct SwapMap {
  SwapProf<SEG> prof;
  uint32_t row_bytes;   // (alpha + 1) * 4
  uint32_t alpha;       // codes above the alphabet read the sentinel row (the
                        // host reports them after the launch)
  __device__ __forceinline__ uint32_t base_lo(uint32_t c) const { return min(c, alpha) * row_bytes; }
  __device__ __forceinline__ uint32_t base_hi(uint32_t c) const { return base_lo(c); }
};

// LDS bytes of the padded matrix (16-byte aligned): the end-cell copy follows.
__host__ __device__ constexpr uint32_t swap_snap_offset(int alpha) {
  return (uint32_t)(((alpha + 1) * (alpha + 1) * 4 + 15) / 16 * 16);
}

// S[q][r] for q, r < alpha, -2^30 where either is the sentinel code alpha.
__device__ __forceinline__ void stage_matrix_padded(const KArgs &a) {
  int32_t *M = (int32_t *)smem;
  const int w = a.alpha + 1;
  for (int k = threadIdx.x; k < w * w; k += blockDim.x) {
    const int q = k / w, r = k % w;
    M[k] = (q < a.alpha && r < a.alpha) ? a.matrix[q * a.alpha + r] : -(1 << 30);
  }
}

__device__ __forceinline__ bool better_swap(int s, int r, int c, int s2, int r2, int c2) {
  return s > s2 || (s == s2 && (r < r2 || (r == r2 && c < c2)));
}

// Task t: pair tasks[t].pair[0], its query streamed over tasks[t].ncols
// columns (the query length rounded up to a block), its reference of at most
// 64*SEG rows striped.
template <int SEG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
void swap_kernel(KArgs a) {
  using O = OpsI32;
  stage_matrix_padded(a);
  __syncthreads();
  // LDS: the padded matrix, then the end-cell copy [SEG][64 lanes]
  const uint32_t snap0 = swap_snap_offset(a.alpha) + (uint32_t)(threadIdx.x & 63) * 4u;
  const LaneCtx L = make_lane<O>(0x1, SEG, (uint32_t)a.gap_extend);
  const Params pr = make_params<O, SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
  const uint32_t sentw = (uint32_t)a.alpha * 0x01010101u;
  uint32_t lazy_steps = 0;
  unsigned long long cols = 0, events = 0;
  for (;;) {
    const int ti = pop_task(a.task_counter);
    if (ti >= a.ntasks) break;
    const Task t = a.tasks[ti];
    const int pid = t.pair[0];
    const PairInfo p = a.pairs[pid];
    SwapMap<SEG> pm;
    pm.row_bytes = (uint32_t)(a.alpha + 1) * 4u;
    pm.alpha = (uint32_t)a.alpha;
    pm.prof.snap = snap0;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const int row = L.l * SEG + j;
      const int code = row < p.n ? min((int)a.ref_res[p.r_off + row], a.alpha) : a.alpha;
      pm.prof.roff[j] = (uint32_t)code * 4u;
    }
    State<SEG> st;
    state_reset(st, 0u);
    const uint8_t *qp = a.query_res + p.q_off;
    const DirectSrc src{qp, qp, p.m, p.m, sentw};
    run_columns<O, SEG, 64, false, false>(st, L, pr, pm, src, t.ncols, nullptr, nullptr, nullptr,
                                          nullptr, lazy_steps);
    cols += (unsigned long long)t.ncols;
    events += st.events;
    // smallest (score desc, row asc, column asc) over the wavefront
    int s = st.rc[0] != 0x7fffffff ? (int)st.S : 0;
    int r = 0x7fffffff, c = 0x7fffffff;
    if (s > 0) {
      int jj = SEG - 1;
#pragma unroll
      for (int j = SEG - 1; j >= 0; --j)
        if ((int)pm.prof.snap_at(j) >= s) jj = j;
      r = L.l * SEG + jj;
      c = st.rc[0];
    } else {
      s = 0;
    }
    for (int d = 1; d < kWave; d <<= 1) {
      const int s2 = __shfl_xor(s, d), r2 = __shfl_xor(r, d), c2 = __shfl_xor(c, d);
      if (better_swap(s2, r2, c2, s, r, c)) { s = s2; r = r2; c = c2; }
    }
    if (L.lane == 0) {
      DevResult res;
      res.score = s;
      res.qend = s > 0 ? c : -1;
      res.rend = s > 0 ? r : -1;
      res.flags = 0;
      a.results[p.out] = res;
    }
  }
  if ((threadIdx.x & 63) == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (events) atomicAdd(&a.stats[2], events);
  }
}

// ================================================================ per-pair kernel

// Each wavefront owns an LDS region [half][alpha+1][SEG][64 lanes]: lane x
// reads and writes only column x, so any sub-group partition works and no
// barrier is needed between building a profile and using it.  ES: bytes per
// entry, the lane type's or 1 (int8 entries, half or a quarter of the LDS).
template <class O, int SEG, int ES = O::kES>
struct PairMap {
  typename std::conditional<ES == 1, ProfLds8<O, kWave>, ProfLds<O, kWave * O::kES>>::type prof;
  uint32_t lo0, hi0;   // bytes: region + lane*ES (+ half offset)
  __device__ __forceinline__ uint32_t base_lo(uint32_t c) const { return lo0 + c * (SEG * kWave * ES); }
  __device__ __forceinline__ uint32_t base_hi(uint32_t c) const { return hi0 + c * (SEG * kWave * ES); }
};

__host__ __device__ constexpr uint32_t pair_region_bytes(int seg, int alpha, int halves, int es) {
  return (uint32_t)(halves * (alpha + 1) * seg * kWave * es);
}

// pids[h]: PairInfo index of this lane's sub-group in half h, or -1.  Rows
// past the query and the sentinel code get the most negative entry: any
// negative score keeps those cells below the alignment's best, since they
// follow every real cell in (column, row) order.
template <class O, int SEG, int ES = O::kES>
__device__ __forceinline__ void build_pair_profile(const KArgs &a, const int pids[2],
                                                   const LaneCtx &L, uint32_t region, int row0) {
  const int32_t *M = (const int32_t *)smem;
  const int nrow = a.alpha + 1;
#pragma unroll
  for (int h = 0; h < O::kHalves; ++h) {
    const int pid = pids[h];
    int m = 0;
    int64_t qo = 0;
    if (pid >= 0) { m = a.pairs[pid].m; qo = a.pairs[pid].q_off; }
    const uint32_t hbase = region + (uint32_t)(h * nrow * SEG * kWave * ES) + L.lane * ES;
    for (int j = 0; j < SEG; ++j) {
      const int row = row0 + L.l * SEG + j;
      int qc = row < m ? (int)a.query_res[qo + row] : -1;
      if (qc >= a.alpha) qc = -1;   // invalid codes are reported by the host check
      for (int c = 0; c < nrow; ++c) {
        const int v = (qc >= 0 && c < a.alpha) ? M[qc * a.alpha + c]
                                               : (ES == 1 ? -128 : (ES == 2 ? -32768 : (int)0x80000000));
        unsigned char *dst = smem + hbase + (c * SEG + j) * kWave * ES;
        if constexpr (ES == 1) *(signed char *)dst = (signed char)v;
        else if constexpr (ES == 2) *(short *)dst = (short)v;
        else *(int *)dst = v;
      }
    }
  }
}

template <class O, int SEG, int PMAX, bool CHUNKED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
void pair_kernel(KArgs a) {
  stage_matrix(a);
  __syncthreads();
  const uint32_t region = matrix_lds_bytes(a.alpha);
  uint32_t lazy_steps = 0;
  unsigned long long cols = 0, events = 0;
  for (;;) {
    const int ti = pop_task(a.task_counter);
    if (ti >= a.ntasks) break;
    const Task t = a.tasks[ti];
    const LaneCtx L = make_lane<O>(t.layout, SEG, (uint32_t)a.gap_extend);
    const Params pr = make_params<O, SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
    PairMap<O, SEG> pm;
    pm.lo0 = region + L.lane * O::kES;
    pm.hi0 = pm.lo0 + (O::kHalves == 2 ? (a.alpha + 1) * SEG * kWave * O::kES : 0);
    const int nch = CHUNKED ? t.nchunks : 1;
    Prev prev;
    prev_reset(prev);
    for (int ch = 0; ch < nch; ++ch) {
      const int row0 = ch * L.P * SEG;
      const int pids[2] = {t.pair[2 * L.sg], t.pair[2 * L.sg + 1]};
      build_pair_profile<O, SEG>(a, pids, L, region, row0);
      State<SEG> st;
      state_reset(st, prev_g0<O>(prev));
      const uint32_t *hb_in = nullptr, *fb_in = nullptr;
      uint32_t *hb_out = nullptr, *fb_out = nullptr;
      if constexpr (CHUNKED) {
        const int64_t base = t.bnd_off + (int64_t)L.sg * t.ncols;
        const int64_t fofs = 4ll * t.ncols;
        uint32_t *rd = a.bnd + (ch & 1) * a.bnd_half;
        uint32_t *wr = a.bnd + ((ch + 1) & 1) * a.bnd_half;
        hb_in = rd + base;
        fb_in = rd + base + fofs;
        if (ch + 1 < nch) { hb_out = wr + base; fb_out = wr + base + fofs; }
      }
      const StreamSrc src{(const uint2 *)(a.streams + t.stream_off) + L.sg};
      run_columns<O, SEG, PMAX, CHUNKED, false>(st, L, pr, pm, src, t.ncols, hb_in, fb_in,
                                                hb_out, fb_out, lazy_steps);
      cols += (unsigned long long)t.ncols;
      events += st.events;
      const int pid[2] = {t.pair[2 * L.sg], t.pair[2 * L.sg + 1]};
      finish<O, SEG>(st, L, pid, a.pairs, a.results, row0, prev, a.sat_cap);
    }
  }
  if ((threadIdx.x & 63) == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (events) atomicAdd(&a.stats[2], events);
  }
}

// Device-planned per-pair kernel: every pair has its own query (one query
// chunk, SEG rows per lane x P lanes at most), 64/P sub-groups of P = 8 or 16
// lanes per wavefront, in int16 mode two alignments per lane.  Task t is
// entries [t*slots, (t+1)*slots) of the planner's longest-first order (entry
// t*slots + s to sub-group s / halves, half s % halves); profiles (ES bytes
// per entry) are built per task in the wavefront's own LDS region; residues
// come from the references themselves.
__host__ __device__ constexpr int pair_direct_waves_per_eu(int seg, int P) {
  return (P == 8 && seg >= 16) ? 3 : 4;
}

template <class O, int SEG, int P, int ES>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(pair_direct_waves_per_eu(SEG, P))))
void pair_direct_kernel(KArgs a) {
  static_assert(P == 8 || P == 16, "sub-groups of 8 or 16 lanes");
  if (a.plan_meta[kMetaErrResidue] | a.plan_meta[kMetaErrPair]) return;
  stage_matrix(a);
  __syncthreads();
  const uint32_t region = matrix_lds_bytes(a.alpha);
  constexpr int kSlotsPerTask = (kWave / P) * O::kHalves;
  const int nvalid = a.plan_meta[kMetaValid];
  const int ntasks = (nvalid + kSlotsPerTask - 1) / kSlotsPerTask;
  const LaneCtx L = P == 8 ? make_lane8<O>(SEG, (uint32_t)a.gap_extend)
                           : make_lane<O>(0xF, SEG, (uint32_t)a.gap_extend);
  const Params pr = make_params<O, SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
  PairMap<O, SEG, ES> pm;
  pm.lo0 = region + L.lane * ES;
  pm.hi0 = pm.lo0 + (O::kHalves == 2 ? (a.alpha + 1) * SEG * kWave * ES : 0);
  const uint32_t sentw = (uint32_t)a.alpha * 0x01010101u;
  uint32_t lazy_steps = 0;
  unsigned long long cols = 0, events = 0, padded = 0;
  for (;;) {
    const int ti = pop_task(a.plan_meta + kMetaCounter);
    if (ti >= ntasks) break;
    int pid[2] = {-1, -1};
    int64_t roff[2] = {0, 0};
    int n[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < O::kHalves; ++h) {
      const int e = ti * kSlotsPerTask + L.sg * O::kHalves + h;
      if (e < nvalid) {
        pid[h] = a.order[e];
        const PairInfo p = a.pairs[pid[h]];
        roff[h] = p.r_off;
        n[h] = p.n;
      }
    }
    int nmax = max(n[0], n[1]);
    for (int d = 1; d < kWave; d <<= 1) nmax = max(nmax, __shfl_xor(nmax, d));
    const int ncols = (nmax + kBlock - 1) / kBlock * kBlock;
    build_pair_profile<O, SEG, ES>(a, pid, L, region, 0);
    Prev prev;
    prev_reset(prev);
    State<SEG> st;
    state_reset(st, 0u);
    const DirectSrc src{a.ref_res + roff[0], a.ref_res + roff[1], n[0], n[1], sentw};
    run_columns<O, SEG, P, false, false>(st, L, pr, pm, src, ncols, nullptr, nullptr, nullptr,
                                         nullptr, lazy_steps);
    cols += (unsigned long long)ncols;
    events += st.events;
    padded += (unsigned long long)min(kSlotsPerTask, nvalid - ti * kSlotsPerTask) * ncols * P * SEG;
    finish<O, SEG>(st, L, pid, a.pairs, a.results, 0, prev, a.sat_cap);
  }
  if ((threadIdx.x & 63) == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (events) atomicAdd(&a.stats[2], events);
    if (padded) atomicAdd(&a.stats[3], padded);
  }
}

// ================================================================ per-pair row pairs

// Pair-score table: word (qa*A1 + qb)*A1 + r (A1 = alpha+1) holds S(qa, r) in
// the low half and S(qb, r) in the high half, -32768 where a code is the
// padding / sentinel code alpha.  Shared by every wavefront of a workgroup; it
// replaces the per-pair query profile, so a lane's rows can be as many as its
// registers hold whatever the alphabet.
__host__ __device__ constexpr uint32_t rp_table_bytes(int alpha) {
  return (uint32_t)((alpha + 1) * (alpha + 1) * (alpha + 1) * 4);
}

__device__ void build_pair_table(const KArgs &a, uint32_t off) {
  const int32_t *M = (const int32_t *)smem;
  const int A1 = a.alpha + 1;
  const int total = A1 * A1 * A1;
  for (int k = threadIdx.x; k < total; k += blockDim.x) {
    const int r = k % A1;
    const int qb = (k / A1) % A1;
    const int qa = k / (A1 * A1);
    const int va = (qa < a.alpha && r < a.alpha) ? M[qa * a.alpha + r] : -32768;
    const int vb = (qb < a.alpha && r < a.alpha) ? M[qb * a.alpha + r] : -32768;
    *(uint32_t *)(smem + off + 4u * k) = ((uint32_t)va & 0xffffu) | ((uint32_t)vb << 16);
  }
}

// Best cell of one alignment so far (identical in every lane of its sub-group).
struct RpBest {
  int s, c, r;
  uint32_t f;
};

// Merges this chunk's records (rows row0 + (2l+h)*SEG + j) into `best`.
template <int SEG, int P>
__device__ __forceinline__ void rp_merge(const State<SEG> &st, int l, int row0, RpBest &best,
                                         int sat_cap) {
  using O = OpsI16;
  int s = 0, c = 0x7fffffff, r = 0x7fffffff;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int sh = st.rc[h] != 0x7fffffff ? O::get(st.S, h) : 0;
    if (sh > 0) {
      int jj = SEG - 1;
#pragma unroll
      for (int j = SEG - 1; j >= 0; --j)
        if (O::get(st.snap[j], h) >= sh) jj = j;
      const int ch = st.rc[h], rh = row0 + (2 * l + h) * SEG + jj;
      if (s <= 0 || better(sh, ch, rh, s, c, r)) { s = sh; c = ch; r = rh; }
    }
  }
  for (int d = 1; d < P; d <<= 1) {
    const int s2 = __shfl_xor(s, d), c2 = __shfl_xor(c, d), r2 = __shfl_xor(r, d);
    if (s2 > 0 && (s <= 0 || better(s2, c2, r2, s, c, r))) { s = s2; c = c2; r = r2; }
  }
  if (s >= sat_cap) best.f |= kFlagNeedsI32;
  if (s > 0 && (best.s <= 0 || better(s, c, r, best.s, best.c, best.r))) {
    best.s = s; best.c = c; best.r = r;
  }
}

// Column loop of one query chunk for the per-pair row-pair kernel: residues
// from the task's stream (the sub-group's low-half word), chunk boundaries as
// in run_columns (written by the sub-group's last lane, low 16 bits).
template <int SEG, bool CHUNKED, int P>
__device__ __forceinline__ void rp_pair_columns(State<SEG> &st, const RpLane &L,
                                                const RpParams &pr, const uint32_t (&qq)[SEG],
                                                const StreamSrc &src, int ncols,
                                                const uint32_t *hb_in, const uint32_t *fb_in,
                                                uint32_t *hb_out, uint32_t *fb_out) {
  const int nblk = ncols / kBlock;
  const bool first = L.l == 0, last = L.l == P - 1;
  uint32_t ev_shared = st.events;
  uint32_t rc = src.get(0).x;
  uint32_t rn = src.get(1).x;
  uint4 hbc, hbn, fbc, fbn;
  if constexpr (CHUNKED) {
    hbc = ((const uint4 *)hb_in)[0];
    hbn = ((const uint4 *)hb_in)[1];
    fbc = ((const uint4 *)fb_in)[0];
    fbn = ((const uint4 *)fb_in)[1];
  }
  for (int b = 0; b < nblk; ++b) {
    const uint32_t r = rc;
    rc = rn;
    rn = src.get(b + 2).x;
    uint4 hbv = make_uint4(0, 0, 0, 0), fbv = make_uint4(0, 0, 0, 0);
    if constexpr (CHUNKED) {
      hbv = hbc; hbc = hbn; hbn = ((const uint4 *)hb_in)[b + 2];
      fbv = fbc; fbc = fbn; fbn = ((const uint4 *)fb_in)[b + 2];
    }
    const uint32_t hin[kBlock] = {hbv.x, hbv.y, hbv.z, hbv.w};
    const uint32_t fin[kBlock] = {fbv.x, fbv.y, fbv.z, fbv.w};
    uint32_t ho[kBlock], fo[kBlock];
#pragma unroll
    for (int k = 0; k < kBlock; ++k) {
      const uint32_t c4 = __builtin_amdgcn_ubfe(r, 8 * k, 8) * 4u;
      const uint32_t ch = first ? (hin[k] & 0xffffu) : 0u;
      const uint32_t cf = first ? (fin[k] & 0xffffu) : 0u;
      rp_column<SEG, CHUNKED, RpPairs<SEG>, P>(st, pr, RpPairs<SEG>{qq, c4}, b * kBlock + k, ch,
                                               cf, ho[k], fo[k], &L);
    }
    if (CHUNKED && hb_out != nullptr && last) {
      ((uint4 *)hb_out)[b] = make_uint4(ho[0], ho[1], ho[2], ho[3]);
      ((uint4 *)fb_out)[b] = make_uint4(fo[0], fo[1], fo[2], fo[3]);
    }
    if (st.events != ev_shared) {
      rp_share_threshold_p<SEG, P>(st, L);
      ev_shared = st.events;
    }
  }
}

// Per-pair kernel in the row-pair layout (int16): one alignment per P-lane
// sub-group (task slot 2*sub_group), 2*P*SEG query rows per chunk, the pair-
// score table in LDS instead of per-pair profiles.  Tasks, residue streams and
// chunk boundaries are those of the host planner's per-pair launches.
// Wavefronts per SIMD: 16 rows per lane, or 12 with chunk boundaries, need
// more than 128 VGPRs.
__host__ __device__ constexpr int rp_pair_waves_per_eu(int seg, bool chunked) {
  return (seg >= 16 || (seg >= 12 && chunked)) ? 3 : 4;
}

template <int SEG, bool CHUNKED, int P>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(rp_pair_waves_per_eu(SEG, CHUNKED))))
void pair_rowpair_kernel(KArgs a) {
  stage_matrix(a);
  __syncthreads();
  const uint32_t off = matrix_lds_bytes(a.alpha);
  build_pair_table(a, off);
  __syncthreads();
  const RpLane L = make_rp_lane<P, SEG>((uint32_t)a.gap_extend);
  const int lane = L.lane, sg = L.sg, l = L.l;
  const int A1 = a.alpha + 1;
  const RpParams pr = make_rp_params<SEG>((uint32_t)a.gap_open, (uint32_t)a.gap_extend);
  unsigned long long cols = 0, events = 0;
  for (;;) {
    const int ti = pop_task(a.task_counter);
    if (ti >= a.ntasks) break;
    const Task t = a.tasks[ti];
    const int pid = t.pair[2 * sg];
    int m = 0;
    int64_t qo = 0;
    if (pid >= 0) {
      const PairInfo p = a.pairs[pid];
      m = p.m;
      qo = p.q_off;
    }
    const int nch = CHUNKED ? t.nchunks : 1;
    RpBest best{0, 0x7fffffff, 0x7fffffff, 0u};
    for (int ch = 0; ch < nch; ++ch) {
      const int row0 = ch * 2 * P * SEG;
      // this lane's row pairs: table rows of (query code of row (2l)*SEG + j,
      // query code of row (2l+1)*SEG + j), alpha past the query's end
      uint32_t qq[SEG];
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const int ra = row0 + 2 * l * SEG + j, rb = ra + SEG;
        const int qa = ra < m ? min((int)a.query_res[qo + ra], a.alpha) : a.alpha;
        const int qb = rb < m ? min((int)a.query_res[qo + rb], a.alpha) : a.alpha;
        qq[j] = off + (uint32_t)((qa * A1 + qb) * A1) * 4u;
      }
      State<SEG> st;
      const uint32_t g0 = best.s > 0 ? (uint32_t)(best.s - 1) : 0u;
      state_reset(st, OpsI16::splat(g0));
      const uint32_t *hb_in = nullptr, *fb_in = nullptr;
      uint32_t *hb_out = nullptr, *fb_out = nullptr;
      if constexpr (CHUNKED) {
        const int64_t base = t.bnd_off + (int64_t)sg * t.ncols;
        const int64_t fofs = 4ll * t.ncols;
        uint32_t *rd = a.bnd + (ch & 1) * a.bnd_half;
        uint32_t *wr = a.bnd + ((ch + 1) & 1) * a.bnd_half;
        hb_in = rd + base;
        fb_in = rd + base + fofs;
        if (ch + 1 < nch) { hb_out = wr + base; fb_out = wr + base + fofs; }
      }
      const StreamSrc src{(const uint2 *)(a.streams + t.stream_off) + sg};
      rp_pair_columns<SEG, CHUNKED, P>(st, L, pr, qq, src, t.ncols, hb_in, fb_in, hb_out, fb_out);
      cols += (unsigned long long)t.ncols;
      events += st.events;
      rp_merge<SEG, P>(st, l, row0, best, a.sat_cap);
    }
    if (l == 0 && pid >= 0) {
      DevResult res;
      res.score = best.s > 0 ? best.s : 0;
      res.qend = best.s > 0 ? best.r : -1;
      res.rend = best.s > 0 ? best.c : -1;
      res.flags = best.f;
      a.results[a.pairs[pid].out] = res;
    }
  }
  if (lane == 0 && a.stats != nullptr) {
    if (cols) atomicAdd(&a.stats[0], cols);
    if (events) atomicAdd(&a.stats[2], events);
  }
}

}  // namespace dev
}  // namespace swk
