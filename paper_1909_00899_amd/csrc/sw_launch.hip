// Residue-stream kernel and the launch dispatchers of libswscan.so.
#include "sw_device.h"
#include "sw_menus.h"

#include <algorithm>

namespace swk {

hipError_t launch_shared_i16(Alg alg, int menu, bool chunked, const KArgs &a, int grid,
                             hipStream_t st, uint32_t mask, size_t lds);
hipError_t launch_shared_i32(Alg alg, int menu, bool chunked, const KArgs &a, int grid,
                             hipStream_t st, uint32_t mask, size_t lds);
hipError_t launch_shared_dual_i32(int menu, bool chunked, const KArgs &a, int grid,
                                  hipStream_t st, uint32_t mask, size_t lds);
hipError_t launch_pair_i16(int seg, int pmax, bool chunked, const KArgs &a, int grid,
                           hipStream_t st, size_t lds);
hipError_t launch_pair_i32(int seg, int pmax, bool chunked, const KArgs &a, int grid,
                           hipStream_t st, size_t lds);
hipError_t launch_direct_i16(int shape, const KArgs &a, int grid, hipStream_t st, size_t lds);
hipError_t launch_direct_i32(int shape, const KArgs &a, int grid, hipStream_t st, size_t lds);
hipError_t launch_rowpair_i16(int seg, bool lds_records, const KArgs &a, int grid,
                              hipStream_t st, size_t lds);
hipError_t launch_pair_direct_i16(int seg, int es, const KArgs &a, int grid, hipStream_t st,
                                  size_t lds);
hipError_t launch_pair_direct8_i16(int seg, const KArgs &a, int grid, hipStream_t st, size_t lds);
hipError_t launch_pair_direct_i32(int seg, const KArgs &a, int grid, hipStream_t st, size_t lds);
hipError_t launch_pair_rowpair_i16(int seg, int lanes, bool chunked, const KArgs &a, int grid,
                                   hipStream_t st, size_t lds);

namespace dev {
// ================================================================ residue streams

// One workgroup per task: block b, slot-half s -> 4 residues (SENT past the end).
__global__ __launch_bounds__(256) void build_streams_kernel(const Task *tasks, const PairInfo *pairs,
                                                            const uint8_t *ref_res, uint8_t *streams,
                                                            int sent) {
  const Task t = tasks[blockIdx.x];
  const int nblk = t.ncols / kBlock;
  uint32_t *dst = (uint32_t *)(streams + t.stream_off);
  for (int k = threadIdx.x; k < nblk * kSlots; k += blockDim.x) {
    const int b = k / kSlots, s = k % kSlots;
    const int pid = tasks[blockIdx.x].pair[s];
    uint32_t w = (uint32_t)sent * 0x01010101u;
    if (pid >= 0) {
      const PairInfo p = pairs[pid];
      w = 0;
#pragma unroll
      for (int q = 0; q < kBlock; ++q) {
        const int i = b * kBlock + q;
        uint32_t c = i < p.n ? (uint32_t)ref_res[p.r_off + i] : (uint32_t)sent;
        c = c < (uint32_t)sent ? c : (uint32_t)sent;   // invalid codes are reported by the host check
        w |= c << (8 * q);
      }
    }
    dst[k] = w;
  }
}

// Sets *flag to 1 if any of the n residues is >= alpha.  Sixteen bytes per
// load between the first and the last 16-byte boundary of the array; the
// bytes before and after (fewer than 16 each) one per thread of the first
// workgroup.
__global__ __launch_bounds__(256) void check_residues_kernel(const uint8_t *p, int64_t n, int alpha,
                                                             int *flag) {
  const int64_t head = min(n, (int64_t)((16 - ((uintptr_t)p & 15)) & 15));
  const int64_t body = (n - head) / 16, tail0 = head + body * 16;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint4 *v = (const uint4 *)(p + head);
  int bad = 0;
  for (int64_t k = tid; k < body; k += stride) {
    const uint4 x = v[k];
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int b = 0; b < 32; b += 8) bad |= (int)((w[j] >> b) & 0xffu) >= alpha;
  }
  if (tid < head) bad |= p[tid] >= alpha;
  if (tid < n - tail0) bad |= p[tail0 + tid] >= alpha;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
// PairInfo of every pair from CSR offsets already on the device.
__global__ __launch_bounds__(256) void build_pairs_kernel(int n_pairs, const int64_t *qoff,
                                                          const int64_t *roff, const int32_t *pq,
                                                          const int32_t *pr, PairInfo *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  const int q = pq ? pq[k] : 0;
  const int r = pr[k];
  PairInfo p;
  p.q_off = qoff[q];
  p.r_off = roff[r];
  p.m = (int)(qoff[q + 1] - qoff[q]);
  p.n = (int)(roff[r + 1] - roff[r]);
  p.out = k;
  p.pad = 0;
  out[k] = p;
}
// ================================================================ device planner
//
// kPlanBlocks workgroups each take a contiguous range of pairs.  Counting and
// placing use LDS atomics only: every workgroup writes its own length
// histogram, one workgroup turns them into per-workgroup start positions of
// every bin, and each workgroup then places its pairs from those starts.

__device__ __forceinline__ int plan_bin(int n) { return min((n + kBlock - 1) / kBlock, kPlanBins - 1); }

__device__ __forceinline__ void plan_range(int n_pairs, int &lo, int &hi) {
  const int chunk = (n_pairs + kPlanBlocks - 1) / kPlanBlocks;
  lo = min(n_pairs, (int)blockIdx.x * chunk);
  hi = min(n_pairs, lo + chunk);
}

// One pair of plan_count_kernel: PairInfo, checks, empty result.  Returns n if
// the pair will run (m > 0 and n > 0), else 0; *m_out = its query length.
// qoff == nullptr: one query (id 0, length m, residues at q_off0); else the
// pair's own query from pq and the query offsets.
__device__ __forceinline__ int plan_one(int k, const int64_t *qoff, int n_queries, int64_t qbytes,
                                        const int64_t *roff, const int32_t *pq,
                                        const int32_t *pr, int n_refs, int64_t ref_bytes, int m,
                                        int64_t q_off0, PairInfo *pairs, DevResult *results,
                                        int32_t *meta, int &m_out) {
  const int q = pq ? pq[k] : 0;
  const int r = pr[k];
  bool ok = r >= 0 && r < n_refs;
  int64_t ro = 0, re = 0, qo = q_off0, qm = m;
  if (qoff == nullptr) {
    ok = ok && q == 0;
  } else {
    ok = ok && q >= 0 && q < n_queries;
    if (ok) {
      qo = qoff[q];
      const int64_t qe = qoff[q + 1];
      ok = qo >= 0 && qo <= qe && qe <= qbytes && qe - qo <= 0x7fffffffll;
      qm = qe - qo;
    }
  }
  if (ok) {
    ro = roff[r];
    re = roff[r + 1];
    ok = ro >= 0 && ro <= re && re <= ref_bytes && re - ro <= 0x7fffffffll;
  }
  if (!ok) {
    atomicOr(&meta[kMetaErrPair], 1);
    ro = re = 0;
    qo = 0;
    qm = 0;
  }
  PairInfo p;
  p.q_off = qo;
  p.r_off = ro;
  p.m = (int)qm;
  p.n = (int)(re - ro);
  p.out = k;
  p.pad = 0;
  pairs[k] = p;
  DevResult v;
  v.score = 0; v.qend = -1; v.rend = -1; v.flags = 0;
  results[k] = v;
  m_out = p.m;
  return p.m > 0 ? p.n : 0;
}

// PairInfo, validation, result initialisation and this workgroup's length
// histogram (block_hist[blockIdx.x][bin]); stats[4] += sum of n, stats[5] +=
// sum of m*n, meta[kMetaMaxM] = largest m, over the pairs that will run.
__global__ __launch_bounds__(1024) void plan_count_kernel(int n_pairs, const int64_t *qoff,
                                                          int n_queries, int64_t qbytes,
                                                          const int64_t *roff, const int32_t *pq,
                                                          const int32_t *pr, int n_refs,
                                                          int64_t ref_bytes, int m, int64_t q_off0,
                                                          PairInfo *pairs, DevResult *results,
                                                          int32_t *block_hist, int32_t *meta,
                                                          unsigned long long *stats) {
  __shared__ int32_t hist[kPlanBins];
  for (int b = threadIdx.x; b < kPlanBins; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  int lo, hi;
  plan_range(n_pairs, lo, hi);
  unsigned long long ns = 0, cs = 0;
  int mmax = 0;
  for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) {
    int mk = 0;
    const int n = plan_one(k, qoff, n_queries, qbytes, roff, pq, pr, n_refs, ref_bytes, m, q_off0,
                           pairs, results, meta, mk);
    if (n > 0) {
      atomicAdd(&hist[plan_bin(n)], 1);
      ns += (unsigned long long)n;
      cs += (unsigned long long)n * (unsigned long long)mk;
      mmax = max(mmax, mk);
    }
  }
  // one atomic per wavefront for each sum and the maximum
  for (int d = 1; d < kWave; d <<= 1) {
    ns += __shfl_xor(ns, d);
    cs += __shfl_xor(cs, d);
    mmax = max(mmax, __shfl_xor(mmax, d));
  }
  if ((threadIdx.x & 63) == 0) {
    if (ns) atomicAdd(&stats[4], ns);
    if (cs) atomicAdd(&stats[5], cs);
    if (mmax) atomicMax(&meta[kMetaMaxM], mmax);
  }
  __syncthreads();
  int32_t *out = block_hist + (size_t)blockIdx.x * kPlanBins;
  for (int b = threadIdx.x; b < kPlanBins; b += blockDim.x) out[b] = hist[b];
}

// One thread per bin: every workgroup's first position inside the bin
// (block_off[w][bin], counted from the bin's start) and the bin's total.
__global__ __launch_bounds__(256) void plan_total_kernel(const int32_t *block_hist,
                                                         int32_t *block_off, int32_t *totals) {
  const int bin = blockIdx.x * blockDim.x + threadIdx.x;
  if (bin >= kPlanBins) return;
  int v[kPlanBlocks];
#pragma unroll
  for (int w = 0; w < kPlanBlocks; ++w) v[w] = block_hist[(size_t)w * kPlanBins + bin];
  int run = 0;
#pragma unroll
  for (int w = 0; w < kPlanBlocks; ++w) {
    block_off[(size_t)w * kPlanBins + bin] = run;
    run += v[w];
  }
  totals[bin] = run;
}

// Places this workgroup's runnable pairs (the same range as plan_count): the
// bins' starts in the longest-first order (an exclusive scan of the totals
// from the longest bin down, redone by every workgroup) plus the workgroup's
// offset inside each bin give LDS cursors.  Workgroup 0 also publishes the
// number of entries and clears the alignment kernel's task counter.
__global__ __launch_bounds__(1024) void plan_scatter_kernel(int n_pairs, const PairInfo *pairs,
                                                            const int32_t *totals,
                                                            const int32_t *block_off,
                                                            int32_t *order, int32_t *meta) {
  constexpr int kPer = kPlanBins / 1024;
  __shared__ int32_t part[1024];
  __shared__ int32_t cursor[kPlanBins];
  const int t = threadIdx.x;
  // thread t owns positions [t*kPer, (t+1)*kPer) of the descending order
  int v[kPer], sum = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    v[q] = totals[kPlanBins - 1 - (t * kPer + q)];
    sum += v[q];
  }
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int x = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  int run = part[t] - sum;   // exclusive prefix of this thread's positions
  const int32_t *off = block_off + (size_t)blockIdx.x * kPlanBins;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int bin = kPlanBins - 1 - (t * kPer + q);
    cursor[bin] = run + off[bin];
    run += v[q];
  }
  if (blockIdx.x == 0 && t == 1023) {
    meta[kMetaValid] = part[1023];
    meta[kMetaCounter] = 0;
  }
  __syncthreads();
  int lo, hi;
  plan_range(n_pairs, lo, hi);
  for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) {
    const PairInfo p = pairs[k];
    if (p.m > 0 && p.n > 0) order[atomicAdd(&cursor[plan_bin(p.n)], 1)] = k;
  }
}

// Segment t of dst (bytes [dst_off[t], dst_off[t+1])) = the same number of
// bytes of src from src_off[t] on, in reverse order; a wavefront per segment
// (grid-stride over the segments), four bytes per lane per step, so a short
// segment (a 150-residue read) is one step and a long one moves 256 bytes a
// step.
__global__ __launch_bounds__(256) void reverse_segments_kernel(int n, const uint8_t *src,
                                                               const int64_t *src_off,
                                                               const int64_t *dst_off,
                                                               uint8_t *dst) {
  const int lane = threadIdx.x & (kWave - 1);
  const int per_block = blockDim.x / kWave;
  const int stride = gridDim.x * per_block;
  for (int t = blockIdx.x * per_block + threadIdx.x / kWave; t < n; t += stride) {
    const int64_t d0 = dst_off[t], len = dst_off[t + 1] - d0, s_last = src_off[t] + len - 1;
    for (int64_t x = 4 * lane; x < len; x += 4 * kWave) {
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (x + b < len) dst[d0 + x + b] = src[s_last - x - b];
    }
  }
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}
// *count += the results that carry a flag of `mask` (one atomic per
// wavefront that saw one).
__global__ __launch_bounds__(256) void count_flag_kernel(int n, const DevResult *r, uint32_t mask,
                                                         int32_t *count) {
  const int stride = gridDim.x * blockDim.x;
  int c = 0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    c += (r[k].flags & mask) != 0 ? 1 : 0;
  for (int d = 1; d < kWave; d <<= 1) c += __shfl_xor(c, d);
  if (c != 0 && (threadIdx.x & 63) == 0) atomicAdd(count, c);
}
// out[k] = the int32 result r32[k] with SW_FLAG_SATURATED for every pair
// whose int16 lanes asked for the rerun.
__global__ __launch_bounds__(256) void merge_rerun_kernel(int n, const DevResult *r32,
                                                          DevResult *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && (out[k].flags & kFlagNeedsI32)) {
    DevResult v = r32[k];
    v.flags = kFlagSaturated;
    out[k] = v;
  }
}
__global__ __launch_bounds__(256) void init_results_kernel(int n, DevResult *r) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    DevResult v;
    v.score = 0; v.qend = -1; v.rend = -1; v.flags = 0;
    r[k] = v;
  }
}
}  // namespace dev

hipError_t launch_reverse_segments(int n, const uint8_t *src, const int64_t *src_off,
                                   const int64_t *dst_off, uint8_t *dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::reverse_segments_kernel, dim3(std::min((n + 3) / 4, 65535)), dim3(256), 0,
                     st, n, src, src_off, dst_off, dst);
  return hipGetLastError();
}

hipError_t launch_init_results(int n, DevResult *r, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::init_results_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, r);
  return hipGetLastError();
}

hipError_t launch_count_flag(int n, const DevResult *r, uint32_t mask, int32_t *count,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = std::min((n + 255) / 256, 1024);
  hipLaunchKernelGGL(dev::count_flag_kernel, dim3(grid), dim3(256), 0, st, n, r, mask, count);
  return hipGetLastError();
}

hipError_t launch_merge_rerun(int n, const DevResult *r32, DevResult *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::merge_rerun_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, r32,
                     out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(dev::fill_u32_kernel, dim3(grid), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_build_pairs(int n_pairs, const int64_t *qoff, const int64_t *roff,
                              const int32_t *pq, const int32_t *pr, PairInfo *out,
                              hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::build_pairs_kernel, dim3((n_pairs + 255) / 256), dim3(256), 0, st,
                     n_pairs, qoff, roff, pq, pr, out);
  return hipGetLastError();
}

hipError_t launch_check_residues(const uint8_t *p, int64_t n, int alpha, int *flag,
                                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  // one 16-byte load per thread per step; at least one workgroup for the
  // unaligned head and tail
  int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n / 16 + 255) / 256, 4096));
  hipLaunchKernelGGL(dev::check_residues_kernel, dim3(grid), dim3(256), 0, st, p, n, alpha, flag);
  return hipGetLastError();
}

hipError_t launch_plan_count(int n_pairs, const int64_t *qoff, int n_queries, int64_t qbytes,
                             const int64_t *roff, const int32_t *pq, const int32_t *pr, int n_refs,
                             int64_t ref_bytes, int m, int64_t q_off0, PairInfo *pairs,
                             DevResult *results, int32_t *block_hist, int32_t *meta,
                             unsigned long long *stats, hipStream_t st) {
  hipLaunchKernelGGL(dev::plan_count_kernel, dim3(kPlanBlocks), dim3(1024), 0, st, n_pairs, qoff,
                     n_queries, qbytes, roff, pq, pr, n_refs, ref_bytes, m, q_off0, pairs, results,
                     block_hist, meta, stats);
  return hipGetLastError();
}

bool pair_direct_has(int seg, int lanes) {
  if (lanes == 8) {
    for (int v : kPair8Segs)
      if (v == seg) return true;
    return false;
  }
  if (lanes != 16) return false;
  for (int v : kPairSegs)
    if (v == seg) return true;
  return false;
}

size_t pair_direct_lds_bytes(Prec prec, int seg, int alpha, int es) {
  const int halves = prec == PREC_I16X2 ? 2 : 1;
  return matrix_lds_bytes(alpha) + (size_t)dev::pair_region_bytes(seg, alpha, halves, es);
}

hipError_t launch_pair_direct(Prec prec, int seg, int lanes, int es, const KArgs &a, int grid,
                              hipStream_t st) {
  if (!pair_direct_has(seg, lanes) || a.order == nullptr || a.plan_meta == nullptr ||
      a.ref_res == nullptr)
    return hipErrorInvalidValue;
  const size_t lds = pair_direct_lds_bytes(prec, seg, a.alpha, es);
  if (prec == PREC_I16X2) {
    if (lanes == 8) return es == 1 ? launch_pair_direct8_i16(seg, a, grid, st, lds) : hipErrorInvalidValue;
    return launch_pair_direct_i16(seg, es, a, grid, st, lds);
  }
  if (lanes != 16 || es != 4) return hipErrorInvalidValue;
  return launch_pair_direct_i32(seg, a, grid, st, lds);
}

hipError_t launch_plan_total(const int32_t *block_hist, int32_t *block_off, int32_t *totals,
                             hipStream_t st) {
  hipLaunchKernelGGL(dev::plan_total_kernel, dim3((kPlanBins + 255) / 256), dim3(256), 0, st,
                     block_hist, block_off, totals);
  return hipGetLastError();
}

hipError_t launch_plan_scatter(int n_pairs, const PairInfo *pairs, const int32_t *totals,
                               const int32_t *block_off, int32_t *order, int32_t *meta,
                               hipStream_t st) {
  static_assert(kPlanBins % 1024 == 0, "plan bins");
  hipLaunchKernelGGL(dev::plan_scatter_kernel, dim3(kPlanBlocks), dim3(1024), 0, st, n_pairs,
                     pairs, totals, block_off, order, meta);
  return hipGetLastError();
}

static int direct_shape_index(int seg, int lanes) {
  for (int k = 0; k < kNumDirectShapes; ++k)
    if (kDirectShapes[k].seg == seg && kDirectShapes[k].lanes == lanes) return k;
  return -1;
}

bool shared_direct_has(Prec, int seg, int lanes) { return direct_shape_index(seg, lanes) >= 0; }

size_t shared_direct_lds_bytes(Prec prec, int seg, int lanes, int alpha) {
  const int es = prec == PREC_I16X2 ? 2 : 4;
  return matrix_lds_bytes(alpha) + (size_t)(alpha + 1) * dev::shared_cstride(seg, lanes, es);
}

hipError_t launch_shared_direct(Prec prec, int seg, int lanes, const KArgs &a, int grid,
                                hipStream_t st) {
  const int k = direct_shape_index(seg, lanes);
  if (k < 0 || a.order == nullptr || a.plan_meta == nullptr || a.ref_res == nullptr)
    return hipErrorInvalidValue;
  const size_t lds = shared_direct_lds_bytes(prec, seg, lanes, a.alpha);
  if (prec == PREC_I16X2) return launch_direct_i16(k, a, grid, st, lds);
  return launch_direct_i32(k, a, grid, st, lds);
}

bool shared_rowpair_has(int seg) { return seg == 4 || seg == 8 || seg == 12 || seg == 16; }

size_t shared_rowpair_lds_bytes(int seg, int alpha) {
  return (matrix_lds_bytes(alpha) + 255) / 256 * 256 + 2 * (size_t)dev::rp_copy_bytes(seg, alpha);
}

// With the end-cell records in LDS as well: one workgroup of 16 wavefronts
// per CU (160 KB of LDS).
static size_t rowpair_lds_records_bytes(int seg, int alpha) {
  return shared_rowpair_lds_bytes(seg, alpha) +
         (size_t)dev::rowpair_waves_per_group(true) * (seg + dev::kRecRows) * 256;
}

bool shared_rowpair_lds_records_fit(int seg, int alpha) {
  return rowpair_lds_records_bytes(seg, alpha) <= 160 * 1024;
}

hipError_t launch_shared_rowpair(int seg, const KArgs &a, int grid, hipStream_t st, int lrec) {
  if (!shared_rowpair_has(seg) || a.order == nullptr || a.plan_meta == nullptr ||
      a.ref_res == nullptr)
    return hipErrorInvalidValue;
  const size_t with = rowpair_lds_records_bytes(seg, a.alpha);
  if (lrec != 0 && with <= 160 * 1024) return launch_rowpair_i16(seg, true, a, grid, st, with);
  return launch_rowpair_i16(seg, false, a, grid, st, shared_rowpair_lds_bytes(seg, a.alpha));
}

bool pair_rowpair_has(int seg, int alpha) {
  return (seg == 4 || seg == 8 || seg == 12 || seg == 16) && pair_rowpair_lds_bytes(alpha) <= 65536;
}

size_t pair_rowpair_lds_bytes(int alpha) {
  return matrix_lds_bytes(alpha) + dev::rp_table_bytes(alpha);
}

hipError_t launch_pair_rowpair(int seg, int lanes, bool chunked, const KArgs &a, int grid,
                               hipStream_t st) {
  if (!pair_rowpair_has(seg, a.alpha) || (lanes != 16 && lanes != 32 && lanes != 64))
    return hipErrorInvalidValue;
  return launch_pair_rowpair_i16(seg, lanes, chunked, a, grid, st, pair_rowpair_lds_bytes(a.alpha));
}

int shared_menu_count() { return kNumSharedMenus; }
SharedMenu shared_menu(int idx) { return kSharedMenus[idx]; }

size_t shared_lds_bytes(Prec prec, int menu, int alpha) {
  const int es = prec == PREC_I16X2 ? 2 : 4;
  const SharedMenu m = kSharedMenus[menu];
  size_t b = matrix_lds_bytes(alpha);
  if (m.seg16) b += (size_t)(alpha + 1) * dev::shared_cstride(m.seg16, 16, es);
  if (m.seg32) b += (size_t)(alpha + 1) * dev::shared_cstride(m.seg32, 32, es);
  if (m.seg64) b += (size_t)(alpha + 1) * dev::shared_cstride(m.seg64, 64, es);
  return b;
}

hipError_t launch_shared(Prec prec, Alg alg, int menu, bool chunked, bool dual, const KArgs &a,
                         int grid, hipStream_t st) {
  if (menu < 0 || menu >= kNumSharedMenus) return hipErrorInvalidValue;
  const size_t lds = shared_lds_bytes(prec, menu, a.alpha);
  if (prec == PREC_I16X2) return dual ? hipErrorInvalidValue : launch_shared_i16(alg, menu, chunked, a, grid, st, 7u, lds);
  if (dual) return alg == ALG_SCAN ? launch_shared_dual_i32(menu, chunked, a, grid, st, 7u, lds)
                                   : hipErrorInvalidValue;
  return launch_shared_i32(alg, menu, chunked, a, grid, st, 7u, lds);
}

bool pair_kernel_has(Prec, int seg, int pmax) {
  bool s = false;
  for (int v : kPairSegs) s |= v == seg;
  return s && (pmax == 16 || pmax == 32 || pmax == 64);
}

size_t pair_lds_bytes(Prec prec, int seg, int alpha) {
  const int es = prec == PREC_I16X2 ? 2 : 4;
  const int halves = prec == PREC_I16X2 ? 2 : 1;
  return matrix_lds_bytes(alpha) + (size_t)dev::pair_region_bytes(seg, alpha, halves, es);
}

hipError_t launch_pair(Prec prec, int seg, int pmax, bool chunked, const KArgs &a, int grid,
                       hipStream_t st) {
  if (!pair_kernel_has(prec, seg, pmax)) return hipErrorInvalidValue;
  const size_t lds = pair_lds_bytes(prec, seg, a.alpha);
  if (prec == PREC_I16X2) return launch_pair_i16(seg, pmax, chunked, a, grid, st, lds);
  return launch_pair_i32(seg, pmax, chunked, a, grid, st, lds);
}

hipError_t launch_build_streams(const Task *tasks, int ntasks, const PairInfo *pairs,
                                const uint8_t *ref_res, uint8_t *streams, int sent_code,
                                hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::build_streams_kernel, dim3(ntasks), dim3(256), 0, st, tasks, pairs,
                     ref_res, streams, sent_code);
  return hipGetLastError();
}

}  // namespace swk
