/*
 * sw.h -- C ABI of the MI355X striped-scan Smith-Waterman library (libswscan.so).
 *
 * Operation (paper: Background section, problem statement; Algorithm 6,
 * "Striped Smith-Waterman Scan"): the optimal LOCAL alignment score of a query
 * q[0..m) against a reference r[0..n) under a substitution matrix S and affine
 * gap penalties, plus the cell where a best alignment ends.
 *
 *   Hd(i,j) = H(i-1,j-1) + S[q_j][r_i]
 *   E(i,j)  = max(E(i-1,j) - GapExtend, H(i-1,j) - GapOpen)
 *   F(i,j)  = max(F(i,j-1) - GapExtend, H(i,j-1) - GapOpen)
 *   H(i,j)  = max(0, Hd(i,j), E(i,j), F(i,j))
 *   score   = max(0, max over all cells of Hd)
 *
 * i runs over the reference (the outer loop of the paper's algorithms), j over
 * the query.  A gap of length L costs GapOpen + (L-1)*GapExtend.  The paper's
 * algorithms require GapExtend <= GapOpen; the library uses
 * min(GapExtend, GapOpen), which gives the same scores for every input
 * (re-opening a gap at every residue already costs GapOpen per residue).
 *
 * End cell (not in the paper, which returns only the maximum): 0-based
 * inclusive (query_end, ref_end) of the Hd cell achieving the score; among
 * ties the smallest ref_end, then the smallest query_end.  (-1, -1) iff the
 * score is 0.
 *
 * Residues are alphabet codes 0..alphabet_size-1 (uint8).  All integers are
 * host-endian.  Every call returns an sw_status code; none aborts, throws or
 * sets errno.  Calls are thread-safe; they serialise on one internal lock per
 * device.  The library uses the HIP device that is current when sw_init (or
 * the first call) runs.
 */
#ifndef SW_H_
#define SW_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SW_OK = 0,
    SW_PENDING = 1,      /* sw_server_poll: request not finished yet              */
    SW_EINVAL = -1,      /* bad argument: NULL pointer, negative length or penalty,
                            residue >= alphabet_size, alphabet_size outside 1..32,
                            bad option value                                      */
    SW_ENOMEM = -2,      /* device or host allocation failed, or a server request
                            can never fit the server's memory budget             */
    SW_EDEVICE = -3,     /* a HIP call failed (text via sw_last_error)            */
    SW_EOVERFLOW = -4,   /* min(m, n) * max(0, max S) >= 2^31 - 1                  */
    SW_ENOENT = -5,      /* unknown or already-collected server ticket            */
    SW_EBUSY = -6        /* server queue full; retry later                        */
} sw_status;

/* Scoring scheme.  matrix is alphabet_size^2 int32, row-major, indexed
 * matrix[query_code * alphabet_size + ref_code] (the paper's query profile
 * holds S[query residue][reference residue]).  gap_open and gap_extend must be
 * >= 0.  The caller owns matrix; the library copies it during each call. */
typedef struct {
    int32_t alphabet_size;      /* 1..32 */
    const int32_t *matrix;
    int32_t gap_open;           /* cost of a gap's first residue         */
    int32_t gap_extend;         /* cost of each further residue          */
} sw_scoring;

#define SW_FLAG_SATURATED 1u    /* int16 lanes saturated; result recomputed in int32 */

typedef struct {
    int32_t score;              /* >= 0 */
    int32_t query_end;          /* 0-based inclusive; -1 iff score == 0 */
    int32_t ref_end;            /* 0-based inclusive; -1 iff score == 0 */
    uint32_t flags;             /* SW_FLAG_* */
} sw_result;

/* Human-readable text of a status code (static storage). */
const char *sw_strerror(int code);

/* Text of the last SW_EDEVICE / SW_ENOMEM error on this thread ("" if none). */
const char *sw_last_error(void);

/* Select and initialise the device (optional; the first call does it with
 * the current device).  Returns SW_EDEVICE if no gfx950 device is usable. */
int sw_init(int device);

/* Release every device buffer the library holds.  Servers must be destroyed
 * first.  The library may be used again afterwards. */
int sw_shutdown(void);

/* ---------------------------------------------------------------------------
 * sw_align -- one pair, one kernel launch ("plain" form of Algorithm 6).
 *
 * The query is striped over one wavefront sub-group (lanes x segLen query rows,
 * paper: Algorithm 6 and the striped layout it inherits); every reference
 * residue is one column step; the vertical-gap correction is the max-plus
 * scan over lanes.  int32 arithmetic, exact while min(m,n)*max S < 2^31-1.
 * query/ref are HOST buffers (copied before return); out is host memory.
 * Empty query or reference is valid and yields {0, -1, -1, 0}.
 * ------------------------------------------------------------------------- */
int sw_align(const uint8_t *query, int32_t query_len,
             const uint8_t *ref, int32_t ref_len,
             const sw_scoring *sc, sw_result *out);

/* ---------------------------------------------------------------------------
 * sw_align_batch -- many pairs of uneven lengths in one persistent launch.
 *
 * Queries and references are CSR: residues concatenated, offsets of length
 * count+1 (int64, nondecreasing, offsets[0] == 0).  Pair k aligns query
 * pair_query[k] (or query 0 if pair_query is NULL) with reference
 * pair_ref[k].  out[k] receives pair k's result (host memory, n_pairs
 * entries).
 *
 * precision: SW_PREC_AUTO runs packed int16x2 lanes (two alignments per
 * 32-bit lane) and recomputes in int32 every pair whose int16 maximum reached
 * 32767 (the int16 result is exact iff its maximum is below 32767, because
 * every H, E and F value is bounded by the running maximum); the recomputed
 * result carries SW_FLAG_SATURATED.  SW_PREC_I32 runs int32 only.
 *
 * Every residue in query_res[0 .. query_off[n_queries]) and
 * ref_res[0 .. ref_off[n_refs]) must be below alphabet_size (SW_EINVAL
 * otherwise), whether or not a pair uses it.
 *
 * device_resident: 0 => the six sequence/offset/pair pointers are host
 * memory; 1 => they are device memory on the library's device (e.g. torch
 * tensors) and must stay valid until the call returns.  The call is
 * synchronous either way.
 * ------------------------------------------------------------------------- */
enum { SW_PREC_AUTO = 0, SW_PREC_I32 = 1 };

typedef struct {
    int32_t n_pairs;
    const uint8_t *query_res; const int64_t *query_off; int32_t n_queries;
    const uint8_t *ref_res;   const int64_t *ref_off;   int32_t n_refs;
    const int32_t *pair_query;   /* n_pairs entries or NULL (=> query 0) */
    const int32_t *pair_ref;     /* n_pairs entries                      */
    int32_t precision;           /* SW_PREC_*                             */
    int32_t device_resident;     /* 0 host, 1 device                      */
    void *stream;                /* hipStream_t to order device-resident inputs
                                    against, or NULL for the default stream */
} sw_batch;

int sw_align_batch(const sw_batch *b, const sw_scoring *sc, sw_result *out);

/* ---------------------------------------------------------------------------
 * sw_align_batch_starts -- start cells of the alignments a batch call found.
 *
 * The paper's method returns only the maximum score (Algorithm 6 keeps Max);
 * start cells are this library's extension.  For pair k with
 * ends[k].score > 0 (ends: the n_pairs results sw_align_batch returned for
 * the same batch and scoring), query_start[k] / ref_start[k] receive the start
 * of an optimal alignment ending at (ends[k].query_end, ends[k].ref_end): of
 * all such alignments, the one with the largest ref_start, then the largest
 * query_start (0-based, inclusive).  Pairs with score 0 get -1, -1.
 *
 * Computed by aligning the reversed prefixes q[0 .. query_end] and
 * r[0 .. ref_end] with the batch path itself (same kernels and precision
 * rules); their optimum must equal ends[k].score, so an end cell that is
 * not the pair's optimum gives SW_EINVAL.  Also SW_EINVAL for NULL arrays,
 * pair ids or offsets out of range, or an end cell outside its sequences.
 * The batch's arrays follow sw_align_batch's rules (device_resident
 * included); ends, query_start and ref_start are host arrays of n_pairs
 * entries owned by the caller.  Synchronous; calls are serialised.
 * ------------------------------------------------------------------------- */
int sw_align_batch_starts(const sw_batch *b, const sw_scoring *sc, const sw_result *ends,
                          int32_t *query_start, int32_t *ref_start);

/* ---------------------------------------------------------------------------
 * sw_align_batch_cigar -- paths (CIGAR runs) of the alignments a batch call
 * found.
 *
 * The paper returns only the score; paths are this library's extension.  For
 * pair k with ends[k].score > 0 and its start cell (query_start[k],
 * ref_start[k]) as sw_align_batch_starts returns it, the path of an
 * alignment of score ends[k].score from the start to the end cell, as runs
 * (length << 4 | op; op SW_CIGAR_M: aligned pairs, SW_CIGAR_I: query
 * residues skipped, SW_CIGAR_D: reference residues skipped; the BAM codes).
 * Of all such alignments, walking back from the end cell, the aligned pair
 * before each aligned pair is the largest (ref index, then query index) on
 * an optimal path; between two aligned pairs the D run comes before the I
 * run.  A gap run of length L costs gap_open + (L - 1) * min(gap_extend,
 * gap_open), the cost the scores are computed with.
 *
 * Output, packed: pair k's runs are cigar[cigar_off[k] .. cigar_off[k+1])
 * (none for score 0); cigar_off has n_pairs + 1 entries, cigar_off[0] = 0.
 * Pair k never needs more than min(A + B - 1, 3 min(A, B) - 2) runs, with
 * A = ref_end - ref_start + 1 and B = query_end - query_start + 1.  If the
 * total exceeds cigar_cap, cigar_off is still filled, cigar is not written,
 * and SW_EINVAL is returned.
 *
 * Computed on the device: one wavefront per pair fills the rectangle between
 * start and end cell, anchored at the start, keeping four decision bits per
 * cell (in LDS when they fit, else in device scratch of at most 1 GiB per
 * launch, up to three launches at once on streams of the library's own),
 * then walks them back from the end cell.
 *
 * SW_EINVAL: NULL arrays, pair ids or offsets out of range, a start cell
 * after its end cell or an end cell outside its sequences, no alignment of
 * score ends[k].score from the start to the end cell, a residue not below
 * alphabet_size inside a rectangle, or too small a cigar_cap.  SW_EOVERFLOW:
 * a rectangle whose anchored scores could leave the kernel's int32 range
 * (about 2^27 / (gap_extend + 1) cells along its sides).  SW_ENOMEM: a
 * rectangle needing more than 2 GiB of decision bits.  The batch's arrays
 * follow sw_align_batch's rules (device_resident included); ends,
 * query_start, ref_start, cigar and cigar_off are host arrays owned by the
 * caller.  Synchronous; calls are serialised with sw_align_batch_starts.
 * ------------------------------------------------------------------------- */
enum { SW_CIGAR_M = 0, SW_CIGAR_I = 1, SW_CIGAR_D = 2 };
int sw_align_batch_cigar(const sw_batch *b, const sw_scoring *sc, const sw_result *ends,
                         const int32_t *query_start, const int32_t *ref_start,
                         uint32_t *cigar, int64_t cigar_cap, int64_t *cigar_off);

/* ---------------------------------------------------------------------------
 * sw_align_batch_global -- end-to-end alignment scores of a batch.
 *
 * Not in the paper (whose problem is local alignment): the same affine gap
 * model without the zero floor.  An alignment is a chain of aligned pairs
 * strictly increasing in both sequences; it scores the substitution scores of
 * its pairs minus gap_open + (L - 1) * min(gap_extend, gap_open) for every
 * run of L skipped residues (between two pairs the skipped reference residues
 * and the skipped query residues are one run each).
 *
 * mode SW_MODE_GLOBAL: every residue of both sequences is aligned or skipped
 *   at a cost, including before the first and after the last pair.
 *   query_end = m - 1, ref_end = n - 1.
 * mode SW_MODE_SEMIGLOBAL: the query end to end as above; reference residues
 *   before the first and after the last pair are free (a read placed inside
 *   a reference window).  query_end = m - 1; ref_end = the smallest
 *   reference prefix end a (-1: the empty prefix) such that the best
 *   alignment of the query inside r[0..a], with the reference residues after
 *   its last pair up to a counted as a gap run, reaches the score.
 * mode SW_MODE_SEMIGLOBAL_REF: the same with the roles swapped: the
 *   reference end to end, query residues before the first and after the last
 *   pair free (a short reference placed inside a long query).  ref_end =
 *   n - 1; query_end = the smallest query prefix end b (-1: the empty
 *   prefix) whose best alignment, with the query residues after its last
 *   pair up to b counted as a gap run, reaches the score.
 * mode SW_MODE_OVERLAP: free end gaps: before the first pair the skipped
 *   residues of one of the two sequences are free and the other's cost a
 *   run, and likewise after the last pair (a dovetail of the two sequences,
 *   or one contained in the other); the empty alignment scores 0.  The end
 *   cell lies on the query's last residue (query_end = m - 1, any ref_end
 *   from -1, the reference after it free) or on the reference's last residue
 *   (ref_end = n - 1, any query_end from -1); of the end cells whose best
 *   alignment reaches the score, the smallest ref_end, then the smallest
 *   query_end.
 *
 * out[k] receives pair k's {score, query_end, ref_end, 0}; scores may be
 * negative.  An empty side gives the charged gap run of the other (or 0).
 * Computed in int32 by one wavefront per pair (the query in 256-column tiles,
 * a max-plus scan over the lanes for the query gap); SW_EOVERFLOW for a pair
 * whose scores could leave that range (about 2^27 / (gap_extend + 1) residues
 * in m + n).  SW_EINVAL for a bad mode, NULL arrays, ids or offsets out of
 * range, or a residue not below alphabet_size.  The batch's arrays follow
 * sw_align_batch's rules (device_resident included; precision is ignored);
 * out is a host array of n_pairs entries.  Synchronous; calls are serialised
 * with sw_align_batch_starts and sw_align_batch_cigar.
 * ------------------------------------------------------------------------- */
enum { SW_MODE_GLOBAL = 0, SW_MODE_SEMIGLOBAL = 1, SW_MODE_SEMIGLOBAL_REF = 2,
       SW_MODE_OVERLAP = 3 };
int sw_align_batch_global(const sw_batch *b, const sw_scoring *sc, int32_t mode,
                          sw_result *out);

/* ---------------------------------------------------------------------------
 * sw_align_batch_global_cigar -- paths of the end-to-end alignments a
 * sw_align_batch_global call found (same batch, scoring and mode; ends: its
 * n_pairs results, or any end cell of the mode with the best score there).
 *
 * Pair k's alignment runs from a virtual start element to its end cell: the
 * element is (-1, -1) for SW_MODE_GLOBAL; (v, -1), v >= -1, r[0..v] being a
 * free reference prefix, for SW_MODE_SEMIGLOBAL and SW_MODE_OVERLAP; (-1, w),
 * q[0..w] being a free query prefix, for SW_MODE_SEMIGLOBAL_REF and
 * SW_MODE_OVERLAP (element coordinates are (ref index, query index)).
 * Walking back from the end, each predecessor is the largest (ref index,
 * then query index) element (aligned pair or virtual start) on an optimal
 * chain, and between two elements, as after the last pair, the D run comes
 * before the I run.  Runs as in sw_align_batch_cigar (packed:
 * cigar[cigar_off[k] .. cigar_off[k+1]), cigar_off[0] = 0; SW_EINVAL with
 * cigar_off filled and cigar untouched when the total exceeds cigar_cap).
 * The path consumes q[query_start[k] .. query_end] and r[ref_start[k] ..
 * ref_end], the start element's coordinates plus one (0, 0 globally).  A
 * pair needs at most (ref_end + 1) + (query_end + 1) + 2 runs.
 *
 * Computed by the path kernel of sw_align_batch_cigar with the boundaries of
 * sw_align_batch_global over r[0..ref_end] x q[0..query_end].  SW_EINVAL: a
 * bad mode, NULL arrays, ids or offsets out of range, an end cell that is
 * not one of the mode's ((m - 1, n - 1) global; query_end = m - 1
 * semi-global; ref_end = n - 1 semi-global the other way; either overlap), a
 * score that is not the optimum there, a residue not below alphabet_size, or
 * too small a cigar_cap; SW_EOVERFLOW and SW_ENOMEM as for
 * sw_align_batch_cigar.  ends, query_start, ref_start, cigar and cigar_off
 * are host arrays owned by the caller.  Synchronous; serialised with the
 * other calls of this group.
 * ------------------------------------------------------------------------- */
int sw_align_batch_global_cigar(const sw_batch *b, const sw_scoring *sc, int32_t mode,
                                const sw_result *ends, int32_t *query_start, int32_t *ref_start,
                                uint32_t *cigar, int64_t cigar_cap, int64_t *cigar_off);

/* Options and statistics for the extended batch call (tests, benchmarks,
 * the autotuner).  Zero-initialise and set what you need. */
enum { SW_PAIRING_AUTO = 0, SW_PAIRING_ALIGNMENTS = 1, SW_PAIRING_ROWS = 2 };
enum { SW_ALG_SCAN = 0,          /* max-plus scan, deferred H fix-up (Algorithm 6) */
       SW_ALG_LAZYF = 1 };       /* lazy-F correction loop (Algorithm 1), comparator */

typedef struct {
    int32_t algorithm;           /* SW_ALG_*                                        */
    int32_t force_lanes;         /* 0 = planner's choice; 16, 32 or 64 = lanes per
                                    alignment for every pair; 8 only for
                                    device-planned batches with one query per
                                    pair (sixteen alignments per wavefront, a
                                    scoring matrix within int8, queries of at
                                    most 152 residues)                           */
    int32_t force_seglen;        /* 0 = planner's choice; else rows per lane (the
                                    query is split into chunks of lanes*seglen rows) */
    int32_t force_kernel;        /* 0 = planner's choice; 1 = shared-query kernel;
                                    2 = per-pair kernel                              */
    int32_t mixed_layout;        /* per-pair kernel: 0 = planner's choice (mixed
                                    unless it models over 15% more work, or the
                                    autotuner's table decides); 1 = mixed: one
                                    rows-per-lane for the batch and 16-, 32- and
                                    64-lane sub-groups inside a wavefront, each
                                    pair on the narrowest that holds its query;
                                    2 = one sub-group width per launch          */
    int32_t int16_cap;           /* 0 = 32767; else a lower saturation threshold for
                                    the int16 pass (tests force the int32 rerun)     */
    int32_t use_graph;           /* 1 = run the device work of the call (uploads,
                                    stream building, alignment kernels) as a
                                    hipGraph: captured on first use, replayed when
                                    a later call has identical parameters; then
                                    kernel_ms spans the whole graph             */
    int32_t planner;             /* 0 = device planner for a batch with one query
                                    (pair_query NULL or n_queries 1) of at most 512
                                    residues and at least 4096 pairs, host planner
                                    otherwise; 1 = host planner; 2 = device planner
                                    (SW_EINVAL if the batch does not qualify).  The
                                    device planner validates, orders and packs the
                                    pairs on the GPU and reads residues straight
                                    from the references; only the query's offsets
                                    and the sets' end offsets are read by the host
                                    before the launch.                             */
    int32_t lane_pairing;        /* int16x2 lanes of device-planned batches: what
                                    the two 16-bit halves of a lane carry.
                                    SW_PAIRING_AUTO = row pairs when no lanes or
                                    seglen are forced and the profile fits 64 KiB
                                    of LDS, else alignment pairs;
                                    SW_PAIRING_ALIGNMENTS = two alignments (one per
                                    half, 16/32/64 lanes per alignment);
                                    SW_PAIRING_ROWS = two row segments of one
                                    alignment (16 lanes, 32 x seglen rows per
                                    alignment or query chunk, seglen 4, 8, 12 or
                                    16): one profile word per row pair and one
                                    more scan step.  Applies to device-planned
                                    batches and to the host planner's per-pair
                                    launches, where AUTO lets the cost model
                                    choose (row pairs need int16 lanes and an
                                    alphabet of at most 24 letters)             */
    int32_t int32_chains;        /* int32 lanes of the shared-query kernel (one
                                    query against many references, scan
                                    algorithm): alignments per sub-group.
                                    SW_CHAINS_AUTO = the library's default (one);
                                    SW_CHAINS_ONE = one; SW_CHAINS_TWO = two
                                    independent column chains, each with its
                                    own state, interleaved in one instruction
                                    stream (results are the same either way)   */
    int32_t striping;            /* which sequence the lanes stripe (host planner):
                                    SW_STRIPE_AUTO = the query (the paper's
                                    layout); SW_STRIPE_QUERY = the query;
                                    SW_STRIPE_SHORTER = for each pair whose
                                    reference is shorter than its query and at
                                    most 2048 residues, the reference, striped
                                    over one 64-lane wavefront (up to 32 rows per
                                    lane) with the query streamed one residue
                                    per column in int32 -- no query chunks at
                                    any query length; the scores are read from
                                    the substitution matrix in LDS, and the end
                                    cell keeps the (ref_end, query_end) order.
                                    Other pairs, the lazy-F algorithm and
                                    batches forced onto the device planner
                                    (planner 2) stripe the query.  Results are
                                    the same either way.                       */
    int32_t reserved[5];
} sw_options;
enum { SW_CHAINS_AUTO = 0, SW_CHAINS_ONE = 1, SW_CHAINS_TWO = 2 };
enum { SW_STRIPE_AUTO = 0, SW_STRIPE_QUERY = 1, SW_STRIPE_SHORTER = 2 };

typedef struct {
    double kernel_ms;            /* device time of the alignment kernels (hipEvents) */
    double total_ms;             /* wall time of the call                           */
    int64_t cells;               /* sum of m*n over pairs                           */
    int64_t padded_cells;        /* cells including lane/row/column padding          */
    int32_t n_rerun;             /* pairs recomputed in int32                        */
    int32_t n_launches;          /* alignment kernel launches                        */
    int64_t lazyf_steps;         /* SW_ALG_LAZYF: inner correction steps executed    */
    int64_t columns;             /* column steps executed (per sub-group)            */
    int32_t lanes_used[3];       /* pairs run with 16 / 32 / 64 lanes                */
    int32_t seglen_max;          /* largest rows-per-lane used                       */
    double prep_ms;              /* host: argument checks, offsets, sequence upload  */
    double plan_ms;              /* host: work planner                               */
    double launch_ms;            /* host: staging uploads and kernel launches        */
    double finish_ms;            /* waiting for the device, results, int32 reruns    */
    int64_t record_events;       /* column steps in which some alignment of a
                                    wavefront set a new running maximum         */
    int32_t graph_hits;          /* use_graph: executions replayed from a cached
                                    graph (no capture)                          */
    int32_t planner_used;        /* 1 = host planner, 2 = device planner        */
    int32_t row_pairs;           /* pairs run in the row-pair lane layout       */
    int32_t lanes8;              /* pairs run with 8 lanes                      */
    int32_t reserved[4];
} sw_stats;

int sw_align_batch_ex(const sw_batch *b, const sw_scoring *sc, const sw_options *opt,
                      sw_result *out, sw_stats *stats);

/* ---------------------------------------------------------------------------
 * sw_align_ex -- sw_align with statistics (for measurement).
 *
 * Same operation, arguments, ownership and errors as sw_align (the plain form
 * of Algorithm 6: one pair, one kernel launch).  If stats is not NULL it is
 * zeroed and then receives kernel_ms (device time of the alignment kernel,
 * from HIP events on the library's stream), total_ms (wall time of the call)
 * and cells (query_len * ref_len); kernel_ms stays 0 for an empty side.
 * ------------------------------------------------------------------------- */
int sw_align_ex(const uint8_t *query, int32_t query_len, const uint8_t *ref, int32_t ref_len,
                const sw_scoring *sc, sw_result *out, sw_stats *stats);

/* ---------------------------------------------------------------------------
 * sw_align_batch_noalloc -- sw_align_batch for callers that cannot allocate.
 *
 * For callers that must not allocate memory during the call: code under HIP
 * stream capture, tight serving loops, hosts that forbid hipMalloc.  Computes
 * exactly what sw_align_batch computes for the same batch and scoring (the
 * same device planner and kernels, in the planner's fixed shapes: the
 * autotuner's table is not consulted), but allocates nothing: no device memory,
 * no pinned host memory and no host heap.  Every buffer of the call lives in
 * one fixed device array of the library (about 53 MiB per device, held from
 * the library's initialisation of a device until the process ends), which
 * bounds the batch to SW_NOALLOC_MAX_PAIRS pairs.
 *
 * Arguments as sw_align_batch, with these restrictions:
 *   - b->device_resident must be 1 (every sequence, offset and pair array is
 *     device memory on the library's device);
 *   - out is DEVICE memory of n_pairs sw_result entries, owned by the caller;
 *   - the batch must be one the device planner takes: one query (pair_query
 *     NULL or n_queries 1) of at most 512 residues, or a query per pair whose
 *     longest fits a compiled per-pair shape (SW_EINVAL otherwise);
 *   - SW_PREC_AUTO: if any pair saturates its int16 lanes, the whole batch is
 *     recomputed in int32 into the scratch array and the saturated pairs'
 *     results are replaced on the device (flag SW_FLAG_SATURATED); a per-pair
 *     batch whose int16 lanes could saturate while no int32 per-pair shape
 *     holds its longest query is refused with SW_EINVAL before any launch.
 * stats (may be NULL) receives kernel_ms, total_ms, cells, n_rerun and the
 * layout counters as sw_align_batch_ex reports them.
 *
 * The array is shared by every call on a device and keeps the last call's
 * contents; the calls serialise on the library's per-device lock, so calls
 * from several threads do not overlap (calls that did overlap on one device
 * would race on it).  Errors: as sw_align_batch, plus SW_EINVAL for host
 * inputs, n_pairs > SW_NOALLOC_MAX_PAIRS or a batch outside the device
 * planner; out holds {0, -1, -1, 0} for every pair after SW_EINVAL from a
 * residue or pair check.  Synchronous.
 * ------------------------------------------------------------------------- */
#define SW_NOALLOC_MAX_PAIRS 1048576
int sw_align_batch_noalloc(const sw_batch *b, const sw_scoring *sc, sw_result *out,
                           sw_stats *stats);

/* ---------------------------------------------------------------------------
 * Autotuner.
 *
 * The planner picks, for each group of pairs, the lanes per alignment (16, 32
 * or 64) and the rows per lane (segLen) from a cost model of the column step
 * (VALU instructions per cell plus the log2(lanes) scan steps per column,
 * amortised over the alignments a wavefront carries).  The autotuner replaces
 * that model by measurement: it runs candidate shapes on the caller's batch
 * (or a seeded sample of it), times the alignment kernels with HIP events and
 * installs the fastest shape per (kernel kind, precision, alphabet size,
 * query-length range) in a process-wide table that every later call consults
 * when no option forces a shape.  The table can be read out and installed
 * again (a cache across processes).
 * ------------------------------------------------------------------------- */
enum { SW_TUNE_SHARED = 0,       /* one query against many references            */
       SW_TUNE_PAIR = 1,         /* a query per pair (per-pair kernel)            */
       SW_TUNE_DEVICE_SHARED = 2,/* device-planned batch with one query           */
       SW_TUNE_DEVICE_PAIR = 3 };/* device-planned batch with a query per pair    */

typedef struct {
    int32_t kind;                /* SW_TUNE_*                                      */
    int32_t precision;           /* SW_PREC_AUTO (int16x2 lanes) or SW_PREC_I32    */
    int32_t alphabet_size;       /* scorings this entry applies to                 */
    int32_t m_lo, m_hi;          /* query lengths covered, inclusive               */
    int32_t lanes;               /* 16, 32 or 64; SW_TUNE_SHARED also 0 = the
                                    planner's per-pair mix of widths              */
    int32_t seglen;              /* rows per lane (SW_TUNE_SHARED with lanes 0:
                                    rows per lane of the 64-lane mode)            */
    int32_t mixed;               /* SW_TUNE_PAIR: 1 = mixed layouts at this seglen
                                    for every per-pair query in [m_lo, m_hi]      */
    int32_t pairing;             /* SW_TUNE_DEVICE_SHARED: SW_PAIRING_ROWS (row
                                    pairs, lanes 16) or SW_PAIRING_ALIGNMENTS
                                    (two alignments per lane, lanes 16 or 32);
                                    other kinds: 0                                */
    int32_t lds_records;         /* SW_TUNE_DEVICE_SHARED with row pairs: 1 = the
                                    end-cell records in LDS, 0 = in registers     */
    double gcups;                /* measured kernel GCUPS of the winner            */
    double model_gcups;          /* measured GCUPS of the cost model's own choice  */
} sw_tune_entry;

/* Tunes the shapes for the pairs of `b` (same arguments as sw_align_batch) and
 * installs the winners.  For the host planner: the shared-query menu and lane
 * mode of the largest query groups, the per-pair shapes per query-length
 * bucket, the mixed layout.  For a batch the device planner takes (one query
 * of at most 512 residues, or a query per pair, at least 4096 pairs): every
 * compiled device-planned shape that holds the query -- row pairs at each
 * rows-per-lane with the end-cell records in LDS or in registers, two
 * alignments per lane at each (rows, lanes) -- or, for a query per pair, the
 * 8- and 16-lane shapes that hold the longest query, each timed on the whole
 * batch (SW_TUNE_DEVICE_* entries for that query length).  sample_cells > 0 caps the cells timed per group (a
 * seeded subset of the group's pairs; 0 = 5e10).  Writes up to `cap` entries to
 * `out` (may be NULL) and their number to *n_out (may be NULL).  Results of
 * later calls are unchanged by tuning: only their speed. */
int sw_autotune(const sw_batch *b, const sw_scoring *sc, int64_t sample_cells,
                sw_tune_entry *out, int32_t cap, int32_t *n_out);

/* Replaces the tuning table (n = 0 clears it, so the cost model decides).
 * SW_EINVAL for entries with an unknown kind, precision or shape. */
int sw_tune_set(const sw_tune_entry *entries, int32_t n);

/* Copies up to `cap` entries of the tuning table; *n_out = their total number. */
int sw_tune_get(sw_tune_entry *out, int32_t cap, int32_t *n_out);

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching request loop.
 *
 * A resident database of references stays in device memory.  Each request is
 * one query against one database reference under one of the server's scoring
 * schemes.  A scheduler thread admits queued requests while the in-flight
 * work fits hbm_budget_bytes and launches them as batches on several HIP
 * streams, so requests that arrive while others run overlap with them on the
 * device.  Results are bit-identical to sw_align_batch on the same pair.
 * ------------------------------------------------------------------------- */
typedef struct sw_server sw_server;

typedef struct {
    size_t hbm_budget_bytes;        /* device bytes the in-flight requests may use */
    int32_t max_queued;             /* requests accepted but not yet collected     */
    const uint8_t *db_res;          /* resident references, CSR, host memory       */
    const int64_t *db_off;
    int32_t n_db;
    const sw_scoring *scorings;     /* n_scorings schemes (copied)                 */
    int32_t n_scorings;
    int32_t max_batch;              /* requests per batch (0 = 16384)              */
    int32_t n_streams;              /* worker threads and streams (0 = 4)          */
    int32_t reserved[6];
} sw_server_config;

int sw_server_create(const sw_server_config *cfg, sw_server **out);

/* Copies the query; returns a ticket.  SW_EBUSY if max_queued requests are
 * outstanding; SW_ENOMEM if the request alone exceeds the budget; SW_EINVAL
 * for a bad ref_id / scoring_id / residue. */
int sw_server_submit(sw_server *s, const uint8_t *query, int32_t query_len,
                     int32_t ref_id, int32_t scoring_id, uint64_t *ticket);

/* SW_OK (result written; the ticket is then forgotten), SW_PENDING, or
 * SW_ENOENT for an unknown or already-collected ticket.  If timestamps_ns is
 * not NULL it receives {submit, admit, done} times (CLOCK_MONOTONIC ns). */
int sw_server_poll(sw_server *s, uint64_t ticket, sw_result *out, int64_t *timestamps_ns);

/* Blocks until every accepted request has finished. */
int sw_server_drain(sw_server *s);

/* Stops the scheduler and frees the server's device memory.  Uncollected
 * tickets are dropped. */
int sw_server_destroy(sw_server *s);

/* Open-loop replay for measurement: submits request k at arrival_ns[k]
 * (nanoseconds after the call starts; nondecreasing) from one thread while
 * another collects completions, then waits for all of them.  Queries are CSR
 * (host), read in place (not copied per request: the buffer must stay
 * unchanged until the call returns).  out[k] gets the result; times_ns[3k..3k+2] = {submit, admit, done}
 * relative to the call's start.  A submit that returns SW_EBUSY is retried
 * until accepted (its submit time is the first attempt).  The collector takes
 * finished requests as the workers report them (no polling of outstanding
 * tickets); one replay at a time per server: a second concurrent call returns
 * SW_EBUSY without submitting anything. */
int sw_server_replay(sw_server *s, int32_t n_requests, const uint8_t *query_res,
                     const int64_t *query_off, const int32_t *ref_id,
                     const int32_t *scoring_id, const int64_t *arrival_ns,
                     sw_result *out, int64_t *times_ns);

#ifdef __cplusplus
}
#endif
#endif /* SW_H_ */
