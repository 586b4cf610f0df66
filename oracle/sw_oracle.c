/*
 * Scalar CPU oracle for local alignment with affine gaps (Smith-Waterman
 * with Gotoh's three-state recurrence).  TEST INFRASTRUCTURE ONLY: nothing in
 * the product path may link, load or call this file.  It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * What it computes (paper: Background section, the local-alignment problem;
 * Algorithm 1 inner loop for the update order; the note under Algorithm 1 that
 * no value may go negative):
 *
 *   H(i,j)   = max(0, Hd(i,j), E(i,j), F(i,j))
 *   Hd(i,j)  = H(i-1,j-1) + S[q_j][r_i]          (diagonal, H(-1,*) = H(*,-1) = 0)
 *   E(i,j)   = max(E(i-1,j) - GapExtend, H(i-1,j) - GapOpen)   (gap along the reference)
 *   F(i,j)   = max(F(i,j-1) - GapExtend, H(i,j-1) - GapOpen)   (gap along the query)
 *
 * i indexes the reference (outer loop, as in both algorithms of the paper),
 * j the query.  A gap of length L therefore costs GapOpen + (L-1)*GapExtend:
 * subtracting GapOpen opens it, each further residue subtracts GapExtend.
 * The score is max over all cells of Hd (the paper keeps the running maximum
 * of H + profile before the E/F maxima are applied), floored at 0.
 *
 * End cell: the paper returns only the score.  This oracle also returns the
 * (query_end, ref_end) of the Hd cell achieving it; on ties the smallest
 * ref_end wins, then the smallest query_end.  That is exactly what a strict ">"
 * gives in a reference-outer, query-inner scan.  Score 0 gives (-1, -1).
 *
 * All arithmetic is int64; inputs are validated by the caller.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <stdatomic.h>

typedef struct {
    int64_t score;
    int64_t query_end;
    int64_t ref_end;
} oracle_result;

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/* One pair.  M is row-major alpha x alpha, indexed M[q_code * alpha + r_code].
 * Returns 0 on success, -1 on allocation failure or bad arguments. */
int oracle_sw(const uint8_t *q, int64_t m, const uint8_t *r, int64_t n,
              const int32_t *M, int32_t alpha, int64_t gap_open,
              int64_t gap_extend, oracle_result *out)
{
    out->score = 0;
    out->query_end = -1;
    out->ref_end = -1;
    if (m < 0 || n < 0 || alpha <= 0) return -1;
    if (m == 0 || n == 0) return 0;

    int64_t *Hprev = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    int64_t *Hcur = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    int64_t *E = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    if (!Hprev || !Hcur || !E) {
        free(Hprev); free(Hcur); free(E);
        return -1;
    }
    for (int64_t j = 0; j < m; ++j) {
        Hprev[j] = 0;
        /* No gap can be open before the first column.  Any value <= -GapOpen
         * behaves the same; 0 - GapOpen - GapExtend keeps it in range. */
        E[j] = -gap_open - gap_extend;
    }

    int64_t best = 0, bi = -1, bj = -1;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t rc = r[i];
        int64_t F = -gap_open - gap_extend;   /* no vertical gap above row 0 */
        for (int64_t j = 0; j < m; ++j) {
            const int64_t diag = (j > 0) ? Hprev[j - 1] : 0;
            const int64_t hd = diag + (int64_t)M[(int64_t)q[j] * alpha + rc];
            if (hd > best) { best = hd; bi = i; bj = j; }
            /* E(i,j) was formed while processing column i-1 (below);
             * F(i,j) was formed while processing row j-1 of this column. */
            int64_t h = max2(max2(0, hd), max2(E[j], F));
            Hcur[j] = h;
            E[j] = max2(E[j] - gap_extend, h - gap_open);   /* E(i+1,j) */
            F = max2(F - gap_extend, h - gap_open);         /* F(i,j+1) */
        }
        int64_t *t = Hprev; Hprev = Hcur; Hcur = t;
    }
    free(Hprev); free(Hcur); free(E);
    if (best > 0) {
        out->score = best;
        out->query_end = bj;
        out->ref_end = bi;
    }
    return 0;
}

/* ---- many pairs over a thread pool -------------------------------------- */

typedef struct {
    int64_t n_pairs;
    const uint8_t *query_res; const int64_t *query_off;
    const uint8_t *ref_res;   const int64_t *ref_off;
    const int32_t *pair_query; const int32_t *pair_ref;
    const int32_t *M; int32_t alpha; int64_t gap_open; int64_t gap_extend;
    oracle_result *out;
    atomic_long next;
    atomic_int failed;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *b = (batch_job *)arg;
    for (;;) {
        long k = atomic_fetch_add(&b->next, 1);
        if (k >= b->n_pairs) break;
        int32_t qi = b->pair_query ? b->pair_query[k] : 0;
        int32_t ri = b->pair_ref[k];
        const uint8_t *q = b->query_res + b->query_off[qi];
        int64_t m = b->query_off[qi + 1] - b->query_off[qi];
        const uint8_t *r = b->ref_res + b->ref_off[ri];
        int64_t n = b->ref_off[ri + 1] - b->ref_off[ri];
        if (oracle_sw(q, m, r, n, b->M, b->alpha, b->gap_open, b->gap_extend,
                      &b->out[k]) != 0)
            atomic_store(&b->failed, 1);
    }
    return NULL;
}

/* Queries and references are CSR (residues + n+1 offsets).  pair_query may
 * be NULL (every pair uses query 0).  Uses n_threads POSIX threads (>= 1).
 * Returns 0, or -1 if any pair failed. */
int oracle_sw_batch(int64_t n_pairs,
                    const uint8_t *query_res, const int64_t *query_off,
                    const uint8_t *ref_res, const int64_t *ref_off,
                    const int32_t *pair_query, const int32_t *pair_ref,
                    const int32_t *M, int32_t alpha,
                    int64_t gap_open, int64_t gap_extend,
                    int32_t n_threads, oracle_result *out)
{
    batch_job b;
    b.n_pairs = n_pairs;
    b.query_res = query_res; b.query_off = query_off;
    b.ref_res = ref_res; b.ref_off = ref_off;
    b.pair_query = pair_query; b.pair_ref = pair_ref;
    b.M = M; b.alpha = alpha; b.gap_open = gap_open; b.gap_extend = gap_extend;
    b.out = out;
    atomic_init(&b.next, 0);
    atomic_init(&b.failed, 0);
    if (n_threads < 1) n_threads = 1;
    if (n_threads == 1) {
        batch_worker(&b);
        return atomic_load(&b.failed) ? -1 : 0;
    }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    if (!th) return -1;
    int started = 0;
    for (int t = 0; t < n_threads; ++t) {
        if (pthread_create(&th[t], NULL, batch_worker, &b) == 0) ++started;
    }
    if (started == 0) batch_worker(&b);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    return atomic_load(&b.failed) ? -1 : 0;
}

/*
 * Alignment path between a start pair (qs, rs) and an end pair (qe, re) of
 * score S (this library's extension: the paper returns only the score).
 *
 * Over the rectangle a = i - rs in [0, A), b = j - qs in [0, B):
 *   M(a,b)  best score of a chain of matched pairs that starts with the start
 *           pair and ends with pair (a,b): S[q][r] of (a,b) plus, unless (a,b)
 *           is the start, the best V(a-1, b-1);
 *   V(x,y)  best over pairs (x',y') <= (x,y) of M(x',y') - g(x-x') - g(y-y'),
 *           g(0) = 0, g(L) = GapOpen + (L-1)*GapExtend (a reference gap and a
 *           query gap between consecutive pairs cost independently);
 * both written out as plain maxima.  The path is read back from the end
 * pair: each predecessor is the largest (a', b') -- reference index first,
 * then query index -- with M(a',b') - g(a-1-a') - g(b-1-b') equal to
 * V(a-1, b-1), i.e. the largest predecessor lying on an optimal chain from
 * the start.  Between two consecutive pairs the skipped reference residues
 * are written first (D), then the skipped query residues (I), then the pair
 * itself (M).
 *
 * ops receives run-length entries (len << 4 | op, op 0 = M, 1 = I, 2 = D) in
 * forward order; returns their count, -1 on bad arguments or allocation
 * failure, -2 if no chain from the start reaches the end with score S.
 */
static int64_t gap_cost(int64_t L, int64_t go, int64_t ge) { return L == 0 ? 0 : go + (L - 1) * ge; }

int64_t oracle_path(const uint8_t *q, const uint8_t *r, const int32_t *Mx, int32_t alpha,
                    int64_t go, int64_t ge, int64_t qs, int64_t rs, int64_t qe, int64_t re,
                    int64_t S, uint32_t *ops, int64_t cap)
{
    if (qe < qs || re < rs || qs < 0 || rs < 0 || alpha <= 0) return -1;
    /* Gotoh's recurrences may close a gap and open the next one at once, so a
     * run of k gaps never costs more than k * go: the scores are those of the
     * extension min(ge, go), and the runs of a path are priced with it. */
    if (ge > go) ge = go;
    const int64_t A = re - rs + 1, B = qe - qs + 1;
    const int64_t NEG = INT64_MIN / 4;
    int64_t *M = (int64_t *)malloc((size_t)(A * B) * sizeof(int64_t));
    int64_t *V = (int64_t *)malloc((size_t)(A * B) * sizeof(int64_t));
    char *rev = (char *)malloc((size_t)(A + B + 1));
    if (!M || !V || !rev) { free(M); free(V); free(rev); return -1; }
#define SC(a, b) ((int64_t)Mx[(int)q[qs + (b)] * alpha + (int)r[rs + (a)]])
    for (int64_t a = 0; a < A; ++a) {
        for (int64_t b = 0; b < B; ++b) {
            int64_t m = NEG;
            if (a == 0 && b == 0) m = SC(0, 0);
            else if (a > 0 && b > 0 && V[(a - 1) * B + (b - 1)] > NEG) m = SC(a, b) + V[(a - 1) * B + (b - 1)];
            M[a * B + b] = m;
            int64_t v = NEG;
            for (int64_t x = 0; x <= a; ++x)
                for (int64_t y = 0; y <= b; ++y)
                    if (M[x * B + y] > NEG) v = max2(v, M[x * B + y] - gap_cost(a - x, go, ge) - gap_cost(b - y, go, ge));
            V[a * B + b] = v;
        }
    }
    int64_t n = 0, a = A - 1, b = B - 1;
    int64_t rc = 0;
    if (M[a * B + b] != S) rc = -2;
    while (rc == 0 && (a > 0 || b > 0)) {
        rev[n++] = 'M';
        const int64_t target = M[a * B + b] - SC(a, b);
        int64_t fx = -1, fy = -1;
        for (int64_t x = a - 1; x >= 0 && fx < 0; --x)
            for (int64_t y = b - 1; y >= 0; --y)
                if (M[x * B + y] > NEG &&
                    M[x * B + y] - gap_cost(a - 1 - x, go, ge) - gap_cost(b - 1 - y, go, ge) == target) {
                    fx = x; fy = y;
                    break;
                }
        if (fx < 0) { rc = -2; break; }
        for (int64_t k = 0; k < b - 1 - fy; ++k) rev[n++] = 'I';
        for (int64_t k = 0; k < a - 1 - fx; ++k) rev[n++] = 'D';
        a = fx;
        b = fy;
    }
    if (rc == 0) rev[n++] = 'M';
#undef SC
    int64_t cnt = 0;
    for (int64_t k = n - 1; rc == 0 && k >= 0;) {
        const char c = rev[k];
        int64_t len = 0;
        while (k >= 0 && rev[k] == c) { ++len; --k; }
        if (cnt >= cap) { rc = -1; break; }
        ops[cnt++] = (uint32_t)(len << 4) | (c == 'M' ? 0u : (c == 'I' ? 1u : 2u));
    }
    free(M); free(V); free(rev);
    return rc ? rc : cnt;
}

/*
 * End-to-end alignments (not in the paper, whose problem is local): an
 * alignment is a chain of aligned pairs (x_1, y_1) < (x_2, y_2) < ... strictly
 * increasing in both the reference index x and the query index y; its score is
 * the sum of S[q_y][r_x] over the pairs minus the cost of every gap run, a run
 * of L skipped residues costing go + (L - 1) * min(ge, go) (Gotoh's
 * recurrences reopen a gap rather than extend it at a higher cost).  Between
 * two pairs, before the first and after the last, the skipped reference
 * residues and the skipped query residues are one run each.
 *
 * mode 0, global: every residue of both sequences is aligned or skipped at a
 *   cost; the chain may be empty (both sequences skipped whole).
 * mode 1, semi-global (fitting): the query end to end as in mode 0, the
 *   reference residues before the first pair and after the last pair are
 *   skipped for free.  End: the smallest reference prefix end a (-1 for the
 *   empty prefix) such that the best such alignment of the query inside
 *   r[0..a] -- counting reference residues after its last pair up to a as a
 *   gap run -- reaches the score.
 *
 * Computed as plain maxima over the chains, no affine recurrence:
 *   W(x, y) = S[q_y][r_x] + best(x - 1, y - 1)    (the best chain ending with pair (x, y))
 *   best(a, b) = max( lead(a, b),  max over x <= a, y <= b of W(x, y) - g(a - x) - g(b - y) )
 * with lead(a, b) the chain before any pair -- residues r[0..a] and q[0..b]
 * skipped: -g(a + 1) - g(b + 1) in mode 0, -g(b + 1) in mode 1 (g(0) = 0) --
 * and best(-1, -1) = 0, best(a, -1) = lead(a, -1), best(-1, b) = lead(-1, b).
 * The inner maximum is taken over y first, then x (one pass per row and one
 * per column), an exact regrouping of the same maximum.  Global score:
 * best(n - 1, m - 1).  Semi-global score: max over a in -1..n-1 of best(a, m - 1).
 */
static int64_t gcost(int64_t L, int64_t go, int64_t ge) { return L <= 0 ? 0 : go + (L - 1) * ge; }

int oracle_endtoend(const uint8_t *q, int64_t m, const uint8_t *r, int64_t n,
                    const int32_t *Mx, int32_t alpha, int64_t go, int64_t ge, int32_t mode,
                    oracle_result *out)
{
    if (m < 0 || n < 0 || alpha <= 0 || (mode != 0 && mode != 1)) return -1;
    if (ge > go) ge = go;
    const int64_t NEG = INT64_MIN / 4;
    /* best and W over (a, b) in -1..n-1 x -1..m-1, stored with a +1 offset */
    const int64_t R = n + 1, C = m + 1;
    int64_t *best = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    int64_t *W = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    int64_t *G = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    if (!best || !W || !G) { free(best); free(W); free(G); return -1; }
#define IX(a, b) (((a) + 1) * C + ((b) + 1))
    for (int64_t a = -1; a < n; ++a) {
        for (int64_t b = -1; b < m; ++b) {
            const int64_t lead = mode == 0 ? -gcost(a + 1, go, ge) - gcost(b + 1, go, ge)
                                           : -gcost(b + 1, go, ge);
            if (a < 0 || b < 0) {
                W[IX(a, b)] = NEG;
                G[IX(a, b)] = NEG;
                best[IX(a, b)] = lead;
                continue;
            }
            W[IX(a, b)] = (int64_t)Mx[(int)q[b] * alpha + (int)r[a]] + best[IX(a - 1, b - 1)];
            /* G(x, b) = max over y <= b of W(x, y) - g(b - y), for this row x = a */
            int64_t g = NEG;
            for (int64_t y = 0; y <= b; ++y) g = max2(g, W[IX(a, y)] - gcost(b - y, go, ge));
            G[IX(a, b)] = g;
            int64_t v = lead;
            for (int64_t x = 0; x <= a; ++x)
                if (G[IX(x, b)] > NEG) v = max2(v, G[IX(x, b)] - gcost(a - x, go, ge));
            best[IX(a, b)] = v;
        }
    }
    if (mode == 0) {
        out->score = best[IX(n - 1, m - 1)];
        out->query_end = m - 1;
        out->ref_end = n - 1;
    } else {
        int64_t s = NEG, at = -1;
        for (int64_t a = -1; a < n; ++a)
            if (best[IX(a, m - 1)] > s) { s = best[IX(a, m - 1)]; at = a; }
        out->score = s;
        out->query_end = m - 1;
        out->ref_end = at;
    }
#undef IX
    free(best); free(W); free(G);
    return 0;
}

/*
 * Path of an end-to-end alignment (mode 0 global, 1 semi-global as in
 * oracle_endtoend), from its end (ref_end, m - 1) back to its start: the
 * chain's elements are the aligned pairs plus a virtual start pair -- (-1, -1)
 * in mode 0, any (v, -1) with v >= -1 in mode 1 (the free reference prefix
 * r[0..v]) -- of value 0.  Walking back from the end, each predecessor is the
 * largest (ref index, then query index) element, virtual ones included, on an
 * optimal chain; between two elements (and after the last pair) the skipped
 * reference residues (D) are written before the skipped query residues (I).
 * Runs go to ops[] as (len << 4 | op), op 0 M, 1 I, 2 D, in forward order;
 * *ref_start receives v + 1 for the virtual start (0 in mode 0).  Returns the
 * number of runs, -1 on bad arguments / allocation failure / too small a cap,
 * -2 if `score` is not the mode's optimum at that end.
 */
int64_t oracle_endtoend_path(const uint8_t *q, int64_t m, const uint8_t *r, int64_t n,
                             const int32_t *Mx, int32_t alpha, int64_t go, int64_t ge,
                             int32_t mode, int64_t ref_end, int64_t score, uint32_t *ops,
                             int64_t cap, int64_t *ref_start)
{
    if (m < 0 || n < 0 || alpha <= 0 || (mode != 0 && mode != 1)) return -1;
    if (ref_end < -1 || ref_end >= n || (mode == 0 && ref_end != n - 1)) return -1;
    if (ge > go) ge = go;
    const int64_t NEG = INT64_MIN / 4;
    const int64_t R = n + 1, C = m + 1;
    int64_t *best = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    int64_t *W = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    int64_t *G = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    char *rev = (char *)malloc((size_t)(n + m + 2));
    if (!best || !W || !G || !rev) { free(best); free(W); free(G); free(rev); return -1; }
#define IX(a, b) (((a) + 1) * C + ((b) + 1))
    for (int64_t a = -1; a < n; ++a) {
        for (int64_t b = -1; b < m; ++b) {
            const int64_t lead = mode == 0 ? -gcost(a + 1, go, ge) - gcost(b + 1, go, ge)
                                           : -gcost(b + 1, go, ge);
            if (a < 0 || b < 0) {
                W[IX(a, b)] = NEG;
                G[IX(a, b)] = NEG;
                best[IX(a, b)] = lead;
                continue;
            }
            W[IX(a, b)] = (int64_t)Mx[(int)q[b] * alpha + (int)r[a]] + best[IX(a - 1, b - 1)];
            int64_t g = NEG;
            for (int64_t y = 0; y <= b; ++y) g = max2(g, W[IX(a, y)] - gcost(b - y, go, ge));
            G[IX(a, b)] = g;
            int64_t v = lead;
            for (int64_t x = 0; x <= a; ++x)
                if (G[IX(x, b)] > NEG) v = max2(v, G[IX(x, b)] - gcost(a - x, go, ge));
            best[IX(a, b)] = v;
        }
    }
    int64_t rc = 0, nrev = 0;
    if (best[IX(ref_end, m - 1)] != score) rc = -2;
    /* walk: the current position (px, py) lies just before the element found
     * last (the end, then each aligned pair); target = best(px, py) */
    int64_t px = ref_end, py = m - 1, target = score, vstart = -1;
    while (rc == 0) {
        int64_t fx = NEG, fy = NEG;
        /* real pairs, largest x first, then largest y */
        for (int64_t x = px; x >= 0 && fx == NEG; --x)
            for (int64_t y = py; y >= 0; --y)
                if (W[IX(x, y)] > NEG &&
                    W[IX(x, y)] - gcost(px - x, go, ge) - gcost(py - y, go, ge) == target) {
                    fx = x; fy = y;
                    break;
                }
        /* a virtual start element beats a real pair only with a larger x */
        int64_t vx = NEG;
        if (mode == 0) {
            if (-gcost(px + 1, go, ge) - gcost(py + 1, go, ge) == target) vx = -1;
        } else {
            for (int64_t v = px; v >= -1 && vx == NEG; --v)
                if (-gcost(px - v, go, ge) - gcost(py + 1, go, ge) == target) vx = v;
        }
        if (vx != NEG && (fx == NEG || vx > fx)) {
            for (int64_t k = 0; k < py - (-1); ++k) rev[nrev++] = 'I';
            for (int64_t k = 0; k < px - vx; ++k) rev[nrev++] = 'D';
            vstart = vx;
            break;
        }
        if (fx == NEG) { rc = -2; break; }
        for (int64_t k = 0; k < py - fy; ++k) rev[nrev++] = 'I';
        for (int64_t k = 0; k < px - fx; ++k) rev[nrev++] = 'D';
        rev[nrev++] = 'M';
        target = W[IX(fx, fy)] - (int64_t)Mx[(int)q[fy] * alpha + (int)r[fx]];
        px = fx - 1;
        py = fy - 1;
    }
#undef IX
    int64_t cnt = 0;
    for (int64_t k = nrev - 1; rc == 0 && k >= 0;) {
        const char c = rev[k];
        int64_t len = 0;
        while (k >= 0 && rev[k] == c) { ++len; --k; }
        if (cnt >= cap) { rc = -1; break; }
        ops[cnt++] = (uint32_t)(len << 4) | (c == 'M' ? 0u : (c == 'I' ? 1u : 2u));
    }
    if (ref_start) *ref_start = vstart + 1;
    free(best); free(W); free(G); free(rev);
    return rc ? rc : cnt;
}
