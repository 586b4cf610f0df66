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
 * residues and the skipped query residues are one run each.  Which of the
 * runs before the first pair and after the last one are charged depends on
 * the mode:
 *
 * mode 0, global: every residue of both sequences is aligned or skipped at a
 *   cost; the chain may be empty (both sequences skipped whole).
 * mode 1, semi-global (the query fitted into the reference): the query end to
 *   end as in mode 0, the reference residues before the first pair and after
 *   the last pair skipped for free.
 * mode 2, semi-global the other way (the reference fitted into the query):
 *   the reference end to end, the query residues before the first and after
 *   the last pair free.
 * mode 3, overlap (free end gaps): before the first pair the skipped residues
 *   of one of the two sequences are free, those of the other cost a run, and
 *   likewise after the last pair -- a dovetail or containment of the two
 *   sequences; the empty chain scores 0.
 *
 * The best alignment that ends at a cell (a, b) -- residues r[0..a] and
 * q[0..b] consumed, those after the last pair up to (a, b) counted as runs --
 * is computed as plain maxima over the chains, no affine recurrence:
 *   W(x, y) = S[q_y][r_x] + best(x - 1, y - 1)    (the best chain ending with pair (x, y))
 *   best(a, b) = max( lead(a, b),  max over x <= a, y <= b of W(x, y) - g(a - x) - g(b - y) )
 * with lead(a, b) the chain before any pair -- residues r[0..a] and q[0..b]
 * skipped: -g(a + 1) - g(b + 1) in mode 0, -g(b + 1) in mode 1, -g(a + 1) in
 * mode 2, -min(g(a + 1), g(b + 1)) in mode 3 (g(0) = 0) -- and best(a, -1) =
 * lead(a, -1), best(-1, b) = lead(-1, b).  The inner maximum is taken over y
 * first, then x (one pass per row and one per column), an exact regrouping
 * of the same maximum.
 *
 * The alignment ends at a cell where the uncharged sequence ends are used up:
 * mode 0 at (n - 1, m - 1); mode 1 at (a, m - 1), a in -1..n-1 (the
 * reference after a is free); mode 2 at (n - 1, b), b in -1..m-1; mode 3 at
 * either kind.  The score is the largest best() over the mode's end cells and
 * the reported end the first of them in (ref_end, query_end) order that
 * reaches it.
 */
static int64_t gcost(int64_t L, int64_t go, int64_t ge) { return L <= 0 ? 0 : go + (L - 1) * ge; }

static int64_t lead_cost(int32_t mode, int64_t a, int64_t b, int64_t go, int64_t ge)
{
    const int64_t ga = gcost(a + 1, go, ge), gb = gcost(b + 1, go, ge);
    switch (mode) {
    case 0: return -ga - gb;
    case 1: return -gb;
    case 2: return -ga;
    default: return ga < gb ? -ga : -gb;
    }
}

/* best(a, b) over (a, b) in -1..n-1 x -1..m-1 (stored with a +1 offset) and
 * W(x, y) of every pair; the caller frees both. */
static int endtoend_tables(const uint8_t *q, int64_t m, const uint8_t *r, int64_t n,
                           const int32_t *Mx, int32_t alpha, int64_t go, int64_t ge, int32_t mode,
                           int64_t **best_out, int64_t **W_out)
{
    const int64_t NEG = INT64_MIN / 4;
    const int64_t R = n + 1, C = m + 1;
    int64_t *best = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    int64_t *W = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    int64_t *G = (int64_t *)malloc((size_t)(R * C) * sizeof(int64_t));
    if (!best || !W || !G) { free(best); free(W); free(G); return -1; }
#define IX(a, b) (((a) + 1) * C + ((b) + 1))
    for (int64_t a = -1; a < n; ++a) {
        for (int64_t b = -1; b < m; ++b) {
            const int64_t lead = lead_cost(mode, a, b, go, ge);
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
#undef IX
    free(G);
    *best_out = best;
    *W_out = W;
    return 0;
}

int oracle_endtoend(const uint8_t *q, int64_t m, const uint8_t *r, int64_t n,
                    const int32_t *Mx, int32_t alpha, int64_t go, int64_t ge, int32_t mode,
                    oracle_result *out)
{
    if (m < 0 || n < 0 || alpha <= 0 || mode < 0 || mode > 3) return -1;
    if (ge > go) ge = go;
    const int64_t NEG = INT64_MIN / 4;
    const int64_t C = m + 1;
    int64_t *best = NULL, *W = NULL;
    if (endtoend_tables(q, m, r, n, Mx, alpha, go, ge, mode, &best, &W)) return -1;
#define IX(a, b) (((a) + 1) * C + ((b) + 1))
    /* the mode's end cells in (ref_end, query_end) order; strict > keeps the first */
    int64_t s = NEG, ea = -1, eb = -1;
    if (mode == 0) {
        s = best[IX(n - 1, m - 1)];
        ea = n - 1;
        eb = m - 1;
    }
    if (mode == 1 || mode == 3) {
        const int64_t last = mode == 1 ? n - 1 : n - 2;   /* mode 3: (n - 1, .) below */
        for (int64_t a = -1; a <= last; ++a)
            if (best[IX(a, m - 1)] > s) { s = best[IX(a, m - 1)]; ea = a; eb = m - 1; }
    }
    if (mode == 2 || mode == 3) {
        for (int64_t b = -1; b < m; ++b)
            if (best[IX(n - 1, b)] > s) { s = best[IX(n - 1, b)]; ea = n - 1; eb = b; }
    }
    out->score = s;
    out->query_end = eb;
    out->ref_end = ea;
#undef IX
    free(best); free(W);
    return 0;
}

/*
 * Path of an end-to-end alignment (modes as in oracle_endtoend), from its end
 * cell (ref_end, query_end) back to its start: the chain's elements are the
 * aligned pairs plus a virtual start element of value 0 -- (-1, -1) in mode 0;
 * any (v, -1), v >= -1, in modes 1 and 3 (the free reference prefix r[0..v]);
 * any (-1, w), w >= -1, in modes 2 and 3 (the free query prefix q[0..w]).
 * Between two consecutive elements, and from the last one to the end cell,
 * the skipped residues of each sequence are one run.  Walking back from the
 * end, each predecessor is the largest (ref index, then query index) element,
 * virtual ones included, on an optimal chain; between two elements (and
 * after the last pair) the skipped reference residues (D) are written before
 * the skipped query residues (I).  Runs go to ops[] as (len << 4 | op), op 0
 * M, 1 I, 2 D, in forward order; *ref_start / *query_start receive the start
 * element's coordinates plus one.  Returns the number of runs, -1 on bad
 * arguments / allocation failure / too small a cap, -2 if `score` is not the
 * mode's best at that end.
 */
int64_t oracle_endtoend_path(const uint8_t *q, int64_t m, const uint8_t *r, int64_t n,
                             const int32_t *Mx, int32_t alpha, int64_t go, int64_t ge,
                             int32_t mode, int64_t query_end, int64_t ref_end, int64_t score,
                             uint32_t *ops, int64_t cap, int64_t *query_start, int64_t *ref_start)
{
    if (m < 0 || n < 0 || alpha <= 0 || mode < 0 || mode > 3) return -1;
    if (ref_end < -1 || ref_end >= n || query_end < -1 || query_end >= m) return -1;
    {
        const int on_q = query_end == m - 1, on_r = ref_end == n - 1;
        const int ok = mode == 0 ? (on_q && on_r) : mode == 1 ? on_q : mode == 2 ? on_r : (on_q || on_r);
        if (!ok) return -1;
    }
    if (ge > go) ge = go;
    const int64_t NEG = INT64_MIN / 4;
    const int64_t C = m + 1;
    int64_t *best = NULL, *W = NULL;
    if (endtoend_tables(q, m, r, n, Mx, alpha, go, ge, mode, &best, &W)) return -1;
    char *rev = (char *)malloc((size_t)(n + m + 2));
    if (!rev) { free(best); free(W); return -1; }
#define IX(a, b) (((a) + 1) * C + ((b) + 1))
    int64_t rc = 0, nrev = 0;
    if (best[IX(ref_end, query_end)] != score) rc = -2;
    /* walk: the current position (px, py) lies just before the element found
     * last (the end, then each aligned pair); target = best(px, py) */
    int64_t px = ref_end, py = query_end, target = score, sx = -1, sy = -1;
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
        /* the largest virtual start element on an optimal chain */
        int64_t vx = NEG, vy = NEG;
        if (mode == 1 || mode == 3)
            for (int64_t v = px; v >= -1 && vx == NEG; --v)
                if (-gcost(px - v, go, ge) - gcost(py + 1, go, ge) == target) { vx = v; vy = -1; }
        if ((mode == 2 || mode == 3) && (vx == NEG || vx < 0))
            for (int64_t w = py; w >= -1; --w)
                if (-gcost(px + 1, go, ge) - gcost(py - w, go, ge) == target) {
                    if (vx == NEG || w > vy) { vx = -1; vy = w; }
                    break;
                }
        if (mode == 0 && -gcost(px + 1, go, ge) - gcost(py + 1, go, ge) == target) { vx = -1; vy = -1; }
        /* a virtual element (x = -1, or y = -1) beats a real pair only with a larger x */
        if (vx != NEG && (fx == NEG || vx > fx)) {
            for (int64_t k = 0; k < py - vy; ++k) rev[nrev++] = 'I';
            for (int64_t k = 0; k < px - vx; ++k) rev[nrev++] = 'D';
            sx = vx;
            sy = vy;
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
    if (ref_start) *ref_start = sx + 1;
    if (query_start) *query_start = sy + 1;
    free(best); free(W); free(rev);
    return rc ? rc : cnt;
}
