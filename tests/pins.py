"""Independent pins for the CPU oracle: definitions that do not share its recurrence.

* ``brute_force`` enumerates every local alignment (a non-empty chain of index
  pairs strictly increasing in both sequences) and scores it directly from the
  definition: substitution scores minus g(L) = GapOpen + (L-1)*GapExtend for
  each horizontal and each vertical gap block between consecutive pairs.
* ``kadane_no_gaps`` is the closed form when gaps can never pay off: the best
  maximum-subarray sum along any diagonal.
* ``lcs`` is the textbook longest-common-subsequence DP, the closed form when
  gaps are free and mismatches never help.
"""
from __future__ import annotations


def gap_cost(L: int, go: int, ge: int) -> int:
    return 0 if L == 0 else go + (L - 1) * ge


def brute_force(q, r, M, go: int, ge: int):
    """(score, query_end, ref_end) by enumerating every chain; tiny inputs only.

    Ties on the score go to the smallest ref_end, then the smallest query_end.
    """
    m, n = len(q), len(r)
    best = [0, -1, -1]

    def consider(score, j, i):
        if score > best[0] or (score == best[0] and score > 0 and (i, j) < (best[2], best[1])):
            best[0], best[1], best[2] = score, j, i

    def extend(i, j, score):
        consider(score, j, i)
        for i2 in range(i + 1, n):
            for j2 in range(j + 1, m):
                s2 = score + int(M[q[j2]][r[i2]]) - gap_cost(i2 - i - 1, go, ge) \
                    - gap_cost(j2 - j - 1, go, ge)
                extend(i2, j2, s2)

    for i in range(n):
        for j in range(m):
            extend(i, j, int(M[q[j]][r[i]]))
    if best[0] <= 0:
        return (0, -1, -1)
    return tuple(best)


def kadane_no_gaps(q, r, M):
    """Best gap-free local alignment: max over diagonals of the max-subarray sum.

    Also returns the end cell (query_end, ref_end) with the smallest ref_end,
    then the smallest query_end, among cells where a best run ends.
    """
    m, n = len(q), len(r)
    best = (0, -1, -1)
    ending = {}
    for i in range(n):
        for j in range(m):
            prev = ending.get((i - 1, j - 1), 0)
            cur = max(prev, 0) + int(M[q[j]][r[i]])
            ending[(i, j)] = cur
    cand = [(-v, i, j) for (i, j), v in ending.items() if v > 0]
    if not cand:
        return best
    v, i, j = min(cand)
    return (-v, j, i)


def lcs(a, b) -> int:
    m, n = len(a), len(b)
    T = [[0] * (n + 1) for _ in range(m + 1)]
    for x in range(m):
        for y in range(n):
            T[x + 1][y + 1] = T[x][y] + 1 if a[x] == b[y] else max(T[x][y + 1], T[x + 1][y])
    return T[m][n]


def brute_force_start(q, r, M, go: int, ge: int):
    """(query_start, ref_start) by enumeration: among every chain scoring the
    optimum and ending at the reported end cell (smallest ref_end, then
    query_end), the largest ref_start, then the largest query_start; (-1, -1)
    when the optimum is 0.  Tiny inputs only."""
    s, qe, re_ = brute_force(q, r, M, go, ge)
    if s <= 0:
        return (-1, -1)
    best = None
    m, n = len(q), len(r)

    def extend(i0, j0, i, j, score):
        nonlocal best
        if (i, j) == (re_, qe) and score == s:
            if best is None or (i0, j0) > best:
                best = (i0, j0)
        for i2 in range(i + 1, n):
            for j2 in range(j + 1, m):
                s2 = score + int(M[q[j2]][r[i2]]) - gap_cost(i2 - i - 1, go, ge) \
                    - gap_cost(j2 - j - 1, go, ge)
                extend(i0, j0, i2, j2, s2)

    for i in range(n):
        for j in range(m):
            extend(i, j, i, j, int(M[q[j]][r[i]]))
    return (best[1], best[0])


def brute_force_path(q, r, M, go: int, ge: int):
    """CIGAR runs of the reported alignment by enumeration: every chain from
    the start pair to the end pair scoring the optimum; of those, the one
    whose pairs, read from the end backwards, are lexicographically largest
    ((ref, query) per pair); rendered as D (skipped reference residues), then
    I (skipped query residues), then M per pair.  Tiny inputs only."""
    s, qe, re_ = brute_force(q, r, M, go, ge)
    if s <= 0:
        return []
    qs, rs = brute_force_start(q, r, M, go, ge)
    best = None

    def extend(chain, score):
        nonlocal best
        i, j = chain[-1]
        if (i, j) == (re_, qe):
            if score == s:
                key = list(reversed(chain))
                if best is None or key > best:
                    best = key
            return
        for i2 in range(i + 1, re_ + 1):
            for j2 in range(j + 1, qe + 1):
                s2 = score + int(M[q[j2]][r[i2]]) - gap_cost(i2 - i - 1, go, ge) \
                    - gap_cost(j2 - j - 1, go, ge)
                extend(chain + [(i2, j2)], s2)

    extend([(rs, qs)], int(M[q[qs]][r[rs]]))
    chain = list(reversed(best))
    ops = ["M"]
    for (i, j), (i2, j2) in zip(chain, chain[1:]):
        ops += ["D"] * (i2 - i - 1) + ["I"] * (j2 - j - 1) + ["M"]
    runs = []
    for o in ops:
        if runs and runs[-1][1] == o:
            runs[-1] = (runs[-1][0] + 1, o)
        else:
            runs.append((1, o))
    return runs


def _endtoend_lead(mode: int, a: int, b: int, go: int, ge: int) -> int:
    """Cost of skipping r[0..a] and q[0..b] before the first pair (the chain
    so far empty): both charged (0), the query only (1), the reference only
    (2), the cheaper of the two (3)."""
    ga, gb = gap_cost(a + 1, go, ge), gap_cost(b + 1, go, ge)
    return (ga + gb, gb, ga, min(ga, gb))[mode]


def _endtoend_ends(mode: int, m: int, n: int):
    """The mode's end cells (ref_end, query_end) in (ref_end, query_end) order:
    where the ends that are charged are used up."""
    cells = set()
    if mode == 0:
        cells.add((n - 1, m - 1))
    if mode in (1, 3):
        cells.update((a, m - 1) for a in range(-1, n))
    if mode in (2, 3):
        cells.update((n - 1, b) for b in range(-1, m))
    return sorted(cells)


def _chains(n: int, m: int):
    chains = [[]]

    def grow(chain):
        i0, j0 = chain[-1] if chain else (-1, -1)
        for i in range(i0 + 1, n):
            for j in range(j0 + 1, m):
                c = chain + [(i, j)]
                chains.append(c)
                grow(c)

    grow([])
    return chains


def brute_force_endtoend(q, r, M, go: int, ge: int, mode: int):
    """(score, query_end, ref_end) of the best end-to-end alignment by
    enumerating every chain of index pairs, the empty chain included, and
    every end cell of the mode, pricing every gap run from the definition
    (runs cost g(L) with the extension clamped to the opening cost).  Modes:
    0 global, 1 semi-global (query end to end, reference ends free), 2 the
    reverse (reference end to end, query ends free), 3 overlap.  The value of
    a chain at an end cell (a, b) counts the runs before its first pair as the
    mode charges them and the residues after its last pair up to (a, b) as a
    run in each sequence; the reported end is the first end cell in
    (ref_end, query_end) order that reaches the best value.  Tiny inputs
    only."""
    m, n = len(q), len(r)
    ge = min(ge, go)
    ends = _endtoend_ends(mode, m, n)
    best_at = {}
    for c in _chains(n, m):
        s = sum(int(M[q[j]][r[i]]) for i, j in c)
        for (i, j), (i2, j2) in zip(c, c[1:]):
            s -= gap_cost(i2 - i - 1, go, ge) + gap_cost(j2 - j - 1, go, ge)
        for a, b in ends:
            if c:
                (fi, fj), (li, lj) = c[0], c[-1]
                if a < li or b < lj:
                    continue
                v = s - _endtoend_lead(mode, fi - 1, fj - 1, go, ge) - \
                    gap_cost(a - li, go, ge) - gap_cost(b - lj, go, ge)
            else:
                v = -_endtoend_lead(mode, a, b, go, ge)
            best_at[(a, b)] = max(best_at.get((a, b), v), v)
    score = max(best_at.values())
    a, b = min(e for e, v in best_at.items() if v == score)
    return score, b, a


def overlap_score_direct(q, r, M, go: int, ge: int) -> int:
    """Overlap score straight from its definition, without end cells: the best
    chain's substitution sum minus its inner runs, minus the cheaper of the
    two runs before its first pair and the cheaper of the two after its last
    pair (the empty chain: 0).  Tiny inputs only."""
    m, n = len(q), len(r)
    ge = min(ge, go)
    best = 0
    for c in _chains(n, m):
        if not c:
            continue
        s = sum(int(M[q[j]][r[i]]) for i, j in c)
        for (i, j), (i2, j2) in zip(c, c[1:]):
            s -= gap_cost(i2 - i - 1, go, ge) + gap_cost(j2 - j - 1, go, ge)
        (fi, fj), (li, lj) = c[0], c[-1]
        s -= min(gap_cost(fi, go, ge), gap_cost(fj, go, ge))
        s -= min(gap_cost(n - 1 - li, go, ge), gap_cost(m - 1 - lj, go, ge))
        best = max(best, s)
    return best


def brute_force_endtoend_path(q, r, M, go: int, ge: int, mode: int):
    """(query_start, ref_start, runs) of the reported end-to-end alignment by
    enumeration: every chain of pairs with a virtual start element of the
    mode ((-1, -1) globally; any (v, -1), a free reference prefix, in modes 1
    and 3; any (-1, w), a free query prefix, in modes 2 and 3) that reaches
    the optimum at the reported end; of those, the one whose elements read
    from the end backwards are lexicographically largest; rendered with D
    before I between elements and after the last pair.  Tiny inputs only."""
    m, n = len(q), len(r)
    ge = min(ge, go)
    score, b_end, a_end = brute_force_endtoend(q, r, M, go, ge, mode)
    best = None
    for c in _chains(a_end + 1, b_end + 1):
        x1, y1 = c[0] if c else (a_end + 1, b_end + 1)
        starts = []
        if mode == 0:
            starts.append((-1, -1))
        if mode in (1, 3):
            starts += [(v, -1) for v in range(-1, x1)]
        if mode in (2, 3):
            starts += [(-1, w) for w in range(-1, y1)]
        for st in set(starts):
            elems = [st] + c
            s = sum(int(M[q[j]][r[i]]) for i, j in c)
            for (i, j), (i2, j2) in zip(elems, elems[1:]):
                s -= gap_cost(i2 - i - 1, go, ge) + gap_cost(j2 - j - 1, go, ge)
            li, lj = elems[-1]
            s -= gap_cost(a_end - li, go, ge) + gap_cost(b_end - lj, go, ge)
            if s == score:
                key = list(reversed(elems))
                if best is None or key > best:
                    best = key
    elems = list(reversed(best))
    ops = []
    for (i, j), (i2, j2) in zip(elems, elems[1:]):
        ops += ["D"] * (i2 - i - 1) + ["I"] * (j2 - j - 1) + ["M"]
    li, lj = elems[-1]
    ops += ["D"] * (a_end - li) + ["I"] * (b_end - lj)
    runs = []
    for o in ops:
        if runs and runs[-1][1] == o:
            runs[-1] = (runs[-1][0] + 1, o)
        else:
            runs.append((1, o))
    return elems[0][1] + 1, elems[0][0] + 1, runs
