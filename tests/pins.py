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


def brute_force_endtoend(q, r, M, go: int, ge: int, mode: int):
    """(score, query_end, ref_end) of the best global (mode 0) or semi-global
    (mode 1: query end to end, reference ends free) alignment by enumerating
    every chain of index pairs, the empty chain included, and pricing every
    gap run from the definition (runs cost g(L) with the extension clamped to
    the opening cost).  Mode 1's ref_end: the smallest prefix end a whose best
    alignment -- the reference residues after the last pair up to a counted as
    a gap run -- reaches the score.  Tiny inputs only."""
    m, n = len(q), len(r)
    ge = min(ge, go)
    chains = [[]]

    def grow(chain):
        i0, j0 = chain[-1] if chain else (-1, -1)
        for i in range(i0 + 1, n):
            for j in range(j0 + 1, m):
                c = chain + [(i, j)]
                chains.append(c)
                grow(c)

    grow([])
    best_at = {}
    for c in chains:
        s = sum(int(M[q[j]][r[i]]) for i, j in c)
        for (i, j), (i2, j2) in zip(c, c[1:]):
            s -= gap_cost(i2 - i - 1, go, ge) + gap_cost(j2 - j - 1, go, ge)
        fi, fj = c[0] if c else (n, m)         # first pair (or past the end)
        li, lj = c[-1] if c else (-1, -1)      # last pair (or before the start)
        if mode == 0:
            if c:
                s -= gap_cost(fi, go, ge) + gap_cost(fj, go, ge)
                s -= gap_cost(n - 1 - li, go, ge) + gap_cost(m - 1 - lj, go, ge)
            else:
                s -= gap_cost(n, go, ge) + gap_cost(m, go, ge)
            best_at[n - 1] = max(best_at.get(n - 1, s), s)
        else:
            s -= (gap_cost(fj, go, ge) + gap_cost(m - 1 - lj, go, ge)) if c else gap_cost(m, go, ge)
            for a in range(li if c else -1, n):
                v = s - (gap_cost(a - li, go, ge) if c else 0)
                best_at[a] = max(best_at.get(a, v), v)
    score = max(best_at.values())
    end = min(a for a, v in best_at.items() if v == score)
    return score, m - 1, end


def brute_force_endtoend_path(q, r, M, go: int, ge: int, mode: int):
    """(ref_start, runs) of the reported end-to-end alignment by enumeration:
    every chain of pairs with its virtual start element ((-1, -1) globally,
    any (v, -1) semi-globally) that reaches the optimum at the reported end;
    of those, the one whose elements read from the end backwards are
    lexicographically largest; rendered with D before I between elements and
    after the last pair.  Tiny inputs only."""
    m, n = len(q), len(r)
    ge = min(ge, go)
    score, _, a_end = brute_force_endtoend(q, r, M, go, ge, mode)
    chains = [[]]

    def grow(chain):
        i0, j0 = chain[-1] if chain else (-1, -1)
        for i in range(i0 + 1, a_end + 1):
            for j in range(j0 + 1, m):
                c = chain + [(i, j)]
                chains.append(c)
                grow(c)

    grow([])
    best = None
    for c in chains:
        starts = [-1] if mode == 0 else list(range(-1, (c[0][0] if c else a_end + 1)))
        for v in starts:
            elems = [(v, -1)] + c
            s = sum(int(M[q[j]][r[i]]) for i, j in c)
            for (i, j), (i2, j2) in zip(elems, elems[1:]):
                s -= gap_cost(i2 - i - 1, go, ge) + gap_cost(j2 - j - 1, go, ge)
            li, lj = elems[-1]
            s -= gap_cost(a_end - li, go, ge) + gap_cost(m - 1 - lj, go, ge)
            if mode == 0 and not c:
                pass        # both runs from the virtual pair: counted just above
            if s == score:
                key = list(reversed(elems))
                if best is None or key > best:
                    best = key
    elems = list(reversed(best))
    ops = []
    for (i, j), (i2, j2) in zip(elems, elems[1:]):
        ops += ["D"] * (i2 - i - 1) + ["I"] * (j2 - j - 1) + ["M"]
    li, lj = elems[-1]
    ops += ["D"] * (a_end - li) + ["I"] * (m - 1 - lj)
    runs = []
    for o in ops:
        if runs and runs[-1][1] == o:
            runs[-1] = (runs[-1][0] + 1, o)
        else:
            runs.append((1, o))
    return elems[0][0] + 1, runs
