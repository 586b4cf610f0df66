"""Pins for the CPU oracle (no GPU).  Each check is independent of the oracle's
own recurrence: brute-force enumeration of all local alignments, a
hand-computed worked example, closed forms (Kadane, LCS) and invariants.
A final test plants plausible mistakes into a copy of the Python oracle and
shows that these pins catch every one of them."""
import inspect
import json
import os
import textwrap

import numpy as np
import pytest

import oracle
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    oracle.build(force=False)


def _both(q, r, M, go, ge):
    a = oracle.align(q, r, M, go, ge)
    b = oracle.gotoh_py(list(q), list(r), M, go, ge)
    assert a == b, (a, b)
    return a


def _case(rng, maxlen=6, alpha=None, symmetric=None):
    alpha = alpha or int(rng.integers(2, 5))
    m = int(rng.integers(1, maxlen + 1))
    n = int(rng.integers(1, maxlen + 1))
    q = rng.integers(0, alpha, size=m).tolist()
    r = rng.integers(0, alpha, size=n).tolist()
    M = rng.integers(-5, 6, size=(alpha, alpha))
    if symmetric if symmetric is not None else rng.random() < 0.5:
        M = np.triu(M) + np.triu(M, 1).T
    go = int(rng.integers(0, 7))
    ge = int(rng.integers(0, go + 1))
    return q, r, M.astype(np.int32), go, ge


# ---------------------------------------------------------------- worked example

def test_worked_example_golden():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    code = {c: k for k, c in enumerate(g["alphabet"])}
    A = len(g["alphabet"])
    M = np.full((A, A), g["mismatch"], dtype=np.int32)
    np.fill_diagonal(M, g["match"])
    q = [code[c] for c in g["query"]]
    r = [code[c] for c in g["ref"]]
    go, ge = g["gap_open"], g["gap_extend"]
    res, hd_cols, h_cols = oracle.gotoh_py(q, r, M, go, ge, tables=True)
    assert hd_cols == g["hdiag_by_column"]
    assert h_cols == g["h_by_column"]
    want = (g["result"]["score"], g["result"]["query_end"], g["result"]["ref_end"])
    assert res == want
    assert oracle.align(q, r, M, go, ge) == want
    assert pins.brute_force(q, r, M, go, ge) == want
    sw = g["swapped_result"]
    assert oracle.align(r, q, M, go, ge) == (sw["score"], sw["query_end"], sw["ref_end"])
    # The other gap convention (open + L*extend) is rejected by this example.
    assert pins.brute_force(q, r, M, go + ge, ge)[0] == g["open_plus_l_extend_score"]


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(6))
def test_brute_force_random(seed):
    rng = np.random.default_rng(1000 + seed)
    for _ in range(120):
        q, r, M, go, ge = _case(rng)
        assert _both(q, r, M, go, ge) == pins.brute_force(q, r, M, go, ge)


def test_brute_force_edge_penalties():
    rng = np.random.default_rng(77)
    for go, ge in [(0, 0), (1, 0), (3, 3), (5, 1), (50, 50)]:
        for _ in range(60):
            q, r, M, _, _ = _case(rng)
            assert _both(q, r, M, go, ge) == pins.brute_force(q, r, M, go, ge)


def test_double_gap_bridge_family():
    """A horizontal and a vertical gap in one block are strictly optimal here
    (match +5 / mismatch -4, GapOpen 11, GapExtend 1, q = A^12 X^k B^12,
    r = A^12 Y^k B^12 with X, Y never matching): checked against the closed form
    of the two alignments that compete (gap-free vs bridged)."""
    A_, B_, X_, Y_ = 0, 1, 2, 3
    M = np.full((4, 4), -4, dtype=np.int32)
    M[A_, A_] = M[B_, B_] = 5
    for k in (11, 12, 16):
        q = [A_] * 12 + [X_] * k + [B_] * 12
        r = [A_] * 12 + [Y_] * k + [B_] * 12
        no_gap = 24 * 5 - 4 * k
        bridged = 24 * 5 - 2 * (11 + (k - 1) * 1)
        want = max(no_gap, bridged, 60)
        s, qe, re_ = oracle.align(q, r, M, 11, 1)
        assert s == want
        assert (qe, re_) == (len(q) - 1, len(r) - 1)
        assert bridged > no_gap  # the gap->gap transition is what wins


# ---------------------------------------------------------------- closed forms

def test_kadane_no_gaps():
    rng = np.random.default_rng(5)
    for _ in range(300):
        q, r, M, _, _ = _case(rng, maxlen=12)
        big = 10 ** 6
        assert _both(q, r, M, big, big) == pins.kadane_no_gaps(q, r, M)


def test_lcs_free_gaps():
    rng = np.random.default_rng(6)
    for _ in range(300):
        alpha = int(rng.integers(2, 5))
        q, r, _, _, _ = _case(rng, maxlen=14, alpha=alpha)
        M = -rng.integers(0, 4, size=(alpha, alpha))
        np.fill_diagonal(M, 1)
        assert _both(q, r, M.astype(np.int32), 0, 0)[0] == pins.lcs(q, r)


# ---------------------------------------------------------------- invariants

def test_gap_extend_clamp():
    rng = np.random.default_rng(7)
    for _ in range(300):
        q, r, M, go, _ = _case(rng, maxlen=10)
        ge = go + int(rng.integers(1, 6))
        assert oracle.align(q, r, M, go, ge) == oracle.align(q, r, M, go, go)


def test_symmetry_and_reversal():
    rng = np.random.default_rng(8)
    for _ in range(300):
        q, r, M, go, ge = _case(rng, maxlen=12, symmetric=True)
        s = oracle.align(q, r, M, go, ge)[0]
        assert oracle.align(r, q, M, go, ge)[0] == s
        assert oracle.align(q[::-1], r[::-1], M, go, ge)[0] == s


def test_self_alignment():
    from paper_1909_00899_amd import workloads
    M = workloads.protein_matrix()
    d = np.diag(M)
    # the protein matrix meets the sufficient condition: diagonal > 0 and
    # every off-diagonal entry below the mean of its two diagonal entries
    assert (d > 0).all()
    assert all(M[a, b] < (d[a] + d[b]) / 2 for a in range(20) for b in range(20) if a != b)
    rng = np.random.default_rng(9)
    for m in (1, 2, 7, 50, 300):
        q = rng.integers(0, 20, size=m)
        assert oracle.align(q, q, M, 11, 1) == (int(d[q].sum()), m - 1, m - 1)
    # the diagonal condition alone is not sufficient
    M2 = np.array([[1, 10], [10, 1]], dtype=np.int32)
    assert oracle.align([0, 1], [0, 1], M2, 5, 1)[0] == 10


def test_bounds_and_monotonicity():
    rng = np.random.default_rng(10)
    for _ in range(300):
        q, r, M, go, ge = _case(rng, maxlen=10)
        s, qe, re_ = oracle.align(q, r, M, go, ge)
        assert 0 <= s <= min(len(q), len(r)) * max(0, int(M.max()))
        assert (s == 0) == (qe == -1) == (re_ == -1)
        if s:
            assert 0 <= qe < len(q) and 0 <= re_ < len(r)
        a = int(rng.integers(0, M.shape[0]))
        assert oracle.align(q + [a], r, M, go, ge)[0] >= s
        assert oracle.align(q, [a] + r, M, go, ge)[0] >= s


def test_empty_inputs():
    M = np.eye(4, dtype=np.int32)
    assert oracle.align([], [1, 2], M, 1, 1) == (0, -1, -1)
    assert oracle.align([1], [], M, 1, 1) == (0, -1, -1)
    assert oracle.gotoh_py([], [], M, 1, 1) == (0, -1, -1)


def test_batch_matches_single():
    from paper_1909_00899_amd import workloads
    w = workloads.random_pairs(64, 20, (0, 40), (0, 60), seed=11)
    out = oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                             w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query,
                             n_threads=4)
    for k in range(w.n_pairs):
        q, r = w.pair(k)
        assert tuple(out[k]) == oracle.align(q, r, w.matrix, w.gap_open, w.gap_extend)


# ---------------------------------------------------------------- planted mistakes

MUTANTS = {
    "open_plus_L_extend": ("E[j] = h - gap_open if e_ext is None else max(e_ext, h - gap_open)",
                           "E[j] = h - gap_open - gap_extend if e_ext is None else "
                           "max(e_ext, h - gap_open - gap_extend)"),
    "no_floor": ("cands = [0, hd]", "cands = [hd]"),
    "drop_E": ("if E[j] is not None:\n                cands.append(E[j])",
               "if False:\n                cands.append(E[j])"),
    "drop_F": ("if F is not None:\n                cands.append(F)",
               "if False:\n                cands.append(F)"),
    "transposed_matrix": ("int(matrix[query[j]][ref[i]])", "int(matrix[ref[i]][query[j]])"),
    "diag_index": ("diag = Hprev[j - 1] if j > 0 else 0", "diag = Hprev[j] if j > 0 else 0"),
    "extend_sign": ("e_ext = E[j] - gap_extend", "e_ext = E[j] + gap_extend"),
    "tie_break_ge": ("if hd > best:", "if hd >= best and hd > 0:"),
    "max_after_gaps": ("            hd_col.append(hd)\n            if hd > best:\n"
                       "                best, bq, br = hd, j, i\n",
                       "            hd_col.append(hd)\n"),
}


def _mutant(name):
    src = textwrap.dedent(inspect.getsource(oracle.gotoh_py))
    old, new = MUTANTS[name]
    assert old in src, name
    src = src.replace(old, new)
    if name == "max_after_gaps":
        src = src.replace("            Hprev = Hcur\n",
                          "            Hprev = Hcur\n"
                          "            for jj, hv in enumerate(Hcur):\n"
                          "                if hv > best:\n"
                          "                    best, bq, br = hv, jj, i\n")
    ns = dict(vars(oracle))
    exec(src, ns)
    return ns["gotoh_py"]


def _pins_catch(fn) -> bool:
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    M = np.full((4, 4), g["mismatch"], dtype=np.int32)
    np.fill_diagonal(M, g["match"])
    if fn([0, 1, 2, 3], [0, 2, 3], M, 2, 1) != (7, 3, 2):
        return True
    rng = np.random.default_rng(4242)
    for _ in range(400):
        q, r, M, go, ge = _case(rng)
        if fn(q, r, M, go, ge) != pins.brute_force(q, r, M, go, ge):
            return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(name):
    assert _pins_catch(oracle.gotoh_py) is False
    assert _pins_catch(_mutant(name)) is True


# ---------------------------------------------------------------- start cells

def _start_via(fn, q, r, M, go, ge):
    """Start cell from an end-cell function ``fn`` applied to the reversed
    prefixes (the construction ``oracle.start_cell`` uses)."""
    s, qe, re_ = oracle.align(q, r, M, go, ge)
    if s <= 0:
        return (-1, -1)
    s2, qe2, re2 = fn(list(q[:qe + 1])[::-1], list(r[:re_ + 1])[::-1], M, go, ge)
    return (qe - qe2, re_ - re2)


def test_start_cell_worked_example():
    # A/A, C against a gap, G/G, T/T: the only alignment scoring 7 starts at (0, 0)
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    M = np.full((4, 4), g["mismatch"], dtype=np.int32)
    np.fill_diagonal(M, g["match"])
    assert oracle.start_cell([0, 1, 2, 3], [0, 2, 3], M, 2, 1) == (0, 0)
    assert pins.brute_force_start([0, 1, 2, 3], [0, 2, 3], M, 2, 1) == (0, 0)


@pytest.mark.parametrize("seed", range(3))
def test_start_cell_brute_force_random(seed):
    rng = np.random.default_rng(3000 + seed)
    ties = 0
    for _ in range(150):
        q, r, M, go, ge = _case(rng)
        want = pins.brute_force_start(q, r, M, go, ge)
        assert oracle.start_cell(q, r, M, go, ge) == want
        # cases where another optimal start exists make the tie rule matter
        if want != (-1, -1) and _start_via(_min_start_end, q, r, M, go, ge) != want:
            ties += 1
    assert ties > 0


def _min_start_end(q, r, M, go, ge):
    """End cell with the tie going to the LAST maximal H_diag in scan order
    (a plausible mistake: it yields the smallest start instead of the largest)."""
    m, n = len(q), len(r)
    Hprev, E = [0] * m, [0] * m
    best, bq, br = 0, -1, -1
    for i in range(n):
        F, Hcur = 0, [0] * m
        for j in range(m):
            hd = (Hprev[j - 1] if j > 0 else 0) + int(M[q[j]][r[i]])
            if hd >= best and hd > 0:
                best, bq, br = hd, j, i
            h = max(0, hd, E[j], F)
            E[j] = max(E[j] - ge, h - go)
            F = max(F - ge, h - go)
            Hcur[j] = h
        Hprev = Hcur
    return (best, bq, br) if best > 0 else (0, -1, -1)


def test_start_cell_pins_catch_planted_mistakes():
    rng = np.random.default_rng(3100)
    cases = [_case(rng) for _ in range(300)]
    want = [pins.brute_force_start(*c) for c in cases]
    # prefixes one residue too short, forward (unreversed) prefixes, and the
    # smallest instead of the largest start are each caught
    short = lambda q, r, M, go, ge: oracle.align(q[1:], r[1:], M, go, ge)  # noqa: E731
    forward = lambda q, r, M, go, ge: oracle.align(q[::-1], r[::-1], M, go, ge)  # noqa: E731
    for fn in (short, forward, _min_start_end):
        got = []
        for c in cases:
            try:
                got.append(_start_via(fn, *c))
            except (IndexError, ValueError):
                got.append(None)
        assert got != want


def test_start_batch_matches_single():
    from paper_1909_00899_amd import workloads
    w = workloads.random_pairs(80, 4, (0, 30), (0, 40), seed=12)
    ends = oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                              w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query)
    st = oracle.start_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref, w.matrix,
                            w.gap_open, w.gap_extend, ends, pair_query=w.pair_query, n_threads=2)
    for k in range(w.n_pairs):
        q, r = w.pair(k)
        assert tuple(st[k]) == oracle.start_cell(q, r, w.matrix, w.gap_open, w.gap_extend)
        if ends[k, 0] > 0:
            assert 0 <= st[k, 0] <= ends[k, 1] and 0 <= st[k, 1] <= ends[k, 2]


# ---------------------------------------------------------------- alignment paths

def _gappy_case(rng):
    alpha = int(rng.integers(2, 4))
    m, n = int(rng.integers(2, 7)), int(rng.integers(2, 7))
    q = rng.integers(0, alpha, size=m).tolist()
    r = rng.integers(0, alpha, size=n).tolist()
    M = rng.integers(-3, 2, size=(alpha, alpha)).astype(np.int32)
    M[np.arange(alpha), np.arange(alpha)] = rng.integers(2, 6, size=alpha)
    go = int(rng.integers(0, 3))
    ge = int(rng.integers(0, go + 1))
    return q, r, M, go, ge


def test_path_extension_above_opening():
    # the scores do not change when gap_extend > gap_open is clamped, so
    # neither may the paths, and a path's runs add up to the score
    rng = np.random.default_rng(31)
    for _ in range(200):
        q, r, M, go, _ = _gappy_case(rng)
        ge = go + int(rng.integers(1, 4))
        s, qe, re_ = oracle.align(q, r, M, go, ge)
        if s <= 0:
            continue
        runs = oracle.path(q, r, M, go, ge)
        assert runs == oracle.path(q, r, M, go, go)
        start = oracle.start_cell(q, r, M, go, ge)
        assert oracle.path_score(q, r, M, go, ge, start, runs) == s


def test_path_double_gap():
    Mb = np.full((4, 4), -10, dtype=np.int32)
    Mb[0, 0] = Mb[1, 1] = 5
    want = [(1, "M"), (1, "D"), (1, "I"), (1, "M")]
    assert pins.brute_force_path([0, 2, 1], [0, 3, 1], Mb, 1, 1) == want
    assert oracle.path([0, 2, 1], [0, 3, 1], Mb, 1, 1) == want


def test_path_worked_example():
    # A/A, C against a gap, G/G, T/T
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    M = np.full((4, 4), g["mismatch"], dtype=np.int32)
    np.fill_diagonal(M, g["match"])
    want = [(1, "M"), (1, "I"), (2, "M")]
    assert oracle.path([0, 1, 2, 3], [0, 2, 3], M, 2, 1) == want
    assert pins.brute_force_path([0, 1, 2, 3], [0, 2, 3], M, 2, 1) == want
    assert oracle.path_score([0, 1, 2, 3], [0, 2, 3], M, 2, 1, (0, 0), want) == 7


@pytest.mark.parametrize("seed", range(3))
def test_path_brute_force_random(seed):
    rng = np.random.default_rng(4000 + seed)
    gaps = 0
    for _ in range(160):
        q, r, M, go, ge = (_gappy_case if _ % 2 else _case)(rng)
        want = pins.brute_force_path(q, r, M, go, ge)
        assert oracle.path(q, r, M, go, ge) == want
        gaps += any(op != "M" for _, op in want)
    assert gaps >= 10


def test_path_consistency_larger():
    """Larger pairs (oracle only): the path starts and ends at the reported
    cells, consumes exactly the rectangle between them and scores the optimum."""
    rng = np.random.default_rng(4100)
    for _ in range(40):
        alpha = int(rng.integers(2, 21))
        m, n = int(rng.integers(1, 60)), int(rng.integers(1, 60))
        q = rng.integers(0, alpha, size=m)
        r = rng.integers(0, alpha, size=n)
        M = rng.integers(-4, 4, size=(alpha, alpha)).astype(np.int32)
        M[np.arange(alpha), np.arange(alpha)] = rng.integers(3, 9, size=alpha)
        go = int(rng.integers(1, 12))
        ge = int(rng.integers(0, go + 1))
        s, qe, re_ = oracle.align(q, r, M, go, ge)
        runs = oracle.path(q, r, M, go, ge)
        if s == 0:
            assert runs == []
            continue
        qs, rs = oracle.start_cell(q, r, M, go, ge)
        assert runs[0][1] == "M" and runs[-1][1] == "M"
        assert sum(L for L, op in runs if op != "D") == qe - qs + 1
        assert sum(L for L, op in runs if op != "I") == re_ - rs + 1
        assert oracle.path_score(q, r, M, go, ge, (qs, rs), runs) == s


def test_path_pins_tell_other_rules_apart():
    """The brute-force pin fixes the tie rule: the smallest instead of the
    largest predecessor, query index before reference index, and the query gap
    written before the reference gap each give other paths on some cases."""
    rng = np.random.default_rng(4200)

    def variant(q, r, M, go, ge, key, igap_first):
        s, qe, re_ = pins.brute_force(q, r, M, go, ge)
        if s <= 0:
            return []
        qs, rs = pins.brute_force_start(q, r, M, go, ge)
        chains = []

        def extend(chain, score):
            i, j = chain[-1]
            if (i, j) == (re_, qe):
                if score == s:
                    chains.append(chain)
                return
            for i2 in range(i + 1, re_ + 1):
                for j2 in range(j + 1, qe + 1):
                    extend(chain + [(i2, j2)], score + int(M[q[j2]][r[i2]]) -
                           pins.gap_cost(i2 - i - 1, go, ge) - pins.gap_cost(j2 - j - 1, go, ge))

        extend([(rs, qs)], int(M[q[qs]][r[rs]]))
        chain = max(chains, key=key)
        ops = ["M"]
        for (i, j), (i2, j2) in zip(chain, chain[1:]):
            d, ins = ["D"] * (i2 - i - 1), ["I"] * (j2 - j - 1)
            ops += (ins + d if igap_first else d + ins) + ["M"]
        runs = []
        for o in ops:
            if runs and runs[-1][1] == o:
                runs[-1] = (runs[-1][0] + 1, o)
            else:
                runs.append((1, o))
        return runs

    rules = {
        "smallest predecessor": (lambda c: [(-i, -j) for i, j in reversed(c)], False),
        "query index first": (lambda c: [(j, i) for i, j in reversed(c)], False),
        "query gap first": (lambda c: list(reversed(c)), True),
    }
    # found by a seeded search: two optimal predecessors where one has the
    # larger reference index and the other the larger query index
    crossing = ([1, 2, 0, 1], [1, 0, 2, 1, 1, 2],
                np.array([[2, -3, -3], [0, 5, 0], [-3, 0, 2]], dtype=np.int32), 1, 0)
    # a reference gap and a query gap between the same two pairs (X, Y never
    # match anything): the bridge beats the mismatch
    Mb = np.full((4, 4), -10, dtype=np.int32)
    Mb[0, 0] = Mb[1, 1] = 5
    bridge = ([0, 2, 1], [0, 3, 1], Mb, 1, 1)
    cases = [crossing, bridge] + [_gappy_case(rng) for _ in range(400)]
    for name, (key, igf) in rules.items():
        assert any(variant(*c, key, igf) != pins.brute_force_path(*c) for c in cases), name


# ---------------------------------------------------------------- end to end

MODES = (0, 1, 2, 3)    # global, semi-global (query fitted), semi-global (reference fitted), overlap


def _tiny(rng):
    alpha = int(rng.integers(2, 4))
    m, n = int(rng.integers(0, 5)), int(rng.integers(0, 6))
    q = rng.integers(0, alpha, size=m).tolist()
    r = rng.integers(0, alpha, size=n).tolist()
    M = rng.integers(-4, 3, size=(alpha, alpha)).astype(np.int32)
    go = int(rng.integers(0, 4))
    ge = int(rng.integers(0, go + 3))      # sometimes above the opening cost
    return q, r, M, go, ge


def test_endtoend_brute_force_random():
    rng = np.random.default_rng(41)
    for _ in range(500):
        q, r, M, go, ge = _tiny(rng)
        for mode in MODES:
            want = pins.brute_force_endtoend(q, r, M, go, ge, mode)
            assert oracle.endtoend(q, r, M, go, ge, mode) == want, (q, r, M.tolist(), go, ge, mode)


def test_overlap_score_from_its_definition():
    # the overlap score without end cells: the cheaper run at each end of the
    # chain, the empty chain 0
    rng = np.random.default_rng(45)
    for _ in range(400):
        q, r, M, go, ge = _tiny(rng)
        assert oracle.endtoend(q, r, M, go, ge, 3)[0] == pins.overlap_score_direct(q, r, M, go, ge)


def test_endtoend_closed_forms():
    rng = np.random.default_rng(42)
    M = np.full((4, 4), -4, dtype=np.int32)
    np.fill_diagonal(M, 5)
    for _ in range(100):
        m = int(rng.integers(1, 30))
        q = rng.integers(0, 4, size=m).tolist()
        go, ge = int(rng.integers(1, 8)), int(rng.integers(0, 3))
        g1 = go + (m - 1) * min(ge, go)
        # a sequence against itself: every residue paired, in every mode
        for mode in MODES:
            assert oracle.endtoend(q, q, M, go, ge, mode) == (5 * m, m - 1, m - 1)
        # against nothing: one gap run where that side is charged
        assert oracle.endtoend(q, [], M, go, ge, 0)[0] == -g1
        assert oracle.endtoend([], q, M, go, ge, 0)[0] == -g1
        assert oracle.endtoend([], q, M, go, ge, 1) == (0, -1, -1)
        assert oracle.endtoend(q, [], M, go, ge, 1) == (-g1, m - 1, -1)
        assert oracle.endtoend(q, [], M, go, ge, 2) == (0, -1, -1)
        assert oracle.endtoend([], q, M, go, ge, 2) == (-g1, -1, m - 1)
        assert oracle.endtoend(q, [], M, go, ge, 3) == (0, -1, -1)
        assert oracle.endtoend([], q, M, go, ge, 3) == (0, -1, -1)
        # a query inside a longer reference: free reference ends, the first
        # occurrence's end; the reverse mode with the roles swapped
        pre = rng.integers(0, 4, size=int(rng.integers(0, 20))).tolist()
        post = rng.integers(0, 4, size=int(rng.integers(0, 20))).tolist()
        r = pre + q + post
        first = min(k for k in range(m - 1, len(r)) if r[k - m + 1:k + 1] == q)
        assert oracle.endtoend(q, r, M, go, ge, 1) == (5 * m, m - 1, first)
        assert oracle.endtoend(r, q, M, go, ge, 2) == (5 * m, first, m - 1)
        # containment is an overlap too
        assert oracle.endtoend(q, r, M, go, ge, 3)[0] == 5 * m
        # a dovetail: the query's suffix is the reference's prefix, the ends
        # mismatching so badly that only the shared part pays
        if len(pre) > 0 and len(post) > 0:
            X = [(c + 1) % 4 for c in pre]
            Z = [(c + 2) % 4 for c in post]
            Mh = np.full((4, 4), -50, dtype=np.int32)
            np.fill_diagonal(Mh, 5)
            s, qe, re_ = oracle.endtoend(X + q, q + Z, Mh, 60, 60, 3)
            assert s >= 5 * m
            assert oracle.align(X + q, q + Z, Mh, 60, 60)[0] >= s
    # free gaps and a +1 identity matrix: every mode = longest common subsequence
    I1 = np.eye(4, dtype=np.int32)
    for _ in range(100):
        q = rng.integers(0, 4, size=int(rng.integers(0, 15))).tolist()
        r = rng.integers(0, 4, size=int(rng.integers(0, 15))).tolist()
        for mode in MODES:
            assert oracle.endtoend(q, r, I1, 0, 0, mode)[0] == pins.lcs(q, r)


def test_dovetail_worked_example():
    # query ACGTT, reference GTTCA (A=0 C=1 G=2 T=3), +5 / -4, GapOpen 6,
    # GapExtend 1 (worked by hand): the query's suffix GTT is the reference's
    # prefix, 15 with both overhangs (the query's AC, the reference's CA)
    # free.  No alignment scores more (15 is also the local optimum), and
    # ending on the reference's last residue instead would pay for CA (8), so
    # the end is the query's last residue against the reference's third
    # (0-based query_end 4, ref_end 2) and the path starts at (2, 0).
    M = np.full((4, 4), -4, dtype=np.int32)
    np.fill_diagonal(M, 5)
    q, r = [0, 1, 2, 3, 3], [2, 3, 3, 1, 0]
    assert oracle.endtoend(q, r, M, 6, 1, 3) == (15, 4, 2)
    assert oracle.endtoend_path(q, r, M, 6, 1, 3) == (2, 0, [(3, "M")])
    assert oracle.align(q, r, M, 6, 1)[0] == 15


def test_endtoend_invariants():
    rng = np.random.default_rng(43)
    for _ in range(300):
        q, r, M, go, ge = _case(rng, maxlen=12)
        Mt = np.ascontiguousarray(np.asarray(M).T)
        g = oracle.endtoend(q, r, M, go, ge, 0)[0]
        sg = oracle.endtoend(q, r, M, go, ge, 1)
        sr = oracle.endtoend(q, r, M, go, ge, 2)
        ov = oracle.endtoend(q, r, M, go, ge, 3)
        assert sg[0] >= g and sr[0] >= g                     # fewer runs are paid
        assert ov[0] >= max(sg[0], sr[0], 0)
        assert oracle.align(q, r, M, go, ge)[0] >= ov[0]      # a local alignment too
        assert oracle.endtoend(q[::-1], r[::-1], M, go, ge, 0)[0] == g
        assert oracle.endtoend(r, q, Mt, go, ge, 0)[0] == g
        # swapping the sequences (and transposing the matrix) swaps the two
        # semi-global modes; the overlap score is symmetric
        t1 = oracle.endtoend(r, q, Mt, go, ge, 1)
        assert (t1[0], t1[2], t1[1]) == sr
        t2 = oracle.endtoend(r, q, Mt, go, ge, 2)
        assert (t2[0], t2[2], t2[1]) == sg
        assert oracle.endtoend(r, q, Mt, go, ge, 3)[0] == ov[0]
        assert oracle.endtoend(q[::-1], r[::-1], M, go, ge, 3)[0] == ov[0]


def test_endtoend_path_brute_force_random():
    rng = np.random.default_rng(44)
    n_cases = n_query_start = 0
    for _ in range(400):
        q, r, M, go, ge = _tiny(rng)
        for mode in MODES:
            want = pins.brute_force_endtoend_path(q, r, M, go, ge, mode)
            got = oracle.endtoend_path(q, r, M, go, ge, mode)
            assert got == want, (q, r, M.tolist(), go, ge, mode, got, want)
            s, qe, re_ = oracle.endtoend(q, r, M, go, ge, mode)
            # the runs add up to the score from the start to the end
            assert _endtoend_runs_score(q, r, M, go, ge, got[:2], got[2], (qe, re_)) == s
            n_query_start += got[0] > 0
            n_cases += 1
    assert n_cases == 1600 and n_query_start > 50


def _endtoend_runs_score(q, r, M, go, ge, start, runs, end):
    ge = min(ge, go)
    j, i = start
    total = 0
    for L, op in runs:
        if op == "M":
            for _ in range(L):
                total += int(M[q[j]][r[i]])
                i += 1
                j += 1
        else:
            total -= go + (L - 1) * ge
            if op == "I":
                j += L
            else:
                i += L
    assert (j - 1, i - 1) == tuple(end)
    return total


def test_endtoend_path_worked_examples():
    M = np.full((4, 4), -2, dtype=np.int32)
    np.fill_diagonal(M, 3)
    # ACGT vs AGT globally: the C skipped
    assert oracle.endtoend_path([0, 1, 2, 3], [0, 2, 3], M, 2, 1, 0) == \
        (0, 0, [(1, "M"), (1, "I"), (2, "M")])
    # GT placed inside ACGTA
    assert oracle.endtoend_path([2, 3], [0, 1, 2, 3, 0], M, 2, 1, 1) == (0, 2, [(2, "M")])
    # ... and ACGTA's GT placed on the reference GT (the reference fitted)
    assert oracle.endtoend_path([0, 1, 2, 3, 0], [2, 3], M, 2, 1, 2) == (2, 0, [(2, "M")])
    # empty sides
    assert oracle.endtoend_path([], [0, 1], M, 2, 1, 0) == (0, 0, [(2, "D")])
    assert oracle.endtoend_path([1], [], M, 2, 1, 1) == (0, 0, [(1, "I")])
    assert oracle.endtoend_path([], [1], M, 2, 1, 2) == (0, 0, [(1, "D")])
    assert oracle.endtoend_path([1, 2], [0, 3], M, 9, 1, 0) == (0, 0, [(2, "M")])
    # the empty overlap: nothing aligned, the query placed before the reference
    assert oracle.endtoend([1, 1], [0, 0], M, 2, 1, 3) == (0, 1, -1)
    assert oracle.endtoend_path([1, 1], [0, 0], M, 2, 1, 3) == (2, 0, [])
