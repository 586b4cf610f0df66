"""Start cells (sw_align_batch_starts): the reversed prefixes ending at each
reported end cell run through the batch path; every start equals the CPU
oracle's (largest ref_start, then largest query_start among the optimal
alignments ending at the end cell), through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    api.load()          # raises if the HIP library is missing: no fallback
    api.sw_init()


def _ends_and_starts(w, **kw):
    out = api.align_workload(w, **kw)
    qs, rs = api.sw_align_batch_starts(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                                       w.matrix, w.gap_open, w.gap_extend, out.results,
                                       pair_query=w.pair_query,
                                       precision=kw.get("precision", api.SW_PREC_AUTO))
    return out.results, np.stack([qs, rs], axis=1)


def _check(w, label, **kw):
    ends, starts = _ends_and_starts(w, **kw)
    want_ends = oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                                   w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query)
    assert (ends[:, :3] == want_ends).all(), label
    want = oracle.start_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                              w.matrix, w.gap_open, w.gap_extend, want_ends,
                              pair_query=w.pair_query)
    bad = np.nonzero((starts != want).any(axis=1))[0]
    if bad.size:
        k = int(bad[0])
        raise AssertionError("%s: %d/%d start mismatches; first pair %d got %s want %s (end %s)" %
                             (label, bad.size, len(want), k, starts[k].tolist(), want[k].tolist(),
                              ends[k].tolist()))
    live = want_ends[:, 0] > 0
    assert (starts[~live] == -1).all()
    assert (starts[live, 0] <= ends[live, 1]).all() and (starts[live, 1] <= ends[live, 2]).all()
    return ends, starts


@pytest.mark.parametrize("alpha,mlen,nlen", [(20, (1, 300), (1, 400)), (4, (1, 200), (1, 500)),
                                             (2, (1, 60), (1, 80))])
def test_starts_random_pairs(alpha, mlen, nlen):
    # two letters: many optimal alignments per end cell, so the tie rule decides
    w = W.random_pairs(700, alpha, mlen, nlen, 880 + alpha)
    _check(w, "random alpha=%d" % alpha)


def test_starts_protein_search_subset_device_planner():
    w = W.protein_search(n_refs=6000)
    ends, starts = _check(w, "protein search", planner=2)
    assert (ends[:, 0] > 0).all()


def test_starts_dna_pairs():
    w = W.dna_pairs(n_pairs=20000, seed=21)
    ends, starts = _check(w, "dna pairs")
    # reads are substrings of their windows: most alignments cover most of the read
    assert np.median(ends[:, 1] - starts[:, 0]) > 100


def test_starts_long_queries_int32_chunked():
    # queries of thousands of residues against short references: chunked
    # per-pair launches of the reversed prefixes, int32 lanes
    w = W.random_pairs(40, 20, (2000, 6000), (50, 400), 890)
    _check(w, "long queries i32", precision=api.SW_PREC_I32)
    _check(w, "long queries auto")


def test_starts_saturated_pairs_rerun_in_int32():
    M = W.protein_matrix().copy()
    np.fill_diagonal(M, 100)
    rng = np.random.default_rng(891)
    q = rng.integers(0, 20, size=700).astype(np.uint8)
    qres = np.concatenate([q, q[100:500]])
    qoff = np.array([0, 700, 1100], dtype=np.int64)
    w = W.Workload("sat", qres, qoff, qres, qoff, np.array([0, 1, 0], np.int32),
                   np.array([0, 1, 1], np.int32), M, 11, 1)
    ends, starts = _check(w, "saturated")
    assert ends[0, 0] > 32767 and ends[0, 3] == api.SW_FLAG_SATURATED
    assert starts[0].tolist() == [0, 0] and starts[1].tolist() == [0, 0]
    assert starts[2].tolist() == [100, 0]          # q[100:500] inside q


def test_starts_device_resident_and_errors():
    import torch
    w = W.random_pairs(300, 20, (0, 200), (0, 300), 892)
    ends, starts = _check(w, "host")
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    qs, rs = api.sw_align_batch_starts(t(w.query_res, torch.uint8), t(w.query_off, torch.int64),
                                       t(w.ref_res, torch.uint8), t(w.ref_off, torch.int64),
                                       t(w.pair_ref, torch.int32), w.matrix, w.gap_open,
                                       w.gap_extend, ends,
                                       pair_query=t(w.pair_query, torch.int32))
    assert (np.stack([qs, rs], axis=1) == starts).all()
    k = int(np.argmax(ends[:, 0]))
    args = (w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref, w.matrix, w.gap_open,
            w.gap_extend)
    wrong = ends.copy()
    wrong[k, 0] += 1                               # not the optimum at that end cell
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_starts(*args, wrong, pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    outside = ends.copy()
    outside[k, 2] = 10 ** 6                        # end cell past the reference
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_starts(*args, outside, pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    qs2, rs2 = api.sw_align_batch_starts(*args, ends, pair_query=w.pair_query)
    assert (np.stack([qs2, rs2], axis=1) == starts).all()


def _one_query(seed, m, n_refs, nlen, alpha, matrix, go=11, ge=1):
    rng = np.random.default_rng(seed)
    q = rng.integers(0, alpha, size=m).astype(np.uint8)
    lens = rng.integers(nlen[0], nlen[1] + 1, size=n_refs)
    refs = [rng.integers(0, alpha, size=int(L)).astype(np.uint8) for L in lens]
    roff = np.zeros(n_refs + 1, dtype=np.int64)
    np.cumsum(lens, out=roff[1:])
    return W.Workload("one_query", q, np.array([0, m], dtype=np.int64), np.concatenate(refs), roff,
                      None, np.arange(n_refs, dtype=np.int32), matrix, go, ge)


@pytest.mark.parametrize("alpha,m", [(2, 200), (4, 512), (20, 97)])
def test_starts_one_query_masked_rows(alpha, m):
    """One query: every pair's reversed prefix is a suffix of the reversed
    query, aligned in one masked row-pair launch (rows before the suffix
    capped at score 0)."""
    rng = np.random.default_rng(900 + alpha)
    M = W.protein_matrix() if alpha == 20 else W.random_matrix(rng, alpha)
    w = _one_query(901 + alpha, m, 3000, (1, 700), alpha, M)
    _check(w, "one query alpha=%d m=%d" % (alpha, m))


def test_starts_one_query_saturated_pairs_take_int32():
    # copies of the query inside the references: with a diagonal of 100 the
    # best score exceeds 32767, so those pairs leave the masked int16 launch
    M = W.protein_matrix().copy()
    np.fill_diagonal(M, 100)
    rng = np.random.default_rng(902)
    q = rng.integers(0, 20, size=450).astype(np.uint8)
    refs = []
    for k in range(400):
        r = rng.integers(0, 20, size=int(rng.integers(50, 900))).astype(np.uint8)
        if k % 7 == 0:
            at = int(rng.integers(0, r.size))
            r = np.concatenate([r[:at], q[k % 50:], r[at:]])
        refs.append(r)
    roff = np.zeros(len(refs) + 1, dtype=np.int64)
    np.cumsum([r.size for r in refs], out=roff[1:])
    w = W.Workload("sat1", q, np.array([0, q.size], np.int64), np.concatenate(refs), roff, None,
                   np.arange(len(refs), dtype=np.int32), M, 11, 1)
    ends, starts = _check(w, "one query, saturated")
    assert (ends[:, 3] == api.SW_FLAG_SATURATED).sum() > 10


def test_starts_one_aligned_query_among_several_and_offsets():
    # pair_query names three queries, but only query 1 aligns anywhere (the
    # other two are empty): the device tables see one query and hand the
    # batch to the one-query launch; then a query whose offsets run past the
    # residue total is refused
    rng = np.random.default_rng(905)
    M = W.random_matrix(rng, 4)
    q = rng.integers(0, 4, size=180).astype(np.uint8)
    qoff = np.array([0, 0, 180, 180], dtype=np.int64)
    lens = rng.integers(50, 400, size=40)
    roff = np.zeros(41, dtype=np.int64)
    np.cumsum(lens, out=roff[1:])
    rres = rng.integers(0, 4, size=int(roff[-1])).astype(np.uint8)
    pr = np.arange(40, dtype=np.int32)
    pq = np.array([1 if k % 3 else (0 if k % 2 else 2) for k in range(40)], dtype=np.int32)
    w = W.Workload("one_aligned", q, qoff, rres, roff, pq, pr, M, 3, 1, {})
    ends, starts = _check(w, "one aligned query")
    assert (ends[pq != 1, 0] == 0).all() and (ends[pq == 1, 0] > 0).all()
    # several aligned queries, one of whose offsets runs past the residues
    w2 = W.random_pairs(200, 4, (20, 120), (20, 200), 906)
    ends2, _ = _check(w2, "several queries")
    k = int(np.argmax(ends2[:, 0]))
    qo = w2.query_off.copy()
    qo[-1] = qo[w2.pair_query[k] + 1] - 1
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_starts(w2.query_res[:qo[-1]], qo, w2.ref_res, w2.ref_off, w2.pair_ref,
                                  w2.matrix, w2.gap_open, w2.gap_extend, ends2,
                                  pair_query=w2.pair_query)
    assert e.value.code == api.SW_EINVAL


@pytest.mark.parametrize("alpha,go,ge", [(4, 6, 1), (2, 2, 3), (4, 1, 1)])
def test_starts_short_queries_long_references(alpha, go, ge):
    # 20-80 residue queries against 500-2000 residue references, each query
    # planted (mutated) near a random place and a second copy elsewhere: the
    # reversed reference prefixes run far past the alignments, so the cut to
    # the span an alignment of the score can have decides most of the work;
    # two letters make many optimal alignments, so the tie rule is exercised
    rng = np.random.default_rng(907 + alpha + 10 * go + 100 * ge)
    M = W.random_matrix(rng, alpha)
    np.fill_diagonal(M, np.abs(np.diag(M)) + 1)
    qs, rs = [], []
    for k in range(300):
        m = int(rng.integers(20, 81))
        n = int(rng.integers(500, 2001))
        q = rng.integers(0, alpha, size=m).astype(np.uint8)
        r = rng.integers(0, alpha, size=n).astype(np.uint8)
        for _ in range(2):
            at = int(rng.integers(0, n - m))
            cp = q.copy()
            flip = rng.random(m) < 0.05
            cp[flip] = rng.integers(0, alpha, size=int(flip.sum()))
            r[at:at + m] = cp
        qs.append(q)
        rs.append(r)
    qoff = np.zeros(301, dtype=np.int64)
    roff = np.zeros(301, dtype=np.int64)
    np.cumsum([x.size for x in qs], out=qoff[1:])
    np.cumsum([x.size for x in rs], out=roff[1:])
    idx = np.arange(300, dtype=np.int32)
    w = W.Workload("short_vs_long", np.concatenate(qs), qoff, np.concatenate(rs), roff, idx,
                   idx.copy(), M, go, ge, {})
    _check(w, "short vs long alpha=%d go=%d ge=%d" % (alpha, go, ge))
