"""Start cells, paths and end-to-end scores at the full benchmark sizes, in
the configuration bench.py times (device-resident sequences): every path of
the 100k protein-search and 1M DNA-pair alignments covers exactly the
rectangle between its start and end cell, has the canonical shape and adds
up to the score (checked for all pairs, vectorised); sampled pairs equal the
CPU oracle's paths, start cells, global / semi-global results and semi-global
paths, and the reference-fitted results with the roles swapped (which equal
the semi-global scores for every pair: the DNA scoring is symmetric)."""
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


def _device(w):
    import torch
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    args = (t(w.query_res, torch.uint8), t(w.query_off, torch.int64), t(w.ref_res, torch.uint8),
            t(w.ref_off, torch.int64), t(w.pair_ref, torch.int32))
    pq = None if w.pair_query is None else t(w.pair_query, torch.int32)
    return args, pq


def _seqs(w, k):
    qi = 0 if w.pair_query is None else int(w.pair_query[k])
    ri = int(w.pair_ref[k])
    return (w.query_res[w.query_off[qi]:w.query_off[qi + 1]],
            w.ref_res[w.ref_off[ri]:w.ref_off[ri + 1]])


def _check_all_paths(w, ends, qs, rs, runs, off):
    """Vectorised over every run of every pair."""
    n = w.n_pairs
    nr = np.diff(off)
    live = ends[:, 0] > 0
    assert (nr[~live] == 0).all() and (nr[live] > 0).all()
    lens = (runs >> 4).astype(np.int64)
    ops = (runs & 15).astype(np.int64)
    assert (lens > 0).all() and (ops <= 2).all()
    pair = np.repeat(np.arange(n), nr)
    first = off[:-1][live]
    last = off[1:][live] - 1
    assert (ops[first] == 0).all() and (ops[last] == 0).all()          # M first and last
    same = pair[1:] == pair[:-1]
    assert not (same & (ops[1:] == ops[:-1])).any()                    # runs merged
    assert not (same & (ops[:-1] == 1) & (ops[1:] == 2)).any()         # D before I
    dq = np.where(ops != 2, lens, 0)
    dr = np.where(ops != 1, lens, 0)
    qspan = np.bincount(pair, dq, minlength=n).astype(np.int64)
    rspan = np.bincount(pair, dr, minlength=n).astype(np.int64)
    assert (qspan[live] == ends[live, 1] - qs[live] + 1).all()
    assert (rspan[live] == ends[live, 2] - rs[live] + 1).all()
    ge = min(w.gap_extend, w.gap_open)
    gaps = np.bincount(pair, np.where(ops != 0, w.gap_open + (lens - 1) * ge, 0),
                       minlength=n).astype(np.int64)
    # residue positions of every aligned pair
    cq = np.cumsum(dq) - dq
    cr = np.cumsum(dr) - dr
    run_first = np.repeat(off[:-1], nr)
    qi = 0 if w.pair_query is None else w.pair_query
    qbase = (w.query_off[qi] if w.pair_query is not None else np.full(n, w.query_off[0])) + qs
    rbase = w.ref_off[w.pair_ref] + rs
    qstart = qbase[pair] + cq - cq[run_first]
    rstart = rbase[pair] + cr - cr[run_first]
    m = ops == 0
    mlen = lens[m]
    within = np.arange(mlen.sum()) - np.repeat(np.cumsum(mlen) - mlen, mlen)
    qpos = np.repeat(qstart[m], mlen) + within
    rpos = np.repeat(rstart[m], mlen) + within
    sub = w.matrix[w.query_res[qpos], w.ref_res[rpos]].astype(np.int64)
    score = np.bincount(np.repeat(pair[m], mlen), sub, minlength=n).astype(np.int64) - gaps
    bad = np.nonzero(live & (score != ends[:, 0]))[0]
    assert bad.size == 0, "%d paths do not add up to their score; first pair %d: %d vs %d" % (
        bad.size, bad[0], score[bad[0]], ends[bad[0], 0])


def _full(w, pick):
    args, pq = _device(w)
    ends = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq).results
    qs, rs = api.sw_align_batch_starts(*args, w.matrix, w.gap_open, w.gap_extend, ends,
                                       pair_query=pq)
    runs, off = api.sw_align_batch_cigar(*args, w.matrix, w.gap_open, w.gap_extend, ends, qs, rs,
                                         pair_query=pq)
    _check_all_paths(w, ends, qs, rs, runs, off)
    for k in pick(ends, qs, rs):
        q, r = _seqs(w, k)
        e = tuple(int(x) for x in ends[k, :3])
        assert oracle.start_cell(q, r, w.matrix, w.gap_open, w.gap_extend, end=e) == \
            (int(qs[k]), int(rs[k])), k
        want = oracle.path(q, r, w.matrix, w.gap_open, w.gap_extend, end=e,
                           start=(int(qs[k]), int(rs[k])))
        assert api.decode_cigar(runs, off, k) == want, k
    return args, pq


def test_protein_search_paths_full_size():
    w = W.protein_search()

    def pick(ends, qs, rs):
        # the oracle's paths are plain maxima over the rectangle: sample the
        # pairs whose rectangles it finishes quickly, and the smallest ones
        area = (ends[:, 1] - qs + 1).astype(np.int64) * (ends[:, 2] - rs + 1)
        order = np.argsort(np.where(ends[:, 0] > 0, area, 1 << 40), kind="stable")
        small = order[:2000]
        small = small[area[small] <= 2500]
        assert small.size >= 40
        return small[:: small.size // 40][:40]

    _full(w, pick)


def test_dna_pairs_paths_and_endtoend_full_size():
    w = W.dna_pairs(n_pairs=1_000_000)
    args, pq = _full(w, lambda ends, qs, rs: [0, 333_333, 999_999])
    glob = api.sw_align_batch_global(*args, w.matrix, w.gap_open, w.gap_extend,
                                     mode=api.SW_MODE_GLOBAL, pair_query=pq)
    semi = api.sw_align_batch_global(*args, w.matrix, w.gap_open, w.gap_extend,
                                     mode=api.SW_MODE_SEMIGLOBAL, pair_query=pq)
    local = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq).results
    assert (semi[:, 0] >= glob[:, 0]).all() and (local[:, 0] >= semi[:, 0]).all()
    assert (glob[:, 1] == 149).all() and (semi[:, 1] == 149).all()
    assert (glob[:, 2] == np.diff(w.ref_off) - 1).all()
    for k in range(0, 1_000_000, 20_000):
        q, r = _seqs(w, k)
        for got, mode in ((glob, 0), (semi, 1)):
            want = oracle.endtoend(q, r, w.matrix, w.gap_open, w.gap_extend, mode)
            assert tuple(int(x) for x in got[k, :3]) == want, (k, mode)
    # the semi-global paths of every pair (device-memory path launches of the
    # most wavefronts they take), sampled against the oracle
    qs, rs, runs, off = api.sw_align_batch_global_cigar(
        *args, w.matrix, w.gap_open, w.gap_extend, semi, mode=api.SW_MODE_SEMIGLOBAL, pair_query=pq)
    for k in range(0, 1_000_000, 20_000):
        q, r = _seqs(w, k)
        want = oracle.endtoend_path(q, r, w.matrix, w.gap_open, w.gap_extend, 1,
                                    end=tuple(int(x) for x in semi[k, :3]))
        assert (int(qs[k]), int(rs[k]), api.decode_cigar(runs, off, k)) == want, k
    # the roles swapped (windows of 300-600 as queries, reads as references;
    # the windows over 512 residues in two tiles, up to 8192 wavefronts)
    swapped = (args[2], args[3], args[0], args[1], pq)
    sref = api.sw_align_batch_global(*swapped, w.matrix, w.gap_open, w.gap_extend,
                                     mode=api.SW_MODE_SEMIGLOBAL_REF, pair_query=args[4])
    assert (sref[:, 0] == semi[:, 0]).all()
    for k in range(0, 1_000_000, 20_000):
        q, r = _seqs(w, k)
        want = oracle.endtoend(r, q, w.matrix, w.gap_open, w.gap_extend,
                               api.SW_MODE_SEMIGLOBAL_REF)
        assert tuple(int(x) for x in sref[k, :3]) == want, k
