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
