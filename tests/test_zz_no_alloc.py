"""sw_align_batch_noalloc (the batch call that allocates nothing: every buffer
in the library's fixed scratch array, results written to a device array)
through the C ABI: its results equal sw_align_batch's exactly on the same
device-resident inputs, on two calls in a row (the second smaller, so the
scratch array holds the first call's contents), for one query (row-pair
kernel), a query per pair (8-lane per-pair kernel), the int32 rerun of
saturated pairs, and its argument errors."""
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
    pq = None if w.pair_query is None else t(w.pair_query, torch.int32)
    return (t(w.query_res, torch.uint8), t(w.query_off, torch.int64), t(w.ref_res, torch.uint8),
            t(w.ref_off, torch.int64), t(w.pair_ref, torch.int32)), pq


def _noalloc(w, precision=api.SW_PREC_AUTO):
    import torch
    args, pq = _device(w)
    out = torch.full((w.n_pairs, 4), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    st = api.sw_align_batch_noalloc(*args, w.matrix, w.gap_open, w.gap_extend, out,
                                    pair_query=pq, precision=precision)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st


def _batch(w, precision=api.SW_PREC_AUTO):
    args, pq = _device(w)
    return api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq,
                              precision=precision)


def _assert_equal(got, want, label):
    bad = np.nonzero((got != want).any(axis=1))[0]
    if bad.size:
        k = int(bad[0])
        raise AssertionError("%s: %d/%d entries differ; first pair %d got %s want %s" %
                             (label, bad.size, len(want), k, got[k].tolist(), want[k].tolist()))


def _oracle_sample(w, got, count=300, seed=0):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(w.n_pairs, size=min(count, w.n_pairs), replace=False))
    sub = w.subset(idx)
    want = oracle.align_batch(sub.query_res, sub.query_off, sub.ref_res, sub.ref_off,
                              sub.pair_ref, sub.matrix, sub.gap_open, sub.gap_extend,
                              pair_query=sub.pair_query)
    _assert_equal(got[idx, :3], want, "oracle sample")


def test_one_query_two_calls_second_smaller():
    w = W.protein_search(n_refs=30_000)
    print("case: protein search 512 x 30000, then x 7000", flush=True)
    got1, st1 = _noalloc(w)
    want1 = _batch(w).results
    _assert_equal(got1, want1, "first call (30000 pairs)")
    assert st1["planner_used"] == 2 and st1["row_pairs"] > 0 and st1["n_rerun"] == 0
    _oracle_sample(w, got1)
    w2 = w.subset(np.arange(11_000, 18_000))
    got2, st2 = _noalloc(w2)
    _assert_equal(got2, _batch(w2).results, "second call (7000 pairs)")
    assert st2["cells"] == w2.cells()
    _oracle_sample(w2, got2, seed=1)


def test_query_per_pair_two_calls_second_smaller():
    w = W.dna_pairs(n_pairs=40_000)
    print("case: DNA pairs 40000, then 9000", flush=True)
    got1, st1 = _noalloc(w)
    _assert_equal(got1, _batch(w).results, "first call (40000 pairs)")
    assert st1["lanes8"] > 0
    _oracle_sample(w, got1)
    w2 = w.subset(np.arange(3_000, 12_000)[::-1])
    got2, _ = _noalloc(w2)
    _assert_equal(got2, _batch(w2).results, "second call (9000 pairs)")
    _oracle_sample(w2, got2, seed=1)


def test_int32_and_random_per_pair_queries():
    # per-pair 20-letter queries of up to 64 residues fit the int32 per-pair
    # shapes too; DNA queries of up to 256 residues
    for alpha, mlen in ((20, (1, 64)), (4, (1, 256))):
        w = W.random_pairs(3000, alpha, mlen, (1, 600), seed=21 + alpha)
        print("case: random per-pair alpha %d, 3000 pairs, int32 then auto" % alpha, flush=True)
        for prec in (api.SW_PREC_I32, api.SW_PREC_AUTO):
            got, _ = _noalloc(w, prec)
            _assert_equal(got, _batch(w, prec).results, "alpha %d precision %d" % (alpha, prec))
        _oracle_sample(w, got)


def test_saturated_pairs_rerun_in_int32():
    # scores of 100 per matching residue: a 512-residue query against copies
    # of itself reaches 51200 > 32767, so those pairs rerun in int32
    rng = np.random.default_rng(7)
    alpha = 8
    M = rng.integers(-30, 20, size=(alpha, alpha)).astype(np.int32)
    np.fill_diagonal(M, 100)
    q = rng.integers(0, alpha, size=512).astype(np.uint8)
    refs = []
    for k in range(600):
        if k % 50 == 0:
            refs.append(q[rng.integers(0, 40):].copy())
        else:
            refs.append(rng.integers(0, alpha, size=int(rng.integers(20, 700))).astype(np.uint8))
    roff = np.zeros(len(refs) + 1, dtype=np.int64)
    np.cumsum([len(r) for r in refs], out=roff[1:])
    w = W.Workload("saturating", q, np.array([0, 512], dtype=np.int64), np.concatenate(refs),
                   roff, None, np.arange(len(refs), dtype=np.int32), M, 11, 1)
    print("case: saturating one-query batch, then its first 120 pairs", flush=True)
    got, st = _noalloc(w)
    want = _batch(w).results
    _assert_equal(got, want, "saturating batch")
    sat = (got[:, 3] & api.SW_FLAG_SATURATED) != 0
    assert sat[::50].all() and st["n_rerun"] == sat.sum() and st["n_launches"] == 2
    assert (got[sat, 0] >= 32767).all()
    _oracle_sample(w, got, count=120)
    w2 = w.subset(np.arange(120))
    got2, st2 = _noalloc(w2)
    _assert_equal(got2, _batch(w2).results, "second, smaller saturating batch")
    sat2 = (got2[:, 3] & api.SW_FLAG_SATURATED) != 0
    assert sat2[::50].all() and st2["n_rerun"] == sat2.sum()


def test_errors():
    import torch
    w = W.random_pairs(50, 4, (1, 100), (1, 100), seed=3)
    args, pq = _device(w)
    out = torch.zeros((w.n_pairs, 4), dtype=torch.int32, device="cuda")
    # host inputs are refused
    with pytest.raises(TypeError):
        api.sw_align_batch_noalloc(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                                   w.matrix, w.gap_open, w.gap_extend, out, pair_query=w.pair_query)
    # a residue outside the alphabet: SW_EINVAL and every result empty
    bad = w.query_res.copy()
    bad[5] = 4
    a2 = list(args)
    a2[0] = torch.from_numpy(bad).cuda()
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_noalloc(*a2, w.matrix, w.gap_open, w.gap_extend, out, pair_query=pq)
    assert e.value.code == api.SW_EINVAL
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == np.array([0, -1, -1, 0], dtype=np.int32)).all()
    # more pairs than the scratch array holds
    n = api.SW_NOALLOC_MAX_PAIRS + 1
    big_pr = torch.zeros(n, dtype=torch.int32, device="cuda")
    big_out = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_noalloc(args[0], args[1], args[2], args[3], big_pr, w.matrix,
                                   w.gap_open, w.gap_extend, big_out)
    assert e.value.code == api.SW_EINVAL
    # per-pair 20-letter queries longer than every per-pair shape: refused
    w3 = W.random_pairs(40, 20, (200, 220), (10, 50), seed=4)
    a3, pq3 = _device(w3)
    out3 = torch.zeros((w3.n_pairs, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_noalloc(*a3, w3.matrix, w3.gap_open, w3.gap_extend, out3,
                                   pair_query=pq3)
    assert e.value.code == api.SW_EINVAL
    # the call still works after the errors
    got, _ = _noalloc(w)
    _assert_equal(got, _batch(w).results, "after errors")
