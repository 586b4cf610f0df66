"""The autotuner on device-planned batches: sw_autotune times every compiled
device-planned shape that holds the query (row pairs with LDS or register
end-cell records, two alignments per lane) or the longest per-pair query (8
and 16 lanes), installs the fastest, and a later sw_align_batch runs that shape
with results equal to the untuned call and to the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    api.load()
    api.sw_init()


@pytest.fixture(autouse=True)
def _keep_table():
    saved = api.tune_get()
    api.tune_set([])
    yield
    api.tune_set(saved)


def _device(w):
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    pq = None if w.pair_query is None else t(w.pair_query, torch.int32)
    return (t(w.query_res, torch.uint8), t(w.query_off, torch.int64), t(w.ref_res, torch.uint8),
            t(w.ref_off, torch.int64), t(w.pair_ref, torch.int32)), pq


def _sample_oracle(w, got, count=400):
    idx = np.sort(np.random.default_rng(9).choice(w.n_pairs, size=count, replace=False))
    sub = w.subset(idx)
    want = oracle.align_batch(sub.query_res, sub.query_off, sub.ref_res, sub.ref_off,
                              sub.pair_ref, sub.matrix, sub.gap_open, sub.gap_extend,
                              pair_query=sub.pair_query)
    assert (got[idx, :3] == want).all()


@pytest.mark.parametrize("m", [512, 300, 100])
def test_tuned_one_query_shape_is_used_and_exact(m):
    w = W.protein_search(n_refs=12_000, m=m)
    d, pq = _device(w)
    base = api.sw_align_batch(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq)
    assert base.stats["planner_used"] == 2
    entries = api.sw_autotune(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq)
    dev = [e for e in entries if e["kind"] == api.SW_TUNE_DEVICE_SHARED]
    assert len(dev) == 1 and dev[0]["m_lo"] == m and dev[0]["gcups"] > 0
    e = dev[0]
    tuned = api.sw_align_batch(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq)
    assert tuned.stats["planner_used"] == 2 and tuned.stats["seglen_max"] == e["seglen"]
    if e["pairing"] == api.SW_PAIRING_ROWS:
        assert tuned.stats["row_pairs"] > 0
    else:
        assert tuned.stats["row_pairs"] == 0
        assert sum(tuned.stats["lanes_used"]) > 0
    assert (tuned.results == base.results).all()
    _sample_oracle(w, tuned.results)


def test_tuned_per_pair_shape_is_used_and_exact():
    w = W.dna_pairs(n_pairs=30_000)
    d, pq = _device(w)
    base = api.sw_align_batch(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq)
    assert base.stats["planner_used"] == 2
    entries = api.sw_autotune(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq)
    dev = [e for e in entries if e["kind"] == api.SW_TUNE_DEVICE_PAIR]
    assert len(dev) == 1 and dev[0]["m_lo"] == int(np.diff(w.query_off).max())
    e = dev[0]
    tuned = api.sw_align_batch(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq)
    assert tuned.stats["seglen_max"] == e["seglen"]
    if e["lanes"] == 8:
        assert tuned.stats["lanes8"] == w.n_pairs
    else:
        assert tuned.stats["lanes_used"][0] == w.n_pairs
    assert (tuned.results == base.results).all()
    _sample_oracle(w, tuned.results)


def test_forced_options_override_the_table():
    w = W.protein_search(n_refs=6000)
    d, pq = _device(w)
    api.tune_set([dict(kind=api.SW_TUNE_DEVICE_SHARED, precision=api.SW_PREC_AUTO,
                       alphabet_size=20, m_lo=512, m_hi=512, lanes=32, seglen=16, mixed=0,
                       pairing=api.SW_PAIRING_ALIGNMENTS, lds_records=0, gcups=1.0,
                       model_gcups=1.0)])
    tuned = api.sw_align_batch(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq)
    assert tuned.stats["row_pairs"] == 0 and tuned.stats["lanes_used"][1] == w.n_pairs
    rows = api.sw_align_batch(*d, w.matrix, w.gap_open, w.gap_extend, pair_query=pq,
                              lane_pairing=api.SW_PAIRING_ROWS)
    assert rows.stats["row_pairs"] == w.n_pairs
    assert (rows.results == tuned.results).all()
    _sample_oracle(w, tuned.results)
