"""GPU parity at the long-and-adversarial workload's stated sizes: 64 queries of
5000-35000 residues (half i.i.d., half poly-residue runs of 50-500), each
against 4 i.i.d. and 4 run-structured references of 200-2000 residues drawn
from the 10k-reference set; protein matrix, GapOpen 11, GapExtend 1, int32.

Both the scan kernel (Algorithm 6) and the lazy-F comparator (Algorithm 1)
must equal the oracle element by element; the queries run as many query
chunks (boundary H and scan carry per column), so every chunk hand-over of
the long path is exercised at full length."""
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


@pytest.fixture(scope="module")
def subset():
    w = W.long_queries_subset(W.long_queries(), per_query=8)
    want = oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                              w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query)
    return w, want


def _check(got, want, label):
    bad = np.nonzero((np.asarray(got)[:, :3] != want).any(axis=1))[0]
    assert bad.size == 0, "%s: %d/%d mismatches, first pair %d got %s want %s" % (
        label, bad.size, len(want), bad[0], got[bad[0], :3].tolist(), want[bad[0]].tolist())


def test_subset_shape(subset):
    w, want = subset
    ql = w.query_lengths()
    assert w.n_pairs == 512
    assert ql.min() >= 5000 and ql.max() <= 35000 and ql.max() > 30000
    rl = w.ref_lengths()
    assert rl.min() >= 200 and rl.max() <= 2000
    assert (want[:, 0] > 0).all()


def test_scan_equals_oracle(subset):
    w, want = subset
    got = api.align_workload(w, precision=api.SW_PREC_I32)
    _check(got.results, want, "scan")


def test_lazyf_equals_oracle(subset):
    w, want = subset
    got = api.align_workload(w, precision=api.SW_PREC_I32, algorithm=api.SW_ALG_LAZYF)
    _check(got.results, want, "lazy-F")
    assert got.stats["lazyf_steps"] > 0


def test_auto_precision_equals_oracle(subset):
    # int16 lanes with the int32 rerun of saturated pairs on the same pairs
    w, want = subset
    got = api.align_workload(w)
    _check(got.results, want, "auto")
