"""Two int32 column chains per sub-group (the shared-query kernel's int32
scan launches with SW_CHAINS_TWO) against one chain and the CPU oracle, element by
element through the C ABI: every lane width, chunked and unchunked queries,
an odd number of pairs (a task whose last sub-group has an empty second
chain), the gap-to-gap family, and the long-and-adversarial workload's
query lengths."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu
ONE, TWO = api.SW_CHAINS_ONE, api.SW_CHAINS_TWO


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    api.load()
    api.sw_init()


def _oracle(w):
    return oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                              w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query)


def _check(got, want, label):
    bad = np.nonzero((np.asarray(got)[:, :3] != want).any(axis=1))[0]
    assert bad.size == 0, "%s: %d/%d mismatches, first pair %d got %s want %s" % (
        label, bad.size, len(want), bad[0], got[bad[0], :3].tolist(), want[bad[0]].tolist())


def _one_query(seed, m, n_refs, nlen, alpha=20, go=11, ge=1):
    rng = np.random.default_rng(seed)
    q = rng.integers(0, alpha, size=m).astype(np.uint8)
    lens = rng.integers(nlen[0], nlen[1] + 1, size=n_refs)
    refs = [rng.integers(0, alpha, size=int(L)).astype(np.uint8) for L in lens]
    roff = np.zeros(n_refs + 1, dtype=np.int64)
    np.cumsum(lens, out=roff[1:])
    M = W.protein_matrix() if alpha == 20 else W.random_matrix(rng, alpha)
    return W.Workload("one_query", q, np.array([0, m], dtype=np.int64), np.concatenate(refs),
                      roff, None, np.arange(n_refs, dtype=np.int32), M, go, ge)


@pytest.mark.parametrize("lanes", [0, 16, 32, 64])
@pytest.mark.parametrize("m", [37, 256, 700])
def test_shared_int32_two_chains_equal_one_and_the_oracle(lanes, m):
    # 301 references: an odd count, so one task's last chain is empty; 700
    # residues run as query chunks at every width
    w = _one_query(3000 + m + lanes, m, 301, (1, 500))
    want = _oracle(w)
    kw = dict(precision=api.SW_PREC_I32, force_kernel=1, force_lanes=lanes)
    two = api.align_workload(w, int32_chains=TWO, **kw)
    _check(two.results, want, "two chains lanes=%d m=%d" % (lanes, m))
    one = api.align_workload(w, int32_chains=ONE, **kw)
    _check(one.results, want, "one chain lanes=%d m=%d" % (lanes, m))
    auto = api.align_workload(w, **kw)
    assert (auto.results == one.results).all()


@pytest.mark.parametrize("lanes,seg", [(16, 4), (32, 4), (64, 4), (16, 8), (64, 8), (32, 12)])
def test_two_chains_every_compiled_shape_chunked(lanes, seg):
    w = _one_query(3100 + lanes + seg, 1500, 120, (20, 300), alpha=4, go=6, ge=1)
    want = _oracle(w)
    got = api.align_workload(w, precision=api.SW_PREC_I32, force_kernel=1, force_lanes=lanes,
                             force_seglen=seg, int32_chains=TWO)
    _check(got.results, want, "lanes=%d seg=%d" % (lanes, seg))


def test_two_chains_gap_to_gap_family():
    # gap-to-gap moves strictly optimal (+5 / -4, GapOpen 11, GapExtend 1):
    # q = X^p A^12 X^k B^12 against r = A^12 Y^k B^12, X and Y mismatching
    # everything; the prefix length p moves the bridge across lane and chunk
    # boundaries
    M = np.full((4, 4), -4, dtype=np.int32)
    np.fill_diagonal(M, 5)
    refs = [np.array([0] * 12 + [3] * k + [2] * 12, dtype=np.uint8) for k in (11, 12, 16)]
    roff = np.zeros(len(refs) + 1, dtype=np.int64)
    np.cumsum([r.size for r in refs], out=roff[1:])
    for k in (11, 12, 16):
        for pre in range(0, 40, 3):
            q = np.array([1] * pre + [0] * 12 + [1] * k + [2] * 12, dtype=np.uint8)
            w = W.Workload("g2g", q, np.array([0, q.size], dtype=np.int64), np.concatenate(refs),
                           roff, None, np.arange(len(refs), dtype=np.int32), M, 11, 1)
            want = _oracle(w)
            for lanes, seg in ((16, 4), (32, 4), (64, 4)):
                got = api.align_workload(w, precision=api.SW_PREC_I32, force_kernel=1,
                                         force_lanes=lanes, force_seglen=seg, int32_chains=TWO)
                _check(got.results, want, "g2g lanes=%d seg=%d k=%d p=%d" % (lanes, seg, k, pre))


def test_long_queries_through_the_shared_kernel():
    # the long-and-adversarial workload's queries (5k-35k residues, query
    # chunks of 512 rows) against 2 of their subset references each (one
    # i.i.d., one run-structured), forced through the shared-query kernel
    # with both chain counts
    w = W.long_queries_subset(W.long_queries(), per_query=8)
    sub = w.subset(np.arange(0, w.n_pairs, 4))    # 2 references per query
    want = _oracle(sub)
    for chains in (ONE, TWO):
        got = api.align_workload(sub, precision=api.SW_PREC_I32, force_kernel=1,
                                 int32_chains=chains)
        _check(got.results, want, "long queries chains=%d" % chains)
