"""Swapped striping (SW_STRIPE_SHORTER: the reference striped over the lanes,
the query streamed as columns, scores read from the matrix) against the CPU
oracle element by element through the C ABI: every rows-per-lane group up to
2048-residue references, ragged lengths, gap penalties with free gaps and an
extension above the opening, tie-heavy inputs where the (ref_end, query_end)
order of the end cell differs from the streamed order, the long-and-adversarial
workload's subset, and mixed batches where only some pairs swap."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu
SWAP = api.SW_STRIPE_SHORTER


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


def _pairs(seed, qlens, rlens, alpha, matrix=None, go=11, ge=1, runs=False):
    rng = np.random.default_rng(seed)

    def seq(L):
        if not runs:
            return rng.integers(0, alpha, size=int(L)).astype(np.uint8)
        out, c = [], int(rng.integers(0, alpha))
        while len(out) < L:
            c = (c + 1 + int(rng.integers(0, alpha - 1))) % alpha
            out += [c] * int(rng.integers(1, 40))
        return np.array(out[:int(L)], dtype=np.uint8)

    qs = [seq(L) for L in qlens]
    rs = [seq(L) for L in rlens]
    qoff = np.zeros(len(qs) + 1, dtype=np.int64)
    roff = np.zeros(len(rs) + 1, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    np.cumsum([r.size for r in rs], out=roff[1:])
    if matrix is None:
        matrix = W.protein_matrix() if alpha == 20 else W.random_matrix(rng, alpha)
    idx = np.arange(len(qs), dtype=np.int32)
    return W.Workload("swap", np.concatenate(qs), qoff, np.concatenate(rs), roff, idx,
                      idx.copy(), np.asarray(matrix, dtype=np.int32), go, ge)


@pytest.mark.parametrize("alpha,go,ge", [(20, 11, 1), (4, 6, 1), (4, 0, 0), (3, 2, 5), (20, 3, 3)])
def test_every_row_group_equals_the_oracle(alpha, go, ge):
    # references in every 256-row group up to 2048 (and 1-row ones), queries
    # longer than their references
    rng = np.random.default_rng(4000 + alpha + go + ge)
    rl = np.concatenate([[1, 2, 255, 256, 257, 2047, 2048],
                         rng.integers(1, 2049, size=73)])
    ql = rl + rng.integers(1, 900, size=rl.size)
    w = _pairs(4001 + alpha, ql, rl, alpha, go=go, ge=ge)
    got = api.align_workload(w, precision=api.SW_PREC_I32, striping=SWAP)
    assert got.stats["seglen_max"] == 32
    _check(got.results, _oracle(w), "alpha=%d go=%d ge=%d" % (alpha, go, ge))


def test_tie_heavy_inputs():
    # poly-residue runs and a two-letter identity: many cells share the
    # maximum, in several rows and columns; the end cell must be the smallest
    # (ref_end, query_end), not the first one in streamed (column) order
    I2 = np.array([[1, -1], [-1, 1]], dtype=np.int32)
    w = _pairs(4100, [400] * 40, [int(x) for x in np.linspace(5, 390, 40)], 2, matrix=I2,
               go=1, ge=1, runs=True)
    want = _oracle(w)
    _check(api.align_workload(w, precision=api.SW_PREC_I32, striping=SWAP).results, want,
           "runs")
    # all-zero sequences: the maximum n is reached at every column from n - 1 on
    zq = np.zeros(3000, dtype=np.uint8)
    zr = [np.zeros(n, dtype=np.uint8) for n in (1, 7, 64, 65, 700, 2048)]
    roff = np.zeros(len(zr) + 1, dtype=np.int64)
    np.cumsum([r.size for r in zr], out=roff[1:])
    wz = W.Workload("zeros", zq, np.array([0, zq.size], dtype=np.int64), np.concatenate(zr),
                    roff, None, np.arange(len(zr), dtype=np.int32), I2, 0, 0)
    got = api.align_workload(wz, precision=api.SW_PREC_I32, striping=SWAP)
    want = _oracle(wz)
    _check(got.results, want, "zeros")
    assert [tuple(x) for x in want] == [(n, n - 1, n - 1) for n in (1, 7, 64, 65, 700, 2048)]


def test_long_queries_subset():
    # the long-and-adversarial subset: 64 queries of 5k-35k residues, 8
    # references of 200-2000 each, int32: every pair swaps
    w = W.long_queries_subset(W.long_queries(), per_query=8)
    got = api.align_workload(w, precision=api.SW_PREC_I32, striping=SWAP)
    _check(got.results, _oracle(w), "long queries swapped")


def test_mixed_batch_only_some_pairs_swap():
    # references longer than the query, or beyond 2048 residues, keep the
    # query striped (and in int16 lanes with AUTO precision); the rest swap
    rng = np.random.default_rng(4200)
    ql = rng.integers(1, 3000, size=200)
    rl = rng.integers(1, 2600, size=200)
    w = _pairs(4201, ql, rl, 20)
    want = _oracle(w)
    for prec in (api.SW_PREC_I32, api.SW_PREC_AUTO):
        got = api.align_workload(w, precision=prec, striping=SWAP)
        _check(got.results, want, "mixed prec=%d" % prec)
        plain = api.align_workload(w, precision=prec, striping=api.SW_STRIPE_QUERY)
        assert (plain.results[:, :3] == got.results[:, :3]).all()
