"""Per-pair launches in the row-pair layout (host planner): one alignment per
16-lane sub-group, the two int16 halves of a lane holding two row segments of
it, scores from the pair-score table instead of per-pair profiles.  Every
result equals the CPU oracle exactly, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu
ROWS = api.SW_PAIRING_ROWS


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    api.load()          # raises if the HIP library is missing: no fallback
    api.sw_init()


def oracle_batch(w):
    return oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                              w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query)


def assert_same(got, want, label=""):
    got3 = np.asarray(got)[:, :3]
    bad = np.nonzero((got3 != want).any(axis=1))[0]
    if bad.size:
        k = int(bad[0])
        raise AssertionError("%s: %d/%d mismatches; first pair %d got %s want %s" %
                             (label, bad.size, len(want), k, got3[k].tolist(), want[k].tolist()))


def _pairs(seed, n, alpha, mlen, nlen, matrix=None, go=11, ge=1, zero_every=0):
    rng = np.random.default_rng(seed)
    M = matrix if matrix is not None else (W.protein_matrix() if alpha == 20 else
                                           W.random_matrix(rng, alpha))
    w = W.random_pairs(n, alpha, mlen, nlen, seed, matrix=M, gap_open=go, gap_extend=ge)
    if zero_every:
        # empty queries and references in between
        ql, rl = np.diff(w.query_off), np.diff(w.ref_off)
        qs = [w.query_res[w.query_off[k]:w.query_off[k + 1]] for k in range(ql.size)]
        rs = [w.ref_res[w.ref_off[k]:w.ref_off[k + 1]] for k in range(rl.size)]
        for k in range(0, len(qs), zero_every):
            qs[k] = qs[k][:0]
        for k in range(1, len(rs), zero_every):
            rs[k] = rs[k][:0]
        qoff = np.zeros(len(qs) + 1, dtype=np.int64)
        np.cumsum([q.size for q in qs], out=qoff[1:])
        roff = np.zeros(len(rs) + 1, dtype=np.int64)
        np.cumsum([r.size for r in rs], out=roff[1:])
        w = W.Workload("zeros", np.concatenate(qs), qoff, np.concatenate(rs), roff, w.pair_query,
                       w.pair_ref, M, go, ge)
    return w


@pytest.mark.parametrize("seg", [4, 8, 12, 16])
def test_row_pairs_every_seglen_with_chunks(seg):
    """Queries up to 1500 residues: one to twelve query chunks of 32*seg rows."""
    w = _pairs(700 + seg, 500, 20, (1, 1500), (1, 400), zero_every=17)
    want = oracle_batch(w)
    got = api.align_workload(w, planner=1, force_kernel=2, lane_pairing=ROWS, force_seglen=seg)
    assert got.stats["row_pairs"] > 0 and got.stats["seglen_max"] == seg
    assert_same(got.results, want, "rows seg=%d" % seg)


@pytest.mark.parametrize("lanes", [32, 64])
@pytest.mark.parametrize("seg", [4, 12, 16])
def test_row_pairs_wide_sub_groups(lanes, seg):
    """32 or 64 lanes per alignment (64 or 128 virtual lanes): the scan's
    row broadcasts and the wave-wide virtual-lane moves, one to several chunks."""
    w = _pairs(710 + lanes + seg, 300, 20, (1, 5000), (1, 300), zero_every=13)
    want = oracle_batch(w)
    got = api.align_workload(w, planner=1, force_kernel=2, lane_pairing=ROWS, force_lanes=lanes,
                             force_seglen=seg)
    assert got.stats["row_pairs"] > 0
    assert_same(got.results, want, "rows lanes=%d seg=%d" % (lanes, seg))


@pytest.mark.parametrize("alpha", [2, 4, 7, 24])
def test_row_pairs_alphabets(alpha):
    w = _pairs(720 + alpha, 400, alpha, (1, 700), (1, 500))
    want = oracle_batch(w)
    got = api.align_workload(w, planner=1, force_kernel=2, lane_pairing=ROWS)
    assert got.stats["row_pairs"] > 0
    assert_same(got.results, want, "rows alpha=%d" % alpha)


def test_row_pairs_chosen_by_the_cost_model_for_protein():
    # 20-letter queries of a few hundred residues: the per-pair profile would
    # allow only 4 rows per lane, so row pairs model less work (in a batch this
    # small the longest queries may still take 64 alignment-pair lanes, whose
    # chain of column steps is shorter)
    w = _pairs(730, 600, 20, (200, 900), (50, 500))
    want = oracle_batch(w)
    got = api.align_workload(w, planner=1, force_kernel=2)
    assert got.stats["row_pairs"] >= w.n_pairs // 2
    assert_same(got.results, want, "auto")
    al = api.align_workload(w, planner=1, force_kernel=2, lane_pairing=api.SW_PAIRING_ALIGNMENTS)
    assert al.stats["row_pairs"] == 0
    assert (al.results == got.results).all()


def test_row_pairs_reruns():
    w = _pairs(740, 400, 20, (10, 900), (10, 300))
    want = oracle_batch(w)
    got = api.align_workload(w, planner=1, force_kernel=2, lane_pairing=ROWS, int16_cap=50)
    assert_same(got.results, want, "cap=50")
    assert got.stats["n_rerun"] == int((want[:, 0] >= 50).sum()) > 0
    # natural saturation: a large diagonal and long self-similar pairs
    M = W.protein_matrix().copy()
    np.fill_diagonal(M, 100)
    rng = np.random.default_rng(741)
    q = rng.integers(0, 20, size=700).astype(np.uint8)
    qres = np.concatenate([q, q[:200]])
    qoff = np.array([0, 700, 900], dtype=np.int64)
    w2 = W.Workload("sat", qres, qoff, qres, qoff, np.array([0, 1, 0], np.int32),
                    np.array([0, 1, 1], np.int32), M, 11, 1)
    want2 = oracle_batch(w2)
    got2 = api.align_workload(w2, planner=1, force_kernel=2, lane_pairing=ROWS)
    assert_same(got2.results, want2, "natural saturation")
    assert want2[0, 0] > 32767 and got2.results[0, 3] == api.SW_FLAG_SATURATED


def test_row_pairs_refused_where_they_do_not_apply():
    w = _pairs(750, 50, 20, (1, 100), (1, 100))
    for kw in ({"precision": api.SW_PREC_I32}, {"force_seglen": 6}):
        with pytest.raises(api.SwError) as e:
            api.align_workload(w, planner=1, force_kernel=2, lane_pairing=ROWS, **kw)
        assert e.value.code == api.SW_EINVAL
    w25 = _pairs(751, 50, 25, (1, 100), (1, 100))
    with pytest.raises(api.SwError):
        api.align_workload(w25, planner=1, force_kernel=2, lane_pairing=ROWS)
    got = api.align_workload(w25, planner=1, force_kernel=2)      # alignment pairs
    assert got.stats["row_pairs"] == 0
    assert_same(got.results, oracle_batch(w25), "alpha=25")


def test_row_pairs_graph_replays_match_eager():
    import torch
    w = _pairs(760, 300, 20, (100, 1200), (20, 300))
    want = oracle_batch(w)
    kw = dict(planner=1, force_kernel=2, lane_pairing=ROWS)
    eager = api.align_workload(w, **kw)
    assert_same(eager.results, want, "eager")
    hits = 0
    for rep in range(4):
        g = api.align_workload(w, use_graph=1, **kw)
        assert (g.results == eager.results).all(), rep
        hits += g.stats["graph_hits"]
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    assert hits >= 3
