"""Device-planned single-query batches (the planner's validation, length
ordering and packing run on the GPU; residues are read from the references
directly): every result equals the CPU oracle exactly, through the C ABI,
and equals the host-planned path."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu
ROWS_PAIRING = api.SW_PAIRING_ROWS

# (rows per lane, lanes) of the compiled device-planned shapes
SHAPES = [(4, 16), (8, 16), (12, 16), (16, 16), (12, 32), (16, 32)]


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


def _device(w):
    import torch
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    pq = None if w.pair_query is None else t(w.pair_query, torch.int32)
    return (t(w.query_res, torch.uint8), t(w.query_off, torch.int64), t(w.ref_res, torch.uint8),
            t(w.ref_off, torch.int64), t(w.pair_ref, torch.int32)), pq


def _run(w, device=True, **kw):
    if device:
        args, pq = _device(w)
    else:
        args, pq = (w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref), w.pair_query
    return api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq, **kw)


def _one_query(seed, m, n_refs, nlen, alpha=20, matrix=None, go=11, ge=1, zero_every=0):
    """One query of length m against n_refs references of lengths U[nlen]
    (every zero_every-th reference empty), pairs in reference order."""
    rng = np.random.default_rng(seed)
    q = rng.integers(0, alpha, size=m).astype(np.uint8)
    lens = rng.integers(nlen[0], nlen[1] + 1, size=n_refs)
    if zero_every:
        lens[::zero_every] = 0
    refs = [rng.integers(0, alpha, size=int(L)).astype(np.uint8) for L in lens]
    roff = np.zeros(n_refs + 1, dtype=np.int64)
    np.cumsum(lens, out=roff[1:])
    M = matrix if matrix is not None else (W.protein_matrix() if alpha == 20 else
                                           W.random_matrix(rng, alpha))
    return W.Workload("one_query", q, np.array([0, m], dtype=np.int64),
                      np.concatenate(refs) if n_refs else np.zeros(0, np.uint8), roff, None,
                      np.arange(n_refs, dtype=np.int32), M, go, ge)


def test_protein_search_device_planned_matches_oracle_and_host_planner():
    w = W.protein_search(n_refs=6000)
    want = oracle_batch(w)
    got = _run(w, planner=2)
    assert got.stats["planner_used"] == 2
    assert_same(got.results, want, "device planner")
    rows = _run(w, planner=2, lane_pairing=api.SW_PAIRING_ROWS)
    assert_same(rows.results, want, "device planner, row pairs")
    assert rows.stats["lanes_used"] == [w.pair_ref.size, 0, 0]
    assert sum(got.stats["lanes_used"]) == w.pair_ref.size
    host = _run(w, planner=1)
    assert host.stats["planner_used"] == 1
    assert (host.results == got.results).all()
    auto = _run(w)                      # 6000 pairs, one query: the device planner
    assert auto.stats["planner_used"] == 2
    assert (auto.results == got.results).all()


def test_host_resident_inputs_device_planned():
    w = W.protein_search(n_refs=1500, seed=7)
    want = oracle_batch(w)
    got = _run(w, device=False, planner=2)
    assert got.stats["planner_used"] == 2
    assert_same(got.results, want, "host-resident")


@pytest.mark.parametrize("pairing", [api.SW_PAIRING_ALIGNMENTS, api.SW_PAIRING_ROWS])
@pytest.mark.parametrize("m", [1, 63, 64, 65, 128, 129, 192, 193, 256, 257, 384, 385, 511, 512])
def test_query_lengths_and_empty_references(m, pairing):
    w = _one_query(40 + m, m, 400, (0, 700), zero_every=7)
    want = oracle_batch(w)
    got = _run(w, planner=2, lane_pairing=pairing)
    assert_same(got.results, want, "m=%d pairing=%d" % (m, pairing))
    assert got.stats["cells"] == int(sum(m * (w.ref_off[k + 1] - w.ref_off[k])
                                         for k in range(w.pair_ref.size)))


@pytest.mark.parametrize("seg,lanes", SHAPES)
@pytest.mark.parametrize("prec", [api.SW_PREC_AUTO, api.SW_PREC_I32])
def test_forced_shapes(seg, lanes, prec):
    m = min(seg * lanes, 300)
    w = _one_query(7 * seg + lanes, m, 300, (1, 400))
    want = oracle_batch(w)
    got = _run(w, planner=2, force_lanes=lanes, force_seglen=seg, precision=prec)
    assert got.stats["seglen_max"] == seg
    assert_same(got.results, want, "seg=%d lanes=%d prec=%d" % (seg, lanes, prec))


@pytest.mark.parametrize("seg", [4, 8, 12, 16])
def test_row_pair_shapes(seg):
    """Two row segments of one alignment per lane: every compiled rows-per-lane,
    queries that fill the 32 virtual lanes exactly, leave the last ones
    empty, or end inside a lane's high half."""
    for m in sorted({32 * seg, 32 * seg - 1, 16 * seg + 1, 16 * seg, 3 * seg + 2}):
        w = _one_query(300 + 7 * seg + m, m, 250, (1, 600), zero_every=11)
        want = oracle_batch(w)
        got = _run(w, planner=2, lane_pairing=api.SW_PAIRING_ROWS, force_seglen=seg)
        assert got.stats["seglen_max"] == seg and got.stats["lanes_used"][0] > 0
        assert_same(got.results, want, "rows seg=%d m=%d" % (seg, m))


def test_row_pairs_refused_where_they_do_not_apply():
    w = _one_query(310, 200, 100, (1, 200))
    for kw in ({"precision": api.SW_PREC_I32}, {"force_lanes": 32}, {"force_seglen": 5}):
        with pytest.raises(api.SwError) as e:
            _run(w, planner=2, lane_pairing=api.SW_PAIRING_ROWS, **kw)
        assert e.value.code == api.SW_EINVAL


def test_references_longer_than_the_last_length_bin():
    # bins cover n <= 4 * 4095; longer references share the last bin
    w = _one_query(50, 100, 64, (1, 300))
    rng = np.random.default_rng(51)
    lens = np.diff(w.ref_off)
    lens[[3, 10, 40]] = [16385, 20001, 17002]
    refs = [rng.integers(0, 20, size=int(L)).astype(np.uint8) for L in lens]
    roff = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=roff[1:])
    w = W.Workload("long_refs", w.query_res, w.query_off, np.concatenate(refs), roff, None,
                   w.pair_ref, w.matrix, w.gap_open, w.gap_extend)
    want = oracle_batch(w)
    for pairing in (api.SW_PAIRING_ALIGNMENTS, api.SW_PAIRING_ROWS):
        got = _run(w, planner=2, lane_pairing=pairing)
        assert_same(got.results, want, "long references, pairing %d" % pairing)


def test_unaligned_reference_ends():
    # every reference length mod 4 and start mod 4 occurs; the last reference
    # ends exactly at the end of the residue buffer
    w = _one_query(60, 200, 257, (1, 13))
    want = oracle_batch(w)
    for pairing in (api.SW_PAIRING_ALIGNMENTS, api.SW_PAIRING_ROWS):
        assert_same(_run(w, planner=2, lane_pairing=pairing).results, want, "short refs")


@pytest.mark.parametrize("pairing", [api.SW_PAIRING_ALIGNMENTS, api.SW_PAIRING_ROWS])
def test_int16_forced_and_natural_reruns(pairing):
    w = _one_query(70, 300, 800, (10, 400))
    want = oracle_batch(w)
    got = _run(w, planner=2, int16_cap=40, lane_pairing=pairing)
    assert_same(got.results, want, "cap=40")
    assert got.stats["n_rerun"] == int((want[:, 0] >= 40).sum())
    assert ((got.results[:, 3] == api.SW_FLAG_SATURATED) == (want[:, 0] >= 40)).all()
    # a matrix whose self-alignment scores pass 32767 in 300 residues
    M = W.protein_matrix().copy()
    np.fill_diagonal(M, 120)
    w2 = _one_query(71, 300, 64, (200, 400), matrix=M)
    refs = [w2.query_res[:250], w2.query_res] + [w2.ref_res[w2.ref_off[k]:w2.ref_off[k + 1]]
                                                  for k in range(2, 64)]
    roff = np.zeros(65, dtype=np.int64)
    np.cumsum([r.size for r in refs], out=roff[1:])
    w2 = W.Workload("saturating", w2.query_res, w2.query_off, np.concatenate(refs), roff, None,
                    w2.pair_ref, M, 11, 1)
    want2 = oracle_batch(w2)
    got2 = _run(w2, planner=2, lane_pairing=pairing)
    assert_same(got2.results, want2, "natural saturation")
    assert want2[1, 0] > 32767 and got2.results[1, 3] == api.SW_FLAG_SATURATED
    assert got2.stats["n_rerun"] == int((want2[:, 0] >= 32767).sum())


def test_pair_query_and_qualification():
    w = _one_query(80, 150, 300, (1, 300))
    want = oracle_batch(w)
    pq = np.zeros(w.pair_ref.size, dtype=np.int32)
    w1 = W.Workload("pq", w.query_res, w.query_off, w.ref_res, w.ref_off, pq, w.pair_ref,
                    w.matrix, w.gap_open, w.gap_extend)
    assert_same(_run(w1, planner=2).results, want, "pair_query zeros")
    # two queries: not device-planned (forced -> SW_EINVAL; auto -> host planner)
    qres = np.concatenate([w.query_res, w.query_res[:20]])
    qoff = np.array([0, 150, 170], dtype=np.int64)
    w2 = W.Workload("two", qres, qoff, w.ref_res, w.ref_off, pq, w.pair_ref, w.matrix,
                    w.gap_open, w.gap_extend)
    with pytest.raises(api.SwError) as e:
        _run(w2, planner=2)
    assert e.value.code == api.SW_EINVAL
    got = _run(w2)
    assert got.stats["planner_used"] == 1
    assert_same(got.results, want, "two queries, all pairs on query 0")
    # a query longer than every compiled shape: host planner (chunked)
    w3 = _one_query(81, 700, 50, (1, 200))
    with pytest.raises(api.SwError):
        _run(w3, planner=2)
    assert_same(_run(w3).results, oracle_batch(w3), "m=700 host planner")


def test_invalid_inputs_rejected_on_device():
    w = _one_query(90, 100, 200, (1, 100))
    bad = w.pair_ref.copy()
    bad[17] = 200                       # reference id out of range
    wb = W.Workload("bad_id", w.query_res, w.query_off, w.ref_res, w.ref_off, None, bad,
                    w.matrix, w.gap_open, w.gap_extend)
    for device in (True, False):
        with pytest.raises(api.SwError) as e:
            _run(wb, device=device, planner=2)
        assert e.value.code == api.SW_EINVAL
    rr = w.ref_res.copy()
    rr[rr.size // 2] = 20               # residue code == alphabet size
    wr = W.Workload("bad_res", w.query_res, w.query_off, rr, w.ref_off, None, w.pair_ref,
                    w.matrix, w.gap_open, w.gap_extend)
    with pytest.raises(api.SwError) as e:
        _run(wr, planner=2)
    assert e.value.code == api.SW_EINVAL
    # the library is still usable afterwards
    assert_same(_run(w, planner=2).results, oracle_batch(w), "after errors")


@pytest.mark.parametrize("pairing", [api.SW_PAIRING_ALIGNMENTS, api.SW_PAIRING_ROWS])
def test_device_planned_graph_replays_match_eager(pairing):
    import torch
    w = W.protein_search(n_refs=5000, seed=9)
    want = oracle_batch(w)
    args, pq = _device(w)
    kw = {"planner": 2, "lane_pairing": pairing}
    eager = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, **kw)
    assert_same(eager.results, want, "eager")
    hits = 0
    for rep in range(4):
        g = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, use_graph=1, **kw)
        assert (g.results == eager.results).all(), rep
        hits += g.stats["graph_hits"]
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        again = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, **kw)
        assert (again.results == eager.results).all(), rep
    assert hits >= 3


# ---------------------------------------------------------------- one query per pair

def _per_pair(seed, n_pairs, alpha, mlen, nlen, n_queries=None, zero_every=0):
    """n_pairs pairs, each with a query drawn from n_queries (default: its own)
    of lengths U[mlen] and its own reference of length U[nlen]."""
    rng = np.random.default_rng(seed)
    nq = n_queries or n_pairs
    qlens = rng.integers(mlen[0], mlen[1] + 1, size=nq)
    rlens = rng.integers(nlen[0], nlen[1] + 1, size=n_pairs)
    if zero_every:
        qlens[::zero_every] = 0
        rlens[1::zero_every] = 0
    qoff = np.zeros(nq + 1, dtype=np.int64)
    np.cumsum(qlens, out=qoff[1:])
    roff = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(rlens, out=roff[1:])
    qres = rng.integers(0, alpha, size=int(qoff[-1])).astype(np.uint8)
    rres = rng.integers(0, alpha, size=int(roff[-1])).astype(np.uint8)
    pq = (np.arange(n_pairs) if n_queries is None else rng.integers(0, nq, size=n_pairs))
    M = W.dna_matrix() if alpha == 4 else (W.protein_matrix() if alpha == 20 else
                                           W.random_matrix(rng, alpha))
    go, ge = (6, 1) if alpha == 4 else (11, 1)
    return W.Workload("per_pair", qres, qoff, rres, roff, pq.astype(np.int32),
                      np.arange(n_pairs, dtype=np.int32), M, go, ge)


def test_dna_pairs_device_planned():
    w = W.dna_pairs(n_pairs=60000)
    want = oracle_batch(w)
    got = _run(w, planner=2)
    # 150-residue reads: 8-lane sub-groups of 19 rows per lane model less work
    assert got.stats["planner_used"] == 2 and got.stats["lanes8"] == w.n_pairs
    assert got.stats["seglen_max"] == 19
    assert_same(got.results, want, "dna pairs, device planner")
    g16 = _run(w, planner=2, force_lanes=16)
    assert g16.stats["lanes_used"][0] == w.n_pairs and g16.stats["lanes8"] == 0
    assert (g16.results == got.results).all()
    assert got.stats["cells"] == w.cells()
    auto = _run(w)
    assert auto.stats["planner_used"] == 2
    assert (auto.results == got.results).all()
    host = _run(w, planner=1)
    assert (host.results == got.results).all()
    hres = _run(w, device=False, planner=2)
    assert (hres.results == got.results).all()


@pytest.mark.parametrize("alpha,mlen", [(4, (1, 256)), (4, (140, 160)), (20, (1, 64)), (7, (30, 100))])
@pytest.mark.parametrize("prec", [api.SW_PREC_AUTO, api.SW_PREC_I32])
def test_per_pair_queries_device_planned(alpha, mlen, prec):
    w = _per_pair(500 + alpha + mlen[1], 900, alpha, mlen, (0, 700), zero_every=13)
    want = oracle_batch(w)
    got = _run(w, planner=2, precision=prec)
    assert got.stats["planner_used"] == 2
    assert_same(got.results, want, "per pair alpha=%d m=%s prec=%d" % (alpha, mlen, prec))


def test_per_pair_shared_queries_and_forced_seglen():
    # queries reused by many pairs; every compiled rows-per-lane that holds them
    w = _per_pair(520, 700, 4, (20, 64), (1, 500), n_queries=37)
    want = oracle_batch(w)
    for seg in (4, 6, 8, 10, 12, 16):
        got = _run(w, planner=2, force_seglen=seg)
        assert got.stats["seglen_max"] == seg
        assert_same(got.results, want, "seg=%d" % seg)


def test_per_pair_not_device_planned_when_queries_too_long():
    w = _per_pair(530, 300, 20, (200, 300), (1, 200))
    with pytest.raises(api.SwError) as e:
        _run(w, planner=2)
    assert e.value.code == api.SW_EINVAL
    got = _run(w)
    assert got.stats["planner_used"] == 1
    assert_same(got.results, oracle_batch(w), "host planner fallback")


def test_per_pair_reruns_and_errors():
    w = _per_pair(540, 600, 20, (10, 64), (10, 300))
    want = oracle_batch(w)
    got = _run(w, planner=2, int16_cap=30)
    assert_same(got.results, want, "cap=30")
    assert got.stats["n_rerun"] == int((want[:, 0] >= 30).sum()) > 0
    bad = w.pair_query.copy()
    bad[5] = w.query_off.size - 1          # query id out of range
    wb = W.Workload("bad_q", w.query_res, w.query_off, w.ref_res, w.ref_off, bad, w.pair_ref,
                    w.matrix, w.gap_open, w.gap_extend)
    with pytest.raises(api.SwError) as e:
        _run(wb, planner=2)
    assert e.value.code == api.SW_EINVAL
    qo = w.query_off.copy()
    qo[3], qo[4] = qo[4], qo[3]            # offsets not nondecreasing
    wo = W.Workload("bad_off", w.query_res, qo, w.ref_res, w.ref_off, w.pair_query, w.pair_ref,
                    w.matrix, w.gap_open, w.gap_extend)
    if qo[3] != qo[4]:
        with pytest.raises(api.SwError) as e:
            _run(wo, planner=2)
        assert e.value.code == api.SW_EINVAL
    assert_same(_run(w, planner=2).results, want, "after errors")


def test_per_pair_graph_replays_match_eager():
    import torch
    w = W.dna_pairs(n_pairs=8000, seed=12)
    want = oracle_batch(w)
    args, pq = _device(w)
    eager = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq, planner=2)
    assert_same(eager.results, want, "eager")
    hits = 0
    for rep in range(4):
        g = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq,
                               planner=2, use_graph=1)
        assert (g.results == eager.results).all(), rep
        hits += g.stats["graph_hits"]
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    assert hits >= 6          # two graphs per call after the first


# ---------------------------------------------------------------- eight-lane sub-groups

def _nonempty(w):
    m = np.diff(w.query_off)[w.pair_query]
    n = np.diff(w.ref_off)[w.pair_ref]
    return int(((m > 0) & (n > 0)).sum())


@pytest.mark.parametrize("seg", [8, 10, 13, 16, 19])
@pytest.mark.parametrize("alpha", [4, 7])
def test_eight_lane_sub_groups_every_seglen(seg, alpha):
    """Sixteen alignments per wavefront, queries up to 8*seg residues (some
    empty), references of every length mod 4 (some empty)."""
    w = _per_pair(900 + seg + alpha, 700, alpha, (1, 8 * seg), (0, 400), zero_every=11)
    want = oracle_batch(w)
    got = _run(w, planner=2, force_lanes=8, force_seglen=seg)
    # pairs with an empty side never reach the kernel
    assert got.stats["lanes8"] == _nonempty(w) and got.stats["seglen_max"] == seg
    assert_same(got.results, want, "8 lanes seg=%d alpha=%d" % (seg, alpha))


def test_eight_lane_sub_groups_protein_and_chosen_shape():
    # 20 letters: the byte profile of 8 rows per lane fits the LDS budget
    w = _per_pair(930, 500, 20, (1, 64), (1, 300), zero_every=9)
    want = oracle_batch(w)
    got = _run(w, planner=2, force_lanes=8)
    assert got.stats["lanes8"] == _nonempty(w) and got.stats["seglen_max"] == 8
    assert_same(got.results, want, "8 lanes protein")
    # unforced: short DNA queries go to eight-lane sub-groups
    w4 = _per_pair(931, 900, 4, (100, 150), (100, 600))
    auto = _run(w4, planner=2)
    assert auto.stats["lanes8"] == w4.n_pairs
    assert_same(auto.results, oracle_batch(w4), "auto")


def test_byte_and_16_bit_profiles_agree():
    """Scores within int8 use byte profile entries (16-lane and 8-lane
    sub-groups); a matrix entry outside int8 keeps 16-bit entries and refuses
    8 lanes."""
    w = _per_pair(940, 600, 4, (1, 150), (1, 500), zero_every=7)
    M2 = w.matrix.copy()
    M2[0, 0] = 200                        # outside int8
    w2 = W.Workload("wide", w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_query,
                    w.pair_ref, M2, w.gap_open, w.gap_extend)
    for ww in (w, w2):
        want = oracle_batch(ww)
        got = _run(ww, planner=2, force_lanes=16)
        assert_same(got.results, want, "16 lanes M00=%d" % ww.matrix[0, 0])
    with pytest.raises(api.SwError) as e:
        _run(w2, planner=2, force_lanes=8)
    assert e.value.code == api.SW_EINVAL
    auto2 = _run(w2, planner=2)
    assert auto2.stats["lanes8"] == 0
    assert_same(auto2.results, oracle_batch(w2), "auto, wide matrix")


def test_eight_lane_reruns_and_refusals():
    w = _per_pair(950, 600, 4, (20, 150), (10, 500))
    want = oracle_batch(w)
    # random DNA pairs score about 6: a cap of 7 sends a good share to int32
    got = _run(w, planner=2, force_lanes=8, int16_cap=7)
    assert_same(got.results, want, "cap=7")
    assert got.stats["n_rerun"] == int((want[:, 0] >= 7).sum()) > 0
    # int32 lanes, queries longer than 152 residues, one query, host planner
    with pytest.raises(api.SwError):
        _run(w, planner=2, force_lanes=8, precision=api.SW_PREC_I32)
    wl = _per_pair(951, 100, 4, (150, 200), (10, 100))
    with pytest.raises(api.SwError):
        _run(wl, planner=2, force_lanes=8)
    w1 = _one_query(952, 100, 300, (1, 200), alpha=4, matrix=W.dna_matrix(), go=6, ge=1)
    with pytest.raises(api.SwError):
        _run(w1, planner=2, force_lanes=8)
    with pytest.raises(api.SwError):
        _run(w, planner=1, force_lanes=8)


def test_eight_lane_graph_replays_match_eager():
    import torch
    w = _per_pair(960, 5000, 4, (140, 152), (300, 600))
    want = oracle_batch(w)
    args, pq = _device(w)
    eager = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq,
                               planner=2, force_lanes=8)
    assert_same(eager.results, want, "eager")
    for rep in range(3):
        g = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq,
                               planner=2, force_lanes=8, use_graph=1)
        assert (g.results == eager.results).all(), rep
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()


# ---------------------------------------------------------------- gap-to-gap regression family

def _bridge_pairs(shifts=range(0, 48, 5)):
    """q = X^s A^12 X^k B^12, r = Y^s A^12 Y^k B^12 (X, Y never match anything):
    for k = 11, 12, 16 the best alignment bridges the middle with a gap in
    each sequence back to back, so a vertical gap followed directly by a
    horizontal one decides the score; the prefix s moves the bridge across
    lane and chunk boundaries."""
    M = np.full((4, 4), -4, dtype=np.int32)
    M[0, 0] = M[1, 1] = 5
    qs, rs = [], []
    for k in (11, 12, 16):
        for s in shifts:
            qs.append(np.array([2] * s + [0] * 12 + [2] * k + [1] * 12, dtype=np.uint8))
            rs.append(np.array([3] * s + [0] * 12 + [3] * k + [1] * 12, dtype=np.uint8))
    qoff = np.zeros(len(qs) + 1, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    roff = np.zeros(len(rs) + 1, dtype=np.int64)
    np.cumsum([r.size for r in rs], out=roff[1:])
    idx = np.arange(len(qs), dtype=np.int32)
    return W.Workload("bridge", np.concatenate(qs), qoff, np.concatenate(rs), roff, idx, idx.copy(),
                      M, 11, 1)


@pytest.mark.parametrize("kw", [
    dict(planner=1, force_kernel=2, force_lanes=16, force_seglen=4),
    dict(planner=1, force_kernel=2, force_lanes=32, force_seglen=4),
    dict(planner=1, force_kernel=2, force_lanes=64, force_seglen=4),
    dict(planner=1, force_kernel=2, force_lanes=16, force_seglen=8),
    dict(planner=1, force_kernel=2, force_lanes=64, force_seglen=8, precision=api.SW_PREC_I32),
    dict(planner=1, force_kernel=2, lane_pairing=ROWS_PAIRING, force_seglen=4),
    dict(planner=1, force_kernel=2, lane_pairing=ROWS_PAIRING, force_seglen=8),
    # device-planned per-pair launches hold the longest query (85) in one chunk
    dict(planner=2, force_lanes=8, force_seglen=13),
    dict(planner=2, force_lanes=8, force_seglen=16),
    dict(planner=2, force_lanes=16, force_seglen=6),
    dict(planner=2, force_lanes=16, force_seglen=8),
    dict(planner=1, algorithm=api.SW_ALG_LAZYF, force_lanes=16, force_seglen=4),
], ids=lambda kw: "-".join("%s%s" % (k[:6], v) for k, v in kw.items()))
def test_gap_to_gap_family_every_layout(kw):
    w = _bridge_pairs()
    want = oracle_batch(w)
    # the bridge beats the ungapped score for every k (78 vs 76, 76 vs 72, 68 vs 60)
    assert set(np.unique(want[:, 0])) == {78, 76, 68}
    got = _run(w, **kw)
    assert_same(got.results, want, "bridge %s" % kw)


def test_gap_to_gap_family_shared_query():
    """One query, the references of the family: row pairs and direct shapes
    of the device-planned shared-query kernel."""
    M = np.full((4, 4), -4, dtype=np.int32)
    M[0, 0] = M[1, 1] = 5
    for s in (0, 9, 17, 40):
        q = np.array([2] * s + [0] * 12 + [2] * 12 + [1] * 12, dtype=np.uint8)
        refs = [np.array([3] * t + [0] * 12 + [3] * k + [1] * 12, dtype=np.uint8)
                for k in (11, 12, 16) for t in range(0, 30, 3)]
        roff = np.zeros(len(refs) + 1, dtype=np.int64)
        np.cumsum([r.size for r in refs], out=roff[1:])
        w = W.Workload("bridge1", q, np.array([0, q.size], np.int64), np.concatenate(refs), roff,
                       None, np.arange(len(refs), dtype=np.int32), M, 11, 1)
        want = oracle_batch(w)
        for kw in (dict(lane_pairing=ROWS_PAIRING, force_seglen=4),
                   dict(lane_pairing=api.SW_PAIRING_ALIGNMENTS, force_lanes=16, force_seglen=8),
                   dict(lane_pairing=api.SW_PAIRING_ALIGNMENTS, force_lanes=32, force_seglen=12)):
            got = _run(w, planner=2, **kw)
            assert_same(got.results, want, "bridge shared s=%d %s" % (s, kw))


def test_results_into_caller_buffers():
    """out= takes a caller's (n_pairs, 4) int32 array, pinned or pageable, and
    the results are those of a fresh array, graph replays included."""
    import torch
    w = W.dna_pairs(n_pairs=5000, seed=31)
    want = _run(w)
    pinned = torch.empty((w.n_pairs, 4), dtype=torch.int32, pin_memory=True).numpy()
    pinned.fill(-7)
    for graph in (0, 1, 1):
        got = _run(w, out=pinned, use_graph=graph)
        assert np.shares_memory(got.results, pinned)
        assert (pinned == want.results).all()
        pinned.fill(-7)
    plain = np.full((w.n_pairs, 4), -7, dtype=np.int32)
    assert (_run(w, out=plain).results == want.results).all()
    with pytest.raises(ValueError):
        _run(w, out=np.zeros((w.n_pairs, 3), dtype=np.int32))
