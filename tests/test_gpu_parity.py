"""GPU parity: every result of the HIP path must equal the CPU oracle exactly
(score, query_end, ref_end), on the same seeded inputs, through the C ABI."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    api.load()          # raises if the HIP library is missing: no fallback
    api.sw_init()


def oracle_batch(w):
    return oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                              w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query)


def assert_same(got, want, w=None, label=""):
    got3 = np.asarray(got)[:, :3]
    bad = np.nonzero((got3 != want).any(axis=1))[0]
    if bad.size:
        k = int(bad[0])
        extra = ""
        if w is not None:
            q, r = w.pair(k)
            extra = " m=%d n=%d" % (q.size, r.size)
        raise AssertionError("%s: %d/%d mismatches; first pair %d got %s want %s%s" %
                             (label, bad.size, len(want), k, got3[k].tolist(),
                              want[k].tolist(), extra))


# ---------------------------------------------------------------- plain kernel

def test_worked_example_plain():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    code = {c: k for k, c in enumerate(g["alphabet"])}
    M = np.full((4, 4), g["mismatch"], dtype=np.int32)
    np.fill_diagonal(M, g["match"])
    q = [code[c] for c in g["query"]]
    r = [code[c] for c in g["ref"]]
    s, qe, re_, fl = api.sw_align(q, r, M, g["gap_open"], g["gap_extend"])
    assert (s, qe, re_) == (g["result"]["score"], g["result"]["query_end"], g["result"]["ref_end"])
    s, qe, re_, fl = api.sw_align(r, q, M, g["gap_open"], g["gap_extend"])
    sw = g["swapped_result"]
    assert (s, qe, re_) == (sw["score"], sw["query_end"], sw["ref_end"])


def test_single_pair_workload_plain():
    w = W.single_pair()
    q, r = w.pair(0)
    got = api.sw_align(q, r, w.matrix, w.gap_open, w.gap_extend)
    assert got[:3] == oracle.align(q, r, w.matrix, w.gap_open, w.gap_extend)


@pytest.mark.parametrize("m", [1, 2, 15, 16, 17, 63, 64, 65, 127, 200, 511, 512, 513, 1100])
def test_plain_query_lengths(m):
    rng = np.random.default_rng(100 + m)
    M = W.protein_matrix()
    for n in (1, 3, 4, 5, 77, 300):
        q = rng.integers(0, 20, size=m)
        r = rng.integers(0, 20, size=n)
        got = api.sw_align(q, r, M, 11, 1)
        assert got[:3] == oracle.align(q, r, M, 11, 1), (m, n)


def test_plain_edge_cases():
    M = W.protein_matrix()
    assert api.sw_align([], [1, 2], M, 11, 1)[:3] == (0, -1, -1)
    neg = -np.ones((20, 20), dtype=np.int32)
    q = np.arange(20)
    assert api.sw_align(q, q, neg, 3, 1)[:3] == (0, -1, -1)
    # self alignment of a long query with every residue matching
    q = np.random.default_rng(3).integers(0, 20, size=700)
    d = np.diag(M)
    assert api.sw_align(q, q, M, 11, 1)[:3] == (int(d[q].sum()), 699, 699)


def test_double_gap_bridge_plain():
    M = np.full((4, 4), -4, dtype=np.int32)
    M[0, 0] = M[1, 1] = 5
    for k in (11, 12, 16):
        q = [0] * 12 + [2] * k + [1] * 12
        r = [0] * 12 + [3] * k + [1] * 12
        assert api.sw_align(q, r, M, 11, 1)[:3] == oracle.align(q, r, M, 11, 1)


def test_gap_extend_above_gap_open_is_clamped():
    rng = np.random.default_rng(9)
    M = W.protein_matrix()
    for _ in range(20):
        q = rng.integers(0, 20, size=int(rng.integers(1, 90)))
        r = rng.integers(0, 20, size=int(rng.integers(1, 90)))
        go = int(rng.integers(0, 6))
        ge = go + int(rng.integers(1, 5))
        assert api.sw_align(q, r, M, go, ge)[:3] == oracle.align(q, r, M, go, ge)


# ---------------------------------------------------------------- batched kernels

def _random_batch(seed, n, alpha, mlen, nlen, go=11, ge=1):
    rng = np.random.default_rng(seed)
    M = W.protein_matrix() if alpha == 20 else W.random_matrix(rng, alpha, symmetric=False)
    return W.random_pairs(n, alpha, mlen, nlen, seed, matrix=M, gap_open=go, gap_extend=ge)


@pytest.mark.parametrize("kernel,layout", [(1, 0), (2, 0), (2, 2)])
@pytest.mark.parametrize("prec", [api.SW_PREC_AUTO, api.SW_PREC_I32])
def test_batch_random_pairs(kernel, layout, prec):
    w = _random_batch(7, 600, 20, (1, 260), (1, 400))
    want = oracle_batch(w)
    got = api.align_workload(w, force_kernel=kernel, precision=prec, mixed_layout=layout)
    assert_same(got.results, want, w, "kernel=%d layout=%d prec=%d" % (kernel, layout, prec))


def test_per_pair_long_queries_many_chunk_counts():
    """One chunked per-pair launch holds tasks of different chunk counts; with
    one width per launch the launches run concurrently on side streams."""
    w = _random_batch(14, 160, 4, (100, 4000), (50, 400), go=6, ge=1)
    want = oracle_batch(w)
    for layout in (0, 2):
        got = api.align_workload(w, force_kernel=2, mixed_layout=layout)
        assert_same(got.results, want, w, "layout=%d" % layout)


@pytest.mark.parametrize("lanes", [16, 32, 64])
@pytest.mark.parametrize("kernel", [1, 2])
def test_batch_forced_lanes(lanes, kernel):
    w = _random_batch(8, 300, 4, (1, 200), (1, 300), go=6, ge=1)
    want = oracle_batch(w)
    got = api.align_workload(w, force_kernel=kernel, force_lanes=lanes)
    assert_same(got.results, want, w, "lanes=%d kernel=%d" % (lanes, kernel))


@pytest.mark.parametrize("lanes,seg", [(16, 4), (32, 4), (64, 4), (16, 8), (64, 8), (32, 12)])
def test_batch_chunked_queries(lanes, seg):
    """Queries longer than lanes*seglen rows run as chunks with boundary carries."""
    w = _random_batch(9, 96, 20, (50, 1500), (20, 300))
    want = oracle_batch(w)
    for kernel in (1, 2):
        got = api.align_workload(w, force_kernel=kernel, force_lanes=lanes, force_seglen=seg)
        assert_same(got.results, want, w, "kernel=%d lanes=%d seg=%d" % (kernel, lanes, seg))


def test_int16_saturation_rerun():
    rng = np.random.default_rng(11)
    M = W.protein_matrix()
    # natural saturation: a 4200-residue self alignment over the letters with
    # diagonal score >= 10 scores above 42000 > 32767
    rich = np.nonzero(np.diag(M) >= 10)[0]
    q = rng.choice(rich, size=4200).astype(np.uint8)
    qs = [q, q[:3300], rng.integers(0, 20, size=300).astype(np.uint8)]
    qres = np.concatenate(qs)
    qoff = np.array([0, 4200, 7500, 7800], dtype=np.int64)
    pq = np.array([0, 1, 2, 0], dtype=np.int32)
    pr = np.array([0, 1, 2, 2], dtype=np.int32)
    got = api.sw_align_batch(qres, qoff, qres, qoff, pr, M, 11, 1, pair_query=pq)
    for k in range(4):
        qq = qres[qoff[pq[k]]:qoff[pq[k] + 1]]
        rr = qres[qoff[pr[k]]:qoff[pr[k] + 1]]
        assert tuple(got.results[k, :3]) == oracle.align(qq, rr, M, 11, 1)
    assert got.results[0, 3] == api.SW_FLAG_SATURATED and got.results[0, 0] > 32767
    assert got.stats["n_rerun"] >= 2


def test_int16_forced_rerun_cap():
    w = _random_batch(12, 400, 20, (10, 200), (10, 300))
    want = oracle_batch(w)
    got = api.align_workload(w, int16_cap=40)
    assert_same(got.results, want, w, "cap=40")
    assert got.stats["n_rerun"] == int((want[:, 0] >= 40).sum())
    assert ((got.results[:, 3] == 1) == (want[:, 0] >= 40)).all()


def test_protein_search_subset():
    w = W.protein_search(n_refs=3000)
    want = oracle_batch(w)
    got = api.align_workload(w)
    assert_same(got.results, want, w, "protein_search")


def test_dna_pairs_subset():
    # 60k pairs: large enough for the planner's multi-threaded sort and packing
    w = W.dna_pairs(n_pairs=60000)
    want = oracle_batch(w)
    got = api.align_workload(w)
    assert_same(got.results, want, w, "dna_pairs")


def test_long_queries_subset_scan_and_lazyf():
    w = W.long_queries(n_queries=4, n_refs=40, qlen=(1500, 3000), rlen=(50, 300))
    want = oracle_batch(w)
    got = api.align_workload(w, precision=api.SW_PREC_I32)
    assert_same(got.results, want, w, "scan")
    lz = api.align_workload(w, precision=api.SW_PREC_I32, algorithm=api.SW_ALG_LAZYF)
    assert_same(lz.results, want, w, "lazyf")
    assert lz.stats["lazyf_steps"] > 0


def test_batch_empty_and_degenerate_pairs():
    M = W.protein_matrix()
    qres = np.array([1, 2, 3, 4, 5], dtype=np.uint8)
    qoff = np.array([0, 0, 5], dtype=np.int64)
    pq = np.array([0, 1, 1], dtype=np.int32)
    pr = np.array([1, 0, 1], dtype=np.int32)
    got = api.sw_align_batch(qres, qoff, qres, qoff, pr, M, 11, 1, pair_query=pq)
    assert got.results[:, :3].tolist() == [[0, -1, -1], [0, -1, -1],
                                          list(oracle.align(qres, qres, M, 11, 1))]


def test_batch_invalid_residue_rejected():
    M = np.eye(4, dtype=np.int32)
    qres = np.array([0, 1, 7], dtype=np.uint8)
    qoff = np.array([0, 3], dtype=np.int64)
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch(qres, qoff, qres, qoff, np.zeros(1, np.int32), M, 2, 1)
    assert e.value.code == api.SW_EINVAL


@pytest.mark.parametrize("shift", [0, 3, 16])
def test_invalid_residue_found_anywhere_in_device_arrays(shift):
    # the residue check reads 16 bytes at a time between the first and last
    # 16-byte boundaries of an array and single bytes outside them: a bad code
    # in the first, last or a middle byte of a reference set that starts off
    # a boundary (and in a query set of 1-40 bytes) is rejected; none is
    # reported without one
    import torch
    dev = torch.device("cuda")
    rng = np.random.default_rng(120 + shift)
    M = np.eye(4, dtype=np.int32)
    n = 5003
    base = rng.integers(0, 4, size=n + shift, dtype=np.uint8)
    q = torch.from_numpy(rng.integers(0, 4, size=40, dtype=np.uint8)).to(dev)
    qoff = torch.tensor([0, 40], dtype=torch.int64, device=dev)
    roff = torch.tensor([0, n], dtype=torch.int64, device=dev)
    pr = torch.zeros(1, dtype=torch.int32, device=dev)

    def run(refs, query=q, query_off=qoff):
        r = torch.from_numpy(refs).to(dev)[shift:]
        return api.sw_align_batch(query, query_off, r, roff, pr, M, 2, 1)

    got = run(base).results
    assert tuple(int(x) for x in got[0, :3]) == \
        oracle.align(q.cpu().numpy(), base[shift:], M, 2, 1)
    for pos in (0, 1, 12, 13, 15, 16, 17, n // 2, n - 17, n - 16, n - 15, n - 2, n - 1):
        bad = base.copy()
        bad[shift + pos] = 4 + pos % 200
        with pytest.raises(api.SwError) as e:
            run(bad)
        assert e.value.code == api.SW_EINVAL, pos
    for m in (1, 15, 16, 17, 40):
        for pos in (0, m - 1):
            qs = rng.integers(0, 4, size=m + shift, dtype=np.uint8)
            qs[shift + pos] = 255
            qd = torch.from_numpy(qs).to(dev)[shift:]
            with pytest.raises(api.SwError) as e:
                run(base, qd, torch.tensor([0, m], dtype=torch.int64, device=dev))
            assert e.value.code == api.SW_EINVAL, (m, pos)


def test_device_resident_inputs_match_host():
    import torch
    w = _random_batch(13, 200, 20, (1, 300), (1, 300))
    want = oracle_batch(w)
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    got = api.sw_align_batch(t(w.query_res, torch.uint8), t(w.query_off, torch.int64),
                             t(w.ref_res, torch.uint8), t(w.ref_off, torch.int64),
                             t(w.pair_ref, torch.int32), w.matrix, w.gap_open, w.gap_extend,
                             pair_query=t(w.pair_query, torch.int32))
    assert_same(got.results, want, w, "device-resident")


# ---------------------------------------------------------------- mixed layouts, graphs

@pytest.mark.parametrize("prec", [api.SW_PREC_AUTO, api.SW_PREC_I32])
@pytest.mark.parametrize("seg", [0, 4, 6])
def test_mixed_layouts(prec, seg):
    """16-, 32- and 64-lane sub-groups of one wavefront (one rows-per-lane per
    launch, each pair on the narrowest sub-group holding its query)."""
    w = _random_batch(21 + seg, 500, 20, (1, 900), (1, 300))
    want = oracle_batch(w)
    got = api.align_workload(w, force_kernel=2, mixed_layout=1, precision=prec,
                             force_seglen=seg)
    assert_same(got.results, want, w, "mixed prec=%d seg=%d" % (prec, seg))
    assert sum(1 for v in got.stats["lanes_used"] if v > 0) >= 2


def test_mixed_layouts_dna_with_rerun():
    w = W.dna_pairs(n_pairs=3000)
    # vary the query lengths: cut every query at a seeded length in [1, 150]
    rng = np.random.default_rng(22)
    cut = rng.integers(1, 151, size=w.pair_query.size)
    qs = [w.query_res[w.query_off[k]:w.query_off[k] + c] for k, c in enumerate(cut)]
    qoff = np.zeros(len(qs) + 1, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    w2 = W.Workload("dna_cut", np.concatenate(qs), qoff, w.ref_res, w.ref_off, w.pair_query,
                    w.pair_ref, w.matrix, w.gap_open, w.gap_extend)
    want = oracle_batch(w2)
    got = api.align_workload(w2, force_kernel=2, mixed_layout=1, int16_cap=60)
    assert_same(got.results, want, w2, "mixed dna cap=60")
    assert got.stats["n_rerun"] == int((want[:, 0] >= 60).sum())


@pytest.mark.parametrize("case", ["shared", "pair", "chunked", "rerun"])
def test_graph_replays_match_eager(case):
    """Captured graphs replayed several times, with eager calls and other
    device work in between, give the eager result every time."""
    import torch
    if case == "shared":
        w, kw = W.protein_search(n_refs=2000), {}
    elif case == "pair":
        w, kw = _random_batch(31, 400, 4, (1, 300), (1, 300), go=6, ge=1), {"force_kernel": 2}
    elif case == "chunked":
        w, kw = _random_batch(32, 64, 20, (300, 1500), (20, 300)), {"force_lanes": 32,
                                                                     "force_seglen": 4}
    else:
        w, kw = _random_batch(33, 300, 20, (10, 200), (10, 300)), {"int16_cap": 40}
    want = oracle_batch(w)
    eager = api.align_workload(w, **kw)
    assert_same(eager.results, want, w, case + " eager")
    hits = 0
    for rep in range(4):
        g = api.align_workload(w, use_graph=1, **kw)
        assert (g.results == eager.results).all(), (case, rep)
        hits += g.stats["graph_hits"]
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        again = api.align_workload(w, **kw)
        assert (again.results == eager.results).all(), (case, rep)
    assert hits >= 3
