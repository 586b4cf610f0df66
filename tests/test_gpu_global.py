"""End-to-end scores (sw_align_batch_global) and paths
(sw_align_batch_global_cigar) in every mode -- global, semi-global with the
query fitted (reference ends free) or the reference fitted (query ends free),
overlap (free end gaps) -- equal the CPU oracle's exactly through the C ABI:
score, end cell (the mode's tie rule), start element and runs."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu
MODES = [api.SW_MODE_GLOBAL, api.SW_MODE_SEMIGLOBAL, api.SW_MODE_SEMIGLOBAL_REF,
         api.SW_MODE_OVERLAP]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.build(force=False)
    api.load()          # raises if the HIP library is missing: no fallback
    api.sw_init()


def _run(w, mode, **kw):
    return api.sw_align_batch_global(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                                     w.matrix, w.gap_open, w.gap_extend, mode=mode,
                                     pair_query=w.pair_query, **kw)


def _check(w, mode, label, pairs=None):
    got = _run(w, mode)
    idx = list(range(w.n_pairs)) if pairs is None else list(pairs)
    want = oracle.endtoend_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                                 w.matrix, w.gap_open, w.gap_extend, mode,
                                 pair_query=w.pair_query, pairs=idx)
    g = got[idx, :3].astype(np.int64)
    bad = np.nonzero((g != want).any(axis=1))[0]
    if bad.size:
        k = int(bad[0])
        raise AssertionError("%s mode %d: %d/%d mismatches; first pair %d got %s want %s" %
                             (label, mode, bad.size, len(idx), idx[k], g[k].tolist(),
                              want[k].tolist()))
    assert (got[:, 3] == 0).all()
    return got


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("alpha,go,ge", [(2, 2, 1), (4, 3, 1), (20, 11, 1), (3, 1, 0),
                                         (4, 2, 5), (4, 0, 0)])
def test_small_pairs_equal_the_oracle(mode, alpha, go, ge):
    # empty sides, one residue, ragged lengths; (2, 5): extension above opening
    rng = np.random.default_rng(970 + alpha + go + 7 * mode)
    M = W.protein_matrix() if alpha == 20 else W.random_matrix(rng, alpha)
    w = W.random_pairs(500, alpha, (0, 60), (0, 70), 971 + alpha + mode, matrix=M,
                       gap_open=go, gap_extend=ge)
    _check(w, mode, "small")


@pytest.mark.parametrize("mode", MODES)
def test_every_column_count(mode):
    # queries of 1-256 residues: 1, 2, 3 and 4 columns per lane, ragged ends
    rng = np.random.default_rng(985 + mode)
    w = W.random_pairs(300, 4, (1, 256), (1, 120), 986 + mode, matrix=W.random_matrix(rng, 4),
                       gap_open=2, gap_extend=1)
    ms = np.diff(w.query_off)
    # up to 160 residues two pairs share a wavefront, 32 lanes each (1-5
    # columns per lane); 161-256 run on 64 lanes (3 or 4 columns per lane)
    assert {int((m + 31) // 32) for m in ms if m <= 160} == {1, 2, 3, 4, 5}
    assert {int((m + 63) // 64) for m in ms if 160 < m <= 256} == {3, 4}
    _check(w, mode, "columns")


@pytest.mark.parametrize("mode", MODES)
def test_dual_pairs_odd_count_uneven_neighbours(mode):
    # an odd number of short-query pairs (the last wavefront holds one pair)
    # whose neighbours in the batch differ greatly in reference length and
    # in columns per lane, so the two halves of a wavefront end far apart
    rng = np.random.default_rng(1990 + mode)
    M = W.random_matrix(rng, 4)
    qs, rs = [], []
    for k in range(41):
        m = int(rng.integers(1, 161)) if k % 3 else int(rng.integers(129, 161))
        n = int(rng.integers(1, 8)) if k % 2 else int(rng.integers(900, 1400))
        qs.append(rng.integers(0, 4, size=m, dtype=np.uint8))
        rs.append(rng.integers(0, 4, size=n, dtype=np.uint8))
    qres = np.concatenate(qs)
    rres = np.concatenate(rs)
    qoff = np.zeros(42, dtype=np.int64)
    roff = np.zeros(42, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    np.cumsum([r.size for r in rs], out=roff[1:])
    idx = np.arange(41, dtype=np.int32)
    w = W.Workload("dual_odd", qres, qoff, rres, roff, idx, idx.copy(), M, 3, 1, {})
    assert w.n_pairs % 2 == 1 and (np.diff(qoff) <= 160).all()
    assert {int((m + 31) // 32) for m in np.diff(qoff)} == {1, 2, 3, 4, 5}
    _check(w, mode, "dual-odd")


def _pairs_of(qlens, rlens, seed, alpha=4, go=3, ge=1):
    rng = np.random.default_rng(seed)
    M = W.random_matrix(rng, alpha)
    qs = [rng.integers(0, alpha, size=int(m), dtype=np.uint8) for m in qlens]
    rs = [rng.integers(0, alpha, size=int(n), dtype=np.uint8) for n in rlens]
    qres, qoff = np.concatenate(qs), np.zeros(len(qs) + 1, dtype=np.int64)
    rres, roff = np.concatenate(rs), np.zeros(len(rs) + 1, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    np.cumsum([r.size for r in rs], out=roff[1:])
    idx = np.arange(len(qs), dtype=np.int32)
    return W.Workload("pairs_of", qres, qoff, rres, roff, idx, idx.copy(), M, go, ge, {})


@pytest.mark.parametrize("mode", MODES)
def test_dual_couples_after_the_reorder(mode):
    # queries up to 160 residues are reordered by columns per lane and rows
    # (more first) before they are coupled two per wavefront: two pairs stay
    # in place (a 1-row pair beside a 1400-row one, 1 and 5 columns per
    # lane); three of different widths leave an uneven couple (5 columns x
    # 1400 rows with 3 x 700) and a lone pair; rows from 1023 on share one
    # bucket, so a crowd of them couples in any order
    w = _pairs_of([20, 150], [1, 1400], 1996 + mode)
    _check(w, mode, "two")
    w = _pairs_of([150, 10, 70], [1400, 3, 700], 1997 + mode)
    _check(w, mode, "three")
    rng = np.random.default_rng(1998 + mode)
    n = 37
    w = _pairs_of(rng.integers(1, 161, size=n), rng.integers(1000, 1600, size=n), 1999 + mode)
    assert (np.diff(w.ref_off) >= 1023).sum() > n // 2
    _check(w, mode, "clamped bucket")


@pytest.mark.parametrize("mode", MODES)
def test_dual_reorder_across_workgroups(mode):
    # 6000 queries up to 160 residues: the reorder's histogram and scatter
    # run in three workgroups that reserve their shares of each bucket
    rng = np.random.default_rng(2003 + mode)
    w = W.random_pairs(6000, 4, (1, 160), (1, 30), 2004 + mode, matrix=W.random_matrix(rng, 4),
                       gap_open=3, gap_extend=1)
    assert (np.diff(w.query_off) <= 160).all()
    _check(w, mode, "reorder x3")


@pytest.mark.parametrize("mode", MODES)
def test_many_tiled_queries_share_wavefronts(mode):
    # 20000 queries of 513-700 residues (two tiles each): one launch of the
    # most wavefronts it takes, each running two or three pairs in turn with
    # its carry slot; a sample against the oracle, every pair against the
    # same pairs run 1000 at a time (as many wavefronts as pairs)
    rng = np.random.default_rng(2010 + mode)
    w = W.random_pairs(20000, 4, (513, 700), (60, 160), 2011 + mode,
                       matrix=W.random_matrix(rng, 4), gap_open=3, gap_extend=1)
    got = _run(w, mode)
    assert (got[:, 3] == 0).all()
    sample = sorted(rng.choice(w.n_pairs, size=150, replace=False).tolist())
    want = oracle.endtoend_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                                 w.matrix, w.gap_open, w.gap_extend, mode,
                                 pair_query=w.pair_query, pairs=sample)
    np.testing.assert_array_equal(got[sample, :3].astype(np.int64), want)
    for lo in range(0, w.n_pairs, 1000):
        part = _run(w.subset(np.arange(lo, lo + 1000)), mode)
        np.testing.assert_array_equal(part, got[lo:lo + 1000])


@pytest.mark.parametrize("mode", MODES)
def test_queries_across_tiles(mode):
    # queries of 257-1600 residues: up to 512 one tile at 5-8 columns per
    # lane, beyond that two to four tiles with carries, as many as 512-column
    # tiles would need, each of the fewest columns per lane (5-8) that cover
    # the query; references from 1 to 400
    rng = np.random.default_rng(980 + mode)
    w = W.random_pairs(120, 4, (257, 1600), (1, 400), 981 + mode, matrix=W.random_matrix(rng, 4),
                       gap_open=3, gap_extend=1)
    ms = np.diff(w.query_off)
    assert {int((m + 63) // 64) for m in ms if m <= 512} == {5, 6, 7, 8}
    tiles = {int(m): int((m + 511) // 512) for m in ms if m > 512}
    assert set(tiles.values()) == {2, 3, 4}
    assert {(m + 64 * t - 1) // (64 * t) for m, t in tiles.items()} == {5, 6, 7, 8}
    _check(w, mode, "tiles")


@pytest.mark.parametrize("mode", MODES)
def test_queries_at_tile_edges(mode):
    # query lengths on both sides of every width edge of the long-query
    # kernel: 5-8 columns per lane in one tile up to 512 residues, then t
    # tiles (t = ceil(m / 512)) of the fewest columns per lane (5-8) that
    # cover the query; references from 1 to 300, some of one residue
    rng = np.random.default_rng(1995 + mode)
    M = W.random_matrix(rng, 4)
    lens = []
    for t in (1, 2, 3, 4):
        for c in (5, 6, 7, 8):
            lens += [64 * c * t, 64 * c * t + 1]
    lens = sorted(set(m for m in lens if m > 256 and m <= 2049) | {257, 2049})
    qs, rs = [], []
    for m in lens:
        for n in (1, int(rng.integers(2, 60)), int(rng.integers(60, 301))):
            qs.append(rng.integers(0, 4, size=m, dtype=np.uint8))
            rs.append(rng.integers(0, 4, size=n, dtype=np.uint8))
    qres, qoff = np.concatenate(qs), np.zeros(len(qs) + 1, dtype=np.int64)
    rres, roff = np.concatenate(rs), np.zeros(len(rs) + 1, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    np.cumsum([r.size for r in rs], out=roff[1:])
    idx = np.arange(len(qs), dtype=np.int32)
    w = W.Workload("tile_edges", qres, qoff, rres, roff, idx, idx.copy(), M, 3, 1, {})
    ms = np.diff(qoff)
    tiles = {int(m): max(1, int((m + 511) // 512)) for m in ms}
    assert set(tiles.values()) == {1, 2, 3, 4, 5}
    assert {(m + 64 * t - 1) // (64 * t) for m, t in tiles.items()} == {5, 6, 7, 8}
    _check(w, mode, "tile edges")


def test_dna_pairs_subset():
    # reads inside their windows: semi-global places each read, global also
    # pays for the window's overhang; every pair scores at least as well
    # semi-globally, and locally better still
    w = W.dna_pairs(n_pairs=2000, seed=25)
    glob = _check(w, api.SW_MODE_GLOBAL, "dna", pairs=range(0, 2000, 50))
    semi = _check(w, api.SW_MODE_SEMIGLOBAL, "dna", pairs=range(0, 2000, 50))
    assert (semi[:, 0] >= glob[:, 0]).all()
    assert np.median(semi[:, 0]) > 100           # 150 bp reads, 2% substitutions
    local = api.align_workload(w).results
    assert (local[:, 0] >= semi[:, 0]).all()


def test_protein_search_sample_and_shared_query():
    w = W.protein_search(n_refs=2000)
    for mode in MODES:
        _check(w, mode, "protein", pairs=range(0, 2000, 200))


def test_device_resident_inputs_and_errors():
    import torch
    w = W.random_pairs(200, 4, (0, 300), (0, 300), 990)
    host = _run(w, api.SW_MODE_SEMIGLOBAL)
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    got = api.sw_align_batch_global(t(w.query_res, torch.uint8), t(w.query_off, torch.int64),
                                    t(w.ref_res, torch.uint8), t(w.ref_off, torch.int64),
                                    t(w.pair_ref, torch.int32), w.matrix, w.gap_open,
                                    w.gap_extend, mode=api.SW_MODE_SEMIGLOBAL,
                                    pair_query=t(w.pair_query, torch.int32))
    assert (got == host).all()
    ref = w.ref_res.copy()
    ref[len(ref) // 2] = 7                       # beyond the 4-letter alphabet
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_global(w.query_res, w.query_off, ref, w.ref_off, w.pair_ref, w.matrix,
                                  w.gap_open, w.gap_extend, mode=api.SW_MODE_GLOBAL,
                                  pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    with pytest.raises(api.SwError) as e:
        _run(w, 5)
    assert e.value.code == api.SW_EINVAL
    again = _run(w, api.SW_MODE_SEMIGLOBAL)
    assert (again == host).all()


def _paths(w, mode, **kw):
    res = _run(w, mode)
    qs, rs, runs, off = api.sw_align_batch_global_cigar(w.query_res, w.query_off, w.ref_res,
                                                        w.ref_off, w.pair_ref, w.matrix,
                                                        w.gap_open, w.gap_extend, res, mode=mode,
                                                        pair_query=w.pair_query, **kw)
    return res, qs, rs, runs, off


def _seqs(w, k):
    qi = 0 if w.pair_query is None else int(w.pair_query[k])
    ri = int(w.pair_ref[k])
    return (w.query_res[w.query_off[qi]:w.query_off[qi + 1]],
            w.ref_res[w.ref_off[ri]:w.ref_off[ri + 1]])


def _check_paths(w, mode, label, pairs=None):
    res, qs, rs, runs, off = _paths(w, mode)
    for k in (range(w.n_pairs) if pairs is None else pairs):
        q, r = _seqs(w, k)
        want = oracle.endtoend_path(q, r, w.matrix, w.gap_open, w.gap_extend, mode,
                                    end=tuple(int(x) for x in res[k, :3]))
        got = (int(qs[k]), int(rs[k]), api.decode_cigar(runs, off, k))
        assert got == want, "%s mode %d pair %d: got %s want %s" % (label, mode, k, got, want)
    return res, qs, rs, runs, off


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("alpha,go,ge", [(2, 2, 1), (4, 3, 1), (20, 11, 1), (3, 1, 0), (4, 2, 5)])
def test_paths_small_pairs_equal_the_oracle(mode, alpha, go, ge):
    # empty sides included (their runs are made by the path planner, no kernel)
    rng = np.random.default_rng(1000 + alpha + go + 7 * mode)
    M = W.protein_matrix() if alpha == 20 else W.random_matrix(rng, alpha)
    w = W.random_pairs(300, alpha, (0, 40), (0, 50), 1001 + alpha + mode, matrix=M,
                       gap_open=go, gap_extend=ge)
    _check_paths(w, mode, "small")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("scale", [1, 1000])
def test_paths_across_tiles_and_in_device_memory(mode, scale):
    # queries of 257-700 residues (one or two 512-column tiles in 16-bit
    # values, two or three 256-column tiles in 32-bit values; rows x tiles
    # beyond the LDS budget, so the decision bits live in device memory) and
    # queries of 20-100 residues with up to 300 rows.  Scale 1000 multiplies
    # the matrix and both penalties: the same optimal paths and ties, values
    # beyond the 16-bit range, so the 32-bit fill runs
    rng = np.random.default_rng(1010 + mode)
    M = W.random_matrix(rng, 4) * scale
    w = W.random_pairs(12, 4, (257, 700), (1, 90), 1011 + mode, matrix=M, gap_open=3 * scale,
                       gap_extend=scale)
    _check_paths(w, mode, "tiles x%d" % scale)
    w = W.random_pairs(12, 4, (20, 100), (170, 300), 1012 + mode, matrix=M, gap_open=3 * scale,
                       gap_extend=scale)
    _check_paths(w, mode, "rows x%d" % scale)


def test_paths_dna_reads_in_windows():
    # semi-global: each read placed inside its window; the path consumes the
    # read and r[ref_start .. ref_end]
    w = W.dna_pairs(n_pairs=400, seed=27)
    res, qs, rs, runs, off = _check_paths(w, api.SW_MODE_SEMIGLOBAL, "dna",
                                          pairs=range(0, 400, 40))
    for k in range(w.n_pairs):
        got = api.decode_cigar(runs, off, k)
        assert qs[k] == 0 and sum(n for n, o in got if o in "MI") == 150
        assert sum(n for n, o in got if o in "MD") == res[k, 2] - rs[k] + 1
    _check_paths(w, api.SW_MODE_GLOBAL, "dna", pairs=range(0, 400, 100))
    _check_paths(w, api.SW_MODE_OVERLAP, "dna", pairs=range(0, 400, 100))
    # the roles swapped: each read is the reference, fitted into its window
    sw = W.Workload("dna_swapped", w.ref_res, w.ref_off, w.query_res, w.query_off,
                    w.pair_ref.copy(), w.pair_query.copy(), w.matrix, w.gap_open, w.gap_extend)
    res2, qs2, rs2, runs2, off2 = _check_paths(sw, api.SW_MODE_SEMIGLOBAL_REF, "dna swapped",
                                               pairs=range(0, 400, 40))
    assert (res2[:, 0] == res[:, 0]).all() and (res2[:, 1] == res[:, 2]).all()
    assert (qs2 == rs).all() and (rs2 == 0).all()


def test_paths_errors():
    w = W.random_pairs(50, 4, (1, 40), (1, 40), 1020)
    res = _run(w, api.SW_MODE_GLOBAL)
    args = (w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref, w.matrix, w.gap_open,
            w.gap_extend)
    bad = res.copy()
    bad[3, 0] += 1                                 # not the optimum
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_global_cigar(*args, bad, mode=api.SW_MODE_GLOBAL,
                                        pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    bad = res.copy()
    bad[3, 2] -= 1                                 # a global end must be (m - 1, n - 1)
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_global_cigar(*args, bad, mode=api.SW_MODE_GLOBAL,
                                        pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    qs, rs, runs, off = api.sw_align_batch_global_cigar(*args, res, mode=api.SW_MODE_GLOBAL,
                                                        pair_query=w.pair_query)
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_global_cigar(*args, res, mode=api.SW_MODE_GLOBAL,
                                        pair_query=w.pair_query, cigar_cap=int(off[-1]) - 1)
    assert e.value.code == api.SW_EINVAL


def test_paths_device_resident_inputs():
    import torch
    w = W.random_pairs(150, 4, (0, 120), (0, 200), 1030)
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    d = (t(w.query_res, torch.uint8), t(w.query_off, torch.int64), t(w.ref_res, torch.uint8),
         t(w.ref_off, torch.int64), t(w.pair_ref, torch.int32))
    pq = t(w.pair_query, torch.int32)
    for mode in MODES:
        res, qs, rs, runs, off = _paths(w, mode)
        res_d = api.sw_align_batch_global(*d, w.matrix, w.gap_open, w.gap_extend, mode=mode,
                                          pair_query=pq)
        assert (res_d == res).all()
        qs_d, rs_d, runs_d, off_d = api.sw_align_batch_global_cigar(*d, w.matrix, w.gap_open,
                                                                    w.gap_extend, res_d,
                                                                    mode=mode, pair_query=pq)
        assert (qs_d == qs).all() and (rs_d == rs).all()
        assert (off_d == off).all() and (runs_d == runs).all()


def test_largest_alphabet_and_overflow_refusal():
    # 32 letters (the largest alphabet): the LDS matrix region at its size
    rng = np.random.default_rng(1040)
    M = rng.integers(-6, 7, size=(32, 32)).astype(np.int32)
    np.fill_diagonal(M, 9)
    w = W.random_pairs(120, 32, (1, 80), (1, 80), 1041, matrix=M, gap_open=5, gap_extend=2)
    for mode in MODES:
        _check(w, mode, "alpha 32")
        _check_paths(w, mode, "alpha 32", pairs=range(0, 120, 10))
    # scores that could leave the kernels' int32 range are refused, not wrapped
    big = np.full((4, 4), -(1 << 27), dtype=np.int32)
    np.fill_diagonal(big, 1 << 26)
    wb = W.random_pairs(4, 4, (10, 20), (10, 20), 1042, matrix=big, gap_open=3, gap_extend=1)
    with pytest.raises(api.SwError) as e:
        _run(wb, api.SW_MODE_GLOBAL)
    assert e.value.code == api.SW_EOVERFLOW


def test_overlap_dovetails_and_reference_fitted_reads():
    # reads that hang off either end of their window: the overlap places the
    # shared part, paying nothing for the overhangs; the same pairs fitted the
    # other way round (the window inside the read) and globally for contrast
    rng = np.random.default_rng(1050)
    qs, rs = [], []
    for k in range(300):
        L = int(rng.integers(40, 120))
        core = rng.integers(0, 4, size=L, dtype=np.uint8)
        hang_q = rng.integers(0, 4, size=int(rng.integers(0, 60)), dtype=np.uint8)
        hang_r = rng.integers(0, 4, size=int(rng.integers(0, 60)), dtype=np.uint8)
        if k % 3 == 0:       # the read's suffix is the window's prefix
            q, r = np.concatenate([hang_q, core]), np.concatenate([core, hang_r])
        elif k % 3 == 1:     # the read's prefix is the window's suffix
            q, r = np.concatenate([core, hang_q]), np.concatenate([hang_r, core])
        else:                # the window inside the read
            q, r = np.concatenate([hang_q, core, hang_r]), core.copy()
        qs.append(q)
        rs.append(r)
    qoff = np.zeros(301, dtype=np.int64)
    roff = np.zeros(301, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    np.cumsum([r.size for r in rs], out=roff[1:])
    idx = np.arange(300, dtype=np.int32)
    w = W.Workload("dovetails", np.concatenate(qs), qoff, np.concatenate(rs), roff, idx,
                   idx.copy(), W.dna_matrix(), 6, 1, {})
    ov = _check(w, api.SW_MODE_OVERLAP, "dovetail")
    assert (ov[:, 0] >= 40).all()                  # at least the shared part, overhangs free
    sr = _check(w, api.SW_MODE_SEMIGLOBAL_REF, "window in read")
    assert (sr[2::3, 0] == np.array([r.size for r in rs[2::3]])).all()   # exact match of the window
    _check(w, api.SW_MODE_GLOBAL, "global")
    assert (ov[:, 0] >= sr[:, 0]).all()
    _check_paths(w, api.SW_MODE_OVERLAP, "dovetail paths", pairs=range(0, 300, 7))
    _check_paths(w, api.SW_MODE_SEMIGLOBAL_REF, "window paths", pairs=range(0, 300, 7))


def test_overlap_and_reference_fitted_end_errors():
    w = W.random_pairs(30, 4, (5, 40), (5, 40), 1060)
    args = (w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref, w.matrix, w.gap_open,
            w.gap_extend)
    for mode in (api.SW_MODE_SEMIGLOBAL_REF, api.SW_MODE_OVERLAP):
        res = _run(w, mode)
        bad = res.copy()
        bad[4, 1] = np.diff(w.query_off)[4] - 2
        bad[4, 2] = np.diff(w.ref_off)[4] - 2      # on neither sequence's last residue
        with pytest.raises(api.SwError) as e:
            api.sw_align_batch_global_cigar(*args, bad, mode=mode, pair_query=w.pair_query)
        assert e.value.code == api.SW_EINVAL
        bad = res.copy()
        bad[6, 0] += 1                             # not the optimum there
        with pytest.raises(api.SwError) as e:
            api.sw_align_batch_global_cigar(*args, bad, mode=mode, pair_query=w.pair_query)
        assert e.value.code == api.SW_EINVAL
