"""Alignment paths (sw_align_batch_cigar): every path equals the CPU oracle's
(canonical predecessor rule, reference gap before query gap) where the oracle
finishes quickly, and at every size the runs cover exactly the rectangle
between start and end cell and add up to the score; through the C ABI.

The path kernel fills rectangles in 16-bit values when their value range
fits and in 32-bit values otherwise.  Scaling the matrix and both gap
penalties by 1000 keeps every optimal path and every tie (all scores scale
alike) but leaves the 16-bit range, so the shape tests run each rectangle
class through both fills."""
import dataclasses

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


def _seqs(w, k):
    qi = 0 if w.pair_query is None else int(w.pair_query[k])
    ri = int(w.pair_ref[k])
    return (w.query_res[w.query_off[qi]:w.query_off[qi + 1]],
            w.ref_res[w.ref_off[ri]:w.ref_off[ri + 1]])


def _scaled(w, k):
    """The same pairs with the matrix and both penalties times k."""
    if k == 1:
        return w
    return dataclasses.replace(w, matrix=(w.matrix * k).astype(np.int32),
                               gap_open=w.gap_open * k, gap_extend=w.gap_extend * k)


def _fits16(w, ends, qs, rs, k):
    """The host's 16-bit rule for pair k's rectangle (4 or 8 columns per lane)."""
    A = int(ends[k, 2] - rs[k] + 1)
    B = int(ends[k, 1] - qs[k] + 1)
    ge = min(w.gap_extend, w.gap_open)
    maxabs = int(np.abs(w.matrix).max())
    tc = 256 if B <= 256 else 512
    span = 5 * (maxabs + w.gap_open) + (A + B + 3 + tc) * ge + 256
    top = min(A, B) * int(max(w.matrix.max(), 0)) + tc * ge + maxabs + 256
    return B > 64 and span < 32768 and top < 32767


def _paths(w):
    ends = api.align_workload(w).results
    qs, rs = api.sw_align_batch_starts(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                                       w.matrix, w.gap_open, w.gap_extend, ends,
                                       pair_query=w.pair_query)
    runs, off = api.sw_align_batch_cigar(w.query_res, w.query_off, w.ref_res, w.ref_off,
                                         w.pair_ref, w.matrix, w.gap_open, w.gap_extend, ends,
                                         qs, rs, pair_query=w.pair_query)
    return ends, qs, rs, runs, off


def _check_properties(w, ends, qs, rs, runs, off, label):
    """What holds at any size: runs cover the rectangle, add up to the score,
    and have the canonical shape (M first and last, D before I between pairs)."""
    for k in range(w.n_pairs):
        got = api.decode_cigar(runs, off, k)
        if ends[k, 0] <= 0:
            assert got == [], (label, k)
            continue
        ops = [o for _, o in got]
        A = ends[k, 2] - rs[k] + 1
        B = ends[k, 1] - qs[k] + 1
        assert ops[0] == "M" and ops[-1] == "M", (label, k, got)
        assert all(x != y for x, y in zip(ops, ops[1:])), (label, k, got)
        assert all(not (x == "I" and y == "D") for x, y in zip(ops, ops[1:])), (label, k, got)
        assert sum(n for n, o in got if o in "MD") == A, (label, k)
        assert sum(n for n, o in got if o in "MI") == B, (label, k)
        q, r = _seqs(w, k)
        s = oracle.path_score(q, r, w.matrix, w.gap_open, w.gap_extend, (qs[k], rs[k]), got)
        assert s == ends[k, 0], (label, k, s, ends[k, 0])


def _check_oracle(w, ends, qs, rs, runs, off, label, pairs):
    for k in pairs:
        q, r = _seqs(w, k)
        want = oracle.path(q, r, w.matrix, w.gap_open, w.gap_extend,
                           end=tuple(int(x) for x in ends[k, :3]), start=(int(qs[k]), int(rs[k])))
        got = api.decode_cigar(runs, off, k)
        assert got == want, "%s: pair %d got %s want %s" % (label, k, got, want)


@pytest.mark.parametrize("alpha,go,ge", [(2, 2, 1), (4, 3, 1), (20, 11, 1), (3, 1, 0),
                                         (4, 2, 5)])
def test_paths_small_pairs_equal_the_oracle(alpha, go, ge):
    # two or three letters and small penalties: many optimal paths, so the tie
    # rule decides; (2, 5): extension above opening
    rng = np.random.default_rng(950 + alpha + go)
    M = W.protein_matrix() if alpha == 20 else W.random_matrix(rng, alpha)
    w = W.random_pairs(600, alpha, (1, 45), (1, 45), 951 + alpha, matrix=M, gap_open=go,
                       gap_extend=ge)
    ends, qs, rs, runs, off = _paths(w)
    _check_properties(w, ends, qs, rs, runs, off, "small")
    _check_oracle(w, ends, qs, rs, runs, off, "small", range(w.n_pairs))


def _gap_family(n_pairs, seed, core, junk, alpha=4, go=2, ge=0):
    """query = X + junk + Y, reference = X + Y: the path crosses a long query
    gap, so the rectangle spans several 256-column tiles."""
    rng = np.random.default_rng(seed)
    M = np.full((alpha, alpha), -3, dtype=np.int32)
    np.fill_diagonal(M, 5)
    qs, rs = [], []
    for k in range(n_pairs):
        x = rng.integers(0, alpha, size=core[0]).astype(np.uint8)
        y = rng.integers(0, alpha, size=core[1]).astype(np.uint8)
        j = rng.integers(0, alpha, size=int(junk[k % len(junk)])).astype(np.uint8)
        qs.append(np.concatenate([x, j, y]))
        rs.append(np.concatenate([x, y]))
    qoff = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum([q.size for q in qs], out=qoff[1:])
    roff = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum([r.size for r in rs], out=roff[1:])
    idx = np.arange(n_pairs, dtype=np.int32)
    return W.Workload("gaps", np.concatenate(qs), qoff, np.concatenate(rs), roff, idx, idx.copy(),
                      M, go, ge)


def test_paths_across_tiles_in_lds():
    # 48 rows x about 300-550 columns in 32-bit values: two or three tiles of
    # 256 columns, decision bits in LDS
    w = _scaled(_gap_family(6, 960, (24, 24), [250, 330, 500]), 1000)
    ends, qs, rs, runs, off = _paths(w)
    _check_properties(w, ends, qs, rs, runs, off, "tiles lds")
    assert (ends[:, 1] - qs + 1 > 256).all()
    assert not any(_fits16(w, ends, qs, rs, k) for k in range(w.n_pairs))
    _check_oracle(w, ends, qs, rs, runs, off, "tiles lds", range(w.n_pairs))


def test_paths_16bit_across_tiles_in_lds():
    # 24 rows x about 540-930 columns in 16-bit values: two tiles of 512
    # columns (8 per lane, 4-byte decision words), decision bits in LDS
    w = _gap_family(6, 965, (12, 12), [520, 600, 750, 900])
    ends, qs, rs, runs, off = _paths(w)
    _check_properties(w, ends, qs, rs, runs, off, "16-bit tiles lds")
    B = ends[:, 1] - qs + 1
    assert ((B > 512) & (B <= 1024)).all() and (ends[:, 2] - rs + 1 <= 40).all()
    assert all(_fits16(w, ends, qs, rs, k) for k in range(w.n_pairs))
    _check_oracle(w, ends, qs, rs, runs, off, "16-bit tiles lds", range(w.n_pairs))


@pytest.mark.parametrize("scale", [1, 1000])
def test_paths_every_column_count(scale):
    # 24-row rectangles whose query spans fall in each columns-per-lane class:
    # in 32-bit values (scale 1000) 1-64, 65-128, 129-192, 193-256 columns
    # (1, 2, 3, 4 columns per lane); in 16-bit values (scale 1) 1-64 columns
    # stay 32-bit, 65-256 take 4 columns per lane, 257-512 take 8
    junk = [10, 40, 70, 100, 140, 150, 200, 230] + ([300, 420] if scale == 1 else [])
    w = _scaled(_gap_family(len(junk), 964, (12, 12), junk), scale)
    ends, qs, rs, runs, off = _paths(w)
    _check_properties(w, ends, qs, rs, runs, off, "columns x%d" % scale)
    B = ends[:, 1] - qs + 1
    if scale == 1:
        assert {int(b <= 64) + 4 * int(64 < b <= 256) + 8 * int(b > 256) for b in B} == {1, 4, 8}
        assert all(_fits16(w, ends, qs, rs, k) == (B[k] > 64) for k in range(w.n_pairs))
    else:
        assert {int((b + 63) // 64) for b in B} == {1, 2, 3, 4}
        assert not any(_fits16(w, ends, qs, rs, k) for k in range(w.n_pairs))
    _check_oracle(w, ends, qs, rs, runs, off, "columns x%d" % scale, range(w.n_pairs))


@pytest.mark.parametrize("scale,junk", [(1, [200, 280]), (1000, [200, 280]), (1, [600, 800])])
def test_paths_in_device_memory(scale, junk):
    # 90 rows x about 290-370 columns (one 512-column tile in 16-bit values,
    # two 256-column tiles in 32-bit ones) or about 690-890 (two 512-column
    # tiles): beyond LDS, decision bits in device memory
    w = _scaled(_gap_family(4, 961, (45, 45), junk), scale)
    ends, qs, rs, runs, off = _paths(w)
    _check_properties(w, ends, qs, rs, runs, off, "device memory")
    A = ends[:, 2] - rs + 1
    B = ends[:, 1] - qs + 1
    if scale == 1:
        assert all(_fits16(w, ends, qs, rs, k) for k in range(w.n_pairs))
        assert (A * ((B + 511) // 512) * 2 > 160).all()
    else:
        assert not any(_fits16(w, ends, qs, rs, k) for k in range(w.n_pairs))
        assert (A * ((B + 255) // 256) > 160).all()
    _check_oracle(w, ends, qs, rs, runs, off, "device memory", range(w.n_pairs))


def test_paths_long_self_alignments():
    # self-alignments: the path is one M run; thousands of rows and columns,
    # several device-memory groups in one call
    rng = np.random.default_rng(962)
    lens = [3000, 1500, 700, 300, 40]
    seqs = [rng.integers(0, 20, size=L).astype(np.uint8) for L in lens]
    off = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    idx = np.arange(len(seqs), dtype=np.int32)
    res = np.concatenate(seqs)
    w = W.Workload("self", res, off, res, off, idx, idx.copy(), W.protein_matrix(), 11, 1)
    ends, qs, rs, runs, off_ = _paths(w)
    for k, L in enumerate(lens):
        assert (qs[k], rs[k]) == (0, 0) and tuple(ends[k, 1:3]) == (L - 1, L - 1)
        assert api.decode_cigar(runs, off_, k) == [(L, "M")]


def test_paths_protein_search_subset():
    w = W.protein_search(n_refs=3000)
    ends, qs, rs, runs, off = _paths(w)
    _check_properties(w, ends, qs, rs, runs, off, "protein")
    area = (ends[:, 1] - qs + 1).astype(np.int64) * (ends[:, 2] - rs + 1)
    small = np.nonzero((ends[:, 0] > 0) & (area <= 1600))[0]
    _check_oracle(w, ends, qs, rs, runs, off, "protein", small[:300])


def test_paths_dna_pairs_subset():
    w = W.dna_pairs(n_pairs=3000, seed=23)
    ends, qs, rs, runs, off = _paths(w)
    _check_properties(w, ends, qs, rs, runs, off, "dna")
    # reads carry indels: most paths have gap runs
    n_gapped = sum(len(api.decode_cigar(runs, off, k)) > 1 for k in range(200))
    assert n_gapped > 20
    _check_oracle(w, ends, qs, rs, runs, off, "dna", range(12))


def test_paths_device_resident_inputs_and_errors():
    import torch
    w = W.random_pairs(300, 4, (0, 60), (0, 80), 963)
    ends, qs, rs, runs, off = _paths(w)
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    runs2, off2 = api.sw_align_batch_cigar(t(w.query_res, torch.uint8), t(w.query_off, torch.int64),
                                           t(w.ref_res, torch.uint8), t(w.ref_off, torch.int64),
                                           t(w.pair_ref, torch.int32), w.matrix, w.gap_open,
                                           w.gap_extend, ends, qs, rs,
                                           pair_query=t(w.pair_query, torch.int32))
    assert (off2 == off).all() and (runs2 == runs).all()
    args = (w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref, w.matrix, w.gap_open,
            w.gap_extend)
    k = int(np.argmax(ends[:, 0]))
    # too small a capacity: offsets still filled
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_cigar(*args, ends, qs, rs, pair_query=w.pair_query,
                                 cigar_cap=int(off[-1]) - 1)
    assert e.value.code == api.SW_EINVAL
    # a start that no alignment of that score leaves from
    bad = qs.copy()
    bad[k] = ends[k, 1]
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_cigar(*args, ends, bad, rs, pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    # a start after the end cell
    bad[k] = ends[k, 1] + 1
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_cigar(*args, ends, bad, rs, pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    # a residue code beyond the alphabet inside a rectangle
    ref = w.ref_res.copy()
    ref[w.ref_off[w.pair_ref[k]] + rs[k]] = 9
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_cigar(w.query_res, w.query_off, ref, w.ref_off, w.pair_ref, w.matrix,
                                 w.gap_open, w.gap_extend, ends, qs, rs, pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL
    # offsets that decrease: a query running past the residue total
    qoff = w.query_off.copy()
    q = int(w.pair_query[k])
    qoff[-1] = qoff[q + 1] - 1
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_cigar(w.query_res[:qoff[-1]], qoff, w.ref_res, w.ref_off, w.pair_ref,
                                 w.matrix, w.gap_open, w.gap_extend, ends, qs, rs,
                                 pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL and "query offsets" in str(e.value)
    roff = w.ref_off.copy()
    r = int(w.pair_ref[k])
    roff[-1] = roff[r + 1] - 1
    with pytest.raises(api.SwError) as e:
        api.sw_align_batch_cigar(w.query_res, w.query_off, w.ref_res[:roff[-1]], roff, w.pair_ref,
                                 w.matrix, w.gap_open, w.gap_extend, ends, qs, rs,
                                 pair_query=w.pair_query)
    assert e.value.code == api.SW_EINVAL and "reference offsets" in str(e.value)
    # the library still works afterwards
    runs3, off3 = api.sw_align_batch_cigar(*args, ends, qs, rs, pair_query=w.pair_query)
    assert (off3 == off).all() and (runs3 == runs).all()
