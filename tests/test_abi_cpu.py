"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/sw.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1909_00899_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "sw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(api.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return api.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert "sw_align" in names and "sw_align_batch" in names
    for n in names:
        assert hasattr(lib, n), n


def test_valu_probe_library_loads(lib):
    # the measurement aid is its own library; built beside libswscan.so
    from paper_1909_00899_amd import valu_probe
    probe = ctypes.CDLL(os.path.join(os.path.dirname(valu_probe.__file__), "libswprobe.so"))
    assert hasattr(probe, "swprobe_valu")
    probe.swprobe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    out = ctypes.c_double(1.0)
    assert probe.swprobe_valu(0, 1, ctypes.byref(out)) != 0     # bad grid: rejected on the host
    assert out.value == 1.0


def test_strerror(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.sw_strerror(code)
    assert lib.sw_strerror(12345) == b"unknown status"


def _sc(M, go=11, ge=1):
    return api.make_scoring(M, go, ge)


def test_sw_align_rejects_bad_arguments(lib):
    M = np.eye(4, dtype=np.int32)
    q = np.array([0, 1, 2], dtype=np.uint8)
    res = api.Result()
    sc, keep = _sc(M)
    # residue outside the alphabet
    bad = np.array([0, 9], dtype=np.uint8)
    assert lib.sw_align(bad.ctypes.data, 2, q.ctypes.data, 3, ctypes.byref(sc), ctypes.byref(res)) == api.SW_EINVAL
    # negative length, NULL out
    assert lib.sw_align(q.ctypes.data, -1, q.ctypes.data, 3, ctypes.byref(sc), ctypes.byref(res)) == api.SW_EINVAL
    assert lib.sw_align(q.ctypes.data, 3, q.ctypes.data, 3, ctypes.byref(sc), None) == api.SW_EINVAL
    # alphabet size, negative penalties
    sc2 = api.Scoring(0, M.ctypes.data, 1, 1)
    assert lib.sw_align(q.ctypes.data, 3, q.ctypes.data, 3, ctypes.byref(sc2), ctypes.byref(res)) == api.SW_EINVAL
    sc3 = api.Scoring(4, M.ctypes.data, -1, 1)
    assert lib.sw_align(q.ctypes.data, 3, q.ctypes.data, 3, ctypes.byref(sc3), ctypes.byref(res)) == api.SW_EINVAL
    # empty sequences are valid and need no device
    assert lib.sw_align(None, 0, q.ctypes.data, 3, ctypes.byref(sc), ctypes.byref(res)) == api.SW_OK
    assert (res.score, res.query_end, res.ref_end) == (0, -1, -1)
    # overflow guard
    big = np.full((4, 4), 2 ** 30, dtype=np.int32)
    scb, kb = _sc(big)
    assert lib.sw_align(q.ctypes.data, 3, q.ctypes.data, 3, ctypes.byref(scb), ctypes.byref(res)) == api.SW_EOVERFLOW


def test_batch_rejects_bad_options(lib):
    M = np.eye(4, dtype=np.int32)
    sc, keep = _sc(M)
    b = api.Batch()
    out = np.zeros((1, 4), dtype=np.int32)
    assert lib.sw_align_batch(None, ctypes.byref(sc), out.ctypes.data) == api.SW_EINVAL
    b.n_pairs = -1
    assert lib.sw_align_batch(ctypes.byref(b), ctypes.byref(sc), out.ctypes.data) == api.SW_EINVAL
    b.n_pairs = 0
    assert lib.sw_align_batch(ctypes.byref(b), ctypes.byref(sc), out.ctypes.data) == api.SW_OK
    opt = api.Options()
    opt.force_lanes = 12
    b.n_pairs = 1
    assert lib.sw_align_batch_ex(ctypes.byref(b), ctypes.byref(sc), ctypes.byref(opt),
                                 out.ctypes.data, None) == api.SW_EINVAL
    opt.force_lanes = 0
    opt.int16_cap = 40000
    assert lib.sw_align_batch_ex(ctypes.byref(b), ctypes.byref(sc), ctypes.byref(opt),
                                 out.ctypes.data, None) == api.SW_EINVAL
    b.precision = 7
    assert lib.sw_align_batch(ctypes.byref(b), ctypes.byref(sc), out.ctypes.data) == api.SW_EINVAL
    opt = api.Options()
    opt.mixed_layout = 3
    b.precision = 0
    assert lib.sw_align_batch_ex(ctypes.byref(b), ctypes.byref(sc), ctypes.byref(opt),
                                 out.ctypes.data, None) == api.SW_EINVAL
    opt = api.Options()
    opt.int32_chains = 3
    assert lib.sw_align_batch_ex(ctypes.byref(b), ctypes.byref(sc), ctypes.byref(opt),
                                 out.ctypes.data, None) == api.SW_EINVAL


def _entry(**kw):
    d = dict(kind=api.SW_TUNE_PAIR, precision=api.SW_PREC_AUTO, alphabet_size=4, m_lo=129,
             m_hi=160, lanes=16, seglen=10, mixed=0, pairing=0, lds_records=0, gcups=1.0,
             model_gcups=1.0)
    d.update(kw)
    return d


def test_tuning_table_round_trip_and_validation(lib, tmp_path):
    try:
        api.tune_set([])
        assert api.tune_get() == []
        good = [_entry(), _entry(kind=api.SW_TUNE_SHARED, alphabet_size=20, m_lo=385, m_hi=512,
                                 lanes=0, seglen=8),
                _entry(kind=api.SW_TUNE_SHARED, alphabet_size=20, m_lo=1, m_hi=64, lanes=16,
                       seglen=4),
                _entry(mixed=1, m_lo=1, m_hi=1000, lanes=64, seglen=16),
                _entry(kind=api.SW_TUNE_DEVICE_SHARED, alphabet_size=20, m_lo=512, m_hi=512,
                       lanes=16, seglen=16, pairing=api.SW_PAIRING_ROWS, lds_records=1),
                _entry(kind=api.SW_TUNE_DEVICE_SHARED, alphabet_size=20, m_lo=300, m_hi=300,
                       lanes=32, seglen=12, pairing=api.SW_PAIRING_ALIGNMENTS),
                _entry(kind=api.SW_TUNE_DEVICE_PAIR, m_lo=150, m_hi=150, lanes=8, seglen=19)]
        api.tune_set(good)
        assert api.tune_get() == good
        path = str(tmp_path / "tune.json")
        api.tune_save(path)
        api.tune_set([])
        api.tune_load(path)
        assert api.tune_get() == good
        bad = [_entry(kind=5), _entry(precision=3), _entry(alphabet_size=0), _entry(m_lo=0),
               _entry(m_lo=10, m_hi=9), _entry(lanes=8), _entry(seglen=7), _entry(mixed=2),
               _entry(kind=api.SW_TUNE_SHARED, lanes=0, seglen=5),
               _entry(kind=api.SW_TUNE_SHARED, lanes=16, seglen=2),
               _entry(kind=api.SW_TUNE_SHARED, mixed=1, lanes=0, seglen=8),
               _entry(kind=api.SW_TUNE_DEVICE_SHARED, lanes=32, seglen=16,
                      pairing=api.SW_PAIRING_ROWS),
               _entry(kind=api.SW_TUNE_DEVICE_SHARED, lanes=16, seglen=16,
                      pairing=api.SW_PAIRING_ROWS, lds_records=2),
               _entry(kind=api.SW_TUNE_DEVICE_SHARED, lanes=16, seglen=16),
               _entry(kind=api.SW_TUNE_DEVICE_PAIR, lanes=8, seglen=19,
                      precision=api.SW_PREC_I32),
               _entry(kind=api.SW_TUNE_DEVICE_PAIR, lanes=32, seglen=8),
               _entry(pairing=api.SW_PAIRING_ROWS)]
        for e in bad:
            with pytest.raises(api.SwError) as ex:
                api.tune_set([e])
            assert ex.value.code == api.SW_EINVAL, e
        assert api.tune_get() == good          # a rejected table leaves the old one
    finally:
        api.tune_set([])


def test_starts_rejects_bad_arguments(lib):
    M = np.eye(4, dtype=np.int32)
    sc, keep = _sc(M)
    b = api.Batch()
    qs = np.zeros(2, dtype=np.int32)
    assert lib.sw_align_batch_starts(None, ctypes.byref(sc), None, qs.ctypes.data,
                                     qs.ctypes.data) == api.SW_EINVAL
    b.n_pairs = 0
    assert lib.sw_align_batch_starts(ctypes.byref(b), ctypes.byref(sc), None, None,
                                     None) == api.SW_OK
    b.n_pairs = 1                                   # ends and outputs missing
    assert lib.sw_align_batch_starts(ctypes.byref(b), ctypes.byref(sc), None, qs.ctypes.data,
                                     qs.ctypes.data) == api.SW_EINVAL
    b.n_pairs = -1
    ends = np.zeros((1, 4), dtype=np.int32)
    assert lib.sw_align_batch_starts(ctypes.byref(b), ctypes.byref(sc), ends.ctypes.data,
                                     qs.ctypes.data, qs.ctypes.data) == api.SW_EINVAL


def test_cigar_rejects_bad_arguments(lib):
    M = np.eye(4, dtype=np.int32)
    sc, keep = _sc(M)
    b = api.Batch()
    z = np.zeros(2, dtype=np.int32)
    off = np.full(3, 7, dtype=np.int64)
    runs = np.zeros(4, dtype=np.uint32)
    assert lib.sw_align_batch_cigar(None, ctypes.byref(sc), None, z.ctypes.data, z.ctypes.data,
                                    runs.ctypes.data, 4, off.ctypes.data) == api.SW_EINVAL
    b.n_pairs = 0
    assert lib.sw_align_batch_cigar(ctypes.byref(b), ctypes.byref(sc), None, None, None, None, 0,
                                    off.ctypes.data) == api.SW_OK
    assert off[0] == 0
    assert lib.sw_align_batch_cigar(ctypes.byref(b), ctypes.byref(sc), None, None, None, None, 0,
                                    None) == api.SW_EINVAL          # no offsets array
    b.n_pairs = 1                                   # arrays missing
    assert lib.sw_align_batch_cigar(ctypes.byref(b), ctypes.byref(sc), None, z.ctypes.data,
                                    z.ctypes.data, runs.ctypes.data, 4,
                                    off.ctypes.data) == api.SW_EINVAL
    b.n_pairs = -1
    assert lib.sw_align_batch_cigar(ctypes.byref(b), ctypes.byref(sc), None, None, None, None, 0,
                                    off.ctypes.data) == api.SW_EINVAL


def test_global_rejects_bad_arguments(lib):
    M = np.eye(4, dtype=np.int32)
    sc, keep = _sc(M)
    b = api.Batch()
    out = np.zeros((2, 4), dtype=np.int32)
    assert lib.sw_align_batch_global(None, ctypes.byref(sc), 0, out.ctypes.data) == api.SW_EINVAL
    b.n_pairs = 0
    assert lib.sw_align_batch_global(ctypes.byref(b), ctypes.byref(sc), 0, None) == api.SW_OK
    assert lib.sw_align_batch_global(ctypes.byref(b), ctypes.byref(sc), 4,
                                     out.ctypes.data) == api.SW_EINVAL        # no such mode
    b.n_pairs = 1                                   # arrays missing
    assert lib.sw_align_batch_global(ctypes.byref(b), ctypes.byref(sc), 1,
                                     out.ctypes.data) == api.SW_EINVAL


def test_global_cigar_rejects_bad_arguments(lib):
    M = np.eye(4, dtype=np.int32)
    sc, keep = _sc(M)
    b = api.Batch()
    off = np.full(3, 7, dtype=np.int64)
    assert lib.sw_align_batch_global_cigar(None, ctypes.byref(sc), 0, None, None, None, None,
                                           0, off.ctypes.data) == api.SW_EINVAL
    b.n_pairs = 0
    for mode in (0, 1, 2, 3):
        off[0] = 7
        assert lib.sw_align_batch_global_cigar(ctypes.byref(b), ctypes.byref(sc), mode, None,
                                               None, None, None, 0, off.ctypes.data) == api.SW_OK
        assert off[0] == 0
    assert lib.sw_align_batch_global_cigar(ctypes.byref(b), ctypes.byref(sc), 4, None, None,
                                           None, None, 0, off.ctypes.data) == api.SW_EINVAL


def test_noalloc_rejects_bad_arguments(lib):
    M = np.eye(4, dtype=np.int32)
    sc, keep = _sc(M)
    q = np.array([0, 1, 2], dtype=np.uint8)
    off = np.array([0, 3], dtype=np.int64)
    pr = np.zeros(1, dtype=np.int32)
    out = np.zeros((1, 4), dtype=np.int32)
    st = api.Stats()
    b = api.Batch(1, q.ctypes.data, off.ctypes.data, 1, q.ctypes.data, off.ctypes.data, 1,
                  None, pr.ctypes.data, api.SW_PREC_AUTO, 0, None)
    # NULL batch or out; host-resident inputs; bad precision; too many pairs:
    # all refused on the host, before any device is touched
    assert lib.sw_align_batch_noalloc(None, ctypes.byref(sc), out.ctypes.data, None) == api.SW_EINVAL
    assert lib.sw_align_batch_noalloc(ctypes.byref(b), ctypes.byref(sc), None, None) == api.SW_EINVAL
    assert lib.sw_align_batch_noalloc(ctypes.byref(b), ctypes.byref(sc), out.ctypes.data,
                                      ctypes.byref(st)) == api.SW_EINVAL
    b.device_resident = 1
    b.precision = 7
    assert lib.sw_align_batch_noalloc(ctypes.byref(b), ctypes.byref(sc), out.ctypes.data, None) == api.SW_EINVAL
    b.precision = api.SW_PREC_AUTO
    b.n_pairs = api.SW_NOALLOC_MAX_PAIRS + 1
    assert lib.sw_align_batch_noalloc(ctypes.byref(b), ctypes.byref(sc), out.ctypes.data, None) == api.SW_EINVAL
    b.n_pairs = 0
    assert lib.sw_align_batch_noalloc(ctypes.byref(b), ctypes.byref(sc), out.ctypes.data, None) == api.SW_OK
