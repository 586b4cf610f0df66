"""Thin ctypes binding of libswscan.so (include/sw.h), same entry-point names.

Argument marshalling only: every alignment step runs in the library's HIP
kernels.  Torch tensors on the GPU may be passed to ``sw_align_batch`` (they
are handed over as device pointers with ``device_resident=1`` and torch's
current stream); numpy arrays are host memory.  If the library is missing the
first call raises ``NativeLibraryError``: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswscan.so")

SW_OK, SW_PENDING, SW_EINVAL, SW_ENOMEM, SW_EDEVICE, SW_EOVERFLOW, SW_ENOENT, SW_EBUSY = \
    0, 1, -1, -2, -3, -4, -5, -6
SW_PREC_AUTO, SW_PREC_I32 = 0, 1
SW_ALG_SCAN, SW_ALG_LAZYF = 0, 1
SW_PAIRING_AUTO, SW_PAIRING_ALIGNMENTS, SW_PAIRING_ROWS = 0, 1, 2
SW_CHAINS_AUTO, SW_CHAINS_ONE, SW_CHAINS_TWO = 0, 1, 2
SW_STRIPE_AUTO, SW_STRIPE_QUERY, SW_STRIPE_SHORTER = 0, 1, 2
SW_FLAG_SATURATED = 1

EXPORTED = ["sw_strerror", "sw_last_error", "sw_init", "sw_shutdown", "sw_align",
            "sw_align_batch", "sw_align_batch_ex", "sw_server_create", "sw_server_submit",
            "sw_server_poll", "sw_server_drain", "sw_server_destroy", "sw_server_replay",
            "sw_autotune", "sw_tune_set", "sw_tune_get", "sw_align_batch_starts",
            "sw_align_batch_cigar", "sw_align_batch_global", "sw_align_batch_global_cigar",
            "sw_align_ex", "sw_align_batch_noalloc"]
SW_NOALLOC_MAX_PAIRS = 1048576


class NativeLibraryError(RuntimeError):
    pass


class SwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, msg))
        self.code = code


class Scoring(ctypes.Structure):
    _fields_ = [("alphabet_size", ctypes.c_int32), ("matrix", ctypes.c_void_p),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("query_end", ctypes.c_int32),
                ("ref_end", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int32),
                ("query_res", ctypes.c_void_p), ("query_off", ctypes.c_void_p),
                ("n_queries", ctypes.c_int32),
                ("ref_res", ctypes.c_void_p), ("ref_off", ctypes.c_void_p),
                ("n_refs", ctypes.c_int32),
                ("pair_query", ctypes.c_void_p), ("pair_ref", ctypes.c_void_p),
                ("precision", ctypes.c_int32), ("device_resident", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("algorithm", ctypes.c_int32), ("force_lanes", ctypes.c_int32),
                ("force_seglen", ctypes.c_int32), ("force_kernel", ctypes.c_int32),
                ("mixed_layout", ctypes.c_int32), ("int16_cap", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("planner", ctypes.c_int32),
                ("lane_pairing", ctypes.c_int32), ("int32_chains", ctypes.c_int32),
                ("striping", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class Stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("cells", ctypes.c_int64), ("padded_cells", ctypes.c_int64),
                ("n_rerun", ctypes.c_int32), ("n_launches", ctypes.c_int32),
                ("lazyf_steps", ctypes.c_int64), ("columns", ctypes.c_int64),
                ("lanes_used", ctypes.c_int32 * 3), ("seglen_max", ctypes.c_int32),
                ("prep_ms", ctypes.c_double), ("plan_ms", ctypes.c_double),
                ("launch_ms", ctypes.c_double), ("finish_ms", ctypes.c_double),
                ("record_events", ctypes.c_int64), ("graph_hits", ctypes.c_int32),
                ("planner_used", ctypes.c_int32), ("row_pairs", ctypes.c_int32),
                ("lanes8", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]

    def as_dict(self) -> dict:
        return {"kernel_ms": self.kernel_ms, "total_ms": self.total_ms, "cells": self.cells,
                "padded_cells": self.padded_cells, "n_rerun": self.n_rerun,
                "n_launches": self.n_launches, "lazyf_steps": self.lazyf_steps,
                "columns": self.columns, "lanes_used": list(self.lanes_used),
                "seglen_max": self.seglen_max, "prep_ms": self.prep_ms, "plan_ms": self.plan_ms,
                "launch_ms": self.launch_ms, "finish_ms": self.finish_ms,
                "record_events": self.record_events, "graph_hits": self.graph_hits,
                "planner_used": self.planner_used, "row_pairs": self.row_pairs,
                "lanes8": self.lanes8}


SW_TUNE_SHARED, SW_TUNE_PAIR, SW_TUNE_DEVICE_SHARED, SW_TUNE_DEVICE_PAIR = 0, 1, 2, 3


class TuneEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("alphabet_size", ctypes.c_int32), ("m_lo", ctypes.c_int32),
                ("m_hi", ctypes.c_int32), ("lanes", ctypes.c_int32), ("seglen", ctypes.c_int32),
                ("mixed", ctypes.c_int32), ("pairing", ctypes.c_int32),
                ("lds_records", ctypes.c_int32), ("gcups", ctypes.c_double),
                ("model_gcups", ctypes.c_double)]
    KEYS = ("kind", "precision", "alphabet_size", "m_lo", "m_hi", "lanes", "seglen", "mixed",
            "pairing", "lds_records", "gcups", "model_gcups")

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in self.KEYS}

    @classmethod
    def from_dict(cls, d: dict) -> "TuneEntry":
        return cls(*[d.get(k, 0) for k in cls.KEYS])


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_queued", ctypes.c_int32),
                ("db_res", ctypes.c_void_p), ("db_off", ctypes.c_void_p),
                ("n_db", ctypes.c_int32), ("scorings", ctypes.c_void_p),
                ("n_scorings", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("reserved", ctypes.c_int32 * 6)]


_lib = None


def load():
    """Load libswscan.so (raises NativeLibraryError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NativeLibraryError("%s is missing; run __graft_entry__.build()" % LIB_PATH)
    # One HIP runtime per process: torch ships its own libamdhip64 (same soname
    # as the system one).  Loading torch first makes this library bind to the
    # runtime torch already mapped instead of mapping a second one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    try:
        lib = ctypes.CDLL(LIB_PATH)
    except OSError as e:
        raise NativeLibraryError("cannot load %s: %s" % (LIB_PATH, e))
    lib.sw_strerror.restype = ctypes.c_char_p
    lib.sw_strerror.argtypes = [ctypes.c_int]
    lib.sw_last_error.restype = ctypes.c_char_p
    lib.sw_last_error.argtypes = []
    lib.sw_init.argtypes = [ctypes.c_int]
    lib.sw_shutdown.argtypes = []
    lib.sw_align.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                             ctypes.POINTER(Scoring), ctypes.POINTER(Result)]
    lib.sw_align_ex.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                ctypes.POINTER(Scoring), ctypes.POINTER(Result),
                                ctypes.POINTER(Stats)]
    lib.sw_align_batch.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring), ctypes.c_void_p]
    lib.sw_align_batch_ex.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring),
                                      ctypes.POINTER(Options), ctypes.c_void_p,
                                      ctypes.POINTER(Stats)]
    lib.sw_align_batch_noalloc.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring),
                                           ctypes.c_void_p, ctypes.POINTER(Stats)]
    lib.sw_align_batch_starts.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring),
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.sw_align_batch_cigar.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring),
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.sw_align_batch_global.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring),
                                          ctypes.c_int32, ctypes.c_void_p]
    lib.sw_align_batch_global_cigar.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring),
                                                ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_void_p]
    lib.sw_autotune.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring), ctypes.c_int64,
                                ctypes.POINTER(TuneEntry), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int32)]
    lib.sw_tune_set.argtypes = [ctypes.POINTER(TuneEntry), ctypes.c_int32]
    lib.sw_tune_get.argtypes = [ctypes.POINTER(TuneEntry), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int32)]
    _bind_server(lib)
    for name in EXPORTED:
        if not hasattr(lib, name):
            raise NativeLibraryError("%s does not export %s" % (LIB_PATH, name))
    _lib = lib
    return lib


def _bind_server(lib):
    lib.sw_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]
    lib.sw_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_uint64)]
    lib.sw_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Result),
                                   ctypes.c_void_p]
    lib.sw_server_drain.argtypes = [ctypes.c_void_p]
    lib.sw_server_destroy.argtypes = [ctypes.c_void_p]
    lib.sw_server_replay.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]


def _strerror(code: int) -> str:
    try:
        return load().sw_strerror(code).decode()
    except NativeLibraryError:
        return "error"


def _check(code: int) -> int:
    if code < 0:
        raise SwError(code, load().sw_last_error().decode())
    return code


def make_scoring(matrix, gap_open: int, gap_extend: int):
    M = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    if M.ndim != 2 or M.shape[0] != M.shape[1]:
        raise ValueError("matrix must be square")
    sc = Scoring(M.shape[0], M.ctypes.data, int(gap_open), int(gap_extend))
    return sc, M  # keep M alive with the struct


def sw_init(device: int = -1) -> None:
    _check(load().sw_init(device))


def sw_align(query, ref, matrix, gap_open: int, gap_extend: int):
    """One pair, one launch.  Returns (score, query_end, ref_end, flags)."""
    q = np.ascontiguousarray(np.asarray(query, dtype=np.uint8))
    r = np.ascontiguousarray(np.asarray(ref, dtype=np.uint8))
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    res = Result()
    _check(load().sw_align(q.ctypes.data if q.size else None, q.size,
                           r.ctypes.data if r.size else None, r.size,
                           ctypes.byref(sc), ctypes.byref(res)))
    return res.score, res.query_end, res.ref_end, res.flags


def sw_align_ex(query, ref, matrix, gap_open: int, gap_extend: int):
    """sw_align with statistics: ((score, query_end, ref_end, flags), stats dict
    with kernel_ms from HIP events, total_ms and cells)."""
    q = np.ascontiguousarray(np.asarray(query, dtype=np.uint8))
    r = np.ascontiguousarray(np.asarray(ref, dtype=np.uint8))
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    res = Result()
    st = Stats()
    _check(load().sw_align_ex(q.ctypes.data if q.size else None, q.size,
                              r.ctypes.data if r.size else None, r.size,
                              ctypes.byref(sc), ctypes.byref(res), ctypes.byref(st)))
    return (res.score, res.query_end, res.ref_end, res.flags), st.as_dict()


def _is_torch_cuda(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


@dataclass
class BatchOutput:
    results: np.ndarray      # (n_pairs, 4) int32: score, query_end, ref_end, flags
    stats: dict


def _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query, precision):
    """sw_batch for numpy (host) or torch CUDA (device-resident) CSR arrays; returns
    the struct, the arrays it points into (keep them alive) and the pair count."""
    dev = _is_torch_cuda(ref_res)
    keep = []
    if dev:
        import torch
        arrs = [query_res, query_off, ref_res, ref_off, pair_ref] + \
            ([] if pair_query is None else [pair_query])
        for a, dt in zip(arrs, [torch.uint8, torch.int64, torch.uint8, torch.int64, torch.int32,
                                torch.int32]):
            if not (_is_torch_cuda(a) and a.dtype == dt and a.is_contiguous()):
                raise TypeError("device-resident inputs must be contiguous CUDA tensors of "
                                "uint8/int64/uint8/int64/int32/int32")
        ptr = lambda a: a.data_ptr() if a.numel() else None  # noqa: E731
        nq, nr, npairs = query_off.numel() - 1, ref_off.numel() - 1, pair_ref.numel()
        stream = torch.cuda.current_stream().cuda_stream
    else:
        query_res = np.ascontiguousarray(np.asarray(query_res, dtype=np.uint8))
        query_off = np.ascontiguousarray(np.asarray(query_off, dtype=np.int64))
        ref_res = np.ascontiguousarray(np.asarray(ref_res, dtype=np.uint8))
        ref_off = np.ascontiguousarray(np.asarray(ref_off, dtype=np.int64))
        pair_ref = np.ascontiguousarray(np.asarray(pair_ref, dtype=np.int32))
        if pair_query is not None:
            pair_query = np.ascontiguousarray(np.asarray(pair_query, dtype=np.int32))
        keep += [query_res, query_off, ref_res, ref_off, pair_ref, pair_query]
        ptr = lambda a: a.ctypes.data if a.size else None  # noqa: E731
        nq, nr, npairs = query_off.size - 1, ref_off.size - 1, pair_ref.size
        stream = None
    b = Batch(npairs, ptr(query_res), ptr(query_off), nq, ptr(ref_res), ptr(ref_off), nr,
              None if pair_query is None else ptr(pair_query), ptr(pair_ref), precision,
              1 if dev else 0, stream)
    return b, keep, npairs


def sw_align_batch(query_res, query_off, ref_res, ref_off, pair_ref, matrix, gap_open: int,
                   gap_extend: int, pair_query=None, precision: int = SW_PREC_AUTO,
                   algorithm: int = SW_ALG_SCAN, force_lanes: int = 0, force_seglen: int = 0,
                   force_kernel: int = 0, mixed_layout: int = 0, int16_cap: int = 0,
                   use_graph: int = 0, planner: int = 0,
                   lane_pairing: int = 0, int32_chains: int = 0, striping: int = 0,
                   out=None) -> BatchOutput:
    """Many pairs in one persistent launch (plus an int32 rerun if needed).

    Sequences are CSR.  Either all six arrays are numpy (host) or all are torch
    CUDA tensors (device-resident; torch's current stream orders them).
    ``out``: optional C-contiguous (n_pairs, 4) int32 host array to receive the
    results (e.g. a view of pinned memory, which the device copies into at
    full link speed); a new array otherwise.
    """
    lib = load()
    b, keep, npairs = _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query,
                                  precision)
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    opt = Options(algorithm, force_lanes, force_seglen, force_kernel, mixed_layout, int16_cap,
                  use_graph, planner, lane_pairing, int32_chains, striping)
    # the library writes every entry (sw_result layout: four int32; flags are
    # small bit sets), so the array is returned as it is, without a copy
    if out is None:
        out = np.empty((max(npairs, 1), 4), dtype=np.int32)
    elif not (isinstance(out, np.ndarray) and out.dtype == np.int32 and
              out.shape == (npairs, 4) and out.flags.c_contiguous and npairs > 0):
        raise ValueError("out must be a C-contiguous (n_pairs, 4) int32 array")
    st = Stats()
    _check(lib.sw_align_batch_ex(ctypes.byref(b), ctypes.byref(sc), ctypes.byref(opt),
                                 out.ctypes.data, ctypes.byref(st)))
    return BatchOutput(out[:npairs], st.as_dict())


def sw_align_batch_noalloc(query_res, query_off, ref_res, ref_off, pair_ref, matrix,
                           gap_open: int, gap_extend: int, out, pair_query=None,
                           precision: int = SW_PREC_AUTO) -> dict:
    """The batch call that allocates nothing (library scratch array only).

    Inputs are torch CUDA tensors as for ``sw_align_batch``; ``out`` is a
    C-contiguous (n_pairs, 4) int32 CUDA tensor that receives the results on
    the device.  Returns the call's statistics.
    """
    lib = load()
    if not (_is_torch_cuda(ref_res)):
        raise TypeError("sw_align_batch_noalloc takes device-resident (torch CUDA) inputs")
    b, keep, npairs = _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query,
                                  precision)
    import torch
    if not (_is_torch_cuda(out) and out.dtype == torch.int32 and out.is_contiguous() and
            tuple(out.shape) == (npairs, 4)):
        raise ValueError("out must be a contiguous (n_pairs, 4) int32 CUDA tensor")
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    st = Stats()
    _check(lib.sw_align_batch_noalloc(ctypes.byref(b), ctypes.byref(sc),
                                      out.data_ptr() if npairs else None, ctypes.byref(st)))
    return st.as_dict()


def sw_align_batch_starts(query_res, query_off, ref_res, ref_off, pair_ref, matrix,
                          gap_open: int, gap_extend: int, results, pair_query=None,
                          precision: int = SW_PREC_AUTO):
    """Start cells of the alignments ``sw_align_batch`` returned (``results``:
    its (n_pairs, 4) int32 array for the same batch and scoring).  Returns
    (query_start, ref_start), two int32 arrays; -1 where the score is 0."""
    lib = load()
    b, keep, npairs = _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query,
                                  precision)
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    ends = np.ascontiguousarray(np.asarray(results, dtype=np.int32))
    if ends.shape != (npairs, 4):
        raise ValueError("results must be the (n_pairs, 4) array of sw_align_batch")
    qs = np.empty(max(npairs, 1), dtype=np.int32)
    rs = np.empty(max(npairs, 1), dtype=np.int32)
    _check(lib.sw_align_batch_starts(ctypes.byref(b), ctypes.byref(sc),
                                     ends.ctypes.data if npairs else None, qs.ctypes.data,
                                     rs.ctypes.data))
    return qs[:npairs], rs[:npairs]


SW_CIGAR_M, SW_CIGAR_I, SW_CIGAR_D = 0, 1, 2
CIGAR_OPS = "MID"


def sw_align_batch_cigar(query_res, query_off, ref_res, ref_off, pair_ref, matrix,
                         gap_open: int, gap_extend: int, results, query_start, ref_start,
                         pair_query=None, cigar_cap=None):
    """Paths of the alignments ``sw_align_batch`` returned, from the start cells
    ``sw_align_batch_starts`` returned.  Returns (runs, offsets): pair k's runs
    are runs[offsets[k]:offsets[k + 1]], each ``length << 4 | op`` (op 0 M,
    1 I, 2 D); ``decode_cigar`` turns them into (length, op letter) lists.
    ``cigar_cap`` overrides the run capacity passed (default: the bound the
    library documents, which always suffices)."""
    lib = load()
    b, keep, npairs = _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query,
                                  SW_PREC_AUTO)
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    ends = np.ascontiguousarray(np.asarray(results, dtype=np.int32))
    qs = np.ascontiguousarray(np.asarray(query_start, dtype=np.int32))
    rs = np.ascontiguousarray(np.asarray(ref_start, dtype=np.int32))
    if ends.shape != (npairs, 4) or qs.shape != (npairs,) or rs.shape != (npairs,):
        raise ValueError("results must be (n_pairs, 4), query_start and ref_start (n_pairs,)")
    # capacity: (query_end + 1) + (ref_end + 1) per pair, one pass (at least
    # A + B - 1 >= the library's bound min(A + B - 1, 3 min(A, B) - 2) for
    # every A x B rectangle; the array is allocated lazily, so only the runs
    # written are touched)
    cap = int(ends[:, 1:3].sum(dtype=np.int64)) + 2 * npairs if cigar_cap is None \
        else int(cigar_cap)
    runs = np.empty(max(cap, 1), dtype=np.uint32)
    off = np.empty(npairs + 1, dtype=np.int64)
    _check(lib.sw_align_batch_cigar(ctypes.byref(b), ctypes.byref(sc),
                                    ends.ctypes.data if npairs else None,
                                    qs.ctypes.data if npairs else None,
                                    rs.ctypes.data if npairs else None, runs.ctypes.data, cap,
                                    off.ctypes.data))
    return runs[:off[-1]], off


SW_MODE_GLOBAL, SW_MODE_SEMIGLOBAL, SW_MODE_SEMIGLOBAL_REF, SW_MODE_OVERLAP = 0, 1, 2, 3


def sw_align_batch_global(query_res, query_off, ref_res, ref_off, pair_ref, matrix,
                          gap_open: int, gap_extend: int, mode: int = SW_MODE_GLOBAL,
                          pair_query=None) -> np.ndarray:
    """End-to-end scores of every pair: global (``SW_MODE_GLOBAL``),
    semi-global with free reference ends (``SW_MODE_SEMIGLOBAL``) or free
    query ends (``SW_MODE_SEMIGLOBAL_REF``), or overlap with free end gaps
    (``SW_MODE_OVERLAP``).  Returns an (n_pairs, 4) int32 array of {score,
    query_end, ref_end, flags}."""
    lib = load()
    b, keep, npairs = _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query,
                                  SW_PREC_AUTO)
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    out = np.empty((max(npairs, 1), 4), dtype=np.int32)
    _check(lib.sw_align_batch_global(ctypes.byref(b), ctypes.byref(sc), int(mode),
                                     out.ctypes.data))
    return out[:npairs]


def sw_align_batch_global_cigar(query_res, query_off, ref_res, ref_off, pair_ref, matrix,
                                gap_open: int, gap_extend: int, results,
                                mode: int = SW_MODE_GLOBAL, pair_query=None, cigar_cap=None):
    """Paths of the alignments ``sw_align_batch_global`` returned (``results``,
    same batch, scoring and mode).  Returns (query_start, ref_start, runs,
    offsets): pair k's runs are runs[offsets[k]:offsets[k + 1]] from its start
    (query_start[k], ref_start[k]) to its end cell."""
    lib = load()
    b, keep, npairs = _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query,
                                  SW_PREC_AUTO)
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    ends = np.ascontiguousarray(np.asarray(results, dtype=np.int32))
    if ends.shape != (npairs, 4):
        raise ValueError("results must be the (n_pairs, 4) array of sw_align_batch_global")
    # capacity: the library's bound, (ref_end + 1) + (query_end + 1) + 2 runs per pair
    if cigar_cap is None:
        span = ends[:, 2].astype(np.int64)
        span += ends[:, 1]
        cap = int(span.sum()) + 4 * npairs
    else:
        cap = int(cigar_cap)
    runs = np.empty(max(cap, 1), dtype=np.uint32)
    off = np.empty(npairs + 1, dtype=np.int64)
    qs = np.empty(max(npairs, 1), dtype=np.int32)
    rs = np.empty(max(npairs, 1), dtype=np.int32)
    _check(lib.sw_align_batch_global_cigar(ctypes.byref(b), ctypes.byref(sc), int(mode),
                                           ends.ctypes.data if npairs else None, qs.ctypes.data,
                                           rs.ctypes.data, runs.ctypes.data, cap,
                                           off.ctypes.data))
    return qs[:npairs], rs[:npairs], runs[:off[-1]], off


def decode_cigar(runs, offsets, k: int) -> list:
    """Pair k's runs as [(length, 'M' | 'I' | 'D'), ...]."""
    seg = runs[offsets[k]:offsets[k + 1]]
    return [(int(v >> 4), CIGAR_OPS[int(v & 15)]) for v in seg]


def align_workload(w, **kw) -> BatchOutput:
    """sw_align_batch on a ``workloads.Workload`` (host arrays)."""
    return sw_align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref, w.matrix,
                          w.gap_open, w.gap_extend, pair_query=w.pair_query, **kw)


def sw_autotune(query_res, query_off, ref_res, ref_off, pair_ref, matrix, gap_open: int,
                gap_extend: int, pair_query=None, precision: int = SW_PREC_AUTO,
                sample_cells: int = 0) -> list:
    """Measures kernel shapes on this batch and installs the fastest (the
    library's process-wide tuning table); returns the new entries."""
    lib = load()
    b, keep, npairs = _make_batch(query_res, query_off, ref_res, ref_off, pair_ref, pair_query,
                                  precision)
    sc, M = make_scoring(matrix, gap_open, gap_extend)
    cap = 256
    out = (TuneEntry * cap)()
    n = ctypes.c_int32(0)
    _check(lib.sw_autotune(ctypes.byref(b), ctypes.byref(sc), int(sample_cells), out, cap,
                           ctypes.byref(n)))
    return [out[k].as_dict() for k in range(min(n.value, cap))]


def autotune_workload(w, **kw) -> list:
    """sw_autotune on a ``workloads.Workload`` (host arrays)."""
    return sw_autotune(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref, w.matrix,
                       w.gap_open, w.gap_extend, pair_query=w.pair_query, **kw)


def tune_get() -> list:
    lib = load()
    n = ctypes.c_int32(0)
    _check(lib.sw_tune_get(None, 0, ctypes.byref(n)))
    out = (TuneEntry * max(n.value, 1))()
    _check(lib.sw_tune_get(out, n.value, ctypes.byref(n)))
    return [out[k].as_dict() for k in range(n.value)]


def tune_set(entries) -> None:
    lib = load()
    arr = (TuneEntry * max(len(entries), 1))(*[TuneEntry.from_dict(e) for e in entries])
    _check(lib.sw_tune_set(arr, len(entries)))


def tune_save(path: str) -> None:
    """Writes the tuning table as JSON (a cache for later processes)."""
    import json
    with open(path, "w") as f:
        json.dump(tune_get(), f, indent=1)


def tune_load(path: str) -> None:
    import json
    with open(path) as f:
        tune_set(json.load(f))


class Server:
    """Continuous-batching request server over a resident reference database."""

    def __init__(self, db_res, db_off, scorings, hbm_budget_bytes: int = 0, max_queued: int = 0,
                 max_batch: int = 0, n_streams: int = 0):
        lib = load()
        self._db_res = np.ascontiguousarray(np.asarray(db_res, dtype=np.uint8))
        self._db_off = np.ascontiguousarray(np.asarray(db_off, dtype=np.int64))
        self._keep = []
        arr = (Scoring * len(scorings))()
        for k, (M, go, ge) in enumerate(scorings):
            sc, Mk = make_scoring(M, go, ge)
            arr[k] = sc
            self._keep.append(Mk)
        self._scorings = arr
        cfg = ServerConfig(hbm_budget_bytes, max_queued, self._db_res.ctypes.data,
                           self._db_off.ctypes.data, self._db_off.size - 1,
                           ctypes.cast(arr, ctypes.c_void_p), len(scorings), max_batch, n_streams)
        h = ctypes.c_void_p()
        _check(lib.sw_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def submit(self, query, ref_id: int, scoring_id: int = 0) -> int:
        q = np.ascontiguousarray(np.asarray(query, dtype=np.uint8))
        t = ctypes.c_uint64()
        rc = load().sw_server_submit(self._h, q.ctypes.data if q.size else None, q.size, ref_id,
                                     scoring_id, ctypes.byref(t))
        if rc == SW_EBUSY:
            return -1
        _check(rc)
        return t.value

    def poll(self, ticket: int):
        """None while pending; else (score, query_end, ref_end, flags, (submit, admit, done) ns)."""
        res = Result()
        ts = (ctypes.c_int64 * 3)()
        rc = load().sw_server_poll(self._h, ticket, ctypes.byref(res), ts)
        if rc == SW_PENDING:
            return None
        _check(rc)
        return res.score, res.query_end, res.ref_end, res.flags, tuple(ts)

    def drain(self) -> None:
        _check(load().sw_server_drain(self._h))

    def replay(self, query_res, query_off, ref_id, scoring_id, arrival_s):
        """Open-loop replay; returns (results (n,4), times_ns (n,3): submit, admit, done)."""
        qres = np.ascontiguousarray(np.asarray(query_res, dtype=np.uint8))
        qoff = np.ascontiguousarray(np.asarray(query_off, dtype=np.int64))
        rid = np.ascontiguousarray(np.asarray(ref_id, dtype=np.int32))
        sid = np.ascontiguousarray(np.asarray(scoring_id, dtype=np.int32))
        arr = np.ascontiguousarray((np.asarray(arrival_s, dtype=np.float64) * 1e9).astype(np.int64))
        n = rid.size
        out = np.zeros((max(n, 1), 4), dtype=np.int32)
        ts = np.zeros((max(n, 1), 3), dtype=np.int64)
        _check(load().sw_server_replay(self._h, n, qres.ctypes.data, qoff.ctypes.data,
                                       rid.ctypes.data, sid.ctypes.data, arr.ctypes.data,
                                       out.ctypes.data, ts.ctypes.data))
        return out[:n].astype(np.int64), ts[:n]

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().sw_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
