"""CPU oracle for affine-gap local alignment (Smith-Waterman / Gotoh).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never loads it, and it shares no code with the HIP path: it has its
own C source (``sw_oracle.c``), its own build step and its own Python loops.

Two implementations of one definition:

* ``sw_oracle.c`` -- scalar int64 Gotoh recurrence, reference-outer /
  query-inner, strict ``>`` for the lexicographically smallest
  (ref_end, query_end) end cell; a pthread pool runs many pairs.
* ``gotoh_py`` -- the same recurrence in pure Python (small cases only), which
  can also return the per-column Hd / H tables for hand-checked examples.

Both follow the paper's problem statement (Background: local alignment with
affine gaps; the update order of the inner loop of Algorithm 1; the remark that
no value may go negative, i.e. the local-alignment floor at zero).  Readings
adopted where the paper is silent are stated in each docstring:

* gap of length L costs GapOpen + (L-1) * GapExtend (subtracting GapOpen opens
  a gap, each further residue subtracts GapExtend);
* the score is the running maximum of H_diag = H(i-1, j-1) + S[q_j][r_i]
  (the paper's Max is taken before the E/F maxima), floored at 0;
* S is indexed [query code][reference code];
* end coordinates are those of the H_diag cell achieving the maximum, smallest
  ref_end first, then smallest query_end; score 0 gives (-1, -1).

Start cells (``start_cell``, ``start_batch``): the end cell of the same
recurrence on the reversed prefixes that end at the reported end cell.
Paths (``path``) and end-to-end scores (``endtoend``: global, semi-global in
either direction and overlap, not in the paper) are plain maxima over chains
of aligned pairs.

Parity status: pinned (brute-force enumeration of all local alignments on tiny
inputs, a hand-computed worked example, closed-form special cases and
invariants; start cells by brute-force enumeration of the optimal alignments
ending at the end cell; see ``tests/test_oracle_pins.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


class _Result(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int64), ("query_end", ctypes.c_int64),
                ("ref_end", ctypes.c_int64)]


def build(force: bool = True) -> str:
    """Compile sw_oracle.c into liboracle.so with gcc -O2 (plain C, pthreads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_sw.restype = ctypes.c_int
        lib.oracle_sw.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_Result)]
        lib.oracle_sw_batch.restype = ctypes.c_int
        lib.oracle_sw_batch.argtypes = [ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int32, ctypes.c_void_p]
        _lib = lib
    return _lib


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint8))


def align(query, ref, matrix, gap_open: int, gap_extend: int) -> Tuple[int, int, int]:
    """One pair with the C oracle.  Returns (score, query_end, ref_end)."""
    q = _u8(query)
    r = _u8(ref)
    M = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    alpha = M.shape[0]
    assert M.shape == (alpha, alpha)
    res = _Result()
    rc = _load().oracle_sw(q.ctypes.data, q.size, r.ctypes.data, r.size, M.ctypes.data,
                           alpha, int(gap_open), int(gap_extend), ctypes.byref(res))
    if rc != 0:
        raise RuntimeError("oracle_sw failed")
    return int(res.score), int(res.query_end), int(res.ref_end)


def align_batch(query_res, query_off, ref_res, ref_off, pair_ref, matrix,
                gap_open: int, gap_extend: int, pair_query=None,
                n_threads: Optional[int] = None) -> np.ndarray:
    """Many pairs with the C oracle over a thread pool.

    Queries and references are CSR (residue bytes + offsets of length count+1).
    Returns an (n_pairs, 3) int64 array of (score, query_end, ref_end).
    """
    qres = _u8(query_res)
    rres = _u8(ref_res)
    qoff = np.ascontiguousarray(np.asarray(query_off, dtype=np.int64))
    roff = np.ascontiguousarray(np.asarray(ref_off, dtype=np.int64))
    pr = np.ascontiguousarray(np.asarray(pair_ref, dtype=np.int32))
    pq = None if pair_query is None else np.ascontiguousarray(np.asarray(pair_query, dtype=np.int32))
    M = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    n_pairs = pr.size
    out = np.zeros((n_pairs, 3), dtype=np.int64)
    if n_threads is None:
        n_threads = min(16, os.cpu_count() or 1)
    rc = _load().oracle_sw_batch(n_pairs, qres.ctypes.data, qoff.ctypes.data,
                                 rres.ctypes.data, roff.ctypes.data,
                                 None if pq is None else pq.ctypes.data, pr.ctypes.data,
                                 M.ctypes.data, M.shape[0], int(gap_open), int(gap_extend),
                                 int(n_threads), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_sw_batch failed")
    return out


def gotoh_py(query: Sequence[int], ref: Sequence[int], matrix, gap_open: int,
             gap_extend: int, tables: bool = False):
    """Pure-Python Gotoh recurrence (small inputs only).

    Same definition and tie-break as the C oracle.  With ``tables=True`` also
    returns the per-column lists of H_diag and H values (column = reference
    position), for checking a hand-computed example cell by cell.
    """
    m, n = len(query), len(ref)
    NEG = None  # "no gap open yet"
    Hprev = [0] * m
    E = [NEG] * m
    best, bq, br = 0, -1, -1
    hd_cols, h_cols = [], []
    for i in range(n):
        F = NEG
        Hcur = [0] * m
        hd_col = []
        for j in range(m):
            diag = Hprev[j - 1] if j > 0 else 0
            hd = diag + int(matrix[query[j]][ref[i]])
            hd_col.append(hd)
            if hd > best:
                best, bq, br = hd, j, i
            cands = [0, hd]
            if E[j] is not None:
                cands.append(E[j])
            if F is not None:
                cands.append(F)
            h = max(cands)
            Hcur[j] = h
            e_ext = E[j] - gap_extend if E[j] is not None else None
            E[j] = h - gap_open if e_ext is None else max(e_ext, h - gap_open)
            f_ext = F - gap_extend if F is not None else None
            F = h - gap_open if f_ext is None else max(f_ext, h - gap_open)
        hd_cols.append(hd_col)
        h_cols.append(list(Hcur))
        Hprev = Hcur
    res = (best, bq, br) if best > 0 else (0, -1, -1)
    if tables:
        return res, hd_cols, h_cols
    return res


# ---------------------------------------------------------------- start cells

def start_cell(query, ref, matrix, gap_open: int, gap_extend: int,
               end: Optional[Tuple[int, int, int]] = None) -> Tuple[int, int]:
    """Start (query_start, ref_start) of the alignment reported by ``align``.

    Reading (the paper returns only Max; start cells are this library's
    extension): of all optimal local alignments that end at the reported end
    cell, the one with the largest ref_start, then the largest query_start.
    Computed as the end cell of the same recurrence on the reversed prefixes
    q[0..query_end] and r[0..ref_end]: every optimal alignment inside those
    prefixes ends at the reported end cell (an earlier end would precede it in
    the (ref_end, query_end) order), and the smallest reversed end is the
    largest forward start.  (-1, -1) when the score is 0.
    """
    q = _u8(query)
    r = _u8(ref)
    s, qe, re_ = align(q, r, matrix, gap_open, gap_extend) if end is None else end
    if s <= 0:
        return (-1, -1)
    s2, qe2, re2 = align(q[:qe + 1][::-1], r[:re_ + 1][::-1], matrix, gap_open, gap_extend)
    if s2 != s:
        raise ValueError("end cell does not belong to an optimal alignment of this pair")
    return (qe - qe2, re_ - re2)


def start_batch(query_res, query_off, ref_res, ref_off, pair_ref, matrix, gap_open: int,
                gap_extend: int, ends, pair_query=None,
                n_threads: Optional[int] = None) -> np.ndarray:
    """``start_cell`` for every pair of a batch, given the batch's (score,
    query_end, ref_end) rows; returns an (n_pairs, 2) int64 array of
    (query_start, ref_start).  The reversed prefixes run through
    ``align_batch``."""
    qres = _u8(query_res)
    rres = _u8(ref_res)
    qoff = np.asarray(query_off, dtype=np.int64)
    roff = np.asarray(ref_off, dtype=np.int64)
    pr = np.asarray(pair_ref, dtype=np.int64)
    pq = np.zeros_like(pr) if pair_query is None else np.asarray(pair_query, dtype=np.int64)
    ends = np.asarray(ends, dtype=np.int64)
    out = np.full((pr.size, 2), -1, dtype=np.int64)
    live = np.nonzero(ends[:, 0] > 0)[0]
    if live.size == 0:
        return out
    qs, rs = [], []
    for k in live:
        qe, re_ = int(ends[k, 1]), int(ends[k, 2])
        q0, r0 = int(qoff[pq[k]]), int(roff[pr[k]])
        qs.append(qres[q0:q0 + qe + 1][::-1])
        rs.append(rres[r0:r0 + re_ + 1][::-1])
    nqoff = np.zeros(live.size + 1, dtype=np.int64)
    np.cumsum([x.size for x in qs], out=nqoff[1:])
    nroff = np.zeros(live.size + 1, dtype=np.int64)
    np.cumsum([x.size for x in rs], out=nroff[1:])
    idx = np.arange(live.size, dtype=np.int32)
    rev = align_batch(np.concatenate(qs), nqoff, np.concatenate(rs), nroff, idx, matrix,
                      gap_open, gap_extend, pair_query=idx, n_threads=n_threads)
    if (rev[:, 0] != ends[live, 0]).any():
        raise ValueError("end cells do not belong to optimal alignments of these pairs")
    out[live, 0] = ends[live, 1] - rev[:, 1]
    out[live, 1] = ends[live, 2] - rev[:, 2]
    return out


# ---------------------------------------------------------------- alignment paths

_OPS = "MID"


def path(query, ref, matrix, gap_open: int, gap_extend: int, end=None, start=None):
    """Alignment path (CIGAR runs) of the reported alignment, from its start
    cell to its end cell: a list of (length, op), op in 'M' (an aligned pair),
    'I' (query residues skipped), 'D' (reference residues skipped).

    Reading (the paper returns only the score): over the rectangle between the
    start and the end pair, walking back from the end, each predecessor pair is
    the largest (ref index, then query index) that lies on an optimal chain from
    the start; between two pairs the reference gap is written before the query
    gap.  Computed by ``oracle_path`` in sw_oracle.c as plain maxima over the
    rectangle (no recurrence shortcuts).  A gap run of length L costs
    gap_open + (L - 1) * min(gap_extend, gap_open): the Gotoh recurrences
    score an extension above the opening cost as a fresh opening.  [] when
    the score is 0.
    """
    q = _u8(query)
    r = _u8(ref)
    M = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    s, qe, re_ = align(q, r, M, gap_open, gap_extend) if end is None else end
    if s <= 0:
        return []
    qs, rs = start_cell(q, r, M, gap_open, gap_extend, end=(s, qe, re_)) if start is None else start
    cap = (qe - qs + 1) + (re_ - rs + 1) + 1
    ops = np.zeros(cap, dtype=np.uint32)
    lib = _load()
    lib.oracle_path.restype = ctypes.c_int64
    lib.oracle_path.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_int64]
    n = lib.oracle_path(q.ctypes.data, r.ctypes.data, M.ctypes.data, M.shape[0], int(gap_open),
                        int(gap_extend), int(qs), int(rs), int(qe), int(re_), int(s),
                        ops.ctypes.data, cap)
    if n < 0:
        raise ValueError("oracle_path failed (%d)" % n)
    return [(int(v >> 4), _OPS[int(v & 15)]) for v in ops[:n]]


def path_score(query, ref, matrix, gap_open: int, gap_extend: int, start, runs) -> int:
    """Score of an alignment given as CIGAR runs from its start cell (a
    direct evaluation: pairs scored from the matrix, each gap run by its
    affine cost)."""
    q, r = _u8(query), _u8(ref)
    M = np.asarray(matrix)
    j, i = start
    gap_extend = min(gap_extend, gap_open)     # as the recurrences price runs
    total = 0
    for L, op in runs:
        if op == "M":
            for _ in range(L):
                total += int(M[q[j]][r[i]])
                i += 1
                j += 1
        else:
            total -= gap_open + (L - 1) * gap_extend
            if op == "I":
                j += L
            else:
                i += L
    return total


def endtoend(query, ref, matrix, gap_open: int, gap_extend: int, mode: int) -> Tuple[int, int, int]:
    """(score, query_end, ref_end) of the best end-to-end alignment, from
    ``oracle_endtoend`` in sw_oracle.c (plain maxima over the chains of aligned
    pairs; gap runs priced with min(gap_extend, gap_open)).  Not in the paper,
    whose problem is local alignment.  Modes: 0 global (both sequences end to
    end; ends (m - 1, n - 1)); 1 semi-global (the query end to end, reference
    ends free; query_end m - 1 and the smallest reference prefix end holding an
    optimal alignment, -1 for the empty prefix); 2 the other semi-global (the
    reference end to end, query ends free; ref_end n - 1 and the smallest
    query prefix end); 3 overlap (the residues before the first pair of one
    sequence free, likewise after the last pair; the end on the last query
    row or the last reference column, the smallest (ref_end, query_end))."""
    q, r = _u8(query), _u8(ref)
    M = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    lib = _load()
    lib.oracle_endtoend.restype = ctypes.c_int
    lib.oracle_endtoend.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.POINTER(_Result)]
    res = _Result()
    rc = lib.oracle_endtoend(q.ctypes.data if q.size else None, q.size,
                             r.ctypes.data if r.size else None, r.size, M.ctypes.data,
                             M.shape[0], int(gap_open), int(gap_extend), int(mode),
                             ctypes.byref(res))
    if rc != 0:
        raise ValueError("oracle_endtoend failed (%d)" % rc)
    return int(res.score), int(res.query_end), int(res.ref_end)


def endtoend_batch(query_res, query_off, ref_res, ref_off, pair_ref, matrix, gap_open: int,
                   gap_extend: int, mode: int, pair_query=None, pairs=None) -> np.ndarray:
    """``endtoend`` for every pair (or the listed ``pairs``) of a CSR batch:
    an (n, 3) int64 array."""
    qo, ro = np.asarray(query_off), np.asarray(ref_off)
    pr = np.asarray(pair_ref)
    idx = range(pr.size) if pairs is None else pairs
    out = []
    for k in idx:
        qi = 0 if pair_query is None else int(pair_query[k])
        ri = int(pr[k])
        out.append(endtoend(query_res[qo[qi]:qo[qi + 1]], ref_res[ro[ri]:ro[ri + 1]], matrix,
                            gap_open, gap_extend, mode))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def endtoend_path(query, ref, matrix, gap_open: int, gap_extend: int, mode: int, end=None):
    """(query_start, ref_start, runs) of the end-to-end alignment (modes as in
    ``endtoend``) reported by ``endtoend`` (or ending at ``end`` = (score,
    query_end, ref_end)): walking back from its end, each predecessor is the
    largest (ref, query) element -- aligned pair or virtual start element:
    (-1, -1) globally, (v, -1) for a free reference prefix r[0..v] in modes 1
    and 3, (-1, w) for a free query prefix q[0..w] in modes 2 and 3 -- on an
    optimal chain; between two elements D is written before I.  The starts are
    the start element's coordinates plus one.  From ``oracle_endtoend_path`` in
    sw_oracle.c (plain maxima over the chains)."""
    q, r = _u8(query), _u8(ref)
    M = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    s, qe, re_ = endtoend(q, r, M, gap_open, gap_extend, mode) if end is None else end
    cap = q.size + r.size + 2
    ops = np.zeros(cap, dtype=np.uint32)
    qs, rs = ctypes.c_int64(0), ctypes.c_int64(0)
    lib = _load()
    lib.oracle_endtoend_path.restype = ctypes.c_int64
    lib.oracle_endtoend_path.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]
    n = lib.oracle_endtoend_path(q.ctypes.data if q.size else None, q.size,
                                 r.ctypes.data if r.size else None, r.size, M.ctypes.data,
                                 M.shape[0], int(gap_open), int(gap_extend), int(mode), int(qe),
                                 int(re_), int(s), ops.ctypes.data, cap, ctypes.byref(qs),
                                 ctypes.byref(rs))
    if n < 0:
        raise ValueError("oracle_endtoend_path failed (%d)" % n)
    return int(qs.value), int(rs.value), [(int(v >> 4), _OPS[int(v & 15)]) for v in ops[:n]]
