"""Seeded synthetic inputs for the alignment workloads.

This module only draws random sequences, matrices and arrival times.  It holds
none of the alignment arithmetic, so both the HIP path and the CPU oracle can
take their inputs from it.  Every generator is deterministic given its seed
(numpy ``default_rng``); integer ranges are inclusive.

The paper measures on mate-rescue alignments of a human whole-genome sample,
which are not available here; these seeded inputs stand in for them with the
shapes, sizes and value distributions of the five benchmark workloads:

* ``single_pair``      256-residue protein query vs a 1024-residue reference.
* ``protein_search``   one 512-residue query vs 100k log-normal references.
* ``dna_pairs``        1M pairs of a mutated 150 bp read vs its 300-600 bp window.
* ``long_queries``     64 queries of 5k-35k residues vs 10k references, half of
                       them built from low-complexity runs.
* ``serving_*``        a resident protein + DNA database and Poisson requests.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PROTEIN_ALPHA = 20
DNA_ALPHA = 4


@dataclass
class Workload:
    """A batch of (query, reference) pairs in CSR form plus one scoring scheme."""
    name: str
    query_res: np.ndarray          # uint8 residue codes, all queries concatenated
    query_off: np.ndarray          # int64, n_queries + 1
    ref_res: np.ndarray            # uint8
    ref_off: np.ndarray            # int64, n_refs + 1
    pair_query: Optional[np.ndarray]  # int32 per pair, None => query 0
    pair_ref: np.ndarray           # int32 per pair
    matrix: np.ndarray             # int32 alpha x alpha, [query code][ref code]
    gap_open: int
    gap_extend: int
    meta: dict = field(default_factory=dict)

    @property
    def n_pairs(self) -> int:
        return int(self.pair_ref.size)

    @property
    def alphabet(self) -> int:
        return int(self.matrix.shape[0])

    def query_lengths(self) -> np.ndarray:
        return np.diff(self.query_off)

    def ref_lengths(self) -> np.ndarray:
        return np.diff(self.ref_off)

    def cells(self) -> int:
        """Real DP cells (sum of m * n over pairs): the GCUPS numerator."""
        ql = self.query_lengths()
        rl = self.ref_lengths()
        pq = np.zeros(self.n_pairs, dtype=np.int64) if self.pair_query is None else self.pair_query
        return int(np.sum(ql[pq].astype(np.int64) * rl[self.pair_ref].astype(np.int64)))

    def pair(self, k: int):
        qi = 0 if self.pair_query is None else int(self.pair_query[k])
        ri = int(self.pair_ref[k])
        q = self.query_res[self.query_off[qi]:self.query_off[qi + 1]]
        r = self.ref_res[self.ref_off[ri]:self.ref_off[ri + 1]]
        return q, r

    def subset(self, idx, name: Optional[str] = None) -> "Workload":
        """Same sequences, only the pairs listed in ``idx``."""
        idx = np.asarray(idx, dtype=np.int64)
        return Workload(name or (self.name + "_subset"), self.query_res, self.query_off,
                        self.ref_res, self.ref_off,
                        None if self.pair_query is None else self.pair_query[idx].copy(),
                        self.pair_ref[idx].copy(), self.matrix, self.gap_open,
                        self.gap_extend, dict(self.meta))


def _csr(seqs):
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    off = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    res = np.concatenate([np.asarray(s, dtype=np.uint8) for s in seqs]) if seqs else \
        np.zeros(0, dtype=np.uint8)
    return res, off


def protein_matrix(seed: int = 10_000) -> np.ndarray:
    """Seeded symmetric 20x20 matrix: diagonal U{4..11}, off-diagonal U{-4..3}.

    The 20 diagonal entries are drawn first, then the 190 upper-triangle
    entries in row-major order, mirrored to the lower triangle.
    """
    rng = np.random.default_rng(seed)
    M = np.zeros((PROTEIN_ALPHA, PROTEIN_ALPHA), dtype=np.int32)
    diag = rng.integers(4, 11, size=PROTEIN_ALPHA, endpoint=True)
    upper = rng.integers(-4, 3, size=PROTEIN_ALPHA * (PROTEIN_ALPHA - 1) // 2, endpoint=True)
    M[np.diag_indices(PROTEIN_ALPHA)] = diag
    iu = np.triu_indices(PROTEIN_ALPHA, k=1)
    M[iu] = upper
    M[(iu[1], iu[0])] = upper
    return M


def dna_matrix(match: int = 1, mismatch: int = -4) -> np.ndarray:
    M = np.full((DNA_ALPHA, DNA_ALPHA), mismatch, dtype=np.int32)
    np.fill_diagonal(M, match)
    return M


def single_pair(m: int = 256, n: int = 1024, seed: int = 0) -> Workload:
    """Plain single pair: i.i.d. uniform 20-letter query (drawn first) and reference."""
    rng = np.random.default_rng(seed)
    q = rng.integers(0, PROTEIN_ALPHA, size=m, dtype=np.uint8)
    r = rng.integers(0, PROTEIN_ALPHA, size=n, dtype=np.uint8)
    qres, qoff = _csr([q])
    rres, roff = _csr([r])
    return Workload("single_pair_%dx%d" % (m, n), qres, qoff, rres, roff, None,
                    np.zeros(1, dtype=np.int32), protein_matrix(), 11, 1,
                    {"seed": seed})


def _lognormal_lengths(rng, count, median=350.0, sigma=0.6, lo=50, hi=5000):
    x = np.exp(rng.normal(np.log(median), sigma, size=count))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def protein_search(n_refs: int = 100_000, m: int = 512, seed: int = 1,
                   sigma: float = 0.6) -> Workload:
    """One query vs many references with non-uniform letter frequencies.

    Frequencies f ~ Dirichlet(2 * ones(20)); query of m residues ~ f; reference
    lengths round(exp(N(ln 350, sigma))) clipped to [50, 5000]; residues ~ f.
    """
    rng = np.random.default_rng(seed)
    f = rng.dirichlet(2.0 * np.ones(PROTEIN_ALPHA))
    q = rng.choice(PROTEIN_ALPHA, size=m, p=f).astype(np.uint8)
    lens = _lognormal_lengths(rng, n_refs, sigma=sigma)
    total = int(lens.sum())
    res = rng.choice(PROTEIN_ALPHA, size=total, p=f).astype(np.uint8)
    roff = np.zeros(n_refs + 1, dtype=np.int64)
    np.cumsum(lens, out=roff[1:])
    qres, qoff = _csr([q])
    return Workload("protein_search_%dx%d" % (m, n_refs), qres, qoff, res, roff, None,
                    np.arange(n_refs, dtype=np.int32), protein_matrix(), 11, 1,
                    {"seed": seed, "freqs": f})


def _mutate_reads(rng, ref_res, ref_off, read_len, sub_p, del_p, ins_p, max_pos):
    """Vectorised read simulation for one chunk of references.

    For each reference a start s ~ U{0..L-read_len-10} is drawn; the reference
    is streamed from s: a uniform random base is inserted before a position
    with probability ins_p, the position is deleted with probability del_p,
    otherwise emitted, substituted by one of the other three bases with
    probability sub_p.  The read is the first ``read_len`` emitted bases.
    Pairs whose window runs out are redrawn.
    """
    n = ref_off.size - 1
    L = np.diff(ref_off)
    out = np.zeros((n, read_len), dtype=np.uint8)
    todo = np.arange(n)
    while todo.size:
        Lt = L[todo]
        s = rng.integers(0, Lt - (read_len + 10), endpoint=True)
        K = max_pos
        pos = s[:, None] + np.arange(K)[None, :]
        inwin = pos < Lt[:, None]
        pos = np.minimum(pos, Lt[:, None] - 1)
        base = ref_res[ref_off[todo][:, None] + pos]
        u = rng.random((todo.size, K, 3))
        ins = u[:, :, 0] < ins_p
        dele = u[:, :, 1] < del_p
        sub = u[:, :, 2] < sub_p
        ins_base = rng.integers(0, 4, size=(todo.size, K), dtype=np.uint8)
        shift = rng.integers(1, 3, size=(todo.size, K), endpoint=True).astype(np.uint8)
        emitted = np.where(sub, (base + shift) % 4, base).astype(np.uint8)
        sym = np.stack([ins_base, emitted], axis=2).reshape(todo.size, 2 * K)
        valid = np.stack([ins & inwin, (~dele) & inwin], axis=2).reshape(todo.size, 2 * K)
        cum = np.cumsum(valid, axis=1)
        ok = cum[:, -1] >= read_len
        take = valid & (cum <= read_len)
        rows = np.nonzero(ok)[0]
        if rows.size:
            sel = sym[rows][take[rows]].reshape(rows.size, read_len)
            out[todo[rows]] = sel
        todo = todo[~ok]
    return out


def dna_pairs(n_pairs: int = 1_000_000, read_len: int = 150, seed: int = 2,
              chunk: int = 100_000) -> Workload:
    """Mutated reads vs their reference windows (DNA, +1/-4, GapOpen 6, GapExtend 1).

    Windows L ~ U{300..600}, ACGT uniform.  Each read is a substring of its
    window with 2% substitutions and 0.5% indels (split evenly between length-1
    insertions and deletions).  Pair k is (query k, reference k).
    """
    rng = np.random.default_rng(seed)
    L = rng.integers(300, 600, size=n_pairs, endpoint=True).astype(np.int64)
    roff = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(L, out=roff[1:])
    rres = rng.integers(0, 4, size=int(roff[-1]), dtype=np.uint8)
    reads = np.zeros((n_pairs, read_len), dtype=np.uint8)
    for a in range(0, n_pairs, chunk):
        b = min(n_pairs, a + chunk)
        sub_off = roff[a:b + 1] - roff[a]
        reads[a:b] = _mutate_reads(rng, rres[roff[a]:roff[b]], sub_off, read_len,
                                   0.02, 0.0025, 0.0025, read_len + 40)
    qoff = np.arange(n_pairs + 1, dtype=np.int64) * read_len
    idx = np.arange(n_pairs, dtype=np.int32)
    return Workload("dna_pairs_%d" % n_pairs, reads.reshape(-1), qoff, rres, roff, idx,
                    idx.copy(), dna_matrix(), 6, 1, {"seed": seed})


def _runs_sequence(rng, length, alpha, run_lo=50, run_hi=500):
    """Low-complexity sequence: runs of one letter, lengths U{run_lo..run_hi},
    each letter uniform and different from the previous run's, truncated."""
    out = np.empty(length, dtype=np.uint8)
    pos, prev = 0, -1
    while pos < length:
        k = int(rng.integers(run_lo, run_hi, endpoint=True))
        if prev < 0:
            c = int(rng.integers(0, alpha))
        else:
            c = int(rng.integers(0, alpha - 1))
            if c >= prev:
                c += 1
        out[pos:pos + k] = c
        pos += k
        prev = c
    return out


def long_queries(n_queries: int = 64, n_refs: int = 10_000, seed: int = 3,
                 qlen=(5000, 35000), rlen=(200, 2000)) -> Workload:
    """Long and adversarial queries vs many references (protein matrix, int32).

    Query lengths U{5000..35000}; the first half i.i.d. uniform, the second half
    built from poly-residue runs of 50-500.  Reference lengths U{200..2000};
    the first half i.i.d., the second half runs.  All query x reference pairs.
    """
    rng = np.random.default_rng(seed)
    ql = rng.integers(qlen[0], qlen[1], size=n_queries, endpoint=True)
    queries = []
    for k in range(n_queries):
        if k < n_queries // 2:
            queries.append(rng.integers(0, PROTEIN_ALPHA, size=int(ql[k]), dtype=np.uint8))
        else:
            queries.append(_runs_sequence(rng, int(ql[k]), PROTEIN_ALPHA))
    rl = rng.integers(rlen[0], rlen[1], size=n_refs, endpoint=True)
    refs = []
    for k in range(n_refs):
        if k < n_refs // 2:
            refs.append(rng.integers(0, PROTEIN_ALPHA, size=int(rl[k]), dtype=np.uint8))
        else:
            refs.append(_runs_sequence(rng, int(rl[k]), PROTEIN_ALPHA))
    qres, qoff = _csr(queries)
    rres, roff = _csr(refs)
    pq = np.repeat(np.arange(n_queries, dtype=np.int32), n_refs)
    pr = np.tile(np.arange(n_refs, dtype=np.int32), n_queries)
    return Workload("long_queries_%dx%d" % (n_queries, n_refs), qres, qoff, rres, roff, pq, pr,
                    protein_matrix(), 11, 1, {"seed": seed, "adversarial_from_query": n_queries // 2,
                                              "adversarial_from_ref": n_refs // 2})


def long_queries_subset(w: Workload, per_query: int = 8, seed: int = 33) -> Workload:
    """Seeded subset: per query, per_query/2 i.i.d. references and per_query/2 run references."""
    rng = np.random.default_rng(seed)
    n_refs = w.ref_off.size - 1
    n_queries = w.query_off.size - 1
    half = n_refs // 2
    idx = []
    for qi in range(n_queries):
        a = rng.choice(half, size=per_query // 2, replace=False)
        b = half + rng.choice(n_refs - half, size=per_query - per_query // 2, replace=False)
        for ri in np.concatenate([a, b]):
            idx.append(qi * n_refs + int(ri))
    return w.subset(np.array(idx), name=w.name + "_subset%d" % len(idx))


@dataclass
class ServingDB:
    """Resident references: a protein family and a DNA family."""
    ref_res: np.ndarray
    ref_off: np.ndarray
    n_protein: int
    n_dna: int
    protein_freqs: np.ndarray


def serving_db(n_protein: int = 25_000, n_dna: int = 25_000, seed: int = 4) -> ServingDB:
    rng = np.random.default_rng(seed)
    f = rng.dirichlet(2.0 * np.ones(PROTEIN_ALPHA))
    plen = _lognormal_lengths(rng, n_protein)
    prot = rng.choice(PROTEIN_ALPHA, size=int(plen.sum()), p=f).astype(np.uint8)
    dlen = rng.integers(300, 600, size=n_dna, endpoint=True).astype(np.int64)
    dna = rng.integers(0, DNA_ALPHA, size=int(dlen.sum()), dtype=np.uint8)
    lens = np.concatenate([plen, dlen])
    off = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return ServingDB(np.concatenate([prot, dna]), off, n_protein, n_dna, f)


@dataclass
class ServingRequests:
    arrival_s: np.ndarray      # float64 seconds from the start, nondecreasing
    is_dna: np.ndarray         # bool
    query_res: np.ndarray
    query_off: np.ndarray
    ref_id: np.ndarray         # int32 index into the resident DB


def serving_requests(db: ServingDB, rate_per_s: float, n_requests: int,
                     seed: int = 40, dna_len=(100, 10_000)) -> ServingRequests:
    """Open-loop Poisson arrivals; each request is protein or DNA with prob. 1/2.

    Protein query lengths log-normal (median 350, sigma 0.6, clipped [50, 5000])
    with the DB's letter frequencies, scored against one uniformly drawn protein
    reference.  DNA query lengths U{100..10000}, uniform bases, scored against
    one uniformly drawn DNA reference.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    arrival = np.cumsum(gaps)
    is_dna = rng.random(n_requests) < 0.5
    plen = _lognormal_lengths(rng, n_requests)
    dlen = rng.integers(dna_len[0], dna_len[1], size=n_requests, endpoint=True)
    lens = np.where(is_dna, dlen, plen).astype(np.int64)
    off = np.zeros(n_requests + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    res = np.empty(int(off[-1]), dtype=np.uint8)
    prot_draw = rng.choice(PROTEIN_ALPHA, size=int(off[-1]), p=db.protein_freqs).astype(np.uint8)
    dna_draw = rng.integers(0, DNA_ALPHA, size=int(off[-1]), dtype=np.uint8)
    mask = np.repeat(is_dna, lens)
    res[:] = np.where(mask, dna_draw, prot_draw)
    pref = rng.integers(0, db.n_protein, size=n_requests)
    dref = db.n_protein + rng.integers(0, db.n_dna, size=n_requests)
    ref_id = np.where(is_dna, dref, pref).astype(np.int32)
    return ServingRequests(arrival, is_dna, res, off, ref_id)


def random_pairs(n_pairs: int, alpha: int, mlen, nlen, seed: int,
                 matrix: Optional[np.ndarray] = None, gap_open: int = 11,
                 gap_extend: int = 1) -> Workload:
    """Independent random pairs with uniform lengths (for tests of edge shapes)."""
    rng = np.random.default_rng(seed)
    ml = rng.integers(mlen[0], mlen[1], size=n_pairs, endpoint=True)
    nl = rng.integers(nlen[0], nlen[1], size=n_pairs, endpoint=True)
    qs = [rng.integers(0, alpha, size=int(k), dtype=np.uint8) for k in ml]
    rs = [rng.integers(0, alpha, size=int(k), dtype=np.uint8) for k in nl]
    qres, qoff = _csr(qs)
    rres, roff = _csr(rs)
    if matrix is None:
        matrix = protein_matrix() if alpha == PROTEIN_ALPHA else random_matrix(rng, alpha)
    idx = np.arange(n_pairs, dtype=np.int32)
    return Workload("random_pairs_%d" % n_pairs, qres, qoff, rres, roff, idx, idx.copy(),
                    np.asarray(matrix, dtype=np.int32), gap_open, gap_extend, {"seed": seed})


def random_matrix(rng, alpha: int, lo: int = -4, hi: int = 5, symmetric: bool = False) -> np.ndarray:
    M = rng.integers(lo, hi, size=(alpha, alpha), endpoint=True).astype(np.int32)
    if symmetric:
        M = np.triu(M) + np.triu(M, 1).T
    return M
