"""Serving loop on the GPU: continuous batching must give, for every request,
exactly the oracle's (and the batch path's) result, alone or in any mix."""
import numpy as np
import pytest

import oracle
from paper_1909_00899_amd import api, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def db():
    return W.serving_db(n_protein=300, n_dna=300, seed=4)


def _scorings():
    return [(W.protein_matrix(), 11, 1), (W.dna_matrix(), 6, 1)]


def _oracle_requests(db, reqs):
    sc = _scorings()
    want = []
    for k in range(reqs.ref_id.size):
        q = reqs.query_res[reqs.query_off[k]:reqs.query_off[k + 1]]
        r = db.ref_res[db.ref_off[reqs.ref_id[k]]:db.ref_off[reqs.ref_id[k] + 1]]
        M, go, ge = sc[1 if reqs.is_dna[k] else 0]
        want.append(oracle.align(q, r, M, go, ge))
    return np.array(want, dtype=np.int64)


def test_replay_mixed_matches_oracle_and_batch(db):
    # the full DNA length range of the serving workload (100 - 10000 bp)
    reqs = W.serving_requests(db, rate_per_s=20000, n_requests=240, seed=41, dna_len=(100, 10_000))
    dlens = np.diff(reqs.query_off)[reqs.is_dna]
    assert dlens.max() > 8000
    want = _oracle_requests(db, reqs)
    sid = reqs.is_dna.astype(np.int32)
    with api.Server(db.ref_res, db.ref_off, _scorings(), n_streams=4, max_batch=64) as srv:
        out, ts = srv.replay(reqs.query_res, reqs.query_off, reqs.ref_id, sid, reqs.arrival_s)
    assert (out[:, :3] == want).all()
    assert (ts[:, 2] >= ts[:, 1]).all() and (ts[:, 1] >= ts[:, 0] - 1000).all()
    # the same pairs alone (one request per server batch) and as one offline batch
    with api.Server(db.ref_res, db.ref_off, _scorings(), n_streams=1, max_batch=1) as srv:
        for k in (0, 5, 17, 99):
            q = reqs.query_res[reqs.query_off[k]:reqs.query_off[k + 1]]
            t = srv.submit(q, int(reqs.ref_id[k]), int(sid[k]))
            srv.drain()
            r = srv.poll(t)
            assert tuple(r[:3]) == tuple(want[k])
    prot = np.nonzero(~reqs.is_dna)[0]
    M, go, ge = _scorings()[0]
    pq = prot.astype(np.int32)
    got = api.sw_align_batch(reqs.query_res, reqs.query_off, db.ref_res, db.ref_off,
                             reqs.ref_id[prot].astype(np.int32), M, go, ge, pair_query=pq)
    assert (got.results[:, :3] == want[prot]).all()


def test_budget_admission_and_errors(db):
    reqs = W.serving_requests(db, rate_per_s=5000, n_requests=40, seed=42, dna_len=(100, 600))
    want = _oracle_requests(db, reqs)
    sid = reqs.is_dna.astype(np.int32)
    # a budget that admits only about one request at a time still completes all
    with api.Server(db.ref_res, db.ref_off, _scorings(), hbm_budget_bytes=80_000,
                    n_streams=3) as srv:
        big = np.zeros(90_000, dtype=np.uint8)
        with pytest.raises(api.SwError) as e:
            srv.submit(big, 0, 0)
        assert e.value.code == api.SW_ENOMEM
        tickets = [srv.submit(reqs.query_res[reqs.query_off[k]:reqs.query_off[k + 1]],
                              int(reqs.ref_id[k]), int(sid[k])) for k in range(40)]
        srv.drain()
        for k, t in enumerate(tickets):
            assert tuple(srv.poll(t)[:3]) == tuple(want[k])
            with pytest.raises(api.SwError) as e:
                srv.poll(t)                      # already collected
            assert e.value.code == api.SW_ENOENT
        with pytest.raises(api.SwError) as e:
            srv.poll(123456789)
        assert e.value.code == api.SW_ENOENT
        with pytest.raises(api.SwError) as e:
            srv.submit([0, 1], 10 ** 6, 0)
        assert e.value.code == api.SW_EINVAL
        with pytest.raises(api.SwError) as e:
            srv.submit([0, 25], 0, 0)           # residue outside the alphabet
        assert e.value.code == api.SW_EINVAL
        # a protein reference (codes up to 19) under the 4-letter DNA scoring
        assert db.ref_res[db.ref_off[0]:db.ref_off[1]].max() >= 4
        with pytest.raises(api.SwError) as e:
            srv.submit([0, 1, 2], 0, 1)
        assert e.value.code == api.SW_EINVAL
        # the same reference under its own scoring is accepted
        t = srv.submit([0, 1, 2], 0, 0)
        srv.drain()
        q = np.array([0, 1, 2], dtype=np.uint8)
        r = db.ref_res[db.ref_off[0]:db.ref_off[1]]
        assert tuple(srv.poll(t)[:3]) == tuple(oracle.align(q, r, *_scorings()[0]))


def test_replay_backlog_fifo_per_class_and_exact(db):
    # every request offered at once with small batches: a deep backlog in
    # every class.  Each class (scoring, and whether the request is long: a
    # query over 1024 residues or over 2^20 cells) is admitted in arrival
    # order, and every result equals the offline batch call's; a sample is
    # checked against the oracle as well
    reqs = W.serving_requests(db, rate_per_s=1e9, n_requests=1500, seed=43, dna_len=(100, 3000))
    sid = reqs.is_dna.astype(np.int32)
    with api.Server(db.ref_res, db.ref_off, _scorings(), n_streams=4, max_batch=48) as srv:
        out, ts = srv.replay(reqs.query_res, reqs.query_off, reqs.ref_id, sid, reqs.arrival_s)
    m = np.diff(reqs.query_off)
    n = np.diff(db.ref_off)[reqs.ref_id]
    cls = 2 * sid + ((m > 1024) | (m * n > (1 << 20)))
    assert len(np.unique(cls)) == 4
    for c in np.unique(cls):
        assert (np.diff(ts[cls == c, 1]) >= 0).all()
    for dna in (False, True):
        # one family's queries and references (the batch call checks every
        # residue it is given)
        sel = np.nonzero(reqs.is_dna == dna)[0]
        qs = [reqs.query_res[reqs.query_off[k]:reqs.query_off[k + 1]] for k in sel]
        qoff = np.zeros(sel.size + 1, dtype=np.int64)
        np.cumsum([q.size for q in qs], out=qoff[1:])
        r0, r1 = (db.n_protein, db.n_protein + db.n_dna) if dna else (0, db.n_protein)
        rres = db.ref_res[db.ref_off[r0]:db.ref_off[r1]]
        roff = db.ref_off[r0:r1 + 1] - db.ref_off[r0]
        M, go, ge = _scorings()[1 if dna else 0]
        got = api.sw_align_batch(np.concatenate(qs), qoff, rres, roff,
                                 (reqs.ref_id[sel] - r0).astype(np.int32), M, go, ge,
                                 pair_query=np.arange(sel.size, dtype=np.int32))
        assert (out[sel, :3] == got.results[:, :3]).all()
    for k in range(0, 1500, 75):
        q = reqs.query_res[reqs.query_off[k]:reqs.query_off[k + 1]]
        r = db.ref_res[db.ref_off[reqs.ref_id[k]]:db.ref_off[reqs.ref_id[k] + 1]]
        M, go, ge = _scorings()[1 if reqs.is_dna[k] else 0]
        assert tuple(out[k, :3]) == tuple(oracle.align(q, r, M, go, ge))
