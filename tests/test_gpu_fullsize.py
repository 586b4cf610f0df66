"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (device-resident inputs, the device planner, results into a pinned host
array, graph replays): every one of the 100k protein-search results and the
1M DNA-pair results equals the CPU oracle's."""
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


def _bench_configuration(w):
    import torch
    dev = torch.device("cuda")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    args = (t(w.query_res, torch.uint8), t(w.query_off, torch.int64), t(w.ref_res, torch.uint8),
            t(w.ref_off, torch.int64), t(w.pair_ref, torch.int32))
    pq = None if w.pair_query is None else t(w.pair_query, torch.int32)
    pinned = torch.empty((w.n_pairs, 4), dtype=torch.int32, pin_memory=True).numpy()
    runs = []
    for graph in (0, 1, 1):
        pinned.fill(-7)
        o = api.sw_align_batch(*args, w.matrix, w.gap_open, w.gap_extend, pair_query=pq,
                               use_graph=graph, out=pinned)
        assert o.stats["planner_used"] == 2
        runs.append(pinned.copy())
    return runs


def _check(w, label):
    want = oracle.align_batch(w.query_res, w.query_off, w.ref_res, w.ref_off, w.pair_ref,
                              w.matrix, w.gap_open, w.gap_extend, pair_query=w.pair_query)
    for k, got in enumerate(_bench_configuration(w)):
        bad = np.nonzero((got[:, :3] != want).any(axis=1))[0]
        assert bad.size == 0, "%s run %d: %d mismatches, first pair %d got %s want %s" % (
            label, k, bad.size, bad[0], got[bad[0]].tolist(), want[bad[0]].tolist())
        assert (got[:, 3] == 0).all()          # no int16 saturation at these scores


def test_protein_search_full_size():
    _check(W.protein_search(), "protein search 512 x 100k")


def test_dna_pairs_full_size():
    _check(W.dna_pairs(n_pairs=1_000_000), "dna pairs 1M")
