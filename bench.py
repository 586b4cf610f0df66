"""Benchmark: batched striped-scan Smith-Waterman on one MI355X.

One step = one sw_align_batch call over the protein-search workload (one
512-residue query vs 100k log-normal references, inputs resident in HBM as
torch tensors): the device planner (pair checks, length ordering and task
packing on the GPU), the persistent int16x2 scan kernel and any int32 reruns,
results copied back.  The call's device work is replayed from a hipGraph
captured during warm-up (identical parameters every step); an eager leg of the
same steps gives the per-launch kernel time for the roofline, and a leg with
the host planner is timed beside it.  The autotuner picks the tile shapes
before the timed region.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain] [--no-serve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS (bit-exact) batched vs plain kernel on one MI355X; p99 latency served"
# Integer VALU peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12
# lane-ops/s for 32-bit ops; packed int16x2 ops do two per lane.
PEAK_I32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PEAK_I16X2_TOPS = 2 * PEAK_I32_TOPS
OPS_PER_CELL = 11   # Algorithm 6 inner loop: 1 add, 6 max, 4 sub
# the alignment kernel of a device-planned int16 single-query batch
KERNEL_NAME = "shared_rowpair_kernel<16, true, false>"


# sources that define the protein-search kernel and its launch: the counter
# summary stays valid while none of them changes
TRAFFIC_SOURCES = ("sw_device.h", "sw_internal.h", "sw_menus.h", "sw_shared_i16.hip",
                   "sw_devplan.cpp")


def _csrc_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(ROOT, "paper_1909_00899_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def _measured_traffic():
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_shared_rowpair_kernel_protein_search.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    return d["hbm_bytes_per_launch"] if d.get("csrc_sha256") == _csrc_sha256() else None


def _probe_peak():
    """Sustained int16x2 VALU rate measured by the probe library (Tops/s), or
    None when it cannot run."""
    try:
        from paper_1909_00899_amd import valu_probe
        return valu_probe.measure() / 1e12
    except (OSError, RuntimeError):
        return None


def _with_measured_peak(roof: dict) -> dict:
    mp = _probe_peak()
    roof["measured_peak"] = None if mp is None else round(mp, 2)
    roof["frac_of_measured_peak"] = None if mp is None else round(roof["achieved"] / mp, 4)
    return roof


def copy_calibration():
    """A plain device copy of 256 MiB, three launches: the known byte count
    against which the HBM counters (FETCH_SIZE, WRITE_SIZE) are scaled."""
    import torch
    n = 256 * 1024 * 1024
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}))


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--n-refs", type=int, default=100_000)
    ap.add_argument("--workload", default="protein_search",
                    choices=["protein_search", "dna_pairs", "long_queries", "serving",
                             "copy_calibration"])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy_calibration":
        return copy_calibration()
    if args.workload == "long_queries":
        return bench_long_queries(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "dna_pairs":
        return bench_dna(args)

    import torch
    from paper_1909_00899_amd import api, workloads as W

    api.load()
    api.sw_init(0)
    dev = torch.device("cuda:0")
    w = W.protein_search(n_refs=args.n_refs)
    cells = w.cells()
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    d = dict(qres=t(w.query_res, torch.uint8), qoff=t(w.query_off, torch.int64),
             rres=t(w.ref_res, torch.uint8), roff=t(w.ref_off, torch.int64),
             pref=t(w.pair_ref, torch.int32))
    torch.cuda.synchronize()

    # tile shapes (lanes per alignment, rows per lane) from the autotuner,
    # measured on this batch before the timed region
    ta = time.perf_counter()
    tuned = api.sw_autotune(d["qres"], d["qoff"], d["rres"], d["roff"], d["pref"], w.matrix,
                            w.gap_open, w.gap_extend) if not args.no_tune else []
    tune_s = time.perf_counter() - ta

    # results land in a pinned host buffer, as a throughput-minded caller
    # would provide (a pageable array is timed beside it)
    pinned = torch.empty((w.n_pairs, 4), dtype=torch.int32, pin_memory=True).numpy()

    def step(graph=0, out=pinned):
        return api.sw_align_batch(d["qres"], d["qoff"], d["rres"], d["roff"], d["pref"],
                                  w.matrix, w.gap_open, w.gap_extend, use_graph=graph, out=out)

    use_graph = 0 if args.no_graph else 1
    for _ in range(args.warmup):
        out = step()
    if use_graph:
        step(1)                      # capture; later identical calls replay it
    torch.cuda.synchronize()
    # eager leg: per-launch kernel time of the alignment kernel (HIP events on
    # the library's stream) for the roofline
    kern_ms = []
    te = time.perf_counter()
    for _ in range(args.steps):
        out = step()
        kern_ms.append(out.stats["kernel_ms"])
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - te) / args.steps * 1e3
    out = api.BatchOutput(out.results.copy(), out.stats)   # the pinned buffer is reused
    # timed region: K whole calls whose device work replays the captured graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        og = step(use_graph)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    gcups = cells / (wall / args.steps) / 1e9
    kms = float(np.mean(kern_ms))
    og_results = og.results.copy()
    tp = time.perf_counter()
    for _ in range(args.steps):
        op = step(use_graph, out=None)
    torch.cuda.synchronize()
    pageable_ms = (time.perf_counter() - tp) / args.steps * 1e3
    achieved_tops = cells * OPS_PER_CELL / (kms / 1e3) / 1e12

    rec = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i16x2",
        "data": "synthetic",
        "config": {"workload": "protein_search: 512-residue query vs 100k refs "
                               "(log-normal median 350, clipped 50-5000), int16x2 + int32 rerun",
                   "pairs": w.n_pairs, "cells": cells, "query_len": 512},
        "roofline": _with_measured_peak(
            {"bound": "alu", "kernel": KERNEL_NAME, "achieved": round(achieved_tops, 3),
             "peak": round(PEAK_I16X2_TOPS, 2), "unit": "Tops/s",
             "frac": round(achieved_tops / PEAK_I16X2_TOPS, 4),
             "traffic": _measured_traffic(),
             "ops_per_cell": OPS_PER_CELL, "kernel_ms": round(kms, 4),
             "kernel_gcups": round(cells / (kms / 1e3) / 1e9, 2)}),
        "stats": {k: out.stats[k] for k in ("n_rerun", "n_launches", "lanes_used",
                                            "seglen_max", "padded_cells", "total_ms", "prep_ms",
                                            "plan_ms", "launch_ms", "finish_ms", "columns",
                                            "record_events", "planner_used")},
        "tuned": {"seconds": round(tune_s, 3),
                  "entries": [{k: (round(v, 1) if isinstance(v, float) else v)
                               for k, v in e.items()} for e in tuned]},
    }
    rec["eager"] = {"ms_per_step": round(eager_ms, 3), "gcups": round(cells / eager_ms / 1e6, 2)}
    # the same calls with the host planner (offsets read back, pairs sorted and
    # packed on the host, residue streams built on the device)
    for _ in range(2):
        oh = api.sw_align_batch(d["qres"], d["qoff"], d["rres"], d["roff"], d["pref"], w.matrix,
                                w.gap_open, w.gap_extend, planner=1)
    torch.cuda.synchronize()
    th = time.perf_counter()
    for _ in range(args.steps):
        oh = api.sw_align_batch(d["qres"], d["qoff"], d["rres"], d["roff"], d["pref"], w.matrix,
                                w.gap_open, w.gap_extend, planner=1)
    torch.cuda.synchronize()
    host_ms = (time.perf_counter() - th) / args.steps * 1e3
    rec["host_planner"] = {"ms_per_step": round(host_ms, 3),
                           "gcups": round(cells / host_ms / 1e6, 2),
                           "kernel_ms": round(oh.stats["kernel_ms"], 4),
                           "same_results": bool(np.array_equal(oh.results, out.results))}
    rec["graph"] = {"used": bool(use_graph), "graph_hits": og.stats["graph_hits"],
                    "same_results_as_eager": bool(np.array_equal(og_results, out.results))}
    rec["pageable_out"] = {"ms_per_step": round(pageable_ms, 3),
                           "gcups": round(cells / pageable_ms / 1e6, 2),
                           "same_results": bool(np.array_equal(op.results, og_results))}
    # start cells of the same alignments: the reversed prefixes ending at every
    # end cell through the batch path (one query per pair)
    api.sw_align_batch_starts(d["qres"], d["qoff"], d["rres"], d["roff"], d["pref"], w.matrix,
                              w.gap_open, w.gap_extend, out.results)
    n_st = max(1, args.steps // 2)
    ts = time.perf_counter()
    for _ in range(n_st):
        qs, rs = api.sw_align_batch_starts(d["qres"], d["qoff"], d["rres"], d["roff"], d["pref"],
                                           w.matrix, w.gap_open, w.gap_extend, out.results)
    st_ms = (time.perf_counter() - ts) / n_st * 1e3
    live = out.results[:, 0] > 0
    pcells = int(((out.results[live, 1].astype(np.int64) + 1) *
                  (out.results[live, 2].astype(np.int64) + 1)).sum())
    rec["starts"] = {"ms_per_call": round(st_ms, 3), "prefix_cells": pcells,
                     "gcups_prefix_cells": round(pcells / st_ms / 1e6, 1),
                     "median_alignment_rows": int(np.median(out.results[live, 1] - qs[live] + 1))}
    rec["paths"] = _paths_leg(api, [d[k] for k in ("qres", "qoff", "rres", "roff", "pref")], None,
                              w, out.results, qs, rs, n_st)

    if not args.no_plain:
        # plain kernel: one 256 x 1024 pair per launch (sw_align_ex: the plain
        # call with the kernel's HIP-event time); the median over 1000 launches
        p = W.single_pair()
        q, r = p.pair(0)
        for _ in range(10):
            api.sw_align_ex(q, r, p.matrix, p.gap_open, p.gap_extend)
        n_pl = 1000
        pk, pw = [], []
        for _ in range(n_pl):
            pres, pst = api.sw_align_ex(q, r, p.matrix, p.gap_open, p.gap_extend)
            pk.append(pst["kernel_ms"])
            pw.append(pst["total_ms"])
        pk_ms = float(np.median(pk))
        pw_ms = float(np.median(pw))
        plain_kernel_gcups = q.size * r.size / (pk_ms / 1e3) / 1e9
        kernel_gcups_batched = cells / (kms / 1e3) / 1e9
        rec["plain"] = {"workload": "single_pair 256x1024 int32, one launch per pair",
                        "launches": n_pl,
                        "kernel_us_median": round(pk_ms * 1e3, 2),
                        "call_us_median": round(pw_ms * 1e3, 2),
                        "kernel_gcups": round(plain_kernel_gcups, 3),
                        "call_gcups": round(q.size * r.size / (pw_ms / 1e3) / 1e9, 3),
                        "batched_over_plain": round(kernel_gcups_batched / plain_kernel_gcups, 1),
                        "same_as_oracle": None}
        if not args.no_cpu:
            import oracle
            rec["plain"]["same_as_oracle"] = bool(
                tuple(pres[:3]) == oracle.align(q, r, p.matrix, p.gap_open, p.gap_extend))

    if not args.no_serve:
        # served latency: a compact open-loop sweep through the server (the
        # full sweep is --workload serving), every result checked against the
        # offline batch call on the same requests
        # (20000 requests per rate: at 200k req/s a shorter run is mostly the
        # tail of its last batches, not the sustained rate; the saturating
        # rate is above the server's capacity, so its achieved rate is the
        # capacity, taken over 100000 requests so that the first, small
        # batches and the last batches' long pairs weigh little against the
        # sustained part)
        rows = _serving_sweep(api, W, [10000, 50000, 200000, SATURATING_RATE],
                              lambda rate: SATURATED_REQUESTS if rate >= SATURATING_RATE else 20000)
        rec["served"] = {"workload": "25k protein + 25k DNA resident refs, Poisson arrivals, "
                                     "20000 requests per rate, 100000 at the saturating rate",
                         "sweep": rows,
                         "served_equals_offline": all(x["served_equals_offline"] for x in rows)}

    if not args.no_cpu:
        import oracle
        # the oracle on the same workload: a bounded sample of references
        n_s = min(w.n_pairs, 20_000)
        sub = w.subset(np.arange(n_s))
        threads = min(16, os.cpu_count() or 1)
        t2 = time.perf_counter()
        want = oracle.align_batch(sub.query_res, sub.query_off, sub.ref_res, sub.ref_off,
                                  sub.pair_ref, sub.matrix, sub.gap_open, sub.gap_extend,
                                  n_threads=threads)
        cs = time.perf_counter() - t2
        # one thread on a smaller sample of the same references
        n_1 = min(w.n_pairs, 2_000)
        sub1 = w.subset(np.arange(n_1))
        t3 = time.perf_counter()
        oracle.align_batch(sub1.query_res, sub1.query_off, sub1.ref_res, sub1.ref_off,
                           sub1.pair_ref, sub1.matrix, sub1.gap_open, sub1.gap_extend, n_threads=1)
        c1 = time.perf_counter() - t3
        rec["cpu_baseline"] = {"value": round(sub.cells() / cs / 1e9, 3), "unit": "GCUPS",
                               "cores": threads, "kind": "oracle",
                               "sample": "first %d of the 100k references (%.2e cells), "
                                         "scalar int64 C oracle, pthreads" % (n_s, sub.cells()),
                               "single_thread": {"value": round(sub1.cells() / c1 / 1e9, 4),
                                                 "unit": "GCUPS",
                                                 "sample": "first %d references (%.2e cells)"
                                                           % (n_1, sub1.cells())},
                               "cpu_model": _cpu_model()}
        rec["parity_sample"] = bool(np.array_equal(out.results[:n_s, :3], want))
    print(json.dumps(rec))


def _paths_leg(api, d, pq, w, ends, qs, rs, reps):
    """sw_align_batch_cigar on the batch's alignments (device-resident
    sequences): whole-call time, rectangle cells per second, run counts."""
    import torch
    call = lambda: api.sw_align_batch_cigar(*d, w.matrix, w.gap_open, w.gap_extend, ends,  # noqa
                                            qs, rs, pair_query=pq)
    runs, off = call()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        runs, off = call()
    ms = (time.perf_counter() - t) / reps * 1e3
    live = ends[:, 0] > 0
    A = (ends[live, 2] - rs[live]).astype(np.int64) + 1
    B = (ends[live, 1] - qs[live]).astype(np.int64) + 1
    cells = int((A * B).sum())
    nr = np.diff(off)[live]
    return {"ms_per_call": round(ms, 3), "alignments": int(live.sum()),
            "rectangle_cells": cells, "gcups_rectangle_cells": round(cells / ms / 1e6, 2),
            "median_rows": int(np.median(A)), "median_cols": int(np.median(B)),
            "runs_total": int(off[-1]), "median_runs": int(np.median(nr)),
            "alignments_per_s": round(live.sum() / ms * 1e3, 1)}


def _endtoend_leg(api, d, pq, w, reps):
    """sw_align_batch_global in every mode on the same pairs (whole calls,
    device-resident sequences): every cell of every pair is computed; the
    reference-fitted mode with the roles swapped (each read, as the
    reference, placed inside its window, as the query)."""
    import torch
    res = {}
    cells = w.cells()
    legs = (("global", api.SW_MODE_GLOBAL, False), ("semiglobal", api.SW_MODE_SEMIGLOBAL, False),
            ("overlap", api.SW_MODE_OVERLAP, False),
            ("semiglobal_ref_swapped", api.SW_MODE_SEMIGLOBAL_REF, True))
    d_fwd, pq_fwd = d, pq
    for name, mode, swapped in legs:
        # swapped: windows as queries, reads as references (same pairs)
        d = [d_fwd[2], d_fwd[3], d_fwd[0], d_fwd[1], pq_fwd] if swapped else d_fwd
        pq = d_fwd[4] if swapped else pq_fwd
        api.sw_align_batch_global(*d, w.matrix, w.gap_open, w.gap_extend, mode=mode, pair_query=pq)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = api.sw_align_batch_global(*d, w.matrix, w.gap_open, w.gap_extend, mode=mode,
                                          pair_query=pq)
        ms = (time.perf_counter() - t) / reps * 1e3
        res[name] = {"ms_per_call": round(ms, 3), "gcups": round(cells / ms / 1e6, 1),
                     "median_score": int(np.median(r[:, 0]))}
        # their paths, from the end cells just found
        api.sw_align_batch_global_cigar(*d, w.matrix, w.gap_open, w.gap_extend, r, mode=mode,
                                        pair_query=pq)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            qs, rs, runs, off = api.sw_align_batch_global_cigar(*d, w.matrix, w.gap_open,
                                                                w.gap_extend, r, mode=mode,
                                                                pair_query=pq)
        pms = (time.perf_counter() - t) / reps * 1e3
        rows = r[:, 2].astype(np.int64) + 1
        pcells = int((rows * (r[:, 1].astype(np.int64) + 1)).sum())
        res[name]["paths"] = {"ms_per_call": round(pms, 3), "cells": pcells,
                              "gcups": round(pcells / pms / 1e6, 1),
                              "median_runs": int(np.median(np.diff(off)))}
    return res


def _device_batch(w):
    import torch
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    d = [t(w.query_res, torch.uint8), t(w.query_off, torch.int64), t(w.ref_res, torch.uint8),
         t(w.ref_off, torch.int64), t(w.pair_ref, torch.int32)]
    pq = None if w.pair_query is None else t(w.pair_query, torch.int32)
    torch.cuda.synchronize()
    return d, pq


def bench_dna(args):
    """Batched DNA pairs: mutated 150 bp reads vs their 300-600 bp windows."""
    import torch
    from paper_1909_00899_amd import api, workloads as W
    api.load()
    api.sw_init(0)
    n = min(args.n_refs * 10, 1_000_000)
    w = W.dna_pairs(n_pairs=n)
    d, pq = _device_batch(w)
    tuned = [] if args.no_tune else api.sw_autotune(*d, w.matrix, w.gap_open, w.gap_extend,
                                                     pair_query=pq)
    pinned = torch.empty((n, 4), dtype=torch.int32, pin_memory=True).numpy()
    step = lambda **kw: api.sw_align_batch(*d, w.matrix, w.gap_open, w.gap_extend,  # noqa
                                           pair_query=pq, **kw)
    use_graph = 0 if args.no_graph else 1
    for _ in range(args.warmup):
        out = step(out=pinned)
    if use_graph:
        step(use_graph=1, out=pinned)          # capture; later identical calls replay it
    torch.cuda.synchronize()
    # eager leg: the alignment kernel's own time (HIP events) for the roofline
    kms = []
    te = time.perf_counter()
    for _ in range(args.steps):
        out = step(out=pinned)
        kms.append(out.stats["kernel_ms"])
    torch.cuda.synchronize()
    eager_wall = (time.perf_counter() - te) / args.steps
    out = api.BatchOutput(out.results.copy(), out.stats)   # the pinned buffer is reused
    # timed region: whole calls replaying the captured graphs, results into
    # pinned host memory
    t0 = time.perf_counter()
    for _ in range(args.steps):
        og = step(use_graph=use_graph, out=pinned)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    same_graph = bool(np.array_equal(og.results, out.results))
    tp = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        op = step(use_graph=use_graph)
    torch.cuda.synchronize()
    pageable_wall = (time.perf_counter() - tp) / max(1, args.steps // 2)
    # the same calls with the host planner
    oh = step(planner=1)
    torch.cuda.synchronize()
    th = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        oh = step(planner=1)
    torch.cuda.synchronize()
    host_wall = (time.perf_counter() - th) / max(1, args.steps // 2)
    cells = w.cells()
    km = float(np.mean(kms))
    ach = cells * OPS_PER_CELL / (km / 1e3) / 1e12
    # start cells and paths of the same alignments
    reps = max(1, args.steps // 4)
    api.sw_align_batch_starts(*d, w.matrix, w.gap_open, w.gap_extend, out.results, pair_query=pq)
    ts = time.perf_counter()
    for _ in range(reps):
        qs, rs = api.sw_align_batch_starts(*d, w.matrix, w.gap_open, w.gap_extend, out.results,
                                           pair_query=pq)
    starts_ms = (time.perf_counter() - ts) / reps * 1e3
    paths = _paths_leg(api, d, pq, w, out.results, qs, rs, reps)
    endtoend = _endtoend_leg(api, d, pq, w, reps)
    print(json.dumps({"metric": METRIC, "value": round(cells / wall / 1e9, 2), "unit": "GCUPS",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(wall * 1e3, 3), "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "i16x2", "data": "synthetic",
                      "config": {"workload": "dna_pairs: %d mutated 150 bp reads vs 300-600 bp "
                                             "windows, +1/-4, GapOpen 6, GapExtend 1" % n,
                                 "pairs": n, "cells": cells},
                      "roofline": _with_measured_peak(
                          {"bound": "alu", "kernel": "pair_direct_kernel",
                           "achieved": round(ach, 3),
                           "peak": round(PEAK_I16X2_TOPS, 2), "unit": "Tops/s",
                           "frac": round(ach / PEAK_I16X2_TOPS, 4), "traffic": None,
                           "kernel_ms": round(km, 3),
                           "kernel_gcups": round(cells / (km / 1e3) / 1e9, 1)}),
                      "stats": {k: out.stats[k] for k in ("n_rerun", "lanes_used", "seglen_max",
                                                          "prep_ms", "plan_ms", "launch_ms",
                                                          "finish_ms", "total_ms",
                                                          "planner_used")},
                      "eager": {"ms_per_step": round(eager_wall * 1e3, 3),
                                "gcups": round(cells / eager_wall / 1e9, 2)},
                      "graph": {"used": bool(use_graph), "same_results_as_eager": same_graph},
                      "pageable_out": {"ms_per_step": round(pageable_wall * 1e3, 3),
                                       "gcups": round(cells / pageable_wall / 1e9, 2),
                                       "same_results": bool(np.array_equal(op.results,
                                                                           out.results))},
                      "host_planner": {"ms_per_step": round(host_wall * 1e3, 3),
                                       "gcups": round(cells / host_wall / 1e9, 2),
                                       "kernel_ms": round(oh.stats["kernel_ms"], 3),
                                       "same_results": bool(np.array_equal(oh.results,
                                                                           out.results))},
                      "starts": {"ms_per_call": round(starts_ms, 3)},
                      "paths": paths,
                      "endtoend": endtoend,
                      "tuned": [{k: (round(v, 1) if isinstance(v, float) else v)
                                 for k, v in e.items()} for e in tuned]}))


def bench_long_queries(args):
    """Scan vs lazy-F (int32) on long i.i.d. and low-complexity queries.

    Per class (query kind x reference kind) two queries of that kind run
    against the 5k references of that kind (10k pairs); the full workload is
    64 queries x 10k references (1.3e13 cells).
    """
    import torch
    import oracle
    from paper_1909_00899_amd import api, workloads as W
    api.load()
    api.sw_init(0)
    full = W.long_queries()
    nq = full.query_off.size - 1
    nr = full.ref_off.size - 1
    half = nr // 2
    rows = {}
    for qkind, qsel in (("iid", (0, 1)), ("runs", (nq // 2, nq // 2 + 1))):
        for rkind, (lo, hi) in (("iid", (0, half)), ("runs", (half, nr))):
            idx = [q * nr + r for q in qsel for r in range(lo, hi)]
            sub = full.subset(np.array(idx))
            d, pq = _device_batch(sub)
            res = {}
            # the scan with two int32 chains per sub-group (the default), with
            # one chain, and the lazy-F comparator
            # and the scan with the references striped and the queries streamed
            for alg, name, chains, stripe in (
                    (api.SW_ALG_SCAN, "scan", api.SW_CHAINS_TWO, api.SW_STRIPE_QUERY),
                    (api.SW_ALG_SCAN, "scan_one_chain", api.SW_CHAINS_ONE, api.SW_STRIPE_QUERY),
                    (api.SW_ALG_SCAN, "scan_swapped", api.SW_CHAINS_AUTO, api.SW_STRIPE_SHORTER),
                    (api.SW_ALG_LAZYF, "lazyf", api.SW_CHAINS_AUTO, api.SW_STRIPE_QUERY)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = api.sw_align_batch(*d, sub.matrix, sub.gap_open, sub.gap_extend,
                                         pair_query=pq, precision=api.SW_PREC_I32, algorithm=alg,
                                         int32_chains=chains, striping=stripe)
                wall = time.perf_counter() - t0
                st = out.stats
                res[name] = {"gcups": round(sub.cells() / wall / 1e9, 1),
                             "kernel_gcups": round(sub.cells() / (st["kernel_ms"] / 1e3) / 1e9, 1),
                             "columns": st["columns"], "lazyf_steps": st["lazyf_steps"],
                             "seglen": st["seglen_max"], "results": out.results}
            lz = res["lazyf"]
            passes = lz["lazyf_steps"] / max(1, lz["columns"]) / max(1, lz["seglen"])
            # the oracle on a seeded sample of the class's pairs (both queries)
            samp = np.random.default_rng(7).choice(sub.n_pairs, size=32, replace=False)
            ws = sub.subset(np.sort(samp))
            want = oracle.align_batch(ws.query_res, ws.query_off, ws.ref_res, ws.ref_off,
                                      ws.pair_ref, ws.matrix, ws.gap_open, ws.gap_extend,
                                      pair_query=ws.pair_query)
            parity = bool(np.array_equal(res["scan"]["results"][np.sort(samp), :3], want) and
                          np.array_equal(lz["results"][np.sort(samp), :3], want))
            rows["query_%s/ref_%s" % (qkind, rkind)] = {
                "pairs": sub.n_pairs, "cells": sub.cells(),
                "query_lens": [int(full.query_off[q + 1] - full.query_off[q]) for q in qsel],
                "scan_gcups": res["scan"]["gcups"], "lazyf_gcups": lz["gcups"],
                "scan_kernel_gcups": res["scan"]["kernel_gcups"],
                "scan_kernel_frac_i32": round(res["scan"]["kernel_gcups"] * OPS_PER_CELL /
                                              (PEAK_I32_TOPS * 1e3), 4),
                "scan_one_chain_gcups": res["scan_one_chain"]["gcups"],
                "scan_one_chain_kernel_gcups": res["scan_one_chain"]["kernel_gcups"],
                "scan_one_chain_kernel_frac_i32": round(
                    res["scan_one_chain"]["kernel_gcups"] * OPS_PER_CELL / (PEAK_I32_TOPS * 1e3), 4),
                "two_chains_equal_one": bool(np.array_equal(res["scan"]["results"],
                                                            res["scan_one_chain"]["results"])),
                "scan_swapped_gcups": res["scan_swapped"]["gcups"],
                "scan_swapped_kernel_gcups": res["scan_swapped"]["kernel_gcups"],
                "scan_swapped_kernel_frac_i32": round(
                    res["scan_swapped"]["kernel_gcups"] * OPS_PER_CELL / (PEAK_I32_TOPS * 1e3), 4),
                "swapped_equal_query_striped": bool(np.array_equal(
                    res["scan_swapped"]["results"], res["scan_one_chain"]["results"])),
                "lazyf_kernel_gcups": lz["kernel_gcups"],
                "lazyf_passes_per_column": round(passes, 3),
                "scan_equals_lazyf": bool(np.array_equal(res["scan"]["results"], lz["results"])),
                "parity_sample_32": parity}
    tot_scan = sum(r["cells"] for r in rows.values()) / sum(
        r["cells"] / r["scan_gcups"] for r in rows.values())
    print(json.dumps({"metric": METRIC, "value": round(tot_scan, 2), "unit": "GCUPS", "n_gpus": 1,
                      "higher_is_better": True, "dtype": "i32", "data": "synthetic",
                      "config": {"workload": "long_queries: per class 2 queries (5k-35k, i.i.d. "
                                             "or poly-residue runs) x 5k refs (200-2000)"},
                      "by_class": rows}))


def _offline_serving(api, db, scor, req):
    """The requests as offline batches (one sw_align_batch per scoring family):
    results in request order and the wall time of the two calls."""
    res = np.zeros((req.ref_id.size, 4), dtype=np.int32)
    fam = []
    for dna in (False, True):
        sel = np.nonzero(req.is_dna == dna)[0]
        if sel.size == 0:
            continue
        qs = [req.query_res[req.query_off[k]:req.query_off[k + 1]] for k in sel]
        qoff = np.zeros(sel.size + 1, dtype=np.int64)
        np.cumsum([q.size for q in qs], out=qoff[1:])
        r0 = 0 if not dna else db.n_protein
        r1 = db.n_protein if not dna else db.n_protein + db.n_dna
        rres = db.ref_res[db.ref_off[r0]:db.ref_off[r1]]
        roff = db.ref_off[r0:r1 + 1] - db.ref_off[r0]
        fam.append((sel, np.concatenate(qs), qoff, rres, roff,
                    (req.ref_id[sel] - r0).astype(np.int32), np.arange(sel.size, dtype=np.int32),
                    scor[1 if dna else 0]))
    t0 = time.perf_counter()
    for sel, qres, qoff, rres, roff, pr, pq, (M, go, ge) in fam:
        res[sel] = api.sw_align_batch(qres, qoff, rres, roff, pr, M, go, ge, pair_query=pq).results
    return res, time.perf_counter() - t0


# An offered rate above the server's capacity (about 1M req/s on this mix),
# and the requests replayed at it.
SATURATING_RATE = 2_000_000
SATURATED_REQUESTS = 100_000


def _serving_sweep(api, W, rates, n_of_rate):
    """Open-loop Poisson replay through the server at each rate; every served
    result is compared with the offline batch call on the same requests."""
    db = W.serving_db()
    scor = [(W.protein_matrix(), 11, 1), (W.dna_matrix(), 6, 1)]
    rows = []
    with api.Server(db.ref_res, db.ref_off, scor, hbm_budget_bytes=8 << 30, n_streams=4,
                    max_batch=16384) as srv:
        for rate in rates:
            n = n_of_rate(rate)
            req = W.serving_requests(db, rate, n, seed=rate)
            sid = req.is_dna.astype(np.int32)
            t0 = time.perf_counter()
            res, ts = srv.replay(req.query_res, req.query_off, req.ref_id, sid, req.arrival_s)
            wall = time.perf_counter() - t0
            lat = (ts[:, 2] - ts[:, 0]) / 1e6
            warm = req.arrival_s >= min(1.0, req.arrival_s[-1] / 4)
            ql = np.diff(req.query_off)
            rl = np.diff(db.ref_off)[req.ref_id]
            cells = float(np.sum(ql.astype(np.float64) * rl))
            off_res, off_wall = _offline_serving(api, db, scor, req)
            rows.append({"rate_per_s": rate, "requests": n,
                         "p50_ms": round(float(np.percentile(lat[warm], 50)), 3),
                         "p99_ms": round(float(np.percentile(lat[warm], 99)), 3),
                         "served_gcups": round(cells / wall / 1e9, 2),
                         "offline_gcups": round(cells / off_wall / 1e9, 2),
                         "achieved_rate": round(n / wall, 1),
                         "served_equals_offline": bool(np.array_equal(res[:, :3],
                                                                      off_res[:, :3]))})
    return rows


def bench_serving(args):
    """Continuous-batching server: Poisson arrivals at a swept rate, p50/p99."""
    from paper_1909_00899_amd import api, workloads as W
    api.load()
    api.sw_init(0)
    rates = [1000, 2000, 5000, 10000, 20000, 50000, 100000, 200000, SATURATING_RATE]
    rows = _serving_sweep(api, W, rates,
                          lambda rate: SATURATED_REQUESTS if rate >= SATURATING_RATE
                          else int(min(20000, max(2000, rate * 3))))
    print(json.dumps({"metric": METRIC, "value": rows[-1]["p99_ms"], "unit": "ms p99",
                      "n_gpus": 1, "higher_is_better": False, "dtype": "i16x2",
                      "data": "synthetic",
                      "config": {"workload": "serving: 25k protein + 25k DNA resident refs, "
                                             "Poisson arrivals, one reference per request"},
                      "sweep": rows,
                      "served_equals_offline": all(r["served_equals_offline"] for r in rows)}))


if __name__ == "__main__":
    main()
