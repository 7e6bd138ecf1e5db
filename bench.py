"""Benchmark: all-pairs posterior matrices of synthetic protein families.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1|nt|c5p|c4]
                [--precision fp32|fp64] [--no-graph] [--no-cpu] [--c4-families F]

The default workload is C3, the largest single-GPU configuration: 1,000
sequences with lengths log-uniform in [50, 1500] (499,500 pairs, 9.1e10
cells).  One step = the whole hot path on device-resident inputs: parameter
tables, pair schedule (cost classes, longest-first queue), the fused
forward / backward / posterior / threshold / MEA kernels, CSR compaction and
the pair-ordered gather.  The CPU baseline times the FP64 oracle on the
seeded C3 sample, and the whole sample (150 uniform pairs and 50 from the top
1 % by cells) gives the measured max |P_gpu - P_oracle|.

After the C3 step, the same run replays a Poisson stream of C4 families
(mean 20 families/s, sizes U{10..500}, lengths U{100..600}; --c4-families,
default 200) through the serving loop and reports its sustained GCUPS and
p50 / p99 family latency under "extra.c4".  --workload c4 runs that stream
alone (--families, default 2000).  Prints one JSON line.
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

METRIC = "all-pairs posterior GCUPS & pairs/s at ≤1e-5 vs FP64 oracle; p99 family latency"
# algorithmic FP32 work per DP cell (both models, both passes, posterior,
# average, MEA, threshold compare)
FLOP_PER_CELL = 67.0
# the same work counted as VALU instructions (an FMA is one), against the
# unpacked issue rate of 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_INSTR_PER_CELL = 49.0
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9
FP32_VALU_PEAK_TFLOPS = 157.3
FP64_VALU_PEAK_TFLOPS = 78.6
KERNEL_SRC = os.path.join(ROOT, "paper_1512_07437_amd", "csrc", "qp_device.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pairs_hbm_traffic.txt")


def kernel_name(cls: int, fp64: bool, ck: bool = False) -> str:
    """Symbol of the persistent pair kernel of one class, as profilers print
    it (ck: the checkpointed FP32 form)."""
    banded = cls >= 8
    r = cls + 1 if not banded else cls - 3
    if ck and not fp64:
        return "qp::k_pairs_ck<%d, %s>" % (4 if banded else r, "true" if banded else "false")
    return "qp::k_pairs<%d, %s, %s>" % (r, "double" if fp64 else "float", "true" if banded else "false")


def class_kernels(B, plan, fp64: bool):
    """Per-class rows (kernel, pairs, cells, average duration, TFLOP/s) of a
    plan's timed runs."""
    classes = []
    for c in range(B.KERNEL_CLASSES):
        c_ms, c_pairs, c_cells, c_r = plan.class_timing(c)
        if c_pairs:
            ck = bool(B.get_tuning()["recompute"][min(c, B.BANDED)])
            classes.append({"class": c, "kernel": kernel_name(c, fp64, ck),
                            "rows_per_lane": c_r, "pairs": c_pairs,
                            "cells": c_cells, "avg_ms": round(c_ms, 4),
                            "tflops": round(c_cells * FLOP_PER_CELL / (c_ms * 1e-3) / 1e12, 3) if c_ms > 0 else None})
    return classes


def consistency_extra(B, W, params, thresh: float, say, reps: int = 3, tree_threshold: int = 200,
                      amplification: float = 3.0):
    """Selective consistency on the device for the C2 family, after the timed
    region: GPU posteriors, the guide tree on their distances, then the
    relaxation of the device-resident all-pairs CSR through the third
    sequences with max(d_xz, d_yz) <= tree_threshold (one pass for 50
    sequences or more, two below), timed with HIP events on the run stream."""
    import torch
    fam = W.c2_family()
    k = len(fam)
    lens = [len(s) for s in fam]
    d_seqs, d_off = B.device_inputs(fam, "cuda:0")
    s = torch.cuda.current_stream()
    plan = B.Plan(lens, params, thresh, nnz_capacity=-1)
    try:
        plan.run(d_seqs.data_ptr(), d_off.data_ptr(), s.cuda_stream)
        dres = plan.sync()
        host = plan.download()
        joins, _ = B.guide_tree(host["dist"], k)
        tdist = B.tree_distance(joins, k)
        d_t = torch.from_numpy(tdist).to("cuda:0")
        passes = 2 if k < 50 else 1
        pair_bytes = np.diff(host["nnz_off"]) * 8 + (np.array([lens[i] for i in host["pair_i"]]) + 1) * 4
        rx = B.Relax(lens, tree_threshold, amplification, passes, thresh, in_capacity=int(dres.nnz))
        try:
            rx.run(dres, int(dres.nnz), d_t.data_ptr(), s.cuda_stream)
            rx.sync()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                rx.run(dres, int(dres.nnz), d_t.data_ptr(), s.cuda_stream)
            e1.record(s)
            out = rx.sync()
            ms = e0.elapsed_time(e1) / reps
            relax_bytes = rx.device_bytes()
        finally:
            rx.close()
    finally:
        plan.close()
    # third sequences selected per pair: z with both tree-guided distances <= T
    D = np.zeros((k, k), dtype=np.int64)
    iu = np.triu_indices(k, 1)
    D[iu] = tdist
    D = D + D.T
    M = (D <= tree_threshold) & ~np.eye(k, dtype=bool)
    Mi = M.astype(np.int64)
    sel = (Mi @ Mi.T)[iu]
    n_pairs = k * (k - 1) // 2
    # algorithmic bytes of a pass: every pair reads, for each selected z, the
    # matrices S_xz and S_zy once (CSR entries and row pointers), and writes
    # its relaxed matrix
    PB = np.zeros((k, k))
    PB[iu] = pair_bytes
    PB = PB + PB.T
    MB = Mi * PB
    read = float(((MB @ Mi.T) + (Mi @ MB.T))[iu].sum() + pair_bytes.sum())
    written = float(int(out.nnz) * 8 + (np.array(lens)[iu[0]] + 1).sum() * 4)
    achieved = (read + written) / (ms * 1e-3) / 1e9
    r = {"workload": "C2: 200 seqs, L ~ U{250..350}, %d pairs" % n_pairs, "tree_threshold": tree_threshold,
         "amplification": amplification, "passes": passes, "ms": round(ms, 3),
         "pairs_per_s": round(n_pairs / (ms * 1e-3), 1), "entries_in": int(dres.nnz), "entries_out": int(out.nnz),
         "z_terms_per_s": round(float(sel.sum()) / (ms * 1e-3), 1),
         "third_sequences_per_pair_mean": round(float(sel.mean()), 2), "device_bytes": relax_bytes,
         "where": "after the timed region, HIP events on the run stream",
         "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                      "frac": round(achieved / 8000.0, 4), "algorithmic_bytes": round(read + written),
                      "what": "per pass: each pair's own matrix and, for each selected z, S_xz and S_zy read "
                              "once (CSR entries and row pointers), the relaxed matrices written"}}
    say("consistency on C2: %s" % r)
    return r


def consistency_cpu_baseline(W, params, thresh: float, tree_threshold: int = 200, amplification: float = 3.0,
                             k_sample: int = 12):
    """The FP64 oracle's relaxation (dense matrices, one pass) timed on one
    core on a bounded sample of the C2 family: its first k_sample sequences,
    their oracle posteriors and the oracle's guide tree as input.  Rate in
    relaxation terms (pair x selected third sequence) per second, the unit of
    the device figure's z_terms_per_s."""
    import oracle
    from oracle import consistency as OC
    from oracle import tree as OT
    fam = W.c2_family()[:k_sample]
    k = len(fam)
    S0, dist = {}, []
    for x in range(k):
        for y in range(x + 1, k):
            r = oracle.pair(fam[x], fam[y], params, per_model=False)
            post = r["post"].copy()
            post[post < thresh] = 0.0
            S0[(x, y)] = post
            dist.append(1.0 - r["ea"])
    joins, _ = OT.wpgma(dist, k)
    tdist = OT.tree_distance(joins, k)
    terms = sum(len(OC.selected(tdist, k, x, y, tree_threshold)) for x in range(k) for y in range(x + 1, k))
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):  # the matrix products on one thread
        t0 = time.perf_counter()
        OC.relax_pass(S0, k, tdist, tree_threshold, amplification, thresh)
        dt = time.perf_counter() - t0
    return {"value": round(terms / dt, 1), "unit": "z-terms/s", "cores": 1, "kind": "oracle",
            "sample": "one pass over the first %d C2 sequences (%d pairs, %d terms, %.2f s), oracle posteriors "
                      "and guide tree as input" % (k, k * (k - 1) // 2, terms, dt)}


def committed_traffic(kernel: str, workload_key: str):
    """HBM bytes per launch (read, write) of `kernel` on `workload_key` from the
    committed counter summary, or None when the summary is missing or was
    taken on a different kernel source than the one built now."""
    import hashlib

    try:
        text = open(TRAFFIC_FILE).read().splitlines()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    src = [ln.split("=", 1)[1].strip() for ln in text if ln.startswith("source_sha256")]
    if not src or src[0] != sha:
        return None
    for ln in text:
        f = ln.split("\t")
        if len(f) == 5 and f[0] == "traffic" and f[1] == kernel and f[2] == workload_key:
            return float(f[3]), float(f[4])
    return None


def workload(name: str):
    from paper_1512_07437_amd import workload as W
    if name == "c1":
        fam = W.c1_family()
        return fam, None, "C1: 8 seqs, L~U{80..120}, 28 pairs", np.arange(28)
    if name == "c2":
        fam = W.c2_family()
        return fam, None, "C2: 200 seqs, L~U{250..350}, 19,900 pairs", W.c2_sample()
    if name == "c3":
        fam = W.c3_family()
        return fam, None, "C3: 1,000 seqs, L log-uniform [50,1500], 499,500 pairs", W.c3_sample(
            [len(s) for s in fam])
    if name == "nt":
        fam = W.nt_workload_family()
        return fam, None, "NT: 200 nucleotide seqs, L~U{250..350}, 19,900 pairs (alphabet 4)", W.c2_sample()
    if name == "c5p":
        ab = W.c5p_pairs()
        fam = [s for pair in ab for s in pair]
        pi = np.arange(0, 2 * len(ab), 2, dtype=np.int32)
        return fam, (pi, pi + 1), ("C5p: 64 independent pairs, L~U{1000..1536}, substitution 0.3, indel 0.05 "
                                   "(precision study within the supported lengths)"), np.arange(len(ab))
    if name == "c5":
        raise SystemExit("C5 (lengths 3000..5000) is disabled: sequences longer than 1536 residues are refused "
                         "by the library until a GPU fault seen on that workload is explained")
    if name == "c5s":
        raise SystemExit("C5 at reduced lengths (1000..1500) overflows the sparse-output estimate, and runs that "
                         "continued after an overflow faulted the GPU; it is not run until that cause is found")
    raise SystemExit("unknown workload " + name)


def _pair_seqs(fam, pairs, p, n_seq):
    from paper_1512_07437_amd import workload as W
    if pairs is None:
        return W.pair_of_index(p, n_seq)
    return int(pairs[0][p]), int(pairs[1][p])


def _err_vs_oracle(res, p, x, y, r):
    from paper_1512_07437_amd import binding as B
    rp, col, val = B.pair_csr(res, p)
    rows = np.repeat(np.arange(len(x)), np.diff(rp))
    return (float(np.abs(val.astype(np.float64) - r["post"][rows, col]).max(initial=0.0)),
            abs((1.0 - res["dist"][p]) - r["ea"]))


def cpu_baseline(fam, pairs, sample, params, res, n_seq, timed=None):
    """FP64 oracle on the sample, and the GPU error there.  The pairs of
    `timed` (default: all of the sample) run one after another on one thread
    and give the single-core rate; the rest of the sample is checked on a
    thread pool (the oracle's C code runs outside the interpreter lock)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    timed = list(sample) if timed is None else list(timed)
    rest = [p for p in sample if p not in set(timed)]
    cells = 0
    worst = ea_worst = 0.0
    t0 = time.perf_counter()
    for p in timed:
        p = int(p)
        i, j = _pair_seqs(fam, pairs, p, n_seq)
        r = oracle.pair(fam[i], fam[j], params, per_model=False)
        cells += len(fam[i]) * len(fam[j])
        e, ea = _err_vs_oracle(res, p, fam[i], fam[j], r)
        worst, ea_worst = max(worst, e), max(ea_worst, ea)
    dt = time.perf_counter() - t0

    def check(p):
        i, j = _pair_seqs(fam, pairs, int(p), n_seq)
        return _err_vs_oracle(res, int(p), fam[i], fam[j], oracle.pair(fam[i], fam[j], params, per_model=False))

    if rest:
        with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as pool:
            for e, ea in pool.map(check, rest):
                worst, ea_worst = max(worst, e), max(ea_worst, ea)
    return cells, dt, worst, ea_worst


def _oracle_pair_cells(job):
    """One sampled pair through the oracle (process-pool worker: imports the
    oracle only, never the GPU library)."""
    import oracle
    x, y, params = job
    oracle.pair(x, y, params, per_model=False)
    return len(x) * len(y)


def cpu_baseline_all_cores(fam, pairs, sample, params, n_seq, workers):
    """The same oracle on the same sample, one pair per task over a pool of
    `workers` freshly started processes; wall time of the whole sample."""
    import multiprocessing as mp_
    from paper_1512_07437_amd import workload as W
    jobs = []
    for p in sample:
        p = int(p)
        i, j = W.pair_of_index(p, n_seq) if pairs is None else (int(pairs[0][p]), int(pairs[1][p]))
        jobs.append((fam[i], fam[j], params))
    from concurrent.futures import ProcessPoolExecutor
    # fresh interpreters (no GPU context inherited); a worker that dies ends
    # the pool with an error instead of being restarted
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp_.get_context("spawn")) as pool:
        list(pool.map(_oracle_pair_cells, jobs[:workers]))  # workers started and warm
        t0 = time.perf_counter()
        cells = sum(pool.map(_oracle_pair_cells, jobs, chunksize=1))
        dt = time.perf_counter() - t0
    return cells, dt


def per_pair_form(B, lens, params, thresh, ii, jj, sample, res, d_seqs, d_off, sp, batched_gcups, peak, say,
                  reps=2):
    """The plain per-pair form (one launch of one wavefront per pair, pair
    order, no graph, no work queue) on the seeded sample of the same family:
    its pairs run one after another, so its rate on the sample is its rate on
    the family.  Its outputs are checked bit for bit against the batched
    run's for the same pairs.  Not part of the timed region."""
    import torch
    si, sj = ii[sample].astype(np.int32), jj[sample].astype(np.int32)
    cells = int(np.sum(lens[si].astype(np.int64) * lens[sj]))
    plan = B.Plan(lens, params, thresh, si, sj)
    try:
        plan.set_per_pair(True)
        plan.run(d_seqs.data_ptr(), d_off.data_ptr(), sp)  # first run: warm-up
        plan.sync()
        plan.timing(reset=True)
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.run(d_seqs.data_ptr(), d_off.data_ptr(), sp)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        kernel_ms, pipe_ms, _ = plan.timing()
        plan.sync()
        pp = plan.download()
    finally:
        plan.close()
    same = True
    for k, p in enumerate(sample):
        a0, a1 = res["nnz_off"][p], res["nnz_off"][p + 1]
        b0, b1 = pp["nnz_off"][k], pp["nnz_off"][k + 1]
        r0, r1 = res["row_off"][p], res["row_off"][p + 1]
        q0, q1 = pp["row_off"][k], pp["row_off"][k + 1]
        same = same and res["dist"][p] == pp["dist"][k] and np.array_equal(res["col"][a0:a1], pp["col"][b0:b1]) \
            and np.array_equal(res["val"][a0:a1], pp["val"][b0:b1]) \
            and np.array_equal(res["row_ptr"][r0:r1], pp["row_ptr"][q0:q1])
    g = cells / dt / 1e9
    say("per-pair form: %d pairs in %.1f ms (%.3f GCUPS)" % (len(sample), dt * 1e3, g))
    return {"gcups": round(g, 4), "pairs_per_s": round(len(sample) / dt, 1),
            "ms_per_pair": round(dt * 1e3 / len(sample), 4), "kernel_span_ms": round(kernel_ms, 3),
            "frac": round(g * FLOP_PER_CELL / 1e3 / peak, 6),
            "batched_speedup": round(batched_gcups / g, 1), "identical_to_batched": bool(same),
            "sample": "%d seeded pairs of the same family (%d cells), one launch per pair" % (len(sample), cells)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--thresh", type=float, default=0.01)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-pair", action="store_true", help="skip the plain per-pair form's measurement")
    ap.add_argument("--families", type=int, default=2000, help="--workload c4: families replayed")
    ap.add_argument("--c4-families", type=int, default=200,
                    help="families of the C4 stream replayed after the C3 step (0: none)")
    ap.add_argument("--slots", type=int, default=4,
                    help="c4: families in flight (the server gives each a 1/slots share of the device's waves; "
                         "4 gave the lowest p50 and p99 at the C4 arrival rate of 2 to 16 tried)")
    ap.add_argument("--rate", type=float, default=20.0, help="c4: mean arrivals per second")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the run, copy this many MiB device-to-device (a known-size kernel that "
                         "calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--orient", default="table", choices=["table", "off", "on"],
                    help="sweep each pair in the orientation the cost model picks (on) or with the first "
                         "sequence as rows (off); default: the tuning table's choice")
    ap.add_argument("--classes", default="table", choices=["table", "serial", "concurrent"],
                    help="kernel classes one after another on the run stream (serial) or side by side on "
                         "forked streams (concurrent); default: the tuning table's choice")
    ap.add_argument("--no-consistency", action="store_true",
                    help="skip the selective-consistency timing on the C2 family after the timed region")
    ap.add_argument("--no-alone", action="store_true",
                    help="skip the pass that times the dominant kernel with the device to itself")
    ap.add_argument("--recompute", default="table",
                    help="FP32 pair-kernel form per class: the tuning table's choice (table), the spilling form "
                         "for every class (none), the checkpointed form wherever it exists (all), or nine "
                         "comma-separated 0/1 flags (the tuning table's recompute entries)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the posterior engine runs one process on one MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    def say(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    import torch

    say("torch %s imported" % torch.__version__)
    from paper_1512_07437_amd import binding as B
    from paper_1512_07437_amd import workload as W

    if args.recompute == "all":
        B.set_tuning(recompute=[1, 1, 1, 1, 1, 0, 0, 0, 1])
    elif args.recompute == "none":
        B.set_tuning(recompute=[0] * 9)
    elif args.recompute != "table":
        flags = [int(v) for v in args.recompute.split(",")]
        if len(flags) != 9:
            raise SystemExit("--recompute takes table, none, all or nine comma-separated flags")
        B.set_tuning(recompute=flags)
    if args.classes != "table":
        B.set_tuning(concurrent_classes=int(args.classes == "concurrent"))
    if args.orient != "table":
        B.set_tuning(orient=int(args.orient == "on"))
    say("pair-kernel forms (1 = checkpointed) per class: %s; classes %s" % (
        B.get_tuning()["recompute"], "concurrent" if B.get_tuning()["concurrent_classes"] else "one after another"))
    if args.workload == "c4":
        out = serve_stream(args, say, args.families)
        print(json.dumps(out), flush=True)
        if out["config"]["failed_families"]:
            sys.exit(1)
        return

    fam, pairs, desc, sample = workload(args.workload)
    mp = W.make_nt_params(0) if args.workload == "nt" else W.make_params(0)
    prec = B.QP_FP64 if args.precision == "fp64" else B.QP_FP32_SCALED
    params = B.make_params(mp, prec)
    lens = np.array([len(s) for s in fam], dtype=np.int32)
    if pairs is None:
        ii, jj = np.triu_indices(len(fam), 1)
    else:
        ii, jj = pairs
    cells = int(np.sum(lens[ii].astype(np.int64) * lens[jj]))
    n_pairs = len(ii)

    dev = torch.device("cuda:0")
    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        say("calibration copy of %d MiB done" % args.calib_copy_mb)
    d_seqs, d_off = B.device_inputs(fam, "cuda:0")
    stream = torch.cuda.current_stream(dev)
    def make_plan(capacity):
        pl = B.Plan(lens, params, args.thresh, None if pairs is None else pairs[0],
                    None if pairs is None else pairs[1], nnz_capacity=capacity)
        pl.set_graph(not args.no_graph)
        return pl

    # c5p: the plan holds the guaranteed output bound, so its runs cannot overflow
    plan = make_plan(-1 if args.workload == "c5p" else 0)
    say("plan: %d pairs, %d cells, %.1f MB device" % (n_pairs, cells, plan.device_bytes() / 1e6))
    sp = stream.cuda_stream
    # the first run checks the estimated sparse-output capacity; if it was too
    # small, a plan sized to the produced entries replaces it
    plan.run(d_seqs.data_ptr(), d_off.data_ptr(), sp)
    st = plan.sync_status()
    if st == B.QP_ENOSPC:
        # continuing after an overflowing run is switched off (such runs were
        # followed by GPU faults whose cause is not identified)
        raise SystemExit("sparse output needed %d entries, more than the plan's estimate; "
                         "this workload is not benchmarked" % plan.needed_nnz)
    if st != B.QP_OK:
        plan.sync()  # raises with the library's message
    for _ in range(args.warmup):
        plan.run(d_seqs.data_ptr(), d_off.data_ptr(), sp)
    torch.cuda.synchronize()
    say("warmup done")
    plan.timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(d_seqs.data_ptr(), d_off.data_ptr(), sp)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kernel_ms, pipe_ms, n_timed = plan.timing()
    plan.sync()
    res = plan.download()
    say("timed %d steps: %.3f ms/step" % (args.steps, dt * 1e3 / args.steps))

    ms_per_step = dt * 1e3 / args.steps
    gcups = cells / (dt / args.steps) / 1e9
    peak = FP64_VALU_PEAK_TFLOPS if prec == B.QP_FP64 else FP32_VALU_PEAK_TFLOPS
    fp64 = prec == B.QP_FP64
    # per-class pair kernels (run concurrently on forked streams); the
    # dominant one is the class with the most cells (the most algorithmic
    # work): a small class sharing the chip with a large one can have the
    # longer span without being what bounds the step
    classes = class_kernels(B, plan, fp64)
    dom = max(classes, key=lambda r: r["cells"]) if classes else None
    achieved = dom["tflops"] if dom else None
    concurrent = bool(B.get_tuning()["concurrent_classes"])
    traffic = committed_traffic(dom["kernel"], args.workload + ("_fp64" if fp64 else "")) if dom else None
    out = {
        "metric": METRIC,
        "value": round(gcups, 3),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if prec == 0 else "fp64",
        "data": "synthetic",
        "config": {"workload": desc, "pairs": n_pairs, "cells": cells, "thresh": args.thresh,
                   "graph": not args.no_graph, "nnz": int(res["nnz"]),
                   "classes": "concurrent" if B.get_tuning()["concurrent_classes"] else "serial",
                   "orient": bool(B.get_tuning()["orient"])},
        "pairs_per_s": round(n_pairs / (dt / args.steps), 1),
        "kernel_ms": round(kernel_ms, 4),
        "pipeline_ms": round(pipe_ms, 4),
        "roofline": {"bound": "alu", "kernel": dom["kernel"] if dom else None,
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": None if achieved is None else round(achieved / peak, 4),
                     "traffic": None if traffic is None else traffic[0] + traffic[1],
                     "traffic_read_write": None if traffic is None else [traffic[0], traffic[1]]},
        "issue_frac": round(gcups * 1e9 * VALU_INSTR_PER_CELL / VALU_ISSUE_PEAK, 4),
        "spill_hbm_gbs": None if traffic is None or not dom else round((traffic[0] + traffic[1]) / (dom["avg_ms"] * 1e-3) / 1e9, 1),
        "pair_kernels": classes,
        "all_classes_tflops": round(cells * FLOP_PER_CELL / (kernel_ms * 1e-3) / 1e12, 3) if kernel_ms > 0 else None,
    }
    if args.workload in ("c2", "nt"):
        # the host-to-host path (qp_posteriors: staging of the sequences, a
        # plan, the run, the CSR copied back into pinned host memory), after
        # the timed region; the first call warms the library's host pools
        B.qp_posteriors(fam, params, args.thresh)
        t_e = time.perf_counter()
        e2e = B.qp_posteriors(fam, params, args.thresh)
        e2e_s = time.perf_counter() - t_e
        out["end_to_end"] = {"ms": round(e2e_s * 1e3, 2), "gcups": round(cells / e2e_s / 1e9, 2),
                             "nnz": int(e2e["nnz"]), "what": "qp_posteriors, host sequences in, host CSR out"}
        del e2e
    if pairs is None and len(fam) > 1:
        # the next stage on the host: guide tree and tree-guided distances
        t_gt = time.perf_counter()
        joins, heights = B.guide_tree(res["dist"], len(fam))
        B.tree_distance(joins, len(fam))
        out["guide_tree"] = {"ms": round((time.perf_counter() - t_gt) * 1e3, 2), "seqs": len(fam),
                             "root_height": round(float(heights[-1]), 6), "where": "host, after the timed region"}
    if not args.no_per_pair and args.workload in ("c2", "c3"):
        # a uniform sample of the family: its rate is the family's
        uni = W.c3_sample(lens, parts=True)[0] if args.workload == "c3" else sample
        out["per_pair_form"] = per_pair_form(B, lens, params, args.thresh, ii, jj, uni, res, d_seqs, d_off, sp,
                                             gcups, peak, say)
    if not args.no_cpu and sample is not None:
        # C3: one core times the 150 uniform pairs of the sample (a bounded
        # share of the work); all 200 are checked against the GPU
        timed = W.c3_sample(lens, parts=True)[0] if args.workload == "c3" else sample
        c_cells, c_dt, worst, ea_worst = cpu_baseline(fam, pairs, sample, mp, res, len(fam), timed)
        say("cpu baseline: %d pairs in %.1f s (%d pairs checked)" % (len(timed), c_dt, len(sample)))
        out["cpu_baseline"] = {"value": round(c_cells / c_dt / 1e9, 6), "unit": "GCUPS", "cores": 1,
                               "kind": "oracle",
                               "sample": "%d seeded pairs of the same family, one thread (%d cells, %.1f s)%s" % (
                                   len(timed), c_cells, c_dt,
                                   "; the uniform part of the 200-pair sample" if args.workload == "c3" else "")}
        out["oracle_checked_pairs"] = int(len(sample))
        out["max_abs_err_vs_oracle"] = worst
        out["max_abs_ea_err_vs_oracle"] = ea_worst
        workers = max(1, min(16, os.cpu_count() or 1))
        if workers > 1:
            try:
                a_cells, a_dt = cpu_baseline_all_cores(fam, pairs, sample, mp, len(fam), workers)
                say("cpu baseline on %d processes: %.1f s" % (workers, a_dt))
                out["cpu_baseline_all_cores"] = {"value": round(a_cells / a_dt / 1e9, 6), "unit": "GCUPS",
                                                 "cores": workers, "kind": "oracle",
                                                 "sample": "the same %d pairs, one per task" % len(sample)}
            except Exception as e:  # the single-core figure above stands on its own
                say("all-core cpu baseline skipped: %s" % e)
    plan.close()
    if concurrent and dom and not args.no_alone:
        # the classes share the device in the timed runs, so each kernel's
        # duration there includes the time it yields to the others; one more
        # plan runs them one after another (same pairs, same outputs) to give
        # the dominant kernel's rate with the device to itself
        B.set_tuning(concurrent_classes=0)
        try:
            alone_plan = B.Plan(lens, params, args.thresh, None if pairs is None else pairs[0],
                                None if pairs is None else pairs[1], nnz_capacity=int(res["nnz"]) + 1024)
            alone_plan.set_graph(not args.no_graph)
            alone_plan.run(d_seqs.data_ptr(), d_off.data_ptr(), sp)
            alone_plan.sync()
            alone_plan.timing(reset=True)
            for _ in range(2):
                alone_plan.run(d_seqs.data_ptr(), d_off.data_ptr(), sp)
            alone_plan.sync()
            a_kernel_ms, _, _ = alone_plan.timing()
            alone = {r["kernel"]: r for r in class_kernels(B, alone_plan, fp64)}
            alone_plan.close()
        finally:
            B.set_tuning(concurrent_classes=1)
        a = alone.get(dom["kernel"])
        if a and a["tflops"]:
            out["roofline_alone"] = {"bound": "alu", "kernel": dom["kernel"], "achieved": a["tflops"], "peak": peak,
                                     "unit": "TFLOP/s", "frac": round(a["tflops"] / peak, 4), "avg_ms": a["avg_ms"],
                                     "what": "the same kernel with the device to itself: the plan's classes run "
                                             "one after another, 2 runs after the timed region",
                                     "classes_one_after_another_ms": round(a_kernel_ms, 4)}
        say("dominant kernel alone: %s" % (out.get("roofline_alone"),))
    del res
    if args.workload in ("c2", "c3") and not args.no_consistency and prec == B.QP_FP32_SCALED:
        out.setdefault("extra", {})["consistency"] = consistency_extra(B, W, params, args.thresh, say)
        if not args.no_cpu:
            out["extra"]["consistency"]["cpu_baseline"] = consistency_cpu_baseline(W, mp, args.thresh)
            say("consistency cpu baseline: %s" % out["extra"]["consistency"]["cpu_baseline"])
    if args.workload == "c3" and args.c4_families > 0 and prec == B.QP_FP32_SCALED:
        # the metric's latency term: the C4 stream through the serving loop
        c4 = serve_stream(args, say, args.c4_families)
        out.setdefault("extra", {})["c4"] = {k: c4[k] for k in (
            "value", "unit", "p50_latency_ms", "p99_latency_ms", "queue_ms_p50_p99", "service_ms_p50_p99",
            "service_split_ms_p50", "offered_gcups", "wall_s", "max_abs_err_vs_oracle",
            "max_abs_ea_err_vs_oracle", "oracle_checked_pairs") if k in c4}
        out["extra"]["c4"]["config"] = c4["config"]
        out["p99_family_latency_ms"] = c4["p99_latency_ms"]
        if c4["config"]["failed_families"]:
            print(json.dumps(out), flush=True)
            sys.exit(1)
    print(json.dumps(out), flush=True)


def serve_stream(args, say, n_families):
    """Replay the Poisson family stream through qp_server_* in real time."""
    import threading

    import torch

    from paper_1512_07437_amd import binding as B
    from paper_1512_07437_amd import workload as W

    mp = W.make_params(0)
    params = B.make_params(mp)
    stream = []
    for t_arr, fam in W.c4_stream(n_families, rate=args.rate):
        stream.append((t_arr, fam))
        if len(stream) % 200 == 0:
            say("generated %d families" % len(stream))
    say("generated %d families" % len(stream))
    free, _ = torch.cuda.mem_get_info()
    srv = B.Server(hbm_budget_bytes=int(free * 0.6), max_slots=args.slots, n_streams=min(args.slots, 16))
    tickets = [None] * len(stream)
    results = [None] * len(stream)

    failed = []
    # oracle spot checks: every check_every-th family keeps its result, and two
    # seeded pairs of each are compared with the FP64 oracle after the run
    check_every = max(1, len(stream) // 10)
    kept = {}

    def waiter():
        for k in range(len(stream)):
            while tickets[k] is None:
                time.sleep(0.0005)
            if tickets[k] < 0:  # its submit failed
                continue
            try:
                res, tm = srv.wait(tickets[k])
                results[k] = (res["n_pairs"], res["nnz"], tm, res["thresh"])
                if k % check_every == 0:
                    kept[k] = res  # spot-checked against the oracle after the stream
            except B.QpError as e:
                failed.append((k, str(e)))

    # a daemon: if the main thread stops early the process still ends
    th = threading.Thread(target=waiter, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for k, (t_arr, fam) in enumerate(stream):
        delay = t_arr - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        try:
            tickets[k] = srv.submit(fam, params, args.thresh)
        except B.QpError as e:
            failed.append((k, "submit: " + str(e)))
            tickets[k] = -1
        if k % 50 == 49:
            say("submitted %d families" % (k + 1))
    th.join()
    t_end = time.perf_counter()
    srv.close()
    done = [r for r in results if r is not None]
    if failed:
        say("%d families failed: %s" % (len(failed), failed[:3]))
    lat = np.array([r[2]["done_s"] - r[2]["submit_s"] for r in done])
    qw = np.array([r[2]["admit_s"] - r[2]["submit_s"] for r in done])   # waiting for a slot / memory
    sv = np.array([r[2]["done_s"] - r[2]["admit_s"] for r in done])     # admitted until downloaded
    cells = sum(r[2]["cells"] for r in done)
    first = min(r[2]["submit_s"] for r in done)
    last = max(r[2]["done_s"] for r in done)
    gcups = cells / (last - first) / 1e9
    out = {
        "metric": METRIC,
        "value": round(gcups, 3),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": len(stream),
        "warmup": 0,
        "ms_per_step": round((last - first) * 1e3 / len(stream), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "C4: Poisson stream, mean %g families/s, k~U{10..500}, L~U{100..600}" % args.rate,
                   "families": len(stream), "failed_families": len(failed), "slots": args.slots,
                   "families_above_requested_thresh": int(sum(r[3] > args.thresh for r in done)),
                   "cells": int(cells), "pairs": int(sum(r[0] for r in done))},
        "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
        "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
        "queue_ms_p50_p99": [round(float(np.percentile(qw, q)) * 1e3, 2) for q in (50, 99)],
        "service_ms_p50_p99": [round(float(np.percentile(sv, q)) * 1e3, 2) for q in (50, 99)],
        "service_split_ms_p50": {k: round(float(np.percentile(v, 50)) * 1e3, 2) for k, v in (
            ("launch", np.array([r[2]["launched_s"] - r[2]["admit_s"] for r in done])),
            ("device", np.array([r[2]["device_s"] - r[2]["launched_s"] for r in done])),
            ("download", np.array([r[2]["done_s"] - r[2]["device_s"] for r in done])))},
        "offered_gcups": round(cells / (stream[-1][0] + 1e-9) / 1e9, 3),
        "wall_s": round(t_end - t0, 2),
    }
    if kept and not args.no_cpu:
        import oracle
        rng = np.random.default_rng(44)
        worst = ea_worst = 0.0
        n_checked = 0
        for k, res in sorted(kept.items()):
            fam = stream[k][1]
            n = len(fam)
            for p in rng.choice(n * (n - 1) // 2, 2, replace=False):
                i, j = W.pair_of_index(int(p), n)
                r = oracle.pair(fam[i], fam[j], mp, per_model=False)
                rp, col, val = B.pair_csr(res, int(p))
                rows = np.repeat(np.arange(len(fam[i])), np.diff(rp))
                worst = max(worst, float(np.abs(val.astype(np.float64) - r["post"][rows, col]).max(initial=0.0)))
                ea_worst = max(ea_worst, abs((1.0 - res["dist"][int(p)]) - r["ea"]))
                n_checked += 1
        out["max_abs_err_vs_oracle"] = worst
        out["max_abs_ea_err_vs_oracle"] = ea_worst
        out["oracle_checked_pairs"] = "%d seeded pairs of %d served families" % (n_checked, len(kept))
    return out


if __name__ == "__main__":
    main()
