#!/usr/bin/env python3
"""Benchmark of the P-DFS / greedy weighted-set-cover hot path on one GPU.

One step = one complete greedy weighted-set-cover solve (every round of
Alg. 1, each round's argmax done by the depth-first search of Alg. 2) of the
h=4, G=20,000 workload (1,000 tumour / 500 normal samples, log-normal gene
rates, 10 planted quadruples, alpha = 1/10), inputs already resident in HBM.

value = h-subsets scored per second: the leaves the search scores (h-subsets
whose cover meets the uncovered tumour samples), summed over all rounds, per
second of solve time, with the paper's empty-intersection pruning (the mode
whose scored set is canonical).  The exact bound-pruned solve of the same
workload (the library default) is timed beside it.

Beside the step: the bound-pruned solve, whole solves of the two smaller
workloads, the pruned-vs-exhaustive first rounds, deeper combinations, the
held-out coverage report, the 32-instance batch (serial plain path, stream
path, one launch per round step; bound and empty mode), the 2,000-request
Poisson stream (served at 20 req/s, and served vs plain at a saturating
rate), and the oracle on every host core (round 1 and the bound-pruned
solve) as the CPU baseline.

Prints one JSON line.  Run with --gpus 1 (the only supported count).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("h-hit subsets scored/s + WSC solve time, batched/served vs plain; "
          "p50/p99 latency")
VALU_PEAK = 256 * 4 * 16 * 2.4e9          # lane-instructions/s (CUs x SIMDs x lanes x clock)
MFMA_I8_PEAK_OPS = 5.0e15                 # dense int8 MFMA, ops/s (2 per multiply-add)

# HBM traffic of the depth-first stage, per launch (one round), from two
# rocprofv3 --pmc runs of two h4_G20000 solves (FETCH_SIZE, WRITE_SIZE; KiB
# summed over both solves' stage kernels), each scaled by what the counter
# reads for a 1 GiB device copy (FETCH_SIZE reads half the bytes, WRITE_SIZE
# all of them); profiles/dfs_stage_h4_G20000_traffic.md.
# Valid for the stage kernels' sources it was taken on (hash below); reported
# as null once they change.
STAGE_SOURCES = ("k_dfs.hip", "k_tri.hip", "dfs_core.h", "slot_reduce.h", "pdfs_dev.h")
STAGE_TRAFFIC = {"sources_sha256_16": "3ce6828f2e443e7f", "workload": "h4_G20000",
                 "bytes_per_launch": (2.0 * 8726112 + 1.0 * 24320177) / 2 * 1024 / 133}


def stage_traffic(workload):
    import hashlib
    h = hashlib.sha256()
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2603_16721_amd", "csrc")
    for f in STAGE_SOURCES:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != STAGE_TRAFFIC["sources_sha256_16"] or \
            workload != STAGE_TRAFFIC["workload"]:
        return None
    return STAGE_TRAFFIC["bytes_per_launch"]


def words(n):
    return (n + 63) // 64


def oracle_subsets_scored(workload):
    """Sum over the rounds of the leaves Alg. 2 scores, from the oracle's stored
    empty-mode solve of the workload (tests/golden/oracle_counters.json), or
    None when none is stored."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_counters.json")
    try:
        with open(path) as f:
            cases = json.load(f)["cases"]
    except OSError:
        return None
    c = cases.get(f"{workload}_empty_all_rounds")
    return None if c is None else int(c["nonempty"][c["h"]])


def dfs_alg_ops(st, h, n_normal, depth3_ops_per_word=4):
    """Algorithmic integer lane-ops of the depth-first kernels for the work they
    were given.  A visited node of depth 3 or 4 costs one W-word AND plus a
    popcount-accumulate, 4 lane-ops per 64-bit word of its round's compacted
    row (W = ceil(|U|/64)); a scored leaf adds its score and comparison (4)
    and, when its normal prefix is non-empty, an AND plus popcount per normal
    word.  depth3_ops_per_word=2 gives the smaller count the h = 4 kernels
    execute for a depth-3 node (a fused and-or emptiness test, no popcount)."""
    w3 = st["dfs_visit_words3"]     # sum of visits x ceil(|U|/64)
    w4 = st["dfs_visit_words4"]
    ops = (depth3_ops_per_word if h == 4 else 4) * w3 + 4 * w4
    ops += 4 * st["dfs_leaves"] + 4 * words(n_normal) * st["dfs_fp_leaves"]
    return ops


# ---- CPU baseline: the oracle (unmodified, pinned) on every host core.  The
# outer loop of a round is cut into shares of first genes (the intervals of
# Sec. III-D) handed to worker processes on request, as the paper's master
# hands out work; the best of the shares under (S desc, tuple asc) is the
# round's answer.
_CPU = {}
SHARE = 32           # first genes per share of the empty-mode round
SHARE_BOUND = 512    # per share of a bound-pruned round (short rounds: fewer hand-offs)


def _cpu_init(T, N, n_tumor, n_normal):
    from oracle import cpu
    _CPU.update(T=T, N=N, nt=n_tumor, nn=n_normal, perm=cpu.order(T, N))


def _cpu_share(args):
    from oracle import cpu
    import numpy as np
    lo, hi, U, h, p, q, mode = args
    b = cpu.best_share(_CPU["T"], _CPU["N"], _CPU["nt"], _CPU["nn"], h, p, q, lo, hi,
                       U=np.asarray(U, dtype=np.uint64), mode=mode, perm=_CPU["perm"])
    key = (b.score, [-i for i in b.sorted_idx]) if b.found else None
    return key, b.sorted_idx, b.tp, b.fp, b.counters["nonempty"][h]


def _cpu_round(pool, G, U, h, p, q, mode, firsts, share):
    """One round over the first-gene shares [lo, lo + share) for lo in
    `firsts`: (best key, sorted tuple, tp, fp), leaves scored."""
    jobs = [(lo, min(lo + share, G), [int(x) for x in U], h, p, q, mode) for lo in firsts]
    best, leaves = None, 0
    for key, idx, tp, fp, ne in pool.imap_unordered(_cpu_share, jobs, chunksize=1):
        leaves += ne
        if key is not None and (best is None or key > best[0]):
            best = (key, idx, tp, fp)
    return best, leaves


def cpu_baseline(inst, T, N, sample_every=4, full=False):
    """The oracle on all host cores: the empty-mode walk of round 1 on a
    stratified sample of first-gene shares (every `sample_every`-th; all of
    them with full=True, median of 3), and the whole bound-pruned greedy
    solve (median of 3).  value = round-1 leaves scored per second."""
    import multiprocessing as mp
    import numpy as np
    from oracle import cpu
    cores = os.cpu_count() or 1
    ctx = mp.get_context("spawn")
    h, p, q = inst.h, inst.alpha_p, inst.alpha_q
    U0 = cpu.full_mask(inst.n_tumor, T.shape[1])
    with ctx.Pool(cores, initializer=_cpu_init, initargs=(T, N, inst.n_tumor, inst.n_normal)) as pool:
        pool.map(_cpu_share, [(0, 1, [int(x) for x in U0], h, p, q, "empty")] * cores)  # warm
        firsts = list(range(0, inst.G, SHARE))
        sample = firsts if full else firsts[::sample_every]
        reps = 3 if full else 1
        rates = []
        for _ in range(reps):
            t0 = time.perf_counter()
            _, leaves = _cpu_round(pool, inst.G, U0, h, p, q, "empty", sample, SHARE)
            dt = time.perf_counter() - t0
            rates.append((leaves / dt, leaves, dt))
            print(f"[bench] oracle round 1 sample: {leaves} leaves in {dt:.1f} s on {cores} cores",
                  file=sys.stderr, flush=True)
        rates.sort()
        rate, leaves, dt = rates[len(rates) // 2]
        # whole bound-pruned solve, round after round
        perm = cpu.order(T, N)
        solves = []
        for _ in range(3):
            U = U0.copy()
            rounds = []
            t0 = time.perf_counter()
            covered = 0
            target = inst.target_covered if inst.target_covered > 0 else inst.n_tumor
            while covered < target:
                best, _ = _cpu_round(pool, inst.G, U, h, p, q, "bound",
                                     list(range(0, inst.G, SHARE_BOUND)), SHARE_BOUND)
                if best is None:
                    break
                genes = [int(perm[i]) for i in best[1]]
                cov = U.copy()
                for g in genes:
                    cov &= T[g]
                U = U & ~cov
                covered = inst.n_tumor - int(sum(bin(int(x)).count("1") for x in U))
                rounds.append((genes, best[2], best[3]))
            solves.append((time.perf_counter() - t0, rounds))
            print(f"[bench] oracle bound solve: {len(rounds)} rounds in {solves[-1][0]:.2f} s",
                  file=sys.stderr, flush=True)
        solves.sort(key=lambda x: x[0])
        solve_s, solve_rounds = solves[1]
    frac = len(sample) / len(firsts)
    return {"value": rate, "unit": "subsets/s", "cores": cores, "kind": "oracle",
            "sample": (f"round 1 of {inst.name}, empty-intersection walk, first-gene shares of "
                       f"{SHARE} sorted positions handed to {cores} worker processes on request; "
                       f"{'all' if full else f'every {sample_every}th'} share ({frac:.2f} of the "
                       f"round): {leaves} leaves in {dt:.1f} s" + (", median of 3" if full else "")),
            "bound_solve_ms": 1e3 * solve_s, "bound_solve_rounds": len(solve_rounds),
            "bound_solve": (f"whole bound-pruned greedy solve, shares of {SHARE_BOUND} first genes "
                            f"per round, median of 3"),
            "_rounds": solve_rounds}


def _gen_request(j):
    from paper_2603_16721_amd import synth
    I = synth.served_request(j)
    T, N = I.packed()
    return j, T, N, I.n_tumor, I.n_normal, I.h


def _gen_batched(i):
    from paper_2603_16721_amd import synth
    I = synth.batched_instance(i)
    T, N = I.packed()
    return i, T, N, I.n_tumor, I.n_normal, I.h


def _pool_map(fn, items):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(16, max(1, (os.cpu_count() or 2) - 1))) as pool:
        return pool.map(fn, items)


def bench_batched(pdfs, data, modes=("bound", "empty")):
    """32 instances: serially through the plain path, the stream path (each
    instance's own launches on 4 streams) and one launch per round step over
    all instances, in bound and empty mode (the batches tuned first)."""
    import torch
    hs = [d[5] for d in data]
    ncap = [d[3] + 1 for d in data]
    out = {"instances": len(data)}
    for mode in modes:
        plain_ms = 0.0
        plain_rounds = []
        for (_, T, N, nt, nn, h) in data:
            with pdfs.Solver(T, N, nt, nn, mode) as s:
                s.wsc(h, 1, 10)                        # warm (allocations)
                torch.cuda.synchronize()
                t = time.perf_counter()
                r, _, _ = s.wsc(h, 1, 10)
                plain_ms += 1e3 * (time.perf_counter() - t)
                plain_rounds.append([(x["genes"], x["tp"], x["fp"]) for x in r])
        row = {"plain_serial_ms": plain_ms}
        reps = 3 if mode == "bound" else 1
        for name, path in (("streams", "streams"), ("one_launch_per_step", "one_launch")):
            b = pdfs.pdfs_batch_create([(T, N, nt, nn) for (_, T, N, nt, nn, _) in data], mode,
                                       autotune=True, path=path)
            try:
                pdfs.pdfs_batch_run(b, hs, 1, 10, n_tumors=ncap)   # warm + tune
                times = []
                for _ in range(reps):
                    t = time.perf_counter()
                    res, st = pdfs.pdfs_batch_run(b, hs, 1, 10, n_tumors=ncap)
                    times.append(1e3 * (time.perf_counter() - t))
            finally:
                pdfs.pdfs_batch_destroy(b)
            same = [[(x["genes"], x["tp"], x["fp"]) for x in r] for r in res] == plain_rounds
            row[name] = {"ms": min(times), "speedup_vs_plain_serial": plain_ms / min(times),
                         "same_results": same, "rounds": st["rounds"]}
            print(f"[bench] batched {mode} {name}: {min(times):.1f} ms vs plain serial "
                  f"{plain_ms:.1f} ms", file=sys.stderr, flush=True)
        # the path a batch takes by default for this mode (path="auto")
        row["default_path"] = "one_launch_per_step" if mode == "bound" else "streams"
        row["default_speedup_vs_plain_serial"] = row[row["default_path"]]["speedup_vs_plain_serial"]
        out[mode] = row
    return out


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x) * 1e3, q))


def _serve_stream(pdfs, data, arrivals, max_active=8):
    """Submits each request at its arrival time to one server (continuous
    batching) and polls until all are done: latencies and span."""
    n_req = len(arrivals)
    srv = pdfs.pdfs_server_create("bound", 0, 0, max_active)
    lat = [None] * n_req
    try:
        tickets = []
        t0 = time.perf_counter()
        j = 0
        pending = set()
        while j < n_req or pending:
            now = time.perf_counter() - t0
            while j < n_req and arrivals[j] <= now:
                (_, T, N, nt, nn, h) = data[j]
                tickets.append(pdfs.pdfs_server_submit(srv, T, N, nt, nn, h, 1, 10))
                pending.add(j)
                j += 1
            for k in list(pending):
                r = pdfs.pdfs_server_poll(srv, tickets[k], cap=data[k][3] + 1)
                if r is not None:
                    lat[k] = r[1]
                    pending.discard(k)
            time.sleep(0.0005)
        span = time.perf_counter() - t0
    finally:
        pdfs.pdfs_server_destroy(srv)
    return lat, span


def _plain_stream(pdfs, data, arrivals):
    """The plain path serving the same arrivals one at a time."""
    lat = []
    t0 = time.perf_counter()
    for j, (_, T, N, nt, nn, h) in enumerate(data):
        now = time.perf_counter() - t0
        if now < arrivals[j]:
            time.sleep(arrivals[j] - now)
        with pdfs.Solver(T, N, nt, nn, "bound") as s:
            s.wsc(h, 1, 10)
        lat.append(time.perf_counter() - t0 - arrivals[j])
    return lat, time.perf_counter() - t0


def bench_served(pdfs, data, saturate=20.0):
    """The seeded Poisson request stream (mean 20 req/s), h in {2,3,4} at
    3:5:2: continuous batching at the stream's own rate, and both the server
    and the plain path (one request at a time) with the arrivals compressed
    `saturate`-fold, where the arrival rate exceeds what either can serve."""
    from paper_2603_16721_amd import synth
    n_req = len(data)
    arrivals = synth.served_arrivals()[:n_req]
    lat, span = _serve_stream(pdfs, data, arrivals)
    out = {"requests": n_req, "latency": "submission to result, wall time", "mode": "bound",
           "at_20_req_per_s": {"served": {"p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                                          "solves_per_s": n_req / span}}}
    print(f"[bench] served at 20 req/s: p50 {_pct(lat, 50):.1f} ms, p99 {_pct(lat, 99):.1f} ms",
          file=sys.stderr, flush=True)
    fast = arrivals / saturate
    lat_s, span_s = _serve_stream(pdfs, data, fast)
    lat_p, span_p = _plain_stream(pdfs, data, fast)
    out[f"at_{20 * saturate:g}_req_per_s"] = {
        "served": {"p50_ms": _pct(lat_s, 50), "p99_ms": _pct(lat_s, 99),
                   "solves_per_s": n_req / span_s},
        "plain_one_at_a_time": {"p50_ms": _pct(lat_p, 50), "p99_ms": _pct(lat_p, 99),
                                "solves_per_s": n_req / span_p}}
    print(f"[bench] saturated ({20 * saturate:g} req/s): served {n_req / span_s:.1f} solves/s, "
          f"plain {n_req / span_p:.1f} solves/s", file=sys.stderr, flush=True)
    return out


def bench_small_solves(pdfs, stream):
    """Whole greedy solves of the two smaller workloads (h2_G500, h3_G5000) in
    both modes: solve time and subsets scored per second (empty mode)."""
    import torch
    from paper_2603_16721_amd import synth
    out = {}
    for name in ("h2_G500", "h3_G5000"):
        wi = synth.WORKLOADS[name]()
        Ti, Ni = wi.packed()
        row = {}
        for mode in ("empty", "bound"):
            with pdfs.Solver(Ti, Ni, wi.n_tumor, wi.n_normal, mode, 0, stream) as sv:
                sv.wsc(wi.h, wi.alpha_p, wi.alpha_q, target=wi.target_covered)
                torch.cuda.synchronize()
                ts = []
                for _ in range(5):
                    t = time.perf_counter()
                    rr, st, _ = sv.wsc(wi.h, wi.alpha_p, wi.alpha_q, target=wi.target_covered)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t)
            dt = sorted(ts)[2]
            row[mode] = {"solve_ms": 1e3 * dt, "rounds": len(rr)}
            if mode == "empty":
                row[mode]["subsets_scored"] = st["nonempty"][wi.h]
                row[mode]["subsets_scored_per_s"] = st["nonempty"][wi.h] / dt
        out[name] = row
        print(f"[bench] {name} solve: empty {row['empty']['solve_ms']:.2f} ms, bound "
              f"{row['bound']['solve_ms']:.2f} ms", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="h4_G20000")
    ap.add_argument("--bound-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-every", type=int, default=4,
                    help="oracle baseline with --cpu-sample: every n-th first-gene share")
    ap.add_argument("--cpu-sample", action="store_true",
                    help="oracle baseline on a sample of round 1 (one pass) instead of the "
                         "whole round (median of 3; ~10 s a pass on 16 cores)")
    ap.add_argument("--no-small-solves", action="store_true",
                    help="skip the whole solves of h2_G500 and h3_G5000")
    ap.add_argument("--no-bound", action="store_true",
                    help="skip the bound-pruning solve (profiling the empty-mode walk alone)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-exhaustive", action="store_true",
                    help="skip the pruned-vs-exhaustive first-round comparison")
    ap.add_argument("--no-deep", action="store_true",
                    help="skip the h = 5, 6 first-round report")
    ap.add_argument("--no-heldout", action="store_true",
                    help="skip the 75/25 held-out coverage report")
    ap.add_argument("--served-requests", type=int, default=2000)
    ap.add_argument("--served-saturate", type=float, default=20.0,
                    help="arrival-rate multiplier of the saturated pass")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; multi-GPU sharding of the search is not "
              "built (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # inputs of the batched and served workloads, generated in worker
    # processes before this process touches the GPU
    data_b = None if args.no_batched else sorted(_pool_map(_gen_batched, range(32)))
    data_s = None if args.no_served else sorted(_pool_map(_gen_request,
                                                          range(args.served_requests)))

    import numpy as np
    import torch

    from paper_2603_16721_amd import pdfs, synth

    torch.cuda.set_device(0)
    inst = synth.WORKLOADS[args.workload]()
    T, N = inst.packed()
    Td = torch.from_numpy(T.view(np.int64)).cuda()
    Nd = torch.from_numpy(N.view(np.int64)).cuda()
    stream = torch.cuda.current_stream()
    h, p, q = inst.h, inst.alpha_p, inst.alpha_q

    def solve(sv):
        rounds, st, _ = sv.wsc(h, p, q, target=inst.target_covered)
        return rounds, st

    # ---- paper's walk (empty-intersection pruning): the timed steps
    sv = pdfs.Solver(Td, Nd, inst.n_tumor, inst.n_normal, "empty", 0, stream.cuda_stream,
                     time_kernels=True)
    for i in range(args.warmup):
        solve(sv)
        print(f"[bench] warmup solve {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        rounds, st = solve(sv)
        stats.append(st)
        print(f"[bench] solve {i + 1}/{args.steps}: {len(rounds)} rounds", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sv.close()
    print(f"[bench] {args.steps} empty-mode solves in {elapsed:.3f} s", file=sys.stderr,
          flush=True)

    scored = stats[0]["nonempty"][h]
    assert all(s["nonempty"][h] == scored for s in stats)
    # the same count from the oracle's stored walk of this solve (every round
    # of Alg. 2 run on the CPU), when one is stored for the workload
    oracle_scored = oracle_subsets_scored(inst.name)
    if oracle_scored is not None:
        assert scored == oracle_scored, (scored, oracle_scored)
    ms_per_step = 1e3 * elapsed / args.steps
    value = scored * args.steps / elapsed

    # dominant stage: the depth-first kernels of each round (HIP events on the
    # library's stream around the main DFS kernel, the bucketing kernels and
    # the depth-4 tile kernel); index 2 = the tile kernel alone
    dfs_ns = sum(s["kernel_ns"][1] for s in stats)
    dfs_launches = sum(s["kernel_launches"][1] for s in stats)
    tile_ns = sum(s["kernel_ns"][2] for s in stats)
    tile_launches = sum(s["kernel_launches"][2] for s in stats)
    ops = sum(dfs_alg_ops(s, h, inst.n_normal) for s in stats)
    ops_exec = sum(dfs_alg_ops(s, h, inst.n_normal, depth3_ops_per_word=2) for s in stats)
    achieved = ops / (dfs_ns * 1e-9) if dfs_ns else 0.0
    achieved_exec = ops_exec / (dfs_ns * 1e-9) if dfs_ns else 0.0
    pair_ns = sum(s["kernel_ns"][0] for s in stats)
    pair_ops = 2 * sum(s["pair_macs"] for s in stats)

    measured_peak = pdfs.pdfs_measure_int_peak(0)
    # the roof is the higher of the datasheet figure and the rate a probe of
    # the kernels' own and + popcount pair reaches on this device
    roof = max(VALU_PEAK, measured_peak)
    traffic = stage_traffic(inst.name)

    # ---- pruned vs exhaustive walk, first greedy round of the two smaller
    # workloads (the exhaustive walk of h4_G20000 visits ~6.7e15 leaves a round)
    exhaustive = None
    if not args.no_exhaustive:
        exhaustive = {}
        for name in ("h2_G500", "h3_G5000"):
            wi = synth.WORKLOADS[name]()
            Ti, Ni = wi.packed()
            row = {}
            for mode in ("none", "empty"):
                svx = pdfs.Solver(Ti, Ni, wi.n_tumor, wi.n_normal, mode, 0, stream.cuda_stream)
                r1, st1, _ = svx.wsc(wi.h, wi.alpha_p, wi.alpha_q, max_rounds=1)
                torch.cuda.synchronize()
                tx = time.perf_counter()
                r1, st1, _ = svx.wsc(wi.h, wi.alpha_p, wi.alpha_q, max_rounds=1)
                torch.cuda.synchronize()
                row[mode] = {"round1_ms": 1e3 * (time.perf_counter() - tx),
                             "visited": st1["visited"][1:wi.h + 1],
                             "nonempty": st1["nonempty"][1:wi.h + 1],
                             "genes": r1[0]["genes"] if r1 else None}
                svx.close()
            row["same_answer"] = row["none"]["genes"] == row["empty"]["genes"]
            row["visited_fraction"] = row["empty"]["visited"][-1] / math.comb(wi.G, wi.h)
            row["pruning_speedup"] = row["none"]["round1_ms"] / row["empty"]["round1_ms"]
            exhaustive[name] = row
            print(f"[bench] exhaustive vs pruned round 1, {name}: "
                  f"{row['none']['round1_ms']:.2f} ms vs {row['empty']['round1_ms']:.2f} ms",
                  file=sys.stderr, flush=True)

    # ---- deeper combinations (h = 5, 6) on the h3_G5000 cohort, first greedy
    # round: the per-lane subtree walk below the pair level
    deep = None
    if not args.no_deep:
        deep = {}
        wi = synth.WORKLOADS["h3_G5000"]()
        Ti, Ni = wi.packed()
        svx = pdfs.Solver(Ti, Ni, wi.n_tumor, wi.n_normal, "empty", 0, stream.cuda_stream)
        for hd in (5, 6):
            svx.wsc(hd, wi.alpha_p, wi.alpha_q, max_rounds=1)
            torch.cuda.synchronize()
            tx = time.perf_counter()
            r1, st1, _ = svx.wsc(hd, wi.alpha_p, wi.alpha_q, max_rounds=1)
            torch.cuda.synchronize()
            dt = time.perf_counter() - tx
            deep[f"h{hd}_G5000_round1"] = {
                "round1_ms": 1e3 * dt, "visited": st1["visited"][1:hd + 1],
                "nonempty": st1["nonempty"][1:hd + 1],
                "leaf_visits_per_s": st1["visited"][hd] / dt,
                "genes": r1[0]["genes"] if r1 else None,
                "tp": r1[0]["tp"] if r1 else None, "fp": r1[0]["fp"] if r1 else None}
            print(f"[bench] h = {hd} round 1 on h3_G5000: {1e3 * dt:.1f} ms, "
                  f"{st1['visited'][hd]:.3e} leaf visits", file=sys.stderr, flush=True)
        svx.close()
        # the whole cover (to the cohort's 95 % target) in bound mode (seed
        # phase, pair filter and bound pruning at every depth)
        svb = pdfs.Solver(Ti, Ni, wi.n_tumor, wi.n_normal, "bound", 0, stream.cuda_stream)
        for hd in (5, 6, 7):
            svb.wsc(hd, wi.alpha_p, wi.alpha_q, max_rounds=1)
            torch.cuda.synchronize()
            tx = time.perf_counter()
            rr, stb, _ = svb.wsc(hd, wi.alpha_p, wi.alpha_q, target=wi.target_covered)
            torch.cuda.synchronize()
            dt = time.perf_counter() - tx
            deep[f"h{hd}_G5000_cover_bound"] = {
                "solve_ms": 1e3 * dt, "rounds": len(rr), "covered": sum(r["tp"] for r in rr),
                "visited": stb["visited"][1:hd + 1], "bound_pruned": stb["bound_pruned"][1:hd + 1]}
            print(f"[bench] h = {hd} cover of h3_G5000 (bound): {len(rr)} rounds in "
                  f"{1e3 * dt:.1f} ms", file=sys.stderr, flush=True)
        svb.close()

    # ---- held-out coverage (accuracy protocol): learn on a 75 % split of the
    # samples with the GPU path, score the frozen combinations on both splits
    held = None
    if not args.no_heldout:
        from paper_2603_16721_amd import heldout
        held = {}
        for name, lit in (("h3_G5000", False), ("h4_G20000", False), ("h3_G5000", True)):
            wi = inst if name == args.workload else synth.WORKLOADS[name]()
            r = heldout.learn_and_evaluate(pdfs, wi, 0.25, seed=16721600, tn_literal=lit)
            r.pop("combos")
            key = name + ("_tn_literal" if lit else "")
            held[key] = r
            print(f"[bench] held-out {key}: {r['combinations']} combinations, test sensitivity "
                  f"{r['test']['sensitivity']:.3f}, specificity {r['test']['specificity']:.3f}",
                  file=sys.stderr, flush=True)

    # ---- exact bound pruning (library default): solve time of the same workload
    bound_ms, same, bound_rounds = None, None, None
    if not args.no_bound:
        svb = pdfs.Solver(Td, Nd, inst.n_tumor, inst.n_normal, "bound", 0, stream.cuda_stream)
        rb, _ = solve(svb)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(args.bound_steps):
            rb2, _ = solve(svb)
        torch.cuda.synchronize()
        bound_ms = 1e3 * (time.perf_counter() - tb) / args.bound_steps
        svb.close()
        same = [(r["genes"], r["tp"], r["fp"]) for r in rb2] == \
            [(r["genes"], r["tp"], r["fp"]) for r in rounds]
        bound_rounds = [(r["genes"], r["tp"], r["fp"]) for r in rb2]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "subsets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": inst.name, "G": inst.G, "n_tumor": inst.n_tumor,
                   "n_normal": inst.n_normal, "h": h, "alpha": f"{p}/{q}",
                   "prune": "empty", "rounds": len(rounds), "subsets_scored_per_solve": scored,
                   "oracle_subsets_scored_per_solve": oracle_scored, "seed": inst.seed},
        "wsc_solve_ms": {"empty": ms_per_step, "bound": bound_ms},
        "bound_matches_empty": same,
        # the same canonical subsets (the empty-mode leaves) over the bound-mode solve time
        "bound_effective_subsets_per_s": (scored / (bound_ms * 1e-3)) if bound_ms else None,
        # Alg. 2's visited depth-h nodes against the C(G,h) subsets of every round
        "visited_fraction": stats[0]["visited"][h] / (len(rounds) * math.comb(inst.G, h)),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": roof / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved / roof,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "traffic_GBps": (traffic / (dfs_ns / max(1, dfs_launches) * 1e-9) / 1e9
                                      if traffic and dfs_ns else None),
                     "kernel": "depth-first stage per round: k_tri_begin, k_dfs<4,W>, "
                               "k_scan_c, k_scatter_c, k_dfs4_tiles<W>",
                     "launches": dfs_launches,
                     "avg_launch_ms": (dfs_ns / max(1, dfs_launches)) * 1e-6,
                     "tile_kernel_avg_ms": (tile_ns / max(1, tile_launches)) * 1e-6,
                     "ops_per_solve": ops // args.steps,
                     "peak_datasheet": VALU_PEAK / 1e12,
                     # the and + popcount pair measured by a probe kernel on this device
                     "peak_measured": measured_peak / 1e12,
                     "frac_of_datasheet": achieved / VALU_PEAK,
                     # depth-3 nodes of h = 4 charged at the and-or test the kernel runs
                     "frac_depth3_executed": achieved_exec / roof},
        "pair_table": {"bound": "mfma", "achieved": pair_ops / max(1e-12, pair_ns * 1e-9) / 1e12,
                       "peak": MFMA_I8_PEAK_OPS / 1e12, "unit": "TOP/s (int8)",
                       "frac": pair_ops / max(1e-12, pair_ns * 1e-9) / MFMA_I8_PEAK_OPS,
                       "avg_launch_ms": pair_ns / max(1, sum(s["kernel_launches"][0]
                                                             for s in stats)) * 1e-6},
    }
    if exhaustive is not None:
        out["exhaustive_vs_pruned_round1"] = exhaustive
    if deep is not None:
        out["deep_round1"] = deep
    if held is not None:
        out["heldout_75_25"] = held
    if not args.no_small_solves:
        out["small_solves"] = bench_small_solves(pdfs, stream.cuda_stream)
    if not args.no_batched:
        print("[bench] batched: 32 instances, plain serial vs batched", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(pdfs, data_b)
    if not args.no_served:
        print(f"[bench] served: {args.served_requests} requests", file=sys.stderr, flush=True)
        out["served"] = bench_served(pdfs, data_s, args.served_saturate)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host cores", file=sys.stderr, flush=True)
        cb = cpu_baseline(inst, T, N, args.cpu_every, not args.cpu_sample)
        rounds_cpu = cb.pop("_rounds")
        if bound_rounds is not None:
            cb["bound_solve_matches_gpu"] = rounds_cpu == bound_rounds
        cb["gpu_bound_solve_speedup"] = (cb["bound_solve_ms"] / bound_ms) if bound_ms else None
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
