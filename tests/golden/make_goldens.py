"""Writes oracle_counters.json: expected values that take the oracle too long
to recompute inside a test.  Calls only oracle/ (and the seeded input
generator); nothing here touches the GPU path.

    python tests/golden/make_goldens.py            # every case
    python tests/golden/make_goldens.py KEY ...    # the named cases, the rest kept
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cpu  # noqa: E402
from paper_2603_16721_amd import synth  # noqa: E402

# ---- whole solves too long for one core: every round's first-gene loop cut
# into shares (the outer-loop intervals of Sec. III-D), run in a process pool
_W = {}


def _share_init(make_name):
    I = synth.WORKLOADS[make_name]()
    T, N = I.packed()
    _W.update(I=I, T=T, N=N, perm=cpu.order(T, N))


def _share_job(args):
    r, lo, hi, U, h = args
    I = _W["I"]
    b = cpu.best_share(_W["T"], _W["N"], I.n_tumor, I.n_normal, h, I.alpha_p, I.alpha_q, lo, hi,
                       U=np.asarray(U, dtype=np.uint64), mode="empty", perm=_W["perm"])
    return r, lo, b


def empty_solve_by_shares(name, step=128, workers=None):
    """The greedy solve of workload `name` in empty-intersection mode (Alg. 2 at
    every round), each round's outer loop cut into shares of `step` first
    genes.  The uncovered mask of every round comes from the oracle's
    bound-mode solve; each round's empty-mode answer, merged over the shares
    under (S desc, tuple asc), must equal that round's bound-mode answer, which
    makes the mask sequence the empty-mode solve's own.  Returns the rounds and
    the per-round counters."""
    I = synth.WORKLOADS[name]()
    T, N = I.packed()
    h = I.h
    seq = cpu.wsc(T, N, I.n_tumor, I.n_normal, h, I.alpha_p, I.alpha_q,
                  target=I.target_covered, mode="bound")
    perm = cpu.order(T, N)
    wt = T.shape[1]
    U = cpu.full_mask(I.n_tumor, wt)
    masks = []
    for rd in seq.rounds:
        masks.append([int(x) for x in U])
        cov = U.copy()
        for g in rd["genes"]:
            cov &= T[g]
        U = U & ~cov
    jobs = [(r, lo, min(lo + step, I.G), masks[r], h)
            for r in range(len(masks)) for lo in range(0, I.G, step)]
    per_round = [dict(best=None, visited=[0] * (cpu.MAX_H + 1), nonempty=[0] * (cpu.MAX_H + 1))
                 for _ in masks]
    done = 0
    t0 = time.time()
    with mp.get_context("fork").Pool(workers or max(1, (os.cpu_count() or 2) - 1),
                                     initializer=_share_init, initargs=(name,)) as pool:
        for r, lo, b in pool.imap_unordered(_share_job, jobs, chunksize=1):
            pr = per_round[r]
            for k in ("visited", "nonempty"):
                pr[k] = [x + y for x, y in zip(pr[k], b.counters[k])]
            if b.found and (pr["best"] is None or
                            (b.score, [-i for i in b.sorted_idx]) >
                            (pr["best"].score, [-i for i in pr["best"].sorted_idx])):
                pr["best"] = b
            done += 1
            if done % 500 == 0:
                print(f"  {name}: {done}/{len(jobs)} shares, {time.time() - t0:.0f} s", flush=True)
    rounds = []
    for r, (rd, pr) in enumerate(zip(seq.rounds, per_round)):
        b = pr["best"]
        assert b is not None and list(b.sorted_idx) == rd["sorted_idx"], (r, b, rd)
        assert (b.tp, b.fp) == (rd["tp"], rd["fp"]), r
        assert list(perm[list(b.sorted_idx)]) == rd["genes"], r
        rounds.append(rd)
    return I, rounds, per_round


def main(keys):
    path = os.path.join(HERE, "oracle_counters.json")
    out = {"source": "oracle/pdfs_oracle.c via tests/golden/make_goldens.py", "cases": {}}
    if keys and os.path.exists(path):
        with open(path) as f:
            out["cases"] = json.load(f)["cases"]
    jobs = [
        # (key, workload, max_rounds, h or None for the workload's own):
        # EMPTY mode = the paper's Alg. 2 walk
        ("h3_G5000_empty_all_rounds", synth.workload_h3_g5000, 0, None),
        ("h4_G20000_empty_round1", synth.workload_h4_g20000, 1, None),
        # deeper combinations on the h3_G5000 cohort (first greedy round)
        ("h5_G5000_empty_round1", synth.workload_h3_g5000, 1, 5),
        ("h6_G5000_empty_round1", synth.workload_h3_g5000, 1, 6),
    ]
    for key, make, maxr, hh in jobs:
        if keys and key not in keys:
            continue
        I = make()
        h = hh or I.h
        T, N = I.packed()
        t0 = time.time()
        r = cpu.wsc(T, N, I.n_tumor, I.n_normal, h, I.alpha_p, I.alpha_q,
                    target=I.target_covered, max_rounds=maxr, mode="empty")
        out["cases"][key] = {"workload": I.name, "seed": I.seed, "h": h, "max_rounds": maxr,
                             "target": I.target_covered, "rounds": r.rounds,
                             "visited": r.counters["visited"], "nonempty": r.counters["nonempty"],
                             "oracle_seconds": round(time.time() - t0, 1)}
        print(key, len(r.rounds), "rounds", round(time.time() - t0, 1), "s", flush=True)
    key = "h4_G20000_empty_all_rounds"
    if not keys or key in keys:
        t0 = time.time()
        I, rounds, per_round = empty_solve_by_shares("h4_G20000")
        tot_v = [sum(pr["visited"][l] for pr in per_round) for l in range(cpu.MAX_H + 1)]
        tot_n = [sum(pr["nonempty"][l] for pr in per_round) for l in range(cpu.MAX_H + 1)]
        out["cases"][key] = {
            "workload": I.name, "seed": I.seed, "h": I.h, "max_rounds": 0,
            "target": I.target_covered, "rounds": rounds, "visited": tot_v, "nonempty": tot_n,
            "per_round_visited": [pr["visited"] for pr in per_round],
            "per_round_nonempty": [pr["nonempty"] for pr in per_round],
            "method": "empty-mode shares of 128 first genes per round, masks from the bound-mode "
                      "solve, every round's merged answer equal to the bound-mode round's",
            "oracle_seconds": round(time.time() - t0, 1)}
        print(key, len(rounds), "rounds", round(time.time() - t0, 1), "s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
