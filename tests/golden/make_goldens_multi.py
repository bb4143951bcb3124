"""Writes batched_oracle.json and served_oracle.json: the oracle's greedy
rounds for every instance of the 32-instance batched workload and for a sample
of the served request stream.  Calls only oracle/ (and the seeded input
generator); nothing here touches the GPU path.

    python tests/golden/make_goldens_multi.py
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SERVED_SAMPLE = list(range(0, 2000, 50))


def _solve(kind, i):
    sys.path.insert(0, ROOT)
    from oracle import cpu
    from paper_2603_16721_amd import synth
    inst = synth.batched_instance(i) if kind == "batched" else synth.served_request(i)
    T, N = inst.packed()
    t0 = time.time()
    r = cpu.wsc(T, N, inst.n_tumor, inst.n_normal, inst.h, inst.alpha_p, inst.alpha_q,
                target=inst.target_covered, mode="bound")
    rounds = [[*x["genes"], x["tp"], x["fp"], x["score_num"]] for x in r.rounds]
    return i, {"name": inst.name, "seed": inst.seed, "G": inst.G, "n_tumor": inst.n_tumor,
               "n_normal": inst.n_normal, "h": inst.h, "rounds": rounds,
               "oracle_seconds": round(time.time() - t0, 2)}


def main():
    jobs = [("batched", i) for i in range(32)] + [("served", j) for j in SERVED_SAMPLE]
    out = {"batched": {}, "served": {}}
    with ProcessPoolExecutor(max(1, (os.cpu_count() or 2) - 1)) as ex:
        futs = {ex.submit(_solve, k, i): (k, i) for k, i in jobs}
        for f in futs:
            k, i = futs[f]
            _, rec = f.result()
            out[k][str(i)] = rec
            print(k, i, len(rec["rounds"]), rec["oracle_seconds"], flush=True)
    fmt = "each round: caller gene ids (sorted order), tp, fp, score_num"
    for k in ("batched", "served"):
        with open(os.path.join(HERE, f"{k}_oracle.json"), "w") as f:
            json.dump({"source": "oracle/pdfs_oracle.c (bound mode) via make_goldens_multi.py",
                       "format": fmt, "instances": out[k]}, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
