"""Writes oracle_counters.json: expected values that take the oracle too long
to recompute inside a test.  Calls only oracle/ (and the seeded input
generator); nothing here touches the GPU path.

    python tests/golden/make_goldens.py            # every case
    python tests/golden/make_goldens.py KEY ...    # the named cases, the rest kept
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cpu  # noqa: E402
from paper_2603_16721_amd import synth  # noqa: E402


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
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
