"""Writes oracle_counters.json: expected values that take the oracle too long
to recompute inside a test.  Calls only oracle/ (and the seeded input
generator); nothing here touches the GPU path.

    python tests/golden/make_goldens.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cpu  # noqa: E402
from paper_2603_16721_amd import synth  # noqa: E402


def main():
    out = {"source": "oracle/pdfs_oracle.c via tests/golden/make_goldens.py", "cases": {}}
    jobs = [
        # (key, workload, max_rounds): EMPTY mode = the paper's Alg. 2 walk
        ("h3_G5000_empty_all_rounds", synth.workload_h3_g5000, 0),
        ("h4_G20000_empty_round1", synth.workload_h4_g20000, 1),
    ]
    for key, make, maxr in jobs:
        I = make()
        T, N = I.packed()
        t0 = time.time()
        r = cpu.wsc(T, N, I.n_tumor, I.n_normal, I.h, I.alpha_p, I.alpha_q,
                    target=I.target_covered, max_rounds=maxr, mode="empty")
        out["cases"][key] = {"workload": I.name, "seed": I.seed, "h": I.h, "max_rounds": maxr,
                             "target": I.target_covered, "rounds": r.rounds,
                             "visited": r.counters["visited"], "nonempty": r.counters["nonempty"],
                             "oracle_seconds": round(time.time() - t0, 1)}
        print(key, len(r.rounds), "rounds", round(time.time() - t0, 1), "s", flush=True)
    with open(os.path.join(HERE, "oracle_counters.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
