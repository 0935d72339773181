"""Write work_units.json: the search work PMS8 does on the benchmark's
instances, counted by the CPU oracle (Algorithm 2 with Algorithm 1 and the
Theorem 1 filter) at the same threshold t the device path uses.

Usage: python tests/golden/make_work_units.py
Calls only the oracle and the seeded instance generator.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1307_0571_amd import instances as I  # noqa: E402

# (l, d, t): t as the device path's threshold rule gives for n=20, m=600
CASES = [(13, 4, 3), (15, 5, 3)]


def main():
    out = {"source": "oracle.solve_b(..., stats=True) on planted instances, n=20, m=600",
           "instances": []}
    for (l, d, t) in CASES:
        for seed in (0, 1, 2, 3, 4):
            inst = I.planted(seed, l, d, 20, 600)
            t0 = time.time()
            res, st = oracle.solve_b(inst.seqs, l, d, t=t, stats=True)
            out["instances"].append({
                "l": l, "d": d, "n": 20, "m": 600, "seed": seed, "t": t,
                "motifs": len(res), "pushes": sum(st["pushes"]),
                "filter_tests": st["filter_tests"], "tuples": st["tuples"],
                "gen_nodes": st["gen_nodes"], "leaves": st["leaves"],
                "verify_tests": st["verify_tests"], "cpu_s": round(time.time() - t0, 2)})
            print(out["instances"][-1], flush=True)
    with open(os.path.join(HERE, "work_units.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
