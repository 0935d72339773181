"""Write the search work PMS8 does on the benchmark's instances, counted by
the CPU oracle (Algorithm 2 with Algorithm 1 and the Theorem 1 filter): the
units the benchmark's roofline charges per launch.

work_units.json          plain (13,4) and (15,5), n=20, m=600, seeds 0-4:
                         full counts at stack size t = 3.
work_units_batched.json  the 256-instance mixed batch: counts on a run of 16
                         consecutive S_1 windows per instance starting at a
                         seeded uniform position (the independent
                         sub-problems of Section 2.3, so the counts of a
                         window set add up; every window is equally likely
                         to be counted), scaled by r / 16, at t = 2 and
                         t = 3 (the benchmark picks the t the device ran).

Usage: python tests/golden/make_work_units.py [plain] [batched] [--threads N]
Calls only the oracle and the seeded instance generator.
"""
import argparse
import json
import os
import random
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1307_0571_amd import instances as I  # noqa: E402

UNITS = ("push_tries", "filter_words", "filter_tests", "compat_pass", "triple_tests",
         "tuples", "gen_nodes", "leaves", "verify_tests")
SAMPLE_WINDOWS = 16


def _units(st):
    return {k: st[k] for k in UNITS}


def plain(threads):
    out = {"source": "oracle.solve_b(..., stats=True) on planted instances, n=20, m=600, "
                     "full counts", "instances": []}
    for (l, d, t) in ((13, 4, 3), (15, 5, 3)):
        for seed in range(5):
            inst = I.planted(seed, l, d, 20, 600)
            t0 = time.time()
            res, st = oracle.solve_b(inst.seqs, l, d, t=t, stats=True, threads=threads)
            e = {"l": l, "d": d, "n": 20, "m": 600, "seed": seed, "t": t, "motifs": len(res),
                 **_units(st), "cpu_s": round(time.time() - t0, 2)}
            out["instances"].append(e)
            print(e, flush=True)
    with open(os.path.join(HERE, "work_units.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def batched(threads):
    insts = I.batch_mix(1000, 256)
    rng = random.Random(20242)
    out = {"source": f"oracle.solve_b(..., stats=True, windows=...) on batch_mix(1000, 256): "
                     f"{SAMPLE_WINDOWS} consecutive S_1 windows per instance from a seeded "
                     "uniform start (random.Random(20242)), counts scaled by r / windows",
           "instances": []}
    for k, x in enumerate(insts):
        r = x.m - x.l + 1
        w0 = rng.randint(0, max(0, r - SAMPLE_WINDOWS))
        w1 = min(r, w0 + SAMPLE_WINDOWS)
        e = {"index": k, "seed": x.seed, "l": x.l, "d": x.d, "n": x.n, "m": x.m,
             "windows": [w0, w1], "by_t": {}}
        t0 = time.time()
        for t in (2, 3):
            _, st = oracle.solve_b(x.seqs, x.l, x.d, t=t, stats=True, threads=threads,
                                   windows=(w0, w1))
            e["by_t"][str(t)] = {u: st[u] * r / (w1 - w0) for u in UNITS}
        e["cpu_s"] = round(time.time() - t0, 2)
        out["instances"].append(e)
        print(k, x.l, x.d, x.n, x.m, e["cpu_s"], flush=True)
    with open(os.path.join(HERE, "work_units_batched.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("groups", nargs="*", default=["plain", "batched"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for g in args.groups:
        {"plain": plain, "batched": batched}[g](args.threads)


if __name__ == "__main__":
    main()
