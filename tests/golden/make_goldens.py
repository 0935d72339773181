"""Write the stored motif sets the GPU parity tests compare against.

Every set here is computed by the CPU oracle (``oracle.solve_a`` for (9,2),
``oracle.solve_b`` elsewhere; both exact, pinned by tests/test_oracle_pins.py)
on instances drawn by the seeded generator, and by nothing else.  For each
instance the file keeps the generator parameters, the number of motifs, the
SHA-256 of the sorted set (each motif followed by a newline), the set itself
when it has at most ``KEEP`` motifs, and the oracle's work counts at the
stack size t it ran with (the units the benchmark's roofline charges).

Usage:  python tests/golden/make_goldens.py [group ...] [--threads N]
Groups: plain (the (9,2), (13,4), (15,5) single instances, n=20, m=600,
seeds 0-4), large ((17,6) seeds 0-2), batched (a seeded sample of the
256-instance mixed batch), serving (a seeded sample of the 10,000-request
served stream), protein (a seeded sample of the 256-instance batch over the
20 amino acids).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import random
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1307_0571_amd import instances as I  # noqa: E402

KEEP = 4096
BATCH_SEED0, BATCH_COUNT = 1000, 256
BATCH_LD = ((11, 3), (13, 4), (15, 5))
SERVE_SEED0, SERVE_COUNT = 2000, 10000
SERVE_LD = ((9, 2), (11, 3), (13, 4), (15, 5), (17, 6))
PROTEIN_SEED0, PROTEIN_COUNT = 3000, 256
PROTEIN_LD = ((11, 4), (13, 5), (15, 6))


def digest(motifs) -> str:
    h = hashlib.sha256()
    for x in motifs:
        h.update(x.encode("ascii") + b"\n")
    return h.hexdigest()


def expected_spurious(l: int, d: int, n: int, m: int, sigma: int = 4) -> float:
    """Appendix C: sigma^l (1 - (1 - N_d / sigma^l)^(m-l+1))^n."""
    nd = sum(math.comb(l, i) * (sigma - 1) ** i for i in range(d + 1))
    p = nd / float(sigma) ** l
    return float(sigma) ** l * (1.0 - (1.0 - p) ** (m - l + 1)) ** n


def entry(inst, threads, t=3, kind="b"):
    t0 = time.time()
    if kind == "a":
        res = oracle.solve_a(inst.seqs, inst.l, inst.d, alphabet=inst.alphabet, threads=threads)
        st = None
    else:
        res, st = oracle.solve_b(inst.seqs, inst.l, inst.d, alphabet=inst.alphabet, t=t,
                                 threads=threads, stats=True)
        st = {k: v for k, v in st.items() if k != "pushes"}
    e = {"seed": inst.seed, "l": inst.l, "d": inst.d, "n": inst.n, "m": inst.m,
         "motif": inst.motif, "count": len(res), "sha256": digest(res),
         "oracle": "solve_a" if kind == "a" else "solve_b", "t": None if kind == "a" else t,
         "stats": st, "cpu_s": round(time.time() - t0, 2), "threads": threads}
    if len(res) <= KEEP:
        e["motifs"] = res
    assert inst.motif in res, "the planted motif must be reported"
    print(json.dumps({k: v for k, v in e.items() if k not in ("motifs", "stats")}), flush=True)
    return e


def group_plain(threads):
    out = []
    for s in range(5):
        out.append(entry(I.planted(s, 9, 2), threads, kind="a"))
    for (l, d) in ((13, 4), (15, 5)):
        for s in range(5):
            out.append(entry(I.planted(s, l, d), threads))
    return {"workload": "planted DNA, n=20, m=600, exactly d substitutions per copy",
            "instances": out}


def group_large(threads):
    out = [entry(I.planted(s, 17, 6), threads) for s in range(3)]
    return {"workload": "(17,6) planted DNA, n=20, m=600", "instances": out}


def batched_sample():
    """Indices into batch_mix(1000, 256): 28 drawn by a seeded RNG plus the
    4 with the largest Appendix C expected number of spurious motifs."""
    insts = I.batch_mix(BATCH_SEED0, BATCH_COUNT, ld=BATCH_LD)
    rng = random.Random(20240)
    picked = set(rng.sample(range(BATCH_COUNT), 28))
    heavy = sorted(range(BATCH_COUNT),
                   key=lambda k: -expected_spurious(insts[k].l, insts[k].d, insts[k].n,
                                                    insts[k].m))
    for k in heavy:
        if len(picked) >= 32:
            break
        picked.add(k)
    return insts, sorted(picked)


def group_batched(threads):
    insts, idx = batched_sample()
    out = []
    for k in idx:
        e = entry(insts[k], threads)
        e["index"] = k
        out.append(e)
    return {"workload": f"batch_mix({BATCH_SEED0}, {BATCH_COUNT}), (l,d) in {list(BATCH_LD)}, "
                        "n in [10,30], m in [300,1000]",
            "sample": "28 seeded (random.Random(20240)) + the 4 largest Appendix C "
                      "expected spurious counts", "instances": out}


def serving_sample():
    """Indices into the served stream: 12 seeded draws among the (9,2),
    (11,3), (13,4) requests and 6 among the (15,5), (17,6) requests whose
    strings number at most 20 (bounded oracle time)."""
    insts = I.batch_mix(SERVE_SEED0, SERVE_COUNT, ld=SERVE_LD, m_range=(200, 1000))
    rng = random.Random(20241)
    light = [k for k, x in enumerate(insts) if x.l <= 13]
    heavy = [k for k, x in enumerate(insts) if x.l >= 15 and x.n <= 20 and x.m <= 700]
    return insts, sorted(rng.sample(light, 12) + rng.sample(heavy, 6))


def group_serving(threads):
    insts, idx = serving_sample()
    out = []
    for k in idx:
        e = entry(insts[k], threads)
        e["index"] = k
        out.append(e)
    return {"workload": f"batch_mix({SERVE_SEED0}, {SERVE_COUNT}), (l,d) in {list(SERVE_LD)}, "
                        "n in [10,30], m in [200,1000]",
            "sample": "12 seeded (random.Random(20241)) of the l <= 13 requests, 6 of the "
                      "l >= 15 requests with n <= 20 and m <= 700", "instances": out}


def group_protein(threads):
    """16 of batch_mix(3000, 256) over the 20 amino acids: 12 seeded draws
    plus the 4 with the largest Appendix C expected number of spurious
    motifs."""
    insts = I.batch_mix(PROTEIN_SEED0, PROTEIN_COUNT, ld=PROTEIN_LD, alphabet=I.PROTEIN)
    rng = random.Random(20242)
    picked = set(rng.sample(range(PROTEIN_COUNT), 12))
    heavy = sorted(range(PROTEIN_COUNT),
                   key=lambda k: -expected_spurious(insts[k].l, insts[k].d, insts[k].n,
                                                    insts[k].m, 20))
    for k in heavy:
        if len(picked) >= 16:
            break
        picked.add(k)
    out = []
    for k in sorted(picked):
        e = entry(insts[k], threads)
        e["index"] = k
        e["alphabet"] = I.PROTEIN
        out.append(e)
    return {"workload": f"batch_mix({PROTEIN_SEED0}, {PROTEIN_COUNT}) over the 20 amino acids, "
                        f"(l,d) in {list(PROTEIN_LD)}, n in [10,30], m in [300,1000]",
            "sample": "12 seeded (random.Random(20242)) + the 4 largest Appendix C "
                      "expected spurious counts", "instances": out}


GROUPS = {"plain": group_plain, "large": group_large, "batched": group_batched,
          "serving": group_serving, "protein": group_protein}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("groups", nargs="*", default=list(GROUPS))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for g in args.groups:
        data = GROUPS[g](args.threads)
        data["source"] = ("oracle (CPU) on the seeded generator's instances; "
                          "tests/golden/make_goldens.py " + g)
        with open(os.path.join(HERE, f"sets_{g}.json"), "w") as f:
            json.dump(data, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
