#!/usr/bin/env python3
"""Benchmark: exact planted motif search on one MI355X.

Default workload (the batched configuration): 256 planted DNA instances,
(l,d) uniform from {(11,3),(13,4),(15,5)}, n uniform in [10,30], m uniform in
[300,1000], exactly d substitutions per planted copy, seeds 1000-1255.  One
step is one device pass of the whole batch (pack, compat bit-matrix, level-1
expansion, persistent search, sort/unique) with the inputs already resident
in HBM, and the copy of every motif set back to the host.  After the timed
steps the same 256 instances are solved the plain way (one device pipeline
run per instance, inputs resident) and timed, for the batched/plain ratio.

Prints one JSON line: `value` is the batched instances/s; beside it the plain
rate, the Hd compares per second, the dominant kernel's roofline and the CPU
oracle timed on a bounded sample of the same workload.

Other workloads: --workload plain (the (13,4)/(15,5) single instances),
serving (a Poisson stream on the served mix), large ((17,6) and (19,7)),
protein (the batched configuration over the 20 amino acids: (l,d) uniform
from {(11,4),(13,5),(15,6)}, same n and m ranges, seeds 3000-3255).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import random
import sys
import threading
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "instances/s and Hd compares/s (mixed l,d), batched vs plain GPU, exact motif set"
# int32 VALU lane-ops/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64
# instruction is 64 lane-ops issued over 4 cycles on one SIMD)
PEAK_INT_TOPS = 256 * 64 * 2.4e9 / 1e12
BATCH_SEED0, BATCH_COUNT = 1000, 256
PROTEIN_SEED0, PROTEIN_LD = 3000, ((11, 4), (13, 5), (15, 6))
SERVE_LD = ((9, 2), (11, 3), (13, 4), (15, 5), (17, 6))


def lane_ops(u: dict, t: int) -> float:
    """Algorithmic VALU lane-ops of one instance's search (1-word l-mers),
    from the oracle's unit counts of the same algorithm at the same t:

    * filter: 2 lane-ops (AND + popcount) per 64-bit row word a push
      touches, plus about 14 per Theorem 1 test (Cd of a survivor that
      passed the 2d bit, against one earlier stack member);
    * generator: 4 lane-ops per pair and per triple suffix test,
      4 (C(t,2) + C(t,3)) per tree node;
    * verification: 5 lane-ops per (candidate, survivor) Hamming test."""
    pairs = t * (t - 1) // 2
    triples = t * (t - 1) * (t - 2) // 6
    return (2.0 * u["filter_words"] + 14.0 * u["triple_tests"] +
            4.0 * (pairs + triples) * u["gen_nodes"] + 5.0 * u["verify_tests"])


TRAFFIC_FILE = os.path.join(HERE, "profiles", "k_search_traffic_batched_256.json")
KERNEL_SRCS = [os.path.join(HERE, "paper_1307_0571_amd", "csrc", f)
               for f in ("pms_kernels.hip", "pms_internal.h", "pms_runtime.cpp")]


def kernel_sha256() -> str:
    """SHA-256 over the kernel source and the launch parameters' sources."""
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_traffic():
    """HBM bytes per k_search launch pair of one batched pass, from the
    committed FETCH_SIZE / WRITE_SIZE counter runs scaled by the copy
    calibration; None once the kernel source differs from the one the
    counters were taken on."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_sha256():
        return None
    return t


def load_json(name):
    path = os.path.join(HERE, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(insts, budget_s: float = 20.0):
    """The oracle (PMS8 written plainly on the CPU, all host threads) on a
    bounded sample of the workload: 8 seeded instances, each on a run of its
    independent S_1 sub-problems (Section 2.3) grown until its share of the
    budget is used, time scaled by r / windows; plus the plain
    sample-driven oracle on one (9,2) instance (n=20, m=600) on one thread."""
    import oracle
    from oracle.oracle import default_threshold
    from paper_1307_0571_amd import instances as I
    cores, model = cpu_info()
    rng = random.Random(99)
    sample = rng.sample(range(len(insts)), min(8, len(insts)))
    per = budget_s / len(sample)
    est = []
    desc = []
    for k in sample:
        x = insts[k]
        r = x.m - x.l + 1
        t = default_threshold(x.n, x.m, x.l, x.d, len(x.alphabet))
        lo, hi, spent, done = 0, 1, 0.0, 0
        while True:
            t0 = time.perf_counter()
            oracle.solve_b(x.seqs, x.l, x.d, alphabet=x.alphabet, t=t, threads=cores,
                           windows=(lo, hi))
            spent += time.perf_counter() - t0
            done += hi - lo
            if hi >= r or spent > per * 0.5:
                break
            lo, hi = hi, min(r, hi + max(1, (hi - lo) * 2))
        est.append(spent * r / done)
        desc.append(f"#{k} ({x.l},{x.d}) n={x.n} m={x.m}: {done}/{r} windows")
    c1 = I.planted(0, 9, 2, 20, 600)
    t0 = time.perf_counter()
    oracle.solve_a(c1.seqs, 9, 2, threads=1)
    c1_s = time.perf_counter() - t0
    return {"value": round(1.0 / (sum(est) / len(est)), 5), "unit": "instances/s",
            "cores": cores, "kind": "oracle", "nproc": cores, "cpu_model": model,
            "sample": "; ".join(desc) + " (time scaled by r / windows done; mean over the 8)",
            "c1_9_2_one_thread_instances_per_s": round(1.0 / c1_s, 3)}


def hd_compares(insts, units, t_of):
    """Compat: every unordered pair of l-mers from different strings, one
    Hd test each; verify: the (candidate, survivor) Hd tests of the oracle's
    count of the same search (sampled windows, scaled)."""
    compat = sum(x.n * (x.n - 1) // 2 * (x.m - x.l + 1) ** 2 for x in insts)
    verify = None
    if units is not None and all(str(t) in u["by_t"] for t, u in zip(t_of, units)):
        verify = sum(units[k]["by_t"][str(t_of[k])]["verify_tests"] for k in range(len(insts)))
    return compat, verify


def run_batched(args, I, pms, insts=None):
    if insts is None:
        insts = I.batch_mix(BATCH_SEED0, args.count)
    probs = [pms.Problem(x.seqs, x.l, x.d, x.alphabet) for x in insts]
    tune = pms.Tune(threshold=args.threshold, waves_per_cu=args.wpc, split=args.split,
                    stage_cap=args.stage_cap, compat_kernel=args.compat_kernel)
    default_rate = None
    tuned_note = "flags"
    if args.autotune:
        # the autotuner proposes search parameters from a 64-instance sample
        # of the batch; the proposal and the defaults are each timed once on
        # the whole batch, and the faster of the two runs the timed steps
        base = tune

        def one_pass(t):
            b0 = pms.Batch(probs, tune=t)
            b0.run()
            b0.results()
            t0 = time.perf_counter()
            b0.run()
            b0.results()
            rate = len(probs) / (time.perf_counter() - t0)
            b0.close()
            return rate

        proposal = pms.autotune(probs, base=base, max_runs=args.tune_runs, sample=64)
        # a sample can favour a threshold the whole batch does not: the
        # proposal is also timed with the base's threshold
        kept_t = pms.Tune(**{**pms.tune_dict(proposal), "threshold": base.threshold})
        cands = [("defaults", base), ("proposal", proposal)]
        if proposal.threshold != base.threshold:
            cands.append(("proposal with the default threshold", kept_t))
        rates = [(one_pass(t), name, t) for name, t in cands]
        default_rate = rates[0][0]
        best = max(rates, key=lambda x: x[0])
        tune = best[2]
        tuned_note = (f"{best[1]} of pms_autotune (64-instance sample) on the whole batch: " +
                      ", ".join(f"{name} {r:.2f}" for r, name, _ in rates) + " instances/s; proposal " +
                      json.dumps({k: v for k, v in pms.tune_dict(proposal).items() if v}))
    b = pms.Batch(probs, tune=tune)
    for _ in range(args.warmup):
        b.run()
        b.results()
    pms.device_synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
        res = b.results()
        phases.append(b.timings())
    pms.device_synchronize()
    elapsed = time.perf_counter() - t0
    for x, r in zip(insts, res):
        if x.motif not in r:
            raise SystemExit(f"planted motif missing in batched instance seed {x.seed}")
    graph_rate = None
    if args.graph_steps > 0:
        b.run(graph=True)
        b.results()
        tg = time.perf_counter()
        for _ in range(args.graph_steps):
            b.run(graph=True)
            rg = b.results()
        graph_rate = args.count * args.graph_steps / (time.perf_counter() - tg)
        if rg != res:
            raise SystemExit("graph replay result differs from the eager run")
    b.close()
    # the same batch from host buffers: validation, encoding, upload, the
    # pipeline and the copy back (pms_solve_batch), PCIe included
    pms.solve_batch(probs, tune=tune)
    th = time.perf_counter()
    hres = pms.solve_batch(probs, tune=tune)
    host_rate = len(probs) / (time.perf_counter() - th)
    if hres != res:
        raise SystemExit("host-buffer result differs from the resident run")
    plain = None
    if not args.no_plain:
        singles = [pms.Batch([p]) for p in probs]  # pms_solve's own setting
        for sb in singles:
            sb.run()
            sb.results()
        pms.device_synchronize()
        tp = time.perf_counter()
        for sb, x in zip(singles, insts):
            sb.run()
            if x.motif not in sb.results()[0]:
                raise SystemExit(f"planted motif missing in plain instance seed {x.seed}")
        plain = time.perf_counter() - tp
        for sb in singles:
            sb.close()
    return (insts, elapsed, phases, plain, graph_rate, [len(r) for r in res], tune, default_rate,
            tuned_note, host_rate)


def batched_main(args, I, pms):
    (insts, elapsed, phases, plain_s, graph_rate, sizes, tune, default_rate, tuned_note,
     host_rate) = run_batched(args, I, pms)
    n = len(insts)
    value = n * args.steps / elapsed
    t_of = [tune.threshold or pms.default_threshold(x.n, x.m, x.l, x.d) for x in insts]
    wu = load_json("work_units_batched.json")
    units = None
    if wu and len(wu["instances"]) >= n and all(
            (e["seed"], e["l"], e["d"], e["n"], e["m"]) == (x.seed, x.l, x.d, x.n, x.m)
            for e, x in zip(wu["instances"], insts)):
        units = wu["instances"][:n]
    search_ms = sum(p[3] for p in phases) / len(phases)
    compat_ms = sum(p[1] for p in phases) / len(phases)
    roofline = None
    if units is not None and all(str(t) in u["by_t"] for t, u in zip(t_of, units)):
        ops = sum(lane_ops(u["by_t"][str(t)], t) for t, u in zip(t_of, units))
        achieved = ops / (search_ms * 1e-3) / 1e12
        tr = load_traffic()
        roofline = {"bound": "alu", "achieved": round(achieved, 5),
                    "peak": round(PEAK_INT_TOPS, 2), "unit": "TOP/s",
                    "frac": round(achieved / PEAK_INT_TOPS, 6),
                    "traffic": tr["hbm_bytes_per_launch"] if tr else None,
                    "kernel": "k_search (the two dispatches of one batched pass)",
                    "avg_launch_ms": round(search_ms, 3),
                    "algorithmic_lane_ops_per_launch": ops,
                    "units": "oracle counts of the same search at the device's t "
                             "(16 consecutive S_1 windows per instance, scaled by r/16)"}
    compat, verify = hd_compares(insts, units, t_of)
    ms_step = elapsed * 1e3 / args.steps
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "instances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 bitwise",
        "data": "synthetic planted DNA instances (seeded generator)",
        "config": {"workload": f"batched: {n} planted DNA instances, (l,d) uniform from "
                               "{(11,3),(13,4),(15,5)}, n in [10,30], m in [300,1000], "
                               f"seeds {BATCH_SEED0}-{BATCH_SEED0 + n - 1}; one step = one "
                               "device pass of the whole batch, inputs resident in HBM",
                   "instances": n,
                   "tune": {k: v for k, v in pms.tune_dict(tune).items()
                            if k in ("threshold", "lmer_words", "triple_filter", "waves_per_cu",
                                     "split", "stage_cap")},
                   "tuned_by": tuned_note},
        "default_tune_instances_per_s": round(default_rate, 3) if default_rate else None,
        "plain_instances_per_s": round(n / plain_s, 3) if plain_s else None,
        "batched_over_plain": round(value / (n / plain_s), 3) if plain_s else None,
        "graph_instances_per_s": round(graph_rate, 3) if graph_rate else None,
        "host_buffers_instances_per_s": round(host_rate, 3),
        "hd_compares_per_s": {
            "compat": round(compat / (ms_step * 1e-3), 1),
            "compat_phase": round(compat / (compat_ms * 1e-3), 1),
            "verify": round(verify / (ms_step * 1e-3), 1) if verify is not None else None,
            "total": round((compat + verify) / (ms_step * 1e-3), 1) if verify is not None else None,
            "verify_units": "oracle count of the same search (sampled windows, scaled)"},
        "phases_ms": {k: round(sum(p[i] for p in phases) / len(phases), 3)
                      for i, k in enumerate(("pack", "compat", "expand", "search", "sort"))},
        "max_motifs_per_instance": max(sizes),
        "roofline": roofline,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(insts, args.cpu_budget)
    print(json.dumps(out), flush=True)


def protein_main(args, I, pms):
    """The batched configuration over the 20 amino acids (five-plane l-mers,
    5-bit keys): batched and plain rates and the CPU oracle beside them."""
    insts = I.batch_mix(PROTEIN_SEED0, args.count, ld=PROTEIN_LD, alphabet=I.PROTEIN)
    (insts, elapsed, phases, plain_s, graph_rate, sizes, tune, default_rate, tuned_note,
     host_rate) = run_batched(args, I, pms, insts)
    n = len(insts)
    value = n * args.steps / elapsed
    out = {"workload": f"protein batched: {n} planted instances over the 20 amino acids, (l,d) "
                       "uniform from {(11,4),(13,5),(15,6)}, n in [10,30], m in [300,1000], "
                       f"seeds {PROTEIN_SEED0}-{PROTEIN_SEED0 + n - 1}; inputs resident in HBM",
           "instances_per_s": round(value, 3), "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
           "steps": args.steps,
           "tune": pms.tune_dict(tune), "tuned_by": tuned_note,
           "default_tune_instances_per_s": round(default_rate, 3) if default_rate else None,
           "plain_instances_per_s": round(n / plain_s, 3) if plain_s else None,
           "batched_over_plain": round(value / (n / plain_s), 3) if plain_s else None,
           "graph_instances_per_s": round(graph_rate, 3) if graph_rate else None,
           "host_buffers_instances_per_s": round(host_rate, 3),
           "phases_ms": {k: round(sum(p[i] for p in phases) / len(phases), 3)
                         for i, k in enumerate(("pack", "compat", "expand", "search", "sort"))},
           "max_motifs_per_instance": max(sizes)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(insts, args.cpu_budget)
    print(json.dumps(out), flush=True)


def plain_main(args, I, pms):
    """The plain single-instance configuration: (13,4) and (15,5), n=20,
    m=600, seeds 0-4, one device pipeline run per instance."""
    tune = pms.Tune(threshold=args.threshold, waves_per_cu=args.wpc, split=args.split)
    configs = [(13, 4), (15, 5)]
    batches = {}
    for s in range(5):
        for (l, d) in configs:
            inst = I.planted(s, l, d, 20, 600)
            batches[(s, l)] = (pms.Batch([pms.Problem(inst.seqs, l, d)], tune=tune), inst)
    wu = load_json("work_units.json")
    units = {(u["l"], u["d"], u["seed"]): u for u in wu["instances"]} if wu else {}
    phases = []

    def step(k, record):
        s = k % 5
        for (l, d) in configs:
            b, inst = batches[(s, l)]
            b.run()
            res = b.results()[0]
            if inst.motif not in res:
                raise SystemExit(f"planted motif missing for seed {s} ({l},{d})")
            if record:
                phases.append(((l, d), s, b.timings()[3]))

    for k in range(args.warmup):
        step(k, False)
    pms.device_synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, True)
    pms.device_synchronize()
    elapsed = time.perf_counter() - t0
    for b, _ in batches.values():
        b.close()
    roofline = None
    t_of = {ld: args.threshold or pms.default_threshold(20, 600, *ld) for ld in configs}
    counted = [(lane_ops(units[(ld[0], ld[1], s)], t_of[ld]), ms) for (ld, s, ms) in phases
               if (ld[0], ld[1], s) in units and units[(ld[0], ld[1], s)]["t"] == t_of[ld]]
    if counted and len(counted) == len(phases):
        ops = sum(o for o, _ in counted) / len(counted)
        avg_ms = sum(ms for _, ms in counted) / len(counted)
        achieved = ops / (avg_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 5),
                    "peak": round(PEAK_INT_TOPS, 2), "unit": "TOP/s",
                    "frac": round(achieved / PEAK_INT_TOPS, 6), "traffic": None,
                    "kernel": "k_search (the two dispatches of one search)",
                    "avg_launch_ms": round(avg_ms, 4),
                    "algorithmic_lane_ops_per_launch": ops,
                    "units": "oracle counts of the same instances at the same t"}
    n_inst = args.steps * len(configs)
    print(json.dumps({"workload": "plain (13,4)+(15,5), n=20, m=600, seeds 0-4",
                      "instances_per_s": round(n_inst / elapsed, 3),
                      "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
                      "search_ms": {f"{ld}": round(sum(ms for (l2, _, ms) in phases if l2 == ld) /
                                                   max(1, sum(1 for p in phases if p[0] == ld)), 3)
                                    for ld in configs},
                      "roofline": roofline}), flush=True)


def large_main(args, I, pms):
    out = {"workload": "large single instances, n=20, m=600"}
    for (l, d, seeds) in ((17, 6, (0, 1, 2)), (19, 7, (0,))):
        for s in seeds:
            inst = I.planted(s, l, d, 20, 600)
            b = pms.Batch([pms.Problem(inst.seqs, l, d)])
            t0 = time.perf_counter()
            b.run()
            res = b.results()[0]
            dt = time.perf_counter() - t0
            b.close()
            if inst.motif not in res:
                raise SystemExit(f"planted motif missing for ({l},{d}) seed {s}")
            out[f"({l},{d}) seed {s}"] = {"s": round(dt, 3), "motifs": len(res)}
            print(json.dumps({f"({l},{d}) seed {s}": out[f"({l},{d}) seed {s}"]}), flush=True)
    print(json.dumps(out), flush=True)


def long_main(args, I, pms):
    """Long strings (up to 8192 windows each): every instance runs with the
    library's choice of compat layout (the whole matrix below 1 GiB, else
    S_1's rows only) and with S_1's rows forced; both must give the same set,
    holding the planted motif.  One warm-up run per layout, then one timed."""
    out = {"workload": "long strings: planted DNA, n 6-20, 4000-8203 characters"}
    cases = ((50, 12, 2, 6, 8203), (47, 9, 1, 12, 8200), (60, 15, 4, 20, 4000),
             (61, 16, 4, 20, 8000), (62, 17, 5, 20, 4000))
    for (seed, l, d, n, m) in cases:
        inst = I.planted(seed, l, d, n, m)
        name = f"({l},{d}) n={n} m={m} seed {seed}"
        row, sets = {}, []
        for mode, label in ((0, "auto"), (2, "s1_rows")):
            b = pms.Batch([pms.Problem(inst.seqs, l, d)], tune=pms.Tune(compat_mode=mode))
            b.run()
            b.results()
            t0 = time.perf_counter()
            b.run()
            res = b.results()[0]
            dt = time.perf_counter() - t0
            ph = b.timings()
            b.close()
            if inst.motif not in res:
                raise SystemExit(f"planted motif missing for {name} ({label})")
            sets.append(res)
            row[label] = {"s": round(dt, 4), "compat_ms": round(ph[1], 3),
                          "search_ms": round(ph[3], 3), "motifs": len(res)}
        if sets[0] != sets[1]:
            raise SystemExit(f"the two compat layouts disagree on {name}")
        row["compat_matrix_bytes"] = (n * (m - l + 1)) * n * ((m - l + 64) // 64) * 8
        out[name] = row
        print(json.dumps({name: row}), flush=True)
    print(json.dumps(out), flush=True)


def serving_main(args, I, pms):
    """A Poisson stream of planted instances with (l,d) uniform from
    {(9,2),(11,3),(13,4),(15,5),(17,6)}, n in [10,30], m in [200,1000].  The
    offered rate is --load times the batched capacity measured on the first
    --count requests of the same stream (one device pass, after a warm-up)."""
    insts = I.batch_mix(2000, args.requests, ld=SERVE_LD, m_range=(200, 1000))
    head = [pms.Problem(x.seqs, x.l, x.d) for x in insts[:max(1, min(args.count, len(insts)))]]
    b = pms.Batch(head)
    b.run()
    b.results()
    t0 = time.perf_counter()
    b.run()
    b.results()
    capacity = len(head) / (time.perf_counter() - t0)
    b.close()
    # the plain rate on the same requests: one device pipeline run each
    singles = [pms.Batch([p]) for p in head]
    for sb in singles:
        sb.run()
        sb.results()
    tp = time.perf_counter()
    for sb in singles:
        sb.run()
        sb.results()
    plain_rate = len(head) / (time.perf_counter() - tp)
    for sb in singles:
        sb.close()
    print(json.dumps({"capacity_instances_per_s": round(capacity, 3),
                      "plain_instances_per_s": round(plain_rate, 3)}), flush=True)
    rate = max(1e-3, args.load * capacity)
    rng = random.Random(7)
    srv = pms.Server(workers=args.workers)
    lock = threading.Lock()
    pending = {}   # ticket -> (submit time, instance)
    done = []      # (latency, instance, result)
    submitting = [True]

    def collect():
        # completion times: poll every outstanding ticket every millisecond,
        # independently of the submitting loop
        while True:
            with lock:
                tickets = list(pending.items())
                more = submitting[0]
            if not tickets and not more:
                return
            for tk, (ts, x) in tickets:
                r = srv.poll(tk)
                if r is not None:
                    done.append((time.perf_counter() - ts, x, r))
                    with lock:
                        del pending[tk]
            time.sleep(0.001)

    th = threading.Thread(target=collect)
    t0 = time.perf_counter()
    th.start()
    next_t = 0.0
    last_report = t0
    for i, x in enumerate(insts):
        next_t += rng.expovariate(rate)
        now = time.perf_counter() - t0
        if next_t > now:
            time.sleep(next_t - now)
        ts = time.perf_counter()
        tk = srv.submit(pms.Problem(x.seqs, x.l, x.d))
        with lock:
            pending[tk] = (ts, x)
        if ts - last_report > 30:
            last_report = ts
            print(json.dumps({"progress": i + 1, "done": len(done)}), flush=True)
    with lock:
        submitting[0] = False
    while th.is_alive():
        th.join(timeout=30)
        if th.is_alive():
            print(json.dumps({"progress": len(insts), "done": len(done)}), flush=True)
    total = time.perf_counter() - t0
    srv.close()
    lat = []
    for (lt, x, r) in done:
        lat.append(lt)
        if x.motif not in r:
            raise SystemExit(f"planted motif missing in served request seed {x.seed}")
    lat.sort()
    print(json.dumps({"workload": "serving", "requests": len(insts), "workers": args.workers,
                      "capacity_instances_per_s": capacity, "offered_rate": rate,
                      "instances_per_s": len(insts) / total,
                      "plain_instances_per_s": plain_rate,
                      "served_over_plain": (len(insts) / total) / plain_rate,
                      "p50_ms": 1e3 * lat[len(lat) // 2],
                      "p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))]}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["batched", "plain", "serving", "large", "protein",
                                           "long"],
                    default="batched")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-plain", action="store_true", help="batched: skip the plain runs")
    ap.add_argument("--graph-steps", type=int, default=1,
                    help="batched: hipGraph replays timed after the eager steps")
    ap.add_argument("--count", type=int, default=BATCH_COUNT,
                    help="instances in the batched workload (serving: capacity sample)")
    ap.add_argument("--wpc", type=int, default=0, help="persistent search waves per CU (0 = auto)")
    ap.add_argument("--split", type=int, default=0, help="part size (0 = auto)")
    ap.add_argument("--threshold", type=int, default=0, help="stack size t (0 = cost model)")
    ap.add_argument("--stage-cap", type=int, default=0, help="staged survivors per tail batch")
    ap.add_argument("--compat-kernel", type=int, default=0,
                    help="compat builder: 1 VALU, 2 int8 MFMA (0 = library default)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="batched: use the flags / defaults instead of pms_autotune")
    ap.add_argument("--tune-runs", type=int, default=24, help="autotuner pipeline runs")
    ap.add_argument("--requests", type=int, default=200, help="serving: number of requests")
    ap.add_argument("--workers", type=int, default=3, help="serving: overlapping passes")
    ap.add_argument("--load", type=float, default=0.7,
                    help="serving: offered rate as a fraction of the batched capacity")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; run with --gpus 1 "
                                   "(the planted motif search shards by instance and by S_1 "
                                   "window, described in the design notes)"}))
        sys.exit(2)
    from paper_1307_0571_amd import instances as I
    from paper_1307_0571_amd import pms
    {"batched": batched_main, "plain": plain_main, "serving": serving_main,
     "large": large_main, "protein": protein_main, "long": long_main}[args.workload](args, I, pms)


if __name__ == "__main__":
    main()
