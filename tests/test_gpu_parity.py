"""GPU path (through the C ABI) against the CPU oracle: identical sorted sets."""
import sys

import pytest

import oracle
from paper_1307_0571_amd import instances as I
from paper_1307_0571_amd import pms

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(inst, tune=None):
    return pms.solve_batch([pms.Problem(inst.seqs, inst.l, inst.d, inst.alphabet)], tune=tune)[0]


SMALL = [
    # (seed, l, d, n, m): several tiles, ragged tails (r not a multiple of 64)
    (1, 6, 1, 5, 70), (2, 7, 2, 6, 130), (3, 8, 2, 8, 200), (4, 9, 2, 10, 257),
    (5, 10, 3, 6, 150), (6, 5, 1, 3, 64), (7, 8, 1, 2, 100), (8, 9, 3, 4, 90),
    (9, 12, 3, 7, 129), (10, 6, 2, 1, 40), (11, 33, 8, 5, 120), (12, 40, 12, 4, 100),
]


@pytest.mark.parametrize("seed,l,d,n,m", SMALL)
def test_small_vs_oracle(seed, l, d, n, m):
    _say(f"case seed={seed} l={l} d={d} n={n} m={m}")
    inst = I.planted(seed, l, d, n, m)
    got = _gpu(inst)
    want = oracle.solve_a(inst.seqs, l, d) if l <= 12 else oracle.solve_b(inst.seqs, l, d)
    assert got == want
    assert inst.motif in got


def test_edge_cases():
    _say("edge cases")
    # m < l: no window, empty set
    assert pms.solve(["ACG", "TTA"], 4, 1) == []
    # one window per string
    assert pms.solve(["ACGT", "ACGT"], 4, 0) == ["ACGT"]
    # d = 0: exact common l-mers
    assert pms.solve(["AACCGT", "CCAATT"], 2, 0) == ["AA", "CC"]
    # a single string: every l-mer within d of one of its windows
    got = pms.solve(["ACGTA"], 3, 1)
    assert got == oracle.solve_a(["ACGTA"], 3, 1)


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_92_full_size(seed):
    _say(f"(9,2) n=20 m=600 seed={seed}")
    inst = I.planted(seed, 9, 2)
    assert _gpu(inst) == oracle.solve_a(inst.seqs, 9, 2)


@pytest.mark.parametrize("l,d", [(13, 4), (15, 5)])
def test_plain_gpu_config_seed0(l, d):
    _say(f"({l},{d}) n=20 m=600 seed=0")
    inst = I.planted(0, l, d)
    want = oracle.solve_b(inst.seqs, l, d, t=3)
    got = _gpu(inst)
    assert got == want
    assert inst.motif in got


@pytest.mark.parametrize("tune", [
    dict(threshold=2), dict(threshold=3), dict(threshold=4), dict(threshold=6),
    dict(triple_filter=-1), dict(lmer_words=2), dict(waves_per_cu=1), dict(out_capacity=1),
    dict(split=1), dict(split=3), dict(split=2047), dict(threshold=4, split=1),
    dict(threshold=5, split=2), dict(threshold=6, split=1), dict(threshold=4, split=5),
    dict(stage_cap=512), dict(stage_cap=4096), dict(threshold=5, stage_cap=512, split=3),
    dict(compat_mode=1), dict(compat_mode=2), dict(compat_mode=2, triple_filter=-1),
    dict(compat_mode=2, threshold=5, split=2), dict(compat_mode=2, threshold=2),
    dict(compat_kernel=2), dict(compat_kernel=2, compat_mode=2), dict(compat_kernel=2, lmer_words=2),
])
def test_output_invariant_under_tuning(tune):
    _say(f"tune {tune}")
    inst = I.planted(21, 11, 3, 12, 300)
    want = oracle.solve_b(inst.seqs, 11, 3)
    assert _gpu(inst, pms.Tune(**tune)) == want


def test_batch_equals_alone():
    _say("batch of mixed instances")
    insts = I.batch_mix(1000, 6, ld=((9, 2), (10, 3), (11, 3)), n_range=(5, 12),
                        m_range=(100, 300))
    probs = [pms.Problem(x.seqs, x.l, x.d) for x in insts]
    batch = pms.solve_batch(probs)
    for x, got in zip(insts, batch):
        assert got == oracle.solve_b(x.seqs, x.l, x.d)
        assert got == _gpu(x)


def test_autotune_then_cached(tmp_path, monkeypatch):
    """The autotuner returns a setting that gives the oracle's sets, writes
    it to the cache file, and tune=None batches of the same shape use it."""
    _say("autotune on a small mixed batch")
    insts = I.batch_mix(1000, 6, ld=((9, 2), (11, 3)), n_range=(6, 10), m_range=(150, 300))
    probs = [pms.Problem(x.seqs, x.l, x.d) for x in insts]
    want = [oracle.solve_b(x.seqs, x.l, x.d) for x in insts]
    t = pms.autotune(probs, max_runs=6, sample=6)
    d = pms.tune_dict(t)
    assert d["s1_begin"] == 0 and d["s1_end"] == 0
    assert pms.solve_batch(probs, tune=t) == want
    assert pms.solve_batch(probs) == want  # tune=None: the cached setting


def test_per_instance_completion():
    """Every instance with search work carries the device time its last work
    item finished; a deep split run gives the same sets and stamps."""
    _say("per-instance completion stamps")
    insts = [I.planted(s, 10, 2, 10, 200) for s in range(3)] + [I.planted(9, 11, 3, 8, 250)]
    want = [oracle.solve_b(x.seqs, x.l, x.d) for x in insts]
    for tune in (None, pms.Tune(threshold=4, split=2)):
        b = pms.Batch([pms.Problem(x.seqs, x.l, x.d) for x in insts], tune=tune)
        try:
            b.run()
            assert b.results() == want
            ticks = [b.work(i)["done_ticks"] for i in range(len(insts))]
            assert all(t > 0 for t in ticks), ticks
        finally:
            b.close()


def test_device_batch_rerun():
    _say("device-resident batch, repeated runs")
    insts = [I.planted(s, 10, 2, 10, 200) for s in range(3)]
    want = [oracle.solve_b(x.seqs, 10, 2) for x in insts]
    b = pms.Batch([pms.Problem(x.seqs, x.l, x.d) for x in insts])
    try:
        for _ in range(3):
            b.run()
            assert b.results() == want
    finally:
        b.close()


def test_graph_replay():
    """hipGraph capture of the pipeline, replayed several times with eager
    runs, host synchronisation and result reads between the replays; every
    replay must give the oracle's sets."""
    _say("hipGraph capture and replay")
    insts = [I.planted(s, 10, 2, 10, 200) for s in range(3)]
    want = [oracle.solve_b(x.seqs, 10, 2) for x in insts]
    b = pms.Batch([pms.Problem(x.seqs, x.l, x.d) for x in insts])
    try:
        for graph in (True, False, True, True, False, True):
            b.run(graph=graph)
            assert b.results() == want, graph
    finally:
        b.close()


def test_graph_replay_on_borrowed_stream():
    _say("hipGraph replay on a caller stream")
    from . import hip_rt
    inst = I.planted(8, 11, 3, 12, 300)
    want = oracle.solve_b(inst.seqs, 11, 3)
    st = hip_rt.stream_create()
    b = pms.Batch([pms.Problem(inst.seqs, 11, 3)])
    try:
        for _ in range(3):
            b.run(stream=st, graph=True)
            assert b.results() == [want]
    finally:
        b.close()
        hip_rt.stream_destroy(st)


def test_caller_workspace():
    """A batch borrows a caller-allocated device workspace of exactly
    pms_batch_workspace_size bytes; one byte less is refused before any
    device work."""
    _say("caller-provided workspace")
    from . import hip_rt
    insts = [I.planted(5, 9, 2, 12, 250), I.planted(6, 11, 3, 10, 300)]
    probs = [pms.Problem(x.seqs, x.l, x.d) for x in insts]
    want = [oracle.solve_a(x.seqs, x.l, x.d) for x in insts]
    size = pms.Batch.workspace_size(probs)
    ws = hip_rt.malloc(size)
    try:
        hip_rt.memset(ws, 0xA5, size)  # stale contents must not matter
        with pytest.raises(pms.PmsError) as e:
            pms.Batch(probs, workspace=(ws, size - 1))
        assert e.value.status == pms.PMS_E_NOMEM
        b = pms.Batch(probs, workspace=(ws, size))
        try:
            for _ in range(2):
                b.run()
                assert b.results() == want
        finally:
            b.close()
    finally:
        hip_rt.device_synchronize()
        hip_rt.free(ws)


def test_caller_workspace_small_output_slots():
    """Output slots smaller than the set (out_capacity 1) with a caller
    workspace: the overflowing instance is solved again alone in library
    memory and the result is still exact."""
    _say("caller workspace, overflowing output slots")
    from . import hip_rt
    inst = I.planted(9, 9, 2, 6, 300)
    want = oracle.solve_a(inst.seqs, 9, 2)
    assert len(want) > 1
    probs = [pms.Problem(inst.seqs, 9, 2)]
    tune = pms.Tune(out_capacity=1)
    size = pms.Batch.workspace_size(probs, tune)
    ws = hip_rt.malloc(size)
    try:
        b = pms.Batch(probs, tune=tune, workspace=(ws, size))
        try:
            b.run()
            assert b.results() == [want]
        finally:
            b.close()
    finally:
        hip_rt.device_synchronize()
        hip_rt.free(ws)


def test_pms_solve_c_entry_and_borrowed_stream():
    """pms_solve itself (the single-instance C entry point), and
    pms_solve_batch on a caller-created stream."""
    _say("pms_solve and a borrowed hip stream")
    import ctypes
    from . import hip_rt
    inst = I.planted(12, 10, 2, 9, 240)
    want = oracle.solve_a(inst.seqs, 10, 2)
    lib = pms.load()
    enc = [s.encode() for s in inst.seqs]
    arr = (ctypes.c_char_p * len(enc))(*enc)
    res = pms._Result()
    assert lib.pms_solve(arr, len(enc), inst.m, b"ACGT", 10, 2, ctypes.byref(res)) == pms.PMS_OK
    assert res.words == 1 and res.l == 10
    assert pms._take(res) == want
    st = hip_rt.stream_create()
    try:
        got = pms.solve_batch([pms.Problem(inst.seqs, 10, 2)], stream=st)
        assert got == [want]
        b = pms.Batch([pms.Problem(inst.seqs, 10, 2)])
        try:
            b.run(stream=st)
            assert b.results() == [want]
        finally:
            b.close()
    finally:
        hip_rt.stream_destroy(st)


# Sizes at the limits of the batched and served configurations: up to 30 and
# 32 strings, strings of 1000 characters, 2048 windows per string (32 words
# per row bitset), and 2d >= l (every pair of l-mers compatible).
@pytest.mark.parametrize("name,seed,l,d,n,m", [
    ("n30_m1000", 40, 9, 2, 30, 1000),
    ("n32", 41, 9, 2, 32, 400),
    ("n31_m1000_11_3", 42, 11, 3, 31, 1000),
    ("r2048", 43, 9, 1, 3, 2056),
    ("2d_ge_l_6_3", 44, 6, 3, 5, 60),
    ("2d_ge_l_7_4", 45, 7, 4, 3, 40),
])
def test_limit_sizes_vs_oracle(name, seed, l, d, n, m):
    _say(f"{name}: seed={seed} l={l} d={d} n={n} m={m}")
    inst = I.planted(seed, l, d, n, m)
    want = oracle.solve_a(inst.seqs, l, d)
    got = _gpu(inst)
    assert got == want
    assert inst.motif in got


# Long strings: 8192 windows per string (128 words per row bitset).  The
# first keeps the whole compat matrix (302 MB); the second's would take
# 1.2 GiB, so only S_1's rows are built and every push tests Hd <= 2d on the
# survivors directly; the third forces that mode on the first instance.
_LONG_WANT = {}


@pytest.mark.parametrize("name,seed,l,d,n,m,solver,tune", [
    ("r8192_12_2", 50, 12, 2, 6, 8203, "b", None),
    ("r8192_n12_auto_s1_rows", 47, 9, 1, 12, 8200, "a", None),
    ("r8192_12_2_s1_rows", 50, 12, 2, 6, 8203, "b", dict(compat_mode=2)),
])
def test_long_sequences_vs_oracle(name, seed, l, d, n, m, solver, tune):
    _say(f"{name}: seed={seed} l={l} d={d} n={n} m={m} tune={tune}")
    inst = I.planted(seed, l, d, n, m)
    key = (seed, l, d, n, m)
    if key not in _LONG_WANT:
        f = oracle.solve_a if solver == "a" else oracle.solve_b
        _LONG_WANT[key] = f(inst.seqs, l, d)
    want = _LONG_WANT[key]
    got = _gpu(inst, pms.Tune(**tune) if tune else None)
    assert got == want
    assert inst.motif in got


# Long strings at the paper's n = 20, on 24 S_1 windows around the planted
# copy (the oracle builds the whole matrix, about 17 s on one core): (16,4)
# at m = 5000, whose whole matrix (1.24 GB) makes the library take S_1's
# rows by itself, and (15,4) at m = 4000 with the whole matrix (0.8 GB) and
# with S_1's rows forced.
@pytest.mark.parametrize("seed,l,d,m,tunes", [
    (61, 16, 4, 5000, (None,)),
    (60, 15, 4, 4000, (None, dict(compat_mode=2))),
])
def test_long_strings_n20_windows_vs_oracle(seed, l, d, m, tunes):
    inst = I.planted(seed, l, d, 20, m)
    a = max(0, inst.starts[0] - 12)
    b = a + 24
    _say(f"long n=20: seed={seed} l={l} d={d} m={m} S1 windows [{a},{b})")
    want = oracle.solve_b(inst.seqs, l, d, windows=(a, b))
    assert inst.motif in want
    for tune in tunes:
        _say(f"  tune {tune}")
        got = _gpu(inst, pms.Tune(s1_begin=a, s1_end=b, **(tune or {})))
        assert got == want


# The int8 MFMA compat builder on sizes across tiles and ragged tails, one and
# two 64-bit planes, 2d >= l (every pair compatible: only the window and
# own-string masks clear bits), 32 strings and 2048 windows per string.
@pytest.mark.parametrize("name,seed,l,d,n,m", [
    ("small_ragged", 4, 9, 2, 10, 257), ("two_words", 11, 33, 8, 5, 120),
    ("l40", 12, 40, 12, 4, 100), ("2d_ge_l_6_3", 44, 6, 3, 5, 60), ("n32", 41, 9, 2, 32, 400),
    ("r2048", 43, 9, 1, 3, 2056), ("n1", 10, 6, 2, 1, 40),
])
def test_mfma_compat_vs_oracle(name, seed, l, d, n, m):
    _say(f"mfma compat {name}: seed={seed} l={l} d={d} n={n} m={m}")
    inst = I.planted(seed, l, d, n, m)
    want = oracle.solve_a(inst.seqs, l, d) if l <= 12 else oracle.solve_b(inst.seqs, l, d)
    assert _gpu(inst, pms.Tune(compat_kernel=2)) == want


# More emitted keys than one LDS sort chunk with two-word keys (l > 32): the
# multi-block sort (HBM bitonic stages, per-chunk merges, compaction).
@pytest.mark.parametrize("seed,l,d,n,m", [(61, 34, 6, 2, 34), (63, 33, 6, 2, 34)])
@pytest.mark.parametrize("ck", [1, 2])
def test_wide_keys_large_output(seed, l, d, n, m, ck):
    _say(f"wide keys, large output: seed={seed} l={l} d={d} n={n} m={m} compat_kernel={ck}")
    inst = I.planted(seed, l, d, n, m)
    want = oracle.solve_b(inst.seqs, l, d)
    assert len(want) > 100000
    assert _gpu(inst, pms.Tune(compat_kernel=ck)) == want


def test_serving_matches_alone():
    _say("serving: continuous batching, each result equals the instance alone")
    insts = I.batch_mix(2000, 12, ld=((9, 2), (10, 2), (11, 3)), n_range=(5, 12),
                        m_range=(100, 300))
    srv = pms.Server(max_wave=4)
    try:
        tickets = [srv.submit(pms.Problem(x.seqs, x.l, x.d)) for x in insts]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for x, g in zip(insts, got):
        assert g == oracle.solve_b(x.seqs, x.l, x.d)
        assert g == _gpu(x)


def test_serving_admission_and_errors():
    _say("serving: admission by device memory, invalid requests, poll")
    inst = I.planted(3, 9, 2, 8, 150)
    one = pms.Batch.workspace_size([pms.Problem(inst.seqs, 9, 2)])
    srv = pms.Server(device_mem_cap=one // 4)  # smaller than the instance's own plan
    try:
        with pytest.raises(pms.PmsError) as e:
            srv.submit(pms.Problem(inst.seqs, 9, 2))
        assert e.value.status == pms.PMS_E_NOMEM
        with pytest.raises(pms.PmsError) as e:
            srv.submit(pms.Problem(inst.seqs, 9, 9))
        assert e.value.status == pms.PMS_E_INVAL
    finally:
        srv.close()
    srv = pms.Server()
    try:
        t = srv.submit(pms.Problem(inst.seqs, 9, 2))
        got = srv.wait(t)
        assert got == oracle.solve_a(inst.seqs, 9, 2)
    finally:
        srv.close()


def test_serving_memory_cap_and_mixed_costs():
    _say("serving: a memory cap that admits about one instance per pass, mixed (l,d)")
    insts = I.batch_mix(2100, 8, ld=((9, 2), (11, 3), (13, 4)), n_range=(6, 10),
                        m_range=(150, 250))
    probs = [pms.Problem(x.seqs, x.l, x.d) for x in insts]
    one = max(pms.Batch.workspace_size([p]) for p in probs)
    srv = pms.Server(device_mem_cap=int(one * 1.2))
    try:
        tickets = [srv.submit(p) for p in probs]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for x, g in zip(insts, got):
        assert g == _gpu(x)
        assert x.motif in g


# S_1 windows are independent sub-problems (Section 2.3): the device search
# restricted to windows [a, b) must return exactly what the oracle finds from
# the same windows.
@pytest.mark.parametrize("seed,l,d,a,b", [
    (0, 13, 4, 100, 140), (1, 15, 5, 0, 24), (2, 15, 5, 570, 586), (3, 11, 3, 7, 8),
])
def test_s1_windows_vs_oracle(seed, l, d, a, b):
    _say(f"({l},{d}) seed={seed} S1 windows [{a},{b})")
    inst = I.planted(seed, l, d)
    want = oracle.solve_b(inst.seqs, l, d, t=3, windows=(a, b))
    got = _gpu(inst, pms.Tune(s1_begin=a, s1_end=b))
    assert got == want


def test_s1_windows_partition_the_result():
    inst = I.planted(4, 13, 4)
    whole = set(_gpu(inst))
    parts = set()
    for a in range(0, 588, 150):
        parts |= set(_gpu(inst, pms.Tune(s1_begin=a, s1_end=a + 150)))
    assert parts == whole


def _is_motif(seqs, mot, d):
    import numpy as np
    code = {c: i for i, c in enumerate("ACGT")}
    M = np.array([code[c] for c in mot], dtype=np.int8)
    l = len(mot)
    for s in seqs:
        a = np.array([code[c] for c in s], dtype=np.int8)
        win = np.lib.stride_tricks.sliding_window_view(a, l)
        if int((win != M).sum(axis=1).min()) > d:
            return False
    return True


# Large instances with 128-bit l-mers: exact parity on a sample of S_1
# windows (the oracle finishes those in seconds), every reported motif
# checked by brute force, and the planted motif found from the window where
# it was planted.
def test_large_19_7_windows_vs_oracle():
    inst = I.planted(0, 19, 7)
    a, b = 40, 46
    _say(f"(19,7) seed=0 S1 windows [{a},{b})")
    want = oracle.solve_b(inst.seqs, 19, 7, t=3, windows=(a, b))
    got = _gpu(inst, pms.Tune(s1_begin=a, s1_end=b, lmer_words=2))
    assert got == want
    st = inst.starts[0]
    got_p = _gpu(inst, pms.Tune(s1_begin=st, s1_end=st + 1))
    assert inst.motif in got_p
    assert all(_is_motif(inst.seqs, x, 7) for x in got_p)
