"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every expected value here comes from a brute-force definition (tests/brute.py),
a closed form, a construction from the proof of Theorem 1, or a hand-worked
fixture under tests/golden/ -- never from the oracle itself.
"""
import json
import os
import random

import numpy as np
import pytest

from paper_1307_0571_amd import instances as I

from . import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _codes_to_str(rows, alpha):
    return ["".join(alpha[c] for c in row) for row in rows]


def _tuples_to_str(tups, alpha):
    return ["".join(alpha[c] for c in t) for t in tups]


# ---------------------------------------------------------------- definition

@pytest.mark.parametrize("l,d,n,m,seed", [
    (6, 1, 20, 600, 0), (7, 1, 20, 600, 1), (8, 1, 20, 600, 2), (8, 2, 20, 120, 3),
    (5, 2, 8, 60, 4), (4, 1, 3, 12, 5),
])
def test_exhaustive_planted(oracle_lib, l, d, n, m, seed):
    """Section 1 definition applied to all of Sigma^l (l <= 8) on planted DNA."""
    inst = I.planted(seed, l, d, n, m)
    want = _tuples_to_str(brute.motifs_exhaustive(inst.codes, l, d, 4), "ACGT")
    assert oracle_lib.solve_a(inst.seqs, l, d) == want
    assert oracle_lib.solve_b(inst.seqs, l, d) == want
    assert inst.motif in want


def test_exhaustive_fuzz(oracle_lib):
    """Random tiny instances over alphabets of size 2..4, any d < l."""
    rng = random.Random(1234)
    for case in range(60):
        a = rng.choice([2, 3, 4])
        alpha = "ACGT"[:a] if a != 3 else "ACG"
        l = rng.randint(1, 6)
        d = rng.randint(0, l - 1)
        n = rng.randint(1, 6)
        m = rng.randint(l, 40)
        inst = I.random_strings(10_000 + case, n, m, alpha)
        want = _tuples_to_str(brute.motifs_exhaustive(inst.codes, l, d, a), alpha)
        got_a = oracle_lib.solve_a(inst.seqs, l, d, alphabet=alpha)
        assert got_a == want, (case, a, l, d, n, m)
        # deep thresholds on loose instances (2d >= l: every pair compatible)
        # cost |windows|^t generator calls; keep those cases shallow
        ts = {1, 2, n} if (2 * d < l or n <= 3) else {1, 2}
        for t in sorted(ts):
            got_b = oracle_lib.solve_b(inst.seqs, l, d, alphabet=alpha, t=t)
            assert got_b == want, (case, a, l, d, n, m, t)


@pytest.mark.parametrize("l,d,n,m,seed", [(6, 1, 12, 200, 30), (7, 2, 8, 90, 31),
                                         (8, 2, 6, 120, 32), (5, 1, 4, 33, 33)])
def test_windows_restriction_bruteforce(oracle_lib, l, d, n, m, seed):
    """oracle_b restricted to S_1 windows [lo, hi) (Section 2.3 sub-problems)
    equals the exhaustive motif set filtered to motifs within d of one of
    those windows, for ranges at both ends, in the middle, single windows and
    empty ranges; the union over a partition of [0, r) is the whole set."""
    inst = I.planted(seed, l, d, n, m)
    r = m - l + 1
    rng = random.Random(seed)
    cuts = sorted({0, r, *(rng.randint(1, r - 1) for _ in range(3))})
    ranges = list(zip(cuts[:-1], cuts[1:])) + [(0, 1), (r - 1, r), (5, 5), (r // 2, r // 2 + 1)]
    whole = set()
    for lo, hi in ranges:
        want = _tuples_to_str(brute.motifs_from_windows(inst.codes, l, d, 4, lo, hi), "ACGT")
        for t in (1, 2, 3):
            got = oracle_lib.solve_b(inst.seqs, l, d, t=t, windows=(lo, hi))
            assert got == want, (lo, hi, t)
        if (lo, hi) in zip(cuts[:-1], cuts[1:]):
            whole |= set(want)
    full = _tuples_to_str(brute.motifs_exhaustive(inst.codes, l, d, 4), "ACGT")
    assert sorted(whole) == full
    assert oracle_lib.solve_b(inst.seqs, l, d, windows=(0, r)) == full


def test_golden_hand_examples(oracle_lib):
    """Hand-worked instances (tests/golden/hand_examples.json)."""
    with open(os.path.join(GOLDEN, "hand_examples.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        for solve in (oracle_lib.solve_a, oracle_lib.solve_b):
            got = solve(c["seqs"], c["l"], c["d"], alphabet=c["alphabet"])
            assert got == sorted(c["motifs"]), c["name"]


# ------------------------------------------------------- distances, Theorem 1

def test_hd_and_cd_definitions(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(300):
        a = int(rng.integers(2, 5))
        l = int(rng.integers(1, 12))
        k = int(rng.integers(2, 6))
        ts = rng.integers(0, a, size=(k, l)).astype(np.uint8)
        assert oracle_lib.hd(ts[0], ts[1]) == brute.hd(ts[0], ts[1])
        assert oracle_lib.cd(ts, a) == brute.consensus_distance(ts.tolist())
        # Cd of two l-mers is their Hamming distance (Section 2.4)
        assert oracle_lib.cd(ts[:2], a) == brute.hd(ts[0], ts[1])


def test_theorem1_bruteforce(oracle_lib):
    """Theorem 1: three l-mers have a common neighbour within budgets (d1,d2,d3)
    iff pairwise Cd <= d_i + d_j and Cd(T) <= d1 + d2 + d3.  Brute-force count
    of common neighbours over all of Sigma^l."""
    rng = np.random.default_rng(11)
    mism = 0
    trials = 0
    for a in (2, 3, 4):
        for _ in range(1200):
            l = int(rng.integers(1, 7))
            ts = rng.integers(0, a, size=(3, l)).astype(np.uint8)
            bud = [int(x) for x in rng.integers(0, l + 1, size=3)]
            exists = len(brute.common_neighbours(ts, bud, a)) > 0
            cond = oracle_lib.theorem1(ts[0], ts[1], ts[2], a, *bud)
            mism += exists != cond
            trials += 1
            if cond:
                w = brute.theorem1_witness(*ts.tolist(), *bud)
                assert w is not None
                for t, b in zip(ts.tolist(), bud):
                    assert brute.hd(w, t) <= b
    assert trials >= 3000 and mism == 0


def test_lemma1_necessary(oracle_lib):
    """Lemma 1: a common neighbour within budgets exists only if Cd(T) <= sum d_i."""
    rng = np.random.default_rng(12)
    for _ in range(600):
        a = int(rng.integers(2, 5))
        l = int(rng.integers(1, 7))
        k = int(rng.integers(2, 6))
        ts = rng.integers(0, a, size=(k, l)).astype(np.uint8)
        bud = [int(x) for x in rng.integers(0, l + 1, size=k)]
        if len(brute.common_neighbours(ts, bud, a)) > 0:
            assert oracle_lib.cd(ts, a) <= sum(bud)


def test_pair_condition(oracle_lib):
    """Section 2.4: a and b share a neighbour within (da, db) iff Hd(a,b) <= da + db."""
    rng = np.random.default_rng(13)
    for _ in range(600):
        a = int(rng.integers(2, 5))
        l = int(rng.integers(1, 7))
        ts = rng.integers(0, a, size=(2, l)).astype(np.uint8)
        bud = [int(x) for x in rng.integers(0, l + 1, size=2)]
        exists = len(brute.common_neighbours(ts, bud, a)) > 0
        assert exists == (oracle_lib.hd(ts[0], ts[1]) <= sum(bud))


# ------------------------------------------------------ Algorithm 1 generator

def _prefix_count(arr: np.ndarray) -> int:
    """Number of distinct prefixes of length 0..l-1 among the rows of arr."""
    if len(arr) == 0:
        return 0
    l = arr.shape[1]
    return sum(len({tuple(r[:p]) for r in arr.tolist()}) for p in range(l))


def test_generator_matches_bruteforce(oracle_lib):
    rng = np.random.default_rng(21)
    for _ in range(400):
        a = int(rng.integers(2, 5))
        l = int(rng.integers(1, 7))
        k = int(rng.integers(1, 6))
        ts = rng.integers(0, a, size=(k, l)).astype(np.uint8)
        bud = [int(x) for x in rng.integers(0, l, size=k)]
        want = brute.common_neighbours(ts, bud, a)
        for tri in (True, False):
            got, nodes = oracle_lib.neighbourhood(ts, bud, a, use_triples=tri)
            assert got.tolist() == want.tolist()
            if tri and k <= 3:
                # no dead ends for |T| <= 3 (Theorem 1 is necessary and
                # sufficient on every suffix): each expanded node is a prefix
                # of some reported leaf
                assert nodes == 1 + a * _prefix_count(want)


def test_neighbourhood_size_closed_form(oracle_lib):
    rng = np.random.default_rng(22)
    for a in (2, 3, 4):
        for l in range(1, 8):
            for d in range(0, l + 1):
                x = rng.integers(0, a, size=(1, l)).astype(np.uint8)
                got, _ = oracle_lib.neighbourhood(x, [d], a)
                assert len(got) == brute.neighbourhood_size(l, d, a)
                assert len({tuple(r) for r in got.tolist()}) == len(got)


# --------------------------------------------------------------- special cases

def test_d0_is_lmer_set_intersection(oracle_lib):
    for seed in range(6):
        inst = I.random_strings(500 + seed, 4, 40, "AC")
        sets = [brute.lmers_of(inst.codes[i:i + 1], 5) for i in range(4)]
        want = sorted(_tuples_to_str(set.intersection(*sets), inst.alphabet))
        assert oracle_lib.solve_a(inst.seqs, 5, 0, alphabet="AC") == want
        assert oracle_lib.solve_b(inst.seqs, 5, 0, alphabet="AC") == want


def test_single_string_is_union_of_balls(oracle_lib):
    inst = I.random_strings(77, 1, 30, "ACGT")
    want = set()
    for w in brute.windows(inst.codes[0], 6):
        want.update(brute.ball(w.tolist(), 2, 4))
    want = sorted(_tuples_to_str(want, "ACGT"))
    assert oracle_lib.solve_a(inst.seqs, 6, 2) == want
    assert oracle_lib.solve_b(inst.seqs, 6, 2) == want


def test_short_strings_and_bad_args(oracle_lib):
    assert oracle_lib.solve_a(["ACG", "ACG"], 4, 1) == []
    assert oracle_lib.solve_b(["ACG", "ACG"], 4, 1) == []
    assert oracle_lib.solve_a(["ACGT"], 4, 0) == ["ACGT"]
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.solve_a(["ACGT"], 4, 4)        # d >= l rejected
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.solve_a(["ACGN"], 2, 0)        # character outside alphabet
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.solve_a(["ACGT", "ACG"], 2, 0)  # unequal lengths


# ------------------------------------------------------------------ invariants

@pytest.mark.parametrize("l,d,seed", [(9, 2, 0), (9, 2, 1), (10, 2, 2)])
def test_planted_full_size_a_equals_b(oracle_lib, l, d, seed):
    inst = I.planted(seed, l, d)
    a = oracle_lib.solve_a(inst.seqs, l, d)
    assert inst.motif in a
    for t in (1, 2, 3, 5):
        assert oracle_lib.solve_b(inst.seqs, l, d, t=t) == a
    assert oracle_lib.solve_b(inst.seqs, l, d, t=3, triple=False) == a


def test_invariances(oracle_lib):
    inst = I.planted(42, 8, 2, 10, 200)
    base = oracle_lib.solve_b(inst.seqs, 8, 2)
    assert inst.motif in base
    seqs = inst.seqs
    # permuting the strings
    perm = [seqs[i] for i in np.random.default_rng(3).permutation(len(seqs))]
    assert oracle_lib.solve_b(perm, 8, 2) == base
    # reversing every string reverses every motif
    rev = oracle_lib.solve_b([s[::-1] for s in seqs], 8, 2)
    assert rev == sorted(x[::-1] for x in base)
    # a bijective relabelling of the alphabet relabels the set
    tr = str.maketrans("ACGT", "GTCA")
    rel = oracle_lib.solve_b([s.translate(tr) for s in seqs], 8, 2)
    assert rel == sorted(x.translate(tr) for x in base)


def test_planted_always_reported(oracle_lib):
    for seed in range(10):
        inst = I.planted(100 + seed, 10, 3, 12, 150)
        got = oracle_lib.solve_b(inst.seqs, 10, 3)
        assert inst.motif in got
        # soundness: every reported motif satisfies the definition directly
        for mot in got:
            code = [inst.alphabet.index(ch) for ch in mot]
            for row in inst.codes:
                w = brute.windows(row, 10)
                assert ((w != np.asarray(code)[None, :]).sum(1) <= 3).any()


def test_generator_plants_exactly_d():
    for seed in range(20):
        inst = I.planted(seed, 15, 5, 20, 600)
        mot = [inst.alphabet.index(c) for c in inst.motif]
        for row, s in zip(inst.codes, inst.starts):
            assert brute.hd(row[s:s + 15].tolist(), mot) == 5
