"""Brute-force definitions used to pin the oracle (numpy, tiny sizes only).

Nothing here calls the oracle or the GPU path: every function applies a
definition of the paper literally, over all of Sigma^l where needed.
"""
from __future__ import annotations

import itertools
from typing import Iterable, List, Sequence

import numpy as np


def all_lmers(l: int, a: int) -> np.ndarray:
    """Every l-mer over codes 0..a-1, in lexicographic order, shape [a^l, l]."""
    idx = np.arange(a ** l, dtype=np.int64)
    out = np.empty((a ** l, l), dtype=np.uint8)
    for p in range(l - 1, -1, -1):
        out[:, p] = idx % a
        idx //= a
    return out


def windows(row: np.ndarray, l: int) -> np.ndarray:
    r = len(row) - l + 1
    if r <= 0:
        return np.zeros((0, l), dtype=np.uint8)
    return np.stack([row[j:j + l] for j in range(r)])


def motifs_exhaustive(codes: np.ndarray, l: int, d: int, a: int) -> List[tuple]:
    """Section 1's definition over all of Sigma^l: M is a motif iff every
    string has a window within Hamming distance d of M."""
    cand = all_lmers(l, a)
    for row in codes:
        w = windows(row, l)
        if len(w) == 0:
            return []
        keep = np.zeros(len(cand), dtype=bool)
        for s in range(0, len(cand), 4096):
            blk = cand[s:s + 4096]
            mism = (blk[:, None, :] != w[None, :, :]).sum(-1)
            keep[s:s + 4096] = (mism <= d).any(1)
        cand = cand[keep]
        if len(cand) == 0:
            break
    return [tuple(int(x) for x in c) for c in cand]


def motifs_from_windows(codes: np.ndarray, l: int, d: int, a: int, lo: int,
                        hi: int) -> List[tuple]:
    """The motifs of Section 1's definition that are also within d of one of
    the S_1 windows lo..hi-1 (the result of the sub-problems of Section 2.3
    for those windows), over all of Sigma^l."""
    full = motifs_exhaustive(codes, l, d, a)
    w = windows(codes[0], l)[lo:hi]
    if len(full) == 0 or len(w) == 0:
        return []
    cand = np.asarray(full, dtype=np.uint8)
    near = ((cand[:, None, :] != w[None, :, :]).sum(-1) <= d).any(1)
    return [tuple(int(x) for x in c) for c in cand[near]]


def common_neighbours(ts: Sequence[Sequence[int]], budgets: Sequence[int], a: int) -> np.ndarray:
    """All M in Sigma^l with Hd(M, T_i) <= budgets[i] for every i."""
    l = len(ts[0])
    cand = all_lmers(l, a)
    ok = np.ones(len(cand), dtype=bool)
    for t, b in zip(ts, budgets):
        ok &= (cand != np.asarray(t, dtype=np.uint8)[None, :]).sum(1) <= b
    return cand[ok]


def hd(x, y) -> int:
    return int(sum(1 for p, q in zip(x, y) if p != q))


def consensus_distance(ts: Sequence[Sequence[int]]) -> int:
    """Definition 1, written out: sum over columns of k - max frequency."""
    k = len(ts)
    total = 0
    for col in zip(*ts):
        counts = {}
        for ch in col:
            counts[ch] = counts.get(ch, 0) + 1
        total += k - max(counts.values())
    return total


def neighbourhood_size(l: int, d: int, a: int) -> int:
    """|N_d(x)| = sum_{i<=d} C(l,i) (a-1)^i (Appendix C/D)."""
    from math import comb
    return sum(comb(l, i) * (a - 1) ** i for i in range(min(d, l) + 1))


def theorem1_witness(t1, t2, t3, d1, d2, d3):
    """The common neighbour built in the proof of Theorem 1 (cases 1 and 2).

    Column types: N0 all equal, N1 T1 differs, N2 T2 differs, N3 T3 differs,
    N4 all distinct.  Returns the constructed l-mer, or None when the
    construction's preconditions (the theorem's conditions) fail.
    """
    T = [list(t1), list(t2), list(t3)]
    D = [d1, d2, d3]
    l = len(t1)
    types = []
    for k in range(l):
        a, b, c = T[0][k], T[1][k], T[2][k]
        if a == b == c:
            types.append(0)
        elif b == c:
            types.append(1)
        elif a == c:
            types.append(2)
        elif a == b:
            types.append(3)
        else:
            types.append(4)
    cols = {i: [k for k in range(l) if types[k] == i] for i in range(5)}
    n = {i: len(cols[i]) for i in range(5)}
    for i in (1, 2, 3):
        if n[i] >= D[i - 1]:
            # case 1: start from T_i, take T_j's character on d_i columns of type N_i
            M = list(T[i - 1])
            other = 1 if i == 1 else 0
            for k in cols[i][:D[i - 1]]:
                M[k] = T[other][k]
            return M
    # case 2: T1 on N0, N2, N3 columns; T2 on N1 columns; split the N4 columns
    M = [None] * l
    for k in range(l):
        if types[k] in (0, 2, 3):
            M[k] = T[0][k]
        elif types[k] == 1:
            M[k] = T[1][k]
    free = list(cols[4])
    for i in range(3):
        need = max(0, n[i + 1] + n[4] - D[i])
        if need > len(free):
            return None
        for _ in range(need):
            k = free.pop()
            M[k] = T[i][k]
    for k in free:
        M[k] = T[0][k]
    return M


def lmers_of(codes: np.ndarray, l: int) -> set:
    out = set()
    for row in codes:
        for w in windows(row, l):
            out.add(tuple(int(x) for x in w))
    return out


def ball(x: Sequence[int], d: int, a: int) -> Iterable[tuple]:
    l = len(x)
    for k in range(d + 1):
        for pos in itertools.combinations(range(l), k):
            for subs in itertools.product(range(a - 1), repeat=k):
                y = list(x)
                for p, s in zip(pos, subs):
                    y[p] = s if s < x[p] else s + 1
                yield tuple(y)
