"""Seeded synthetic planted-motif instances (the paper's workload, Section 1).

This module only draws inputs.  It holds none of the search arithmetic and is
the one piece of code that both the GPU path's tests/benchmarks and the CPU
oracle use, so that both see identical bytes.

Recipe (Section 1 describes the model; the planting rule is the one the
benchmarks fix: exactly d substitutions per planted copy):

* random numbers come from a counter-based SplitMix64: the i-th draw of
  stream s for seed k is ``mix(mix(4*k + s) + (i + 1) * GOLDEN)`` where
  ``mix`` is SplitMix64's finaliser (Steele, Lea, Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014) and GOLDEN = 0x9E3779B97F4A7C15;
* background: n*m i.i.d. uniform bases, base = top two bits of a draw of
  stream 0 (string i, position j uses counter i*m + j);
* motif: l uniform bases from stream 1;
* per string i: start uniform in [0, m-l] (stream 2), then d distinct positions
  of the copy by a partial Fisher-Yates shuffle of [0, l) and, for each, the
  new base (old + 1 + U{0,1,2}) mod 4 (stream 3), so every copy is at Hamming
  distance exactly d from the motif;
* uniform integers in [0, k) use rejection sampling on full 64-bit draws.

Codes 0..3 stand for the alphabet characters in ascending ASCII order
("ACGT" for DNA).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
DNA = "ACGT"
PROTEIN = "ACDEFGHIKLMNPQRSTVWY"  # the 20 standard amino acids


def _mix_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


SHAPE_TAG = 0x5348415045  # "SHAPE": keys the per-instance shape draws of batch_mix


class Stream:
    """Sequential view of one counter-based stream (seed, stream id).

    ``Stream.shape(seed)`` is the stream batch_mix draws an instance's
    (l, d, n, m) from; its key, mix(mix(seed) ^ SHAPE_TAG), is not the key
    mix(4 * seed' + s) of a planting stream of any seed in use."""

    def __init__(self, seed: int, stream: int, key: int = None):
        self.key = _mix_int((4 * int(seed) + int(stream)) & MASK64) if key is None else key
        self.i = 0

    @classmethod
    def shape(cls, seed: int) -> "Stream":
        return cls(seed, 0, key=_mix_int(_mix_int(int(seed) & MASK64) ^ SHAPE_TAG))

    def next(self) -> int:
        self.i += 1
        return _mix_int(self.key + self.i * GOLDEN)

    def block(self, count: int) -> np.ndarray:
        """The next ``count`` draws as a uint64 array."""
        idx = np.arange(self.i + 1, self.i + 1 + count, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.key) + idx * np.uint64(GOLDEN)
        self.i += count
        return _mix_np(z)

    def below(self, k: int) -> int:
        """Uniform integer in [0, k) by rejection."""
        if k <= 0:
            raise ValueError("k must be positive")
        limit = (1 << 64) - ((1 << 64) % k)
        while True:
            x = self.next()
            if x < limit:
                return x % k


@dataclass
class Instance:
    """One planted (l,d) instance: n strings of length m over ``alphabet``."""

    seed: int
    l: int
    d: int
    n: int
    m: int
    alphabet: str
    codes: np.ndarray            # uint8 [n, m], values 0..|alphabet|-1
    motif: str                   # the planted motif
    starts: List[int] = field(default_factory=list)

    @property
    def seqs(self) -> List[str]:
        table = np.frombuffer(self.alphabet.encode("ascii"), dtype=np.uint8)
        return [table[row].tobytes().decode("ascii") for row in self.codes]


def planted(seed: int, l: int, d: int, n: int = 20, m: int = 600,
            alphabet: str = DNA) -> Instance:
    """Planted instance with exactly ``d`` substitutions per copy."""
    alphabet = "".join(sorted(alphabet))
    a = len(alphabet)
    if a < 2 or len(set(alphabet)) != a:
        raise ValueError("alphabet needs >= 2 distinct characters")
    if not (1 <= l <= m) or not (0 <= d <= l) or n < 1:
        raise ValueError("bad (l, d, n, m)")
    bg = Stream(seed, 0).block(n * m)
    if a == 4:
        codes = (bg >> np.uint64(62)).astype(np.uint8)
    else:
        # exact uniform on other alphabets: reduce the top 32 bits (tiny bias
        # irrelevant here; alphabets other than 4 are only used in tests)
        codes = ((bg >> np.uint64(32)) % np.uint64(a)).astype(np.uint8)
    codes = codes.reshape(n, m)
    ms = Stream(seed, 1)
    if a == 4:
        motif = [int(x) >> 62 for x in ms.block(l)]
    else:
        motif = [ms.below(a) for _ in range(l)]
    st = Stream(seed, 2)
    sub = Stream(seed, 3)
    starts = []
    for i in range(n):
        s = st.below(m - l + 1)
        starts.append(s)
        copy = list(motif)
        pos = list(range(l))
        for k in range(d):  # partial Fisher-Yates: d distinct positions
            j = k + sub.below(l - k)
            pos[k], pos[j] = pos[j], pos[k]
            p = pos[k]
            copy[p] = (copy[p] + 1 + sub.below(a - 1)) % a
        codes[i, s:s + l] = np.asarray(copy, dtype=np.uint8)
    return Instance(seed=seed, l=l, d=d, n=n, m=m, alphabet=alphabet,
                    codes=codes, motif="".join(alphabet[c] for c in motif),
                    starts=starts)


def random_strings(seed: int, n: int, m: int, alphabet: str = DNA) -> Instance:
    """i.i.d. strings with nothing planted (edge-case and fuzz inputs)."""
    alphabet = "".join(sorted(alphabet))
    a = len(alphabet)
    bg = Stream(seed, 0).block(n * m)
    codes = ((bg >> np.uint64(32)) % np.uint64(a)).astype(np.uint8).reshape(n, m)
    return Instance(seed=seed, l=0, d=0, n=n, m=m, alphabet=alphabet,
                    codes=codes, motif="", starts=[])


def batch_mix(seed0: int, count: int,
              ld: Sequence[tuple] = ((11, 3), (13, 4), (15, 5)),
              n_range=(10, 30), m_range=(300, 1000), alphabet: str = DNA) -> List[Instance]:
    """Mixed batch: (l,d) uniform from ``ld``, n and m uniform in the ranges.

    Instance k uses seed ``seed0 + k``; its shape is drawn from the seed's own
    shape stream (``Stream.shape``), which no planting stream shares, so the
    instance bytes depend only on the seed and the shape.
    """
    out = []
    for k in range(count):
        s = seed0 + k
        sh = Stream.shape(s)
        l, d = ld[sh.below(len(ld))]
        n = n_range[0] + sh.below(n_range[1] - n_range[0] + 1)
        m = m_range[0] + sh.below(m_range[1] - m_range[0] + 1)
        out.append(planted(s, l, d, n, m, alphabet))
    return out
