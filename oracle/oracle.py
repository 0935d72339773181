"""ctypes front end of the C oracle (test infrastructure only).

Characters are mapped to codes by their rank in the alphabet sorted by ASCII
value, so byte-lexicographic order of motif strings equals the order of their
code arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pms_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class OracleError(RuntimeError):
    pass


class _Stats(ctypes.Structure):
    _fields_ = [
        ("pushes", ctypes.c_int64 * 65),
        ("tuples", ctypes.c_int64),
        ("gen_nodes", ctypes.c_int64),
        ("leaves", ctypes.c_int64),
        ("motifs", ctypes.c_int64),
        ("filter_tests", ctypes.c_int64),
        ("verify_tests", ctypes.c_int64),
        ("push_tries", ctypes.c_int64),
        ("filter_words", ctypes.c_int64),
        ("compat_pass", ctypes.c_int64),
        ("triple_tests", ctypes.c_int64),
    ]


def library_path() -> str:
    return _LIB


def build() -> str:
    """Compile the oracle with gcc (plain -O3, portable code)."""
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall",
           "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u8pp = ctypes.POINTER(u8p)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_a.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, u8pp, i64p]
    lib.oracle_a.restype = ctypes.c_int
    lib.oracle_b.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8pp, i64p,
                             ctypes.POINTER(_Stats)]
    lib.oracle_b.restype = ctypes.c_int
    lib.oracle_b_windows.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int64, ctypes.c_int64, u8pp, i64p,
                                     ctypes.POINTER(_Stats)]
    lib.oracle_b_windows.restype = ctypes.c_int
    lib.oracle_hd.argtypes = [u8p, u8p, ctypes.c_int]
    lib.oracle_hd.restype = ctypes.c_int
    lib.oracle_cd.argtypes = [ctypes.POINTER(u8p), ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_cd.restype = ctypes.c_int
    lib.oracle_theorem1.argtypes = [u8p, u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int]
    lib.oracle_theorem1.restype = ctypes.c_int
    lib.oracle_neighbourhood.argtypes = [ctypes.POINTER(u8p), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                         ctypes.c_int, u8pp, i64p, i64p]
    lib.oracle_neighbourhood.restype = ctypes.c_int
    lib.oracle_free.argtypes = [ctypes.c_void_p]
    lib.oracle_free.restype = None
    _lib = lib
    return lib


def encode(seqs: Sequence[str], alphabet: str) -> Tuple[np.ndarray, str]:
    """Strings -> uint8 code matrix [n, m]; codes are ASCII ranks in the alphabet."""
    alpha = "".join(sorted(alphabet))
    if len(set(alpha)) != len(alpha):
        raise OracleError("duplicate alphabet character")
    if not seqs:
        raise OracleError("no strings")
    m = len(seqs[0])
    if any(len(s) != m for s in seqs):
        raise OracleError("strings must share one length")
    table = np.full(256, 255, dtype=np.uint8)
    for i, ch in enumerate(alpha):
        table[ord(ch)] = i
    raw = np.frombuffer("".join(seqs).encode("latin-1"), dtype=np.uint8)
    codes = table[raw].reshape(len(seqs), m)
    if (codes == 255).any():
        raise OracleError("character outside the alphabet")
    return np.ascontiguousarray(codes), alpha


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _decode(buf, count: int, l: int, alpha: str) -> List[str]:
    if count == 0:
        return []
    arr = np.ctypeslib.as_array(buf, shape=(count * l,)).copy()
    table = np.frombuffer(alpha.encode("ascii"), dtype=np.uint8)
    chars = table[arr].tobytes().decode("ascii")
    return [chars[i * l:(i + 1) * l] for i in range(count)]


def _threads(threads):
    if threads is None:
        return max(1, min(16, os.cpu_count() or 1))
    return int(threads)


def _codes_arg(seqs, alphabet, codes):
    if codes is not None:
        c = np.ascontiguousarray(codes, dtype=np.uint8)
        return c, "".join(sorted(alphabet))
    return encode(seqs, alphabet)


def solve_a(seqs: Sequence[str] = None, l: int = 0, d: int = 0, alphabet: str = "ACGT",
            threads: int = None, codes: np.ndarray = None) -> List[str]:
    """Sorted motif set by enumerating the d-neighbourhood of every S_1 window."""
    lib = _load()
    c, alpha = _codes_arg(seqs, alphabet, codes)
    n, m = c.shape
    out = ctypes.POINTER(ctypes.c_uint8)()
    cnt = ctypes.c_int64(0)
    rc = lib.oracle_a(_ptr(c), n, m, len(alpha), l, d, _threads(threads),
                      ctypes.byref(out), ctypes.byref(cnt))
    if rc != 0:
        raise OracleError(f"oracle_a failed ({rc})")
    try:
        return _decode(out, cnt.value, l, alpha)
    finally:
        lib.oracle_free(out)


def solve_b(seqs: Sequence[str] = None, l: int = 0, d: int = 0, alphabet: str = "ACGT",
            t: int = None, triple: bool = True, threads: int = None,
            codes: np.ndarray = None, stats: bool = False, windows=None):
    """Sorted motif set by PMS8 (Algorithm 2 with Algorithm 1 and Theorem 1).

    ``windows=(lo, hi)`` restricts the run to the S_1 windows lo..hi-1 (the
    independent sub-problems of Section 2.3); the result is then the motifs
    found from those windows only."""
    lib = _load()
    c, alpha = _codes_arg(seqs, alphabet, codes)
    n, m = c.shape
    if t is None:
        t = default_threshold(n, m, l, d, len(alpha))
    out = ctypes.POINTER(ctypes.c_uint8)()
    cnt = ctypes.c_int64(0)
    st = _Stats()
    if windows is None:
        rc = lib.oracle_b(_ptr(c), n, m, len(alpha), l, d, int(t), int(bool(triple)),
                          _threads(threads), ctypes.byref(out), ctypes.byref(cnt),
                          ctypes.byref(st))
    else:
        rc = lib.oracle_b_windows(_ptr(c), n, m, len(alpha), l, d, int(t), int(bool(triple)),
                                  _threads(threads), int(windows[0]), int(windows[1]),
                                  ctypes.byref(out), ctypes.byref(cnt), ctypes.byref(st))
    if rc != 0:
        raise OracleError(f"oracle_b failed ({rc})")
    try:
        res = _decode(out, cnt.value, l, alpha)
    finally:
        lib.oracle_free(out)
    if stats:
        info = {
            "pushes": [int(x) for x in st.pushes],
            "tuples": st.tuples, "gen_nodes": st.gen_nodes, "leaves": st.leaves,
            "motifs": st.motifs, "filter_tests": st.filter_tests,
            "verify_tests": st.verify_tests, "push_tries": st.push_tries,
            "filter_words": st.filter_words, "compat_pass": st.compat_pass,
            "triple_tests": st.triple_tests, "t": t,
        }
        return res, info
    return res


def default_threshold(n: int, m: int, l: int, d: int, a: int = 4) -> int:
    """Threshold t minimising the cost model of Appendix D over t = 1..n.

    Time_s(t) = n l sum_{k<=t} (m-l+1)^k p^{k(k-1)/2},  p = N_2d / |S|^l;
    Time_p(t) = T_t N_d q^{t-1} l with T_t = (m-l+1)^t p^{t(t-1)/2}, q = N_d/N_2d.
    """
    from math import comb, log, exp
    r = m - l + 1
    if r <= 0:
        return 1

    def nd(dd):
        return sum(comb(l, i) * (a - 1) ** i for i in range(0, min(dd, l) + 1))

    p = nd(2 * d) / float(a) ** l
    q = nd(d) / nd(2 * d)
    best, best_cost = 1, None
    ts = 0.0
    for t in range(1, n + 1):
        lt = t * log(r) + (t * (t - 1) / 2) * log(p) if p > 0 else -1e300
        ts += n * l * exp(min(lt, 700))
        tp = exp(min(lt + log(nd(d)) + (t - 1) * log(q) if q > 0 else -1e300, 700)) * l
        cost = ts + tp
        if best_cost is None or cost < best_cost:
            best, best_cost = t, cost
    return best


def hd(a: Sequence[int], b: Sequence[int]) -> int:
    lib = _load()
    x = np.ascontiguousarray(a, dtype=np.uint8)
    y = np.ascontiguousarray(b, dtype=np.uint8)
    return lib.oracle_hd(_ptr(x), _ptr(y), len(x))


def cd(ts: Sequence[Sequence[int]], a: int) -> int:
    lib = _load()
    arrs = [np.ascontiguousarray(t, dtype=np.uint8) for t in ts]
    ptrs = (ctypes.POINTER(ctypes.c_uint8) * len(arrs))(*[_ptr(x) for x in arrs])
    return lib.oracle_cd(ptrs, len(arrs), len(arrs[0]), a)


def theorem1(a, b, c, alphabet_size: int, d1: int, d2: int, d3: int) -> bool:
    lib = _load()
    x, y, z = (np.ascontiguousarray(v, dtype=np.uint8) for v in (a, b, c))
    return bool(lib.oracle_theorem1(_ptr(x), _ptr(y), _ptr(z), len(x), alphabet_size,
                                    d1, d2, d3))


def neighbourhood(ts: Sequence[Sequence[int]], budgets: Sequence[int], alphabet_size: int,
                  use_triples: bool = True):
    """Algorithm 1 alone: common neighbours of ``ts`` (codes) within ``budgets``.

    Returns (array [count, l] of codes in generation order, tree nodes visited).
    """
    lib = _load()
    arrs = [np.ascontiguousarray(t, dtype=np.uint8) for t in ts]
    l = len(arrs[0])
    ptrs = (ctypes.POINTER(ctypes.c_uint8) * len(arrs))(*[_ptr(x) for x in arrs])
    bud = (ctypes.c_int * len(arrs))(*[int(b) for b in budgets])
    out = ctypes.POINTER(ctypes.c_uint8)()
    cnt = ctypes.c_int64(0)
    nodes = ctypes.c_int64(0)
    rc = lib.oracle_neighbourhood(ptrs, len(arrs), l, alphabet_size, bud, int(bool(use_triples)),
                                  ctypes.byref(out), ctypes.byref(cnt), ctypes.byref(nodes))
    if rc != 0:
        raise OracleError(f"oracle_neighbourhood failed ({rc})")
    try:
        if cnt.value == 0:
            return np.zeros((0, l), dtype=np.uint8), nodes.value
        arr = np.ctypeslib.as_array(out, shape=(cnt.value * l,)).copy().reshape(cnt.value, l)
        return arr, nodes.value
    finally:
        lib.oracle_free(out)
