"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function include/pms.h declares, and rejects invalid input before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_1307_0571_amd import instances as I
from paper_1307_0571_amd import pms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pms.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pms_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pms.LIB_PATH):
        from paper_1307_0571_amd import build
        build.build()
    return pms.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_and_version(lib):
    assert b"gfx950" in lib.pms_version()
    for code in range(-8, 1):
        assert pms.strerror(code)
    assert pms.strerror(pms.PMS_E_ALPHABET).startswith("character")


def _status(seqs, l, d, alphabet="ACGT", m=None):
    lib = pms.load()
    enc = [s.encode() for s in seqs]
    arr = (ctypes.c_char_p * max(1, len(enc)))(*enc)
    res = pms._Result()
    mm = len(seqs[0]) if m is None else m
    return lib.pms_solve(arr, len(seqs), mm, alphabet.encode(), l, d, ctypes.byref(res))


def test_rejects_invalid_input(lib):
    ok = ["ACGTACGT", "TTGACGTA"]
    assert _status(ok, 4, 4) == pms.PMS_E_INVAL           # d >= l
    assert _status(ok, 0, 0) == pms.PMS_E_INVAL           # l < 1
    assert _status(ok, 4, -1) == pms.PMS_E_INVAL          # d < 0
    assert _status(["ACGTACGT", "ACGTACG"], 4, 1, m=8) == pms.PMS_E_INVAL  # short string
    assert _status(["ACGTACGT", "ACGTACGTA"], 4, 1, m=8) == pms.PMS_E_INVAL  # long string
    assert _status(["ACGTNCGT", "ACGTACGT"], 4, 1) == pms.PMS_E_ALPHABET
    assert _status(["acgtacgt", "ACGTACGT"], 4, 1) == pms.PMS_E_ALPHABET  # case-sensitive
    assert _status(ok, 4, 1, alphabet="ACGA") == pms.PMS_E_ALPHABET      # repeated letter
    assert _status(["AB", "BA"], 1, 0, alphabet="A") == pms.PMS_E_ALPHABET  # one letter
    big = "".join(chr(ord("A") + i) for i in range(26)) + "012345!"      # 33 letters
    assert _status(["ABCD", "DCBA"], 2, 1, alphabet=big) == pms.PMS_E_UNSUPPORTED
    assert _status(["A" * 80, "C" * 80], 65, 3) == pms.PMS_E_UNSUPPORTED   # l > 64
    many = I.random_strings(1, 33, 20).seqs
    assert _status(many, 5, 1) == pms.PMS_E_UNSUPPORTED                   # n > 32
    long = I.random_strings(2, 2, 8210).seqs
    assert _status(long, 10, 2) == pms.PMS_E_UNSUPPORTED                  # m - l + 1 > 8192


def test_null_arguments(lib):
    res = pms._Result()
    assert lib.pms_solve(None, 1, 4, b"ACGT", 2, 0, ctypes.byref(res)) == pms.PMS_E_INVAL
    arr = (ctypes.c_char_p * 1)(b"ACGT")
    assert lib.pms_solve(arr, 1, 4, b"ACGT", 2, 0, None) == pms.PMS_E_INVAL
    assert lib.pms_solve_batch(None, 1, None, None, None) == pms.PMS_E_INVAL
    assert lib.pms_batch_destroy(None) == pms.PMS_OK


def test_default_threshold_range(lib):
    for (l, d) in [(9, 2), (11, 3), (13, 4), (15, 5), (17, 6), (19, 7), (50, 21)]:
        t = pms.default_threshold(20, 600, l, d)
        assert 2 <= t <= 8
    # more windows per string -> never a larger threshold (Appendix D: t falls with m)
    assert pms.default_threshold(20, 2000, 15, 5) <= pms.default_threshold(20, 300, 15, 5)


def _ws(problems, tune=None):
    mar = pms._Marshal(problems)
    sz = ctypes.c_size_t(0)
    t = ctypes.byref(tune) if tune is not None else None
    return pms.load().pms_batch_workspace_size(mar.arr, len(problems), t, ctypes.byref(sz))


def test_alphabet_limits_host_only(lib):
    P = I.PROTEIN
    prot = I.random_strings(1, 4, 60, P).seqs
    assert _ws([pms.Problem(prot, 11, 4, P)]) == pms.PMS_OK
    assert _ws([pms.Problem(prot, 24, 9, P)]) == pms.PMS_OK         # 2 words of 12 5-bit codes
    assert _ws([pms.Problem(prot, 25, 9, P)]) == pms.PMS_E_UNSUPPORTED
    a16 = "ABCDEFGHIJKLMNOP"
    s16 = I.random_strings(2, 3, 60, a16).seqs
    assert _ws([pms.Problem(s16, 32, 9, a16)]) == pms.PMS_OK        # 2 words of 16 4-bit codes
    assert _ws([pms.Problem(s16, 33, 9, a16)]) == pms.PMS_E_UNSUPPORTED  # 32-bit planes
    for a in ("01", "ACG"):
        assert _ws([pms.Problem(I.random_strings(3, 3, 40, a).seqs, 8, 2, a)]) == pms.PMS_OK
    dna = I.random_strings(4, 3, 60).seqs
    # one batch: l > 32 and a large alphabet never share one (no l-mer class holds both)
    assert _ws([pms.Problem(dna, 40, 9), pms.Problem(prot, 11, 4, P)]) == pms.PMS_E_UNSUPPORTED
    assert _ws([pms.Problem(dna, 20, 5), pms.Problem(prot, 11, 4, P)]) == pms.PMS_OK


def test_expected_motifs_one_window_is_the_ball(lib):
    # n = 1, m = l: Appendix C's expectation is exact, the motif set being
    # the d-ball of the one window, sum_i C(l,i) (sigma-1)^i l-mers; the
    # oracle's set size fixes it for every alphabet size
    import oracle
    for seed, alpha, l, d in [(1, "ACGT", 6, 2), (2, I.PROTEIN, 4, 2), (3, "01", 10, 3),
                              (4, "ACG", 7, 2), (5, "ABCDEFGH", 5, 3)]:
        inst = I.random_strings(seed, 1, l, alpha)
        want = len(oracle.solve_a(inst.seqs, l, d, alphabet=alpha))
        assert round(pms.expected_motifs(1, l, l, d, len(alpha))) == want
        assert round(pms.expected_motifs(1, l, l, d, 0)) == round(pms.expected_motifs(1, l, l, d, 4))


def test_default_threshold_any_alphabet(lib):
    for sigma in (2, 3, 4, 8, 20, 32):
        for (l, d) in [(9, 2), (13, 5), (17, 7)]:
            assert 2 <= pms.default_threshold(20, 600, l, d, sigma) <= 8
    # the same Appendix D model as the oracle's (at its best stack size of 3 and up)
    from oracle.oracle import default_threshold
    for sigma in (8, 20, 32):
        for (l, d) in [(9, 2), (11, 3), (15, 5), (20, 8)]:
            want = default_threshold(20, 600, l, d, sigma)
            if want >= 3:
                assert pms.default_threshold(20, 600, l, d, sigma) == want


def test_workspace_size_is_host_only(lib):
    inst = I.planted(3, 9, 2, 10, 200)
    mar = pms._Marshal([pms.Problem(inst.seqs, 9, 2)])
    sz = ctypes.c_size_t(0)
    assert lib.pms_batch_workspace_size(mar.arr, 1, None, ctypes.byref(sz)) == pms.PMS_OK
    r = 200 - 9 + 1
    # at least the compat bit-matrix: N * n * ceil(r/64) words
    assert sz.value >= (10 * r) * 10 * ((r + 63) // 64) * 8


def test_tune_validation_is_host_only(lib):
    inst = I.planted(3, 9, 2, 10, 200)
    mar = pms._Marshal([pms.Problem(inst.seqs, 9, 2)])
    sz = ctypes.c_size_t(0)

    def st(**kw):
        t = pms.Tune(**kw)
        return lib.pms_batch_workspace_size(mar.arr, 1, ctypes.byref(t), ctypes.byref(sz))

    assert st() == pms.PMS_OK
    assert st(s1_begin=5, s1_end=9) == pms.PMS_OK
    assert st(s1_begin=0, s1_end=10_000) == pms.PMS_OK          # clamped to the last window
    assert st(s1_begin=9, s1_end=5) == pms.PMS_E_INVAL
    assert st(s1_begin=-1, s1_end=5) == pms.PMS_E_INVAL
    assert st(split=2048) == pms.PMS_E_INVAL
    assert st(split=1) == pms.PMS_OK
    assert st(compat_kernel=2) == pms.PMS_OK                 # the int8 MFMA builder
    assert st(compat_kernel=3) == pms.PMS_E_INVAL
    assert st(compat_mode=2) == pms.PMS_OK
    assert st(compat_mode=3) == pms.PMS_E_INVAL


def test_autotune_argument_checks(lib):
    out = pms.Tune()
    base = pms.Tune(split=7)
    # no instances: the base comes back, nothing runs on a device
    assert lib.pms_autotune(None, 0, ctypes.byref(base), 4, 4, ctypes.byref(out)) == pms.PMS_OK
    assert out.split == 7
    assert lib.pms_autotune(None, 1, None, 4, 4, ctypes.byref(out)) == pms.PMS_E_INVAL
    assert lib.pms_autotune(None, 0, None, 4, 4, None) == pms.PMS_E_INVAL


def test_compat_layout_choice_is_host_only(lib):
    # the whole matrix while it stays under 1 GiB, S_1's rows above (section
    # 2.2's memory bound): n = 20 at 4000 characters keeps the whole 0.8 GB
    # matrix, at 5000 characters (1.24 GB) only S_1's rows, as if forced
    def ws(m, mode):
        inst = I.planted(61, 16, 4, 20, m)
        mar = pms._Marshal([pms.Problem(inst.seqs, 16, 4)])
        sz = ctypes.c_size_t(0)
        t = pms.Tune(compat_mode=mode)
        assert lib.pms_batch_workspace_size(mar.arr, 1, ctypes.byref(t), ctypes.byref(sz)) == pms.PMS_OK
        return sz.value
    whole = (20 * 3985) * 20 * ((3985 + 63) // 64) * 8
    assert ws(4000, 0) == ws(4000, 1) >= whole
    assert ws(4000, 2) < ws(4000, 0) - whole // 2
    assert ws(5000, 0) == ws(5000, 2) < ws(5000, 1)


def test_expected_motifs_matches_oracle_means(lib):
    # Appendix C: over i.i.d. uniform strings the expected number of l-mers
    # within d of some window of every string; the mean of the oracle's set
    # sizes over 200 seeds must agree within 4 standard errors plus 3% (the
    # expectation treats overlapping windows as independent)
    import statistics
    import oracle
    for (n, m, l, d, alpha) in [(4, 40, 6, 1, "ACGT"), (5, 60, 7, 2, "ACGT"), (3, 30, 5, 1, "ACG"),
                                (4, 50, 8, 2, "01"), (3, 40, 4, 1, I.PROTEIN)]:
        cs = [len(oracle.solve_a(I.random_strings(s, n, m, alpha).seqs, l, d, alphabet=alpha))
              for s in range(200)]
        mean, se = statistics.mean(cs), statistics.stdev(cs) / len(cs) ** 0.5
        e = pms.expected_motifs(n, m, l, d, len(alpha))
        assert abs(mean - e) <= 4 * se + 0.03 * e, (n, m, l, d, len(alpha), mean, se, e)
