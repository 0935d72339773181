"""GPU path over alphabets other than DNA, through the C ABI, against the CPU
oracle: identical sorted sets.  Section 1 states the problem over any
alphabet, Section 2.1 stores an l-mer in l * ceil(log2 |alphabet|) bits, and
Theorem 1 holds for any alphabet (Section 2.4).  Up to 4 letters run in the
two-plane class (children limited to the alphabet's codes); 5 to 32 letters
in the five-plane class with B-bit keys."""
import string
import sys

import pytest

import oracle
from paper_1307_0571_amd import instances as I
from paper_1307_0571_amd import pms

pytestmark = pytest.mark.gpu

P = I.PROTEIN
A8 = "ABCDEFGH"
A16 = "ABCDEFGHIJKLMNOP"
A32 = string.ascii_uppercase + "012345"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _want(inst):
    if inst.n == 1 or inst.l <= 6:
        return oracle.solve_a(inst.seqs, inst.l, inst.d, alphabet=inst.alphabet)
    return oracle.solve_b(inst.seqs, inst.l, inst.d, alphabet=inst.alphabet)


def _gpu(inst, tune=None):
    return pms.solve_batch([pms.Problem(inst.seqs, inst.l, inst.d, inst.alphabet)], tune=tune)[0]


CASES = [
    # (name, seed, alphabet, l, d, n, m)
    ("protein_11_4", 1, P, 11, 4, 10, 300),
    ("protein_13_5", 2, P, 13, 5, 20, 600),
    ("protein_15_6", 3, P, 15, 6, 12, 400),
    ("protein_9_4", 23, P, 9, 4, 8, 200),
    ("protein_10_5", 21, P, 10, 5, 10, 200),
    ("protein_8_4_2d_ge_l", 24, P, 8, 4, 5, 40),
    ("protein_17_7", 10, P, 17, 7, 10, 300),
    ("protein_n1", 30, P, 5, 1, 1, 20),
    ("a32_24_9_two_key_words", 5, A32, 24, 9, 6, 150),
    ("a32_12_6", 26, A32, 12, 6, 8, 150),
    ("a8_22_7_word_boundary", 6, A8, 22, 7, 6, 150),
    ("a16_20_7_word_boundary", 7, A16, 20, 7, 6, 150),
    ("a16_32_12_full_width", 27, A16, 32, 12, 4, 60),
    ("binary_14_2", 8, "01", 14, 2, 5, 100),
    ("binary_34_3_wide", 31, "01", 34, 3, 4, 50),
    ("ternary_10_2", 9, "ACG", 10, 2, 6, 80),
]


@pytest.mark.parametrize("name,seed,alpha,l,d,n,m", CASES)
def test_alphabet_vs_oracle(name, seed, alpha, l, d, n, m):
    _say(f"{name}: seed={seed} |alphabet|={len(alpha)} l={l} d={d} n={n} m={m}")
    inst = I.planted(seed, l, d, n, m, alphabet=alpha)
    want = _want(inst)
    got = _gpu(inst)
    assert got == want
    assert inst.motif in got


@pytest.mark.parametrize("name,seed,alpha,l,d,n,m", [c for c in CASES if c[0] in (
    "protein_13_5", "protein_8_4_2d_ge_l", "a32_24_9_two_key_words", "a16_32_12_full_width",
    "binary_34_3_wide", "ternary_10_2", "a8_22_7_word_boundary")])
def test_alphabet_mfma_compat(name, seed, alpha, l, d, n, m):
    _say(f"mfma compat {name}")
    inst = I.planted(seed, l, d, n, m, alphabet=alpha)
    assert _gpu(inst, pms.Tune(compat_kernel=2)) == _want(inst)


def test_packed_keys_layout():
    # pms_solve's packed keys: B-bit codes, floor(64 / B) characters per
    # word, first character in the top bits
    import ctypes
    for seed, alpha, l, d, n, m, B in [(24, P, 8, 4, 5, 40, 5), (6, A8, 22, 7, 6, 150, 3),
                                       (27, A16, 32, 12, 4, 60, 4)]:
        _say(f"packed keys |alphabet|={len(alpha)} l={l}")
        inst = I.planted(seed, l, d, n, m, alphabet=alpha)
        lib = pms.load()
        arr = (ctypes.c_char_p * n)(*[x.encode() for x in inst.seqs])
        res = pms._Result()
        assert lib.pms_solve(arr, n, m, alpha.encode(), l, d, ctypes.byref(res)) == pms.PMS_OK
        try:
            cpw = 64 // B
            assert res.words == (l + cpw - 1) // cpw
            raw = ctypes.string_at(res.motifs, res.count * l).decode()
            mots = [raw[i * l:(i + 1) * l] for i in range(res.count)]
            assert mots == _want(inst)
            for i, mot in enumerate(mots):
                want = [0] * res.words
                for p, ch in enumerate(mot):
                    want[p // cpw] |= alpha.index(ch) << (64 - B * (p % cpw + 1))
                assert [res.packed[i * res.words + q] for q in range(res.words)] == want
        finally:
            lib.pms_result_free(ctypes.byref(res))


@pytest.mark.parametrize("tune", [
    dict(threshold=2), dict(threshold=3), dict(threshold=4), dict(threshold=5),
    dict(threshold=5, split=1), dict(triple_filter=-1), dict(compat_mode=2),
    dict(stage_cap=512), dict(waves_per_cu=1), dict(out_capacity=1), dict(split=2),
    dict(compat_kernel=2), dict(compat_kernel=2, compat_mode=2),
])
def test_protein_invariant_under_tuning(tune):
    _say(f"protein tune {tune}")
    inst = I.planted(21, 10, 5, 10, 200, alphabet=P)
    want = _want(inst)
    assert _gpu(inst, pms.Tune(**tune)) == want


def test_mixed_alphabets_in_one_batch():
    _say("one batch: DNA, protein, ternary and 32 letters")
    insts = [I.planted(40, 10, 2, 6, 150), I.planted(41, 11, 4, 10, 300, alphabet=P),
             I.planted(42, 9, 2, 6, 80, alphabet="ACG"), I.planted(43, 12, 3, 8, 200),
             I.planted(44, 12, 6, 8, 150, alphabet=A32)]
    got = pms.solve_batch([pms.Problem(x.seqs, x.l, x.d, x.alphabet) for x in insts])
    for x, g in zip(insts, got):
        assert g == _want(x)


def test_serving_mixed_classes():
    # l > 32 and large alphabets never share a pass; every request is served
    _say("serving: DNA l > 32, protein and DNA requests together")
    insts = [I.planted(50, 33, 8, 5, 120), I.planted(51, 11, 4, 10, 300, alphabet=P),
             I.planted(52, 10, 2, 6, 150), I.planted(53, 40, 12, 4, 100),
             I.planted(54, 9, 4, 8, 200, alphabet=P), I.planted(55, 12, 6, 8, 150, alphabet=A32)]
    srv = pms.Server(max_wave=8)
    try:
        tickets = [srv.submit(pms.Problem(x.seqs, x.l, x.d, x.alphabet)) for x in insts]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for x, g in zip(insts, got):
        assert g == _want(x)
