"""pms_solve_device_noalloc (the entry point for callers that cannot
allocate device memory) through the C ABI, against pms_solve_batch on the
same instances: identical sorted sets, on consecutive calls that reuse the
library's fixed scratch array (the second call smaller than the first)."""
import ctypes
import sys

import pytest

from paper_1307_0571_amd import instances as I
from paper_1307_0571_amd import pms

from . import hip_rt

pytestmark = pytest.mark.gpu

DNA = "ACGT"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _lib():
    lib = pms.load()
    vp = ctypes.c_void_p
    lib.pms_solve_device_noalloc.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                                             ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64,
                                             vp, vp]
    lib.pms_solve_device_noalloc.restype = ctypes.c_int
    lib.pms_noalloc_scratch_bytes.argtypes = []
    lib.pms_noalloc_scratch_bytes.restype = ctypes.c_size_t
    return lib


def _decode(raw: bytes, count: int, l: int, words: int):
    keys = [int.from_bytes(raw[8 * i:8 * i + 8], "little") for i in range(count * words)]
    out = []
    for i in range(count):
        k = keys[i * words:(i + 1) * words]
        out.append("".join(DNA[(k[p >> 5] >> (62 - 2 * (p & 31))) & 3] for p in range(l)))
    return out


def _noalloc(seqs, l, d, keys_cap=1 << 16, stream=None):
    """Returns (status, count or negative status, motifs)."""
    lib = _lib()
    n, m = len(seqs), len(seqs[0])
    words = 1 if l <= 32 else 2
    raw = "".join(seqs).encode("ascii")
    d_chars = hip_rt.malloc(max(1, len(raw)))
    d_keys = hip_rt.malloc(max(1, keys_cap) * 8 * words)
    d_count = hip_rt.malloc(8)
    try:
        if raw:
            hip_rt.copy_to_device(d_chars, raw)
        hip_rt.memset(d_count, 0x7F, 8)
        rc = lib.pms_solve_device_noalloc(d_chars, n, m, b"ACGT", l, d, d_keys, keys_cap, d_count,
                                          stream)
        if rc != pms.PMS_OK:
            return rc, None, None
        if stream:
            hip_rt.stream_synchronize(stream)
        else:
            hip_rt.device_synchronize()
        count = int.from_bytes(hip_rt.copy_from_device(d_count, 8), "little", signed=True)
        motifs = None
        if count >= 0:
            motifs = _decode(hip_rt.copy_from_device(d_keys, max(1, count) * 8 * words), count,
                             l, words)
        return rc, count, motifs
    finally:
        hip_rt.device_synchronize()
        hip_rt.free(d_chars)
        hip_rt.free(d_keys)
        hip_rt.free(d_count)


def _existing(inst):
    return pms.solve_batch([pms.Problem(inst.seqs, inst.l, inst.d)])[0]


def test_noalloc_two_calls_second_smaller():
    big = I.planted(3, 13, 4, 20, 600)
    small = I.planted(4, 9, 2, 8, 200)
    for inst in (big, small):
        _say(f"noalloc ({inst.l},{inst.d}) n={inst.n} m={inst.m} seed={inst.seed}")
        rc, count, got = _noalloc(inst.seqs, inst.l, inst.d)
        assert rc == pms.PMS_OK
        want = _existing(inst)
        assert count == len(want)
        assert got == want
        assert inst.motif in got


def test_noalloc_wide_lmers_and_stream():
    st = hip_rt.stream_create()
    try:
        for inst in (I.planted(11, 33, 8, 5, 120), I.planted(12, 10, 3, 6, 150)):
            _say(f"noalloc on a stream ({inst.l},{inst.d}) n={inst.n} m={inst.m}")
            rc, count, got = _noalloc(inst.seqs, inst.l, inst.d, stream=st)
            assert rc == pms.PMS_OK
            assert got == _existing(inst)
    finally:
        hip_rt.stream_destroy(st)


def test_noalloc_s1_rows_mode():
    # the whole compat matrix (130 MB) would take over a quarter of the
    # scratch array, so only S_1's rows are built
    inst = I.planted(13, 9, 1, 16, 2000)
    _say(f"noalloc S_1-row compat ({inst.l},{inst.d}) n={inst.n} m={inst.m}")
    rc, count, got = _noalloc(inst.seqs, inst.l, inst.d)
    assert rc == pms.PMS_OK
    assert got == _existing(inst)
    assert inst.motif in got


def test_noalloc_limits_and_errors():
    _say("noalloc limits")
    lib = _lib()
    assert lib.pms_noalloc_scratch_bytes() == 256 << 20
    # larger than the scratch array (8191 windows per string: 512 MiB of
    # work items alone): refused on the host, nothing enqueued
    huge = I.random_strings(5, 4, 8200)
    rc, _, _ = _noalloc(huge.seqs, 10, 2, keys_cap=16)
    assert rc == pms.PMS_E_NOMEM
    # invalid arguments are refused on the host
    rc, _, _ = _noalloc(["ACGTACGT", "ACGTACGT"], 4, 4)
    assert rc == pms.PMS_E_INVAL
    # a character outside the alphabet is reported through the count
    rc, count, _ = _noalloc(["ACGTACGTNA", "ACGTACGTAA"], 4, 1)
    assert rc == pms.PMS_OK and count == pms.PMS_E_ALPHABET
    # more motifs than output slots
    inst = I.planted(6, 9, 2, 6, 300)
    want = _existing(inst)
    assert len(want) > 1
    rc, count, _ = _noalloc(inst.seqs, 9, 2, keys_cap=len(want) - 1)
    assert rc == pms.PMS_OK and count == pms.PMS_E_NOMEM
    # exactly enough slots, and m < l (empty set)
    rc, count, got = _noalloc(inst.seqs, 9, 2, keys_cap=len(want))
    assert count == len(want) and got == want
    rc, count, got = _noalloc(["ACG", "TTA"], 4, 1)
    assert rc == pms.PMS_OK and count == 0 and got == []
