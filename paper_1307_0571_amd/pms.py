"""Python binding of libpms (ctypes).  Argument marshalling only: every step
of the search runs in the library's HIP kernels.

One HIP runtime per process: libpms is built against the system ROCm, and
the torch wheel bundles its own HIP runtime under the same soname, so a
process that loads libpms must not also load torch's runtime.  Device memory
comes from the library itself (or from a caller workspace pointer allocated
in the same runtime); streams are passed as raw hipStream_t handles."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpms.so")

PMS_OK = 0
PMS_E_INVAL = -1
PMS_E_ALPHABET = -2
PMS_E_UNSUPPORTED = -3
PMS_E_NOMEM = -4
PMS_E_DEVICE = -5
PMS_E_AGAIN = -6
PMS_E_ABORTED = -7
PMS_E_TIMEOUT = -8


class PmsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})" if what else strerror(status))


class _Instance(ctypes.Structure):
    _fields_ = [("seqs", ctypes.POINTER(ctypes.c_char_p)), ("n", ctypes.c_int32),
                ("m", ctypes.c_int32), ("alphabet", ctypes.c_char_p),
                ("l", ctypes.c_int32), ("d", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("l", ctypes.c_int32), ("words", ctypes.c_int32),
                ("motifs", ctypes.POINTER(ctypes.c_char)),
                ("packed", ctypes.POINTER(ctypes.c_uint64))]


class Tune(ctypes.Structure):
    """Search parameters (0 = automatic); none of them changes the result
    except s1_begin / s1_end, which restrict the search to those S_1 windows."""
    _fields_ = [("threshold", ctypes.c_int32), ("lmer_words", ctypes.c_int32),
                ("triple_filter", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("compat_kernel", ctypes.c_int32), ("split", ctypes.c_int32),
                ("s1_begin", ctypes.c_int32), ("s1_end", ctypes.c_int32),
                ("stage_cap", ctypes.c_int32), ("compat_mode", ctypes.c_int32),
                ("out_capacity", ctypes.c_int64)]

    def __init__(self, threshold=0, lmer_words=0, triple_filter=0, waves_per_cu=0,
                 compat_kernel=0, split=0, s1_begin=0, s1_end=0, out_capacity=0, stage_cap=0,
                 compat_mode=0):
        super().__init__(threshold, lmer_words, triple_filter, waves_per_cu, compat_kernel,
                         split, s1_begin, s1_end, stage_cap, compat_mode, out_capacity)


class Work(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "compat_pairs", "items", "pushes", "filter_words", "triple_tests", "tuples",
        "gen_evals", "candidates", "verify_tests", "motifs_emitted", "done_ticks")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class _StreamConfig(ctypes.Structure):
    _fields_ = [("device_mem_cap", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_wave", ctypes.c_int32), ("tune", Tune), ("workers", ctypes.c_int32)]


_lib = None


def _foreign_hip_runtime() -> Optional[str]:
    """Path of a HIP runtime other than the system one already mapped here."""
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line and "/opt/rocm" not in line:
                    return line.split()[-1]
    except OSError:
        pass
    return None


def load():
    """Load libpms.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    other = _foreign_hip_runtime()
    if other:
        raise RuntimeError(f"another HIP runtime is already loaded ({other}); libpms needs the "
                           "system ROCm runtime: load it in a process that does not import torch")
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1307_0571_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.pms_solve.argtypes = [P(ctypes.c_char_p), ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                              ctypes.c_int32, ctypes.c_int32, P(_Result)]
    lib.pms_solve_batch.argtypes = [P(_Instance), ctypes.c_int32, P(_Result), P(Tune), vp]
    lib.pms_batch_create.argtypes = [P(_Instance), ctypes.c_int32, P(Tune), vp, ctypes.c_size_t,
                                     P(vp)]
    lib.pms_batch_workspace_size.argtypes = [P(_Instance), ctypes.c_int32, P(Tune),
                                             P(ctypes.c_size_t)]
    lib.pms_batch_run.argtypes = [vp, vp, ctypes.c_int32]
    lib.pms_batch_results.argtypes = [vp, P(_Result)]
    lib.pms_batch_timings.argtypes = [vp, P(ctypes.c_float)]
    lib.pms_batch_destroy.argtypes = [vp]
    lib.pms_batch_work.argtypes = [vp, ctypes.c_int32, P(Work)]
    lib.pms_stream_create.argtypes = [P(_StreamConfig), P(vp)]
    lib.pms_stream_submit.argtypes = [vp, P(_Instance), P(ctypes.c_uint64)]
    lib.pms_stream_poll.argtypes = [vp, ctypes.c_uint64, P(_Result)]
    lib.pms_stream_wait.argtypes = [vp, ctypes.c_uint64, P(_Result), ctypes.c_int64]
    lib.pms_stream_destroy.argtypes = [vp]
    lib.pms_result_free.argtypes = [P(_Result)]
    lib.pms_result_free.restype = None
    lib.pms_strerror.argtypes = [ctypes.c_int]
    lib.pms_strerror.restype = ctypes.c_char_p
    lib.pms_version.restype = ctypes.c_char_p
    lib.pms_autotune.argtypes = [P(_Instance), ctypes.c_int32, P(Tune), ctypes.c_int32,
                                 ctypes.c_int32, P(Tune)]
    lib.pms_default_threshold.argtypes = [ctypes.c_int] * 5
    lib.pms_expected_motifs.argtypes = [ctypes.c_int] * 5
    lib.pms_expected_motifs.restype = ctypes.c_double
    lib.pms_device_count.argtypes = [P(ctypes.c_int32)]
    lib.pms_device_synchronize.argtypes = []
    for f in ("pms_solve", "pms_solve_batch", "pms_batch_create", "pms_batch_workspace_size",
              "pms_batch_run", "pms_batch_results", "pms_batch_timings", "pms_batch_destroy",
              "pms_stream_create", "pms_stream_submit", "pms_stream_poll", "pms_stream_wait",
              "pms_stream_destroy", "pms_default_threshold", "pms_batch_work",
              "pms_device_count", "pms_device_synchronize", "pms_autotune"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load().pms_strerror(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def device_count() -> int:
    n = ctypes.c_int32(0)
    _check(load().pms_device_count(ctypes.byref(n)), "pms_device_count")
    return int(n.value)


def device_synchronize() -> None:
    _check(load().pms_device_synchronize(), "pms_device_synchronize")


def default_threshold(n: int, m: int, l: int, d: int, sigma: int = 4) -> int:
    return int(load().pms_default_threshold(n, m, l, d, sigma))


def expected_motifs(n: int, m: int, l: int, d: int, sigma: int = 4) -> float:
    return float(load().pms_expected_motifs(n, m, l, d, sigma))


@dataclass
class Problem:
    """One instance: strings, motif length l, distance d, alphabet."""
    seqs: Sequence[str]
    l: int
    d: int
    alphabet: str = "ACGT"


class _Marshal:
    """Keeps the C views of a list of problems alive."""

    def __init__(self, problems: Sequence[Problem]):
        self.keep = []
        self.arr = (_Instance * max(1, len(problems)))()
        for i, p in enumerate(problems):
            enc = [s.encode("latin-1") for s in p.seqs]
            seqs = (ctypes.c_char_p * max(1, len(enc)))(*enc)
            alpha = p.alphabet.encode("latin-1")
            self.keep.append((enc, seqs, alpha))
            m = len(p.seqs[0]) if len(p.seqs) else 0
            self.arr[i] = _Instance(seqs, len(p.seqs), m, alpha, p.l, p.d)
        self.count = len(problems)


def _take(res: _Result) -> List[str]:
    lib = load()
    try:
        if res.count == 0:
            return []
        raw = ctypes.string_at(res.motifs, res.count * res.l).decode("latin-1")
        return [raw[i * res.l:(i + 1) * res.l] for i in range(res.count)]
    finally:
        lib.pms_result_free(ctypes.byref(res))


def _check(rc: int, what: str):
    if rc != PMS_OK:
        raise PmsError(rc, what)


def autotune(problems: Sequence[Problem], base: Optional[Tune] = None, max_runs: int = 16,
             sample: int = 32) -> Tune:
    """pms_autotune: the fastest setting for this shape of batch (cached for
    later tune=None calls on batches of the same shape)."""
    mar = _Marshal(problems)
    out = Tune()
    _check(load().pms_autotune(mar.arr, mar.count, ctypes.byref(base) if base else None,
                               max_runs, sample, ctypes.byref(out)), "pms_autotune")
    return out


def tune_dict(t: Tune) -> dict:
    return {n: int(getattr(t, n)) for n, _ in Tune._fields_}


def solve(seqs: Sequence[str], l: int, d: int, alphabet: str = "ACGT") -> List[str]:
    """pms_solve: the sorted motif set of one instance."""
    return solve_batch([Problem(seqs, l, d, alphabet)])[0]


def _stream_ptr(stream) -> Optional[int]:
    """A raw hipStream_t handle (int) or None for the library's own stream."""
    if stream is None:
        return None
    return int(stream)


def solve_batch(problems: Sequence[Problem], tune: Optional[Tune] = None,
                stream=None) -> List[List[str]]:
    """pms_solve_batch: every instance in one device pass."""
    lib = load()
    mar = _Marshal(problems)
    res = (_Result * max(1, mar.count))()
    rc = lib.pms_solve_batch(mar.arr, mar.count, res, ctypes.byref(tune) if tune else None,
                             _stream_ptr(stream))
    _check(rc, "pms_solve_batch")
    return [_take(res[i]) for i in range(mar.count)]


class Batch:
    """Device-resident batch: inputs uploaded once, then run many times.

    ``workspace`` (optional) is a (device pointer, bytes) pair the library
    borrows instead of allocating; ``Batch.workspace_size`` gives the size."""

    def __init__(self, problems: Sequence[Problem], tune: Optional[Tune] = None,
                 workspace=None):
        lib = load()
        self.mar = _Marshal(problems)
        self.tune = tune
        ptr, size = (None, 0) if workspace is None else (int(workspace[0]), int(workspace[1]))
        tp = ctypes.byref(tune) if tune else None
        h = ctypes.c_void_p()
        _check(lib.pms_batch_create(self.mar.arr, self.mar.count, tp, ptr, size, ctypes.byref(h)),
               "pms_batch_create")
        self.h = h

    @staticmethod
    def workspace_size(problems: Sequence[Problem], tune: Optional[Tune] = None) -> int:
        mar = _Marshal(problems)
        sz = ctypes.c_size_t(0)
        _check(load().pms_batch_workspace_size(mar.arr, mar.count,
                                               ctypes.byref(tune) if tune else None,
                                               ctypes.byref(sz)), "pms_batch_workspace_size")
        return int(sz.value)

    def run(self, stream=None, graph: bool = False):
        _check(load().pms_batch_run(self.h, _stream_ptr(stream), int(graph)), "pms_batch_run")

    def results(self) -> List[List[str]]:
        res = (_Result * max(1, self.mar.count))()
        _check(load().pms_batch_results(self.h, res), "pms_batch_results")
        return [_take(res[i]) for i in range(self.mar.count)]

    def timings(self) -> List[float]:
        arr = (ctypes.c_float * 5)()
        _check(load().pms_batch_timings(self.h, arr), "pms_batch_timings")
        return list(arr)

    def work(self, i: int = 0) -> dict:
        w = Work()
        _check(load().pms_batch_work(self.h, i, ctypes.byref(w)), "pms_batch_work")
        return w.as_dict()

    def close(self):
        if getattr(self, "h", None):
            load().pms_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """pms_stream_*: continuous batching of submitted instances."""

    def __init__(self, device_mem_cap: int = 0, max_inflight: int = 0, max_wave: int = 0,
                 tune: Optional[Tune] = None, workers: int = 0):
        lib = load()
        cfg = _StreamConfig(device_mem_cap, max_inflight, max_wave, tune or Tune(), workers)
        h = ctypes.c_void_p()
        _check(lib.pms_stream_create(ctypes.byref(cfg), ctypes.byref(h)), "pms_stream_create")
        self.h = h
        self._keep = {}

    def submit(self, p: Problem) -> int:
        mar = _Marshal([p])
        t = ctypes.c_uint64(0)
        _check(load().pms_stream_submit(self.h, mar.arr, ctypes.byref(t)), "pms_stream_submit")
        return int(t.value)

    def poll(self, ticket: int):
        res = _Result()
        rc = load().pms_stream_poll(self.h, ticket, ctypes.byref(res))
        if rc == PMS_E_AGAIN:
            return None
        _check(rc, "pms_stream_poll")
        return _take(res)

    def wait(self, ticket: int, timeout_us: int = -1) -> List[str]:
        res = _Result()
        _check(load().pms_stream_wait(self.h, ticket, ctypes.byref(res), timeout_us),
               "pms_stream_wait")
        return _take(res)

    def close(self):
        if getattr(self, "h", None):
            load().pms_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
