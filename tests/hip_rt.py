"""Minimal ctypes access to the system HIP runtime (the one libpms is linked
against), for tests that hand the library a borrowed stream or a caller
workspace.  Importing this module loads no GPU code; the first call does."""
from __future__ import annotations

import ctypes
import os

_LIB = "/opt/rocm/lib/libamdhip64.so"
_hip = None


def _rt():
    global _hip
    if _hip is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} is missing")
        _hip = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        _hip.hipMalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t]
        _hip.hipFree.argtypes = [vp]
        _hip.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(vp), ctypes.c_uint]
        _hip.hipStreamDestroy.argtypes = [vp]
        _hip.hipStreamSynchronize.argtypes = [vp]
        _hip.hipMemset.argtypes = [vp, ctypes.c_int, ctypes.c_size_t]
        _hip.hipDeviceSynchronize.argtypes = []
        _hip.hipMemcpy.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int]
        for f in ("hipMalloc", "hipFree", "hipStreamCreateWithFlags", "hipStreamDestroy",
                  "hipStreamSynchronize", "hipMemset", "hipDeviceSynchronize", "hipMemcpy"):
            getattr(_hip, f).restype = ctypes.c_int
    return _hip


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with HIP error {rc}")


def malloc(nbytes: int) -> int:
    p = ctypes.c_void_p()
    _check(_rt().hipMalloc(ctypes.byref(p), nbytes), "hipMalloc")
    return int(p.value)


def free(ptr: int) -> None:
    _check(_rt().hipFree(ctypes.c_void_p(ptr)), "hipFree")


def memset(ptr: int, value: int, nbytes: int) -> None:
    _check(_rt().hipMemset(ctypes.c_void_p(ptr), value, nbytes), "hipMemset")


def copy_to_device(dst: int, data: bytes) -> None:
    buf = ctypes.create_string_buffer(data, len(data))
    _check(_rt().hipMemcpy(ctypes.c_void_p(dst), buf, len(data), 1), "hipMemcpy H2D")


def copy_from_device(src: int, nbytes: int) -> bytes:
    buf = ctypes.create_string_buffer(nbytes)
    _check(_rt().hipMemcpy(buf, ctypes.c_void_p(src), nbytes, 2), "hipMemcpy D2H")
    return buf.raw


def stream_create() -> int:
    s = ctypes.c_void_p()
    _check(_rt().hipStreamCreateWithFlags(ctypes.byref(s), 1), "hipStreamCreateWithFlags")
    return int(s.value)


def stream_destroy(s: int) -> None:
    _check(_rt().hipStreamDestroy(ctypes.c_void_p(s)), "hipStreamDestroy")


def stream_synchronize(s: int) -> None:
    _check(_rt().hipStreamSynchronize(ctypes.c_void_p(s)), "hipStreamSynchronize")


def device_synchronize() -> None:
    _check(_rt().hipDeviceSynchronize(), "hipDeviceSynchronize")
