"""ctypes binding of libbmprobe.so: the device's vector-ALU issue rate, the
measured counterpart of the path kernels' roofline peak (one wave64 instruction
per CU per clock).  A measurement aid of the benchmark, not part of the method."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbmprobe.so")
_lib = None


class ProbeError(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbmprobe.so not built (run python -m paper_1409_4923_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        L.bmp_valu_probe.restype = ctypes.c_int
        L.bmp_valu_probe.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        L.bmp_last_error.restype = ctypes.c_char_p
        L.bmp_last_error.argtypes = []
        _lib = L
    return _lib


def valu_probe(mix: int, iters: int, d_out: int, n_out: int, stream: int) -> float:
    """Lane-operations per second for mix 0 (FMA chains), 1 (FMA + compare +
    select) or 2 (FMA + exp2); d_out: n_out device floats (a multiple of 256)."""
    r = ctypes.c_double(0.0)
    rc = lib().bmp_valu_probe(mix, iters, d_out, n_out, stream, ctypes.byref(r))
    if rc != 0:
        raise ProbeError("libbmprobe error %d: %s" % (rc, lib().bmp_last_error().decode()))
    return r.value
