"""Build-and-load helper for the oracle's C core (test infrastructure only).

The C core (``csrc/oracle_core.c``) is compiled with gcc into
``oracle/_build/liboracle.so``.  ``build()`` always recompiles; ``lib()``
compiles only when the shared object is missing.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle_core.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_SO = os.path.join(_OUT_DIR, "liboracle.so")
_lib = None


def build():
    os.makedirs(_OUT_DIR, exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_F32 = ctypes.POINTER(ctypes.c_float)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.oracle_line_segments.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, _I32, _D, _D]
        L.oracle_line_segments.restype = ctypes.c_int
        for name in ("oracle_project", "oracle_backproject"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, _D, _D, _D, _D, _D]
            f.restype = None
        L.oracle_nlm.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, _D]
        L.oracle_nlm.restype = None
        L.oracle_bm3d_ref_axis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32]
        L.oracle_bm3d_ref_axis.restype = ctypes.c_int
        L.oracle_bm3d_groups.argtypes = [ctypes.c_int, _F32, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_float, ctypes.c_int, _I32, _I32, _I32]
        L.oracle_bm3d_groups.restype = None
        L.oracle_bm3d_keep.argtypes = [ctypes.c_int, _F32, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       _I32, _I32, _F32, ctypes.c_float, _U8, _I32]
        L.oracle_bm3d_keep.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the C core's OpenMP loops; returns the previous count."""
    L = lib()
    prev = int(L.oracle_max_threads())
    L.oracle_set_threads(int(n))
    return prev


def dptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def iptr(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_I32)


def fptr(a):
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_F32)


def u8ptr(a):
    assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_U8)
