"""Build and load the generator's C helper (gcc, OpenMP)."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "stgen_scatter.c")
_LIB = os.path.join(_HERE, "_lib", "libstgen.so")
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-std=c11", _SRC, "-o", _LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.stgen_row_bounds.argtypes = [i32, i32, i32, P, P]
        L.stgen_row_bounds.restype = None
        L.stgen_pattern.argtypes = [i32, i32, i32, P, P, P, ctypes.c_int, P, P, P, P]
        L.stgen_pattern.restype = None
        L.stgen_scatter.argtypes = [i32, i32, P, i64, i64, P, ctypes.c_int, P, P, P, P, P, P, P, P]
        L.stgen_scatter.restype = None
        _lib = L
    return _lib
