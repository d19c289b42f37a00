"""Loader for the oracle's plain-C band routines (builds them with gcc if absent)."""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "band.c")
_LIB = os.path.join(_HERE, "liboracle_band.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile band.c with gcc (IEEE semantics: no fast-math, no -march)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = build()
            L = ctypes.CDLL(path)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int64)
            L.band_lu.argtypes = [ctypes.c_long, ctypes.c_long, dp, dp]
            L.band_lu.restype = ctypes.c_long
            L.band_solve.argtypes = [ctypes.c_long, ctypes.c_long, dp, ctypes.c_long, dp]
            L.band_solve.restype = None
            L.netlist_residual_ld.argtypes = [
                ctypes.c_long, ctypes.c_long, ip, ip, dp, ctypes.c_long, ip, ip, dp,
                ctypes.c_long, dp, ctypes.c_long, dp, ctypes.c_void_p, dp]
            L.netlist_residual_ld.restype = None
            _lib = L
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def iptr(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
