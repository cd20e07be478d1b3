"""Loader for the oracle's plain-C direct-sum helper (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "direct.c")
_LIB = os.path.join(_HERE, "_oracle_direct.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C helper with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        _lib = ctypes.CDLL(path)
        _lib.oracle_direct.restype = None
        _lib.oracle_direct.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return _lib


def direct(kernel: int, xt: np.ndarray, ys: np.ndarray, dens: np.ndarray, out: np.ndarray,
           shift=None) -> None:
    """out[t] += sum_s K(x_t - (y_s + shift)) dens[s]; zero-separation pairs skipped."""
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.float64)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous
    k = 1 if kernel == 1 else 3
    assert xt.shape[0] * k == out.size and ys.shape[0] * k == dens.size
    if xt.shape[0] == 0 or ys.shape[0] == 0:
        return
    sh = None
    if shift is not None:
        sh = np.ascontiguousarray(shift, dtype=np.float64)
    lib().oracle_direct(kernel, xt.shape[0], xt.ctypes.data, ys.shape[0], ys.ctypes.data,
                        dens.ctypes.data, None if sh is None else sh.ctypes.data, out.ctypes.data)
