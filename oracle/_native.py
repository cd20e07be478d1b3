"""Loader for the oracle's plain-C direct-sum helper (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "direct.c")
_SRC_EWALD = os.path.join(_HERE, "csrc", "ewald_tp.c")
_LIB = os.path.join(_HERE, "_oracle_direct.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C helper with gcc (OpenMP, no fast-math)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_EWALD))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, _SRC_EWALD, "-o", tmp, "-lm"])
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
        _lib.tp_ewald_targets.restype = None
        _lib.tp_ewald_targets.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
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


def tp_ewald_targets(kernel: int, targets: np.ndarray, sources: np.ndarray, dens: np.ndarray,
                     xi: float = 10.6, tol_x: float = 5.8) -> np.ndarray:
    """The triply periodic sum (k = 0 removed) at a few targets from many sources through structure
    factors (csrc/ewald_tp.c).  dens: [N, k] or [R, N, k]; returns [T, k] or [R, T, k].  Real space
    to rc = 5.3/xi (at most half the period: erfc(5.3) ~ 7e-14), Fourier space to |k| <= 2 xi tol_x
    (e^{-x^2}(1 + x^2) ~ 1e-13 at x = 5.8)."""
    xt = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1, 3)
    ys = np.ascontiguousarray(sources, dtype=np.float64).reshape(-1, 3)
    k = 1 if kernel == 1 else 3
    d = np.asarray(dens, dtype=np.float64)
    single = d.ndim < 3 and not (d.ndim == 2 and k == 1 and d.shape[0] != ys.shape[0])
    d = np.ascontiguousarray(d.reshape(-1, ys.shape[0], k))
    R = d.shape[0]
    assert 1 <= R <= 16 and R * k <= 64
    rc = 5.3 / xi
    assert rc <= 0.5
    kint = int(np.ceil(2.0 * xi * tol_x / (2.0 * np.pi)))
    out = np.zeros((R, xt.shape[0], k))
    lib().tp_ewald_targets(kernel, R, xt.shape[0], xt.ctypes.data, ys.shape[0], ys.ctypes.data, d.ctypes.data,
                           xi, rc, kint, out.ctypes.data)
    return out[0] if single else out
