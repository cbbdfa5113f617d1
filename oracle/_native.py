"""Loader for the oracle's plain-C pair loops (``csrc/oracle_pairs.c``).

Test infrastructure only.  The shared object is built with gcc (no fast-math,
no FP contraction) into this directory; ``build()`` always recompiles, ``lib()``
compiles only when the object is missing or older than its source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle_pairs.c")
_LIB = os.path.join(_HERE, "liboracle_pairs.so")
_handle = None


def build() -> str:
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _handle
    if _handle is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        h = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        h.oracle_direct_sum.argtypes = [i64, d, d, d, i64, d, d, d, d, i64,
                                        ctypes.c_int32, ctypes.c_double, d]
        h.oracle_direct_sum.restype = None
        h.oracle_kernel_pairs.argtypes = [i64, d, d, d, ctypes.c_int32,
                                          ctypes.c_double, d]
        h.oracle_kernel_pairs.restype = None
        _handle = h
    return _handle


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def direct_sum(targets: np.ndarray, sources: np.ndarray, sigma: np.ndarray,
               kernel_id: int, param: float) -> np.ndarray:
    """phi[i, c] = sum_j K(t_i, s_j) sigma[j, c] in float64 (eq. (1))."""
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.float64).T)
    s = np.ascontiguousarray(np.asarray(sources, dtype=np.float64).T)
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    if sig.ndim == 1:
        sig = sig[:, None]
    nt, ns, r = t.shape[1], s.shape[1], sig.shape[1]
    assert sig.shape[0] == ns
    out = np.zeros((nt, r), dtype=np.float64)
    if nt == 0 or ns == 0:
        return out
    lib().oracle_direct_sum(nt, _dp(t[0]), _dp(t[1]), _dp(t[2]), ns,
                            _dp(s[0]), _dp(s[1]), _dp(s[2]), _dp(sig), r,
                            int(kernel_id), float(param), _dp(out))
    return out


def kernel_values(diff: np.ndarray, kernel_id: int, param: float) -> np.ndarray:
    """K evaluated at target-minus-source differences ``diff`` (..., 3)."""
    diff = np.asarray(diff, dtype=np.float64)
    shape = diff.shape[:-1]
    d = np.ascontiguousarray(diff.reshape(-1, 3).T)
    out = np.empty(d.shape[1], dtype=np.float64)
    if out.size:
        lib().oracle_kernel_pairs(out.size, _dp(d[0]), _dp(d[1]), _dp(d[2]),
                                  int(kernel_id), float(param), _dp(out))
    return out.reshape(shape)
