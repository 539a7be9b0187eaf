"""Loads the oracle's plain C pair sums (oracle/pairsum.c) through ctypes.

The shared object is compiled with gcc on first use if it is missing (it is
test infrastructure, so compiling it on demand is fine); `build()` in the
repository entry point also compiles it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pairsum.c")
_SO = os.path.join(_HERE, "_build", "liboracle_pairsum.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            d = ctypes.POINTER(ctypes.c_double)
            i64 = ctypes.c_int64
            lib.oracle_charge_sums.argtypes = [i64, d, i64, d, d, ctypes.POINTER(i64), d, d]
            lib.oracle_charge_sums.restype = None
            lib.oracle_layer_sums.argtypes = [i64, d, i64, d, d, d, d, d, d]
            lib.oracle_layer_sums.restype = None
            _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def charge_sums(targets, sources, charges, skip=None):
    """phi (nt,), field (nt,3) from point charges; skip[t] = source index to omit."""
    lib = _load()
    t = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1, 3)
    s = np.ascontiguousarray(sources, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(charges, dtype=np.float64).reshape(-1)
    assert q.shape[0] == s.shape[0]
    phi = np.zeros(t.shape[0])
    field = np.zeros((t.shape[0], 3))
    sk = None
    if skip is not None:
        skip = np.ascontiguousarray(skip, dtype=np.int64)
        assert skip.shape[0] == t.shape[0]
        sk = skip.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    lib.oracle_charge_sums(t.shape[0], _dp(t), s.shape[0], _dp(s), _dp(q), sk, _dp(phi), _dp(field))
    return phi, field


def layer_sums(targets, points, normals, Q, D):
    """phi, field from single-layer charges Q and double-layer strengths D."""
    lib = _load()
    t = np.ascontiguousarray(targets, dtype=np.float64).reshape(-1, 3)
    y = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    n = np.ascontiguousarray(normals, dtype=np.float64).reshape(-1, 3)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    phi = np.zeros(t.shape[0])
    field = np.zeros((t.shape[0], 3))
    lib.oracle_layer_sums(t.shape[0], _dp(t), y.shape[0], _dp(y), _dp(n), _dp(Q), _dp(D), _dp(phi), _dp(field))
    return phi, field
