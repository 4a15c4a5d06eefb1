"""ctypes loader for the plain-C FP64 oracle (cpu_ref.c).  Test
infrastructure only, like the rest of this package."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "cpu_ref.c")
LIB = os.path.join(_HERE, "libcpu_ref.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile cpu_ref.c with gcc (OpenMP) into oracle/libcpu_ref.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-D_GNU_SOURCE", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        i64, i32, f64, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64
        P = ctypes.c_void_p
        lib.oracle_gaussian_input.argtypes = [i64, i32, u64, P]
        lib.oracle_gaussian_input.restype = None
        lib.oracle_ffp.argtypes = [i64, P, P, f64, i32, i32, P, f64, f64, f64, i32, P]
        lib.oracle_ffp.restype = ctypes.c_int
        lib.oracle_philox4x64_10.argtypes = [P, u64, u64, P]
        lib.oracle_philox4x64_10.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def gaussian_input(N, d, seed):
    X = np.empty((N, d), dtype=np.float64)
    _load().oracle_gaussian_input(int(N), int(d), ctypes.c_uint64(int(seed)), _ptr(X))
    return X


def philox4x64_10(ctr, k0, k1):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    o = np.empty(4, dtype=np.uint64)
    _load().oracle_philox4x64_10(_ptr(c), ctypes.c_uint64(int(k0)), ctypes.c_uint64(int(k1)), _ptr(o))
    return o


def ffp_from_input(rowptr, colidx, N, tau, K, X, alpha=1.0, theta=0.1, eps=1e-3, ddof=0):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    d = X.shape[1]
    out = np.empty_like(X)
    rc = _load().oracle_ffp(int(N), _ptr(rowptr), _ptr(colidx), float(tau), int(K), int(d),
                            _ptr(X), float(alpha), float(theta), float(eps), int(ddof), _ptr(out))
    if rc != 0:
        raise MemoryError("oracle_ffp: allocation failed")
    return out
