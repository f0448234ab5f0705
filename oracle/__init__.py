"""Plain FP64 CPU oracle for the continuous (box) Gauss transform.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU path (``paper_2305_07165_amd``) and never imports it.

``oracle_u`` returns, at every Gauss-Legendre node of the requested leaves,

    u(x) = sum_S int_S G(x - y; delta) s_S(y) dy

with s_S the tensor Legendre interpolant of the samples on leaf S (Eq. (bgt)
with the leaf model of Eq. (papprox)), computed by the plain definition in
``oracle.c`` (Lemma directbox with adaptive Gauss-Legendre 1D integrals).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (strict IEEE, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_box_fgt.restype = ctypes.c_int64
        lib.oracle_box_fgt.argtypes = [ctypes.c_int, ctypes.c_int64, i32p, i32p,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_double, f64p, ctypes.c_int64, i64p,
                                       f64p, ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_gauss_legendre.restype = None
        lib.oracle_gauss_legendre.argtypes = [ctypes.c_int, f64p, f64p]
        _lib = lib
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def oracle_u(levels, coords, p: int, delta: float, sigma, periodic: bool = False,
             targets=None, rcut: float = 0.0, nthreads: int = 0,
             return_pairs: bool = False):
    """u at the nodes of ``targets`` (default: every leaf), ``[nt, p**d]``."""
    lib = _load()
    levels = np.ascontiguousarray(levels, dtype=np.int32)
    coords = np.ascontiguousarray(coords, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    n, d = coords.shape
    if sigma.shape != (n, p ** d):
        raise ValueError(f"sigma has shape {sigma.shape}, expected {(n, p ** d)}")
    if targets is None:
        tp = None
        nt = n
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tp = _ptr(targets, ctypes.c_int64)
        nt = len(targets)
    u = np.zeros((nt, p ** d), dtype=np.float64)
    npair = lib.oracle_box_fgt(d, n, _ptr(levels, ctypes.c_int32), _ptr(coords, ctypes.c_int32),
                               p, float(delta), int(bool(periodic)), float(rcut),
                               _ptr(sigma, ctypes.c_double), nt, tp,
                               _ptr(u, ctypes.c_double), int(nthreads))
    if npair < 0:
        raise RuntimeError(f"oracle_box_fgt failed ({npair})")
    return (u, int(npair)) if return_pairs else u


def threads_used() -> int:
    return int(_load().oracle_threads())


def gauss_legendre(n: int):
    lib = _load()
    x = np.zeros(n)
    w = np.zeros(n)
    lib.oracle_gauss_legendre(n, _ptr(x, ctypes.c_double), _ptr(w, ctypes.c_double))
    return x, w
