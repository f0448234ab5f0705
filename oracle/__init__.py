"""Plain FP64 CPU oracle for the continuous (box) Gauss transform.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU path (``paper_2305_07165_amd``) and never imports it.

``oracle_u`` returns, at every Gauss-Legendre node of the requested leaves,

    u(x) = sum_S int_S G(x - y; delta) s_S(y) dy

with s_S the tensor Legendre interpolant of the samples on leaf S (Eq. (bgt)
with the leaf model of Eq. (papprox)), computed by the plain definition in
``oracle.c`` (Lemma directbox with adaptive Gauss-Legendre 1D integrals).
``oracle_u_boxes`` returns the same u at the nodes of arbitrary target boxes
(the boxes of an output tree, Section 4.2).  ``oracle_interp`` evaluates a
function given by values on a tree's leaves (the leaf model of Eq. (papprox))
at arbitrary points, in numpy.  ``oracle_point`` is the discrete transform of
Eq. (pgt) summed directly over source points.
"""

from __future__ import annotations

import ctypes
import math
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
        lib.oracle_box_fgt_boxes.restype = ctypes.c_int64
        lib.oracle_box_fgt_boxes.argtypes = [ctypes.c_int, ctypes.c_int64, i32p, i32p,
                                             ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_double, f64p, ctypes.c_int64, i32p, i32p,
                                             f64p, ctypes.c_int]
        lib.oracle_point_fgt.restype = ctypes.c_int64
        lib.oracle_point_fgt.argtypes = [ctypes.c_int, ctypes.c_int64, f64p, f64p, ctypes.c_int64,
                                         f64p, ctypes.c_double, ctypes.c_double, f64p, ctypes.c_int]
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


def oracle_u_boxes(levels, coords, p: int, delta: float, sigma, blevels, bcoords,
                   periodic: bool = False, rcut: float = 0.0, nthreads: int = 0):
    """u at the nodes of the boxes (blevels, bcoords), ``[nbox, p**d]``; the
    sources are the leaves (levels, coords) with samples sigma."""
    lib = _load()
    levels = np.ascontiguousarray(levels, dtype=np.int32)
    coords = np.ascontiguousarray(coords, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    blevels = np.ascontiguousarray(blevels, dtype=np.int32)
    bcoords = np.ascontiguousarray(bcoords, dtype=np.int32)
    n, d = coords.shape
    if sigma.shape != (n, p ** d) or bcoords.shape != (len(blevels), d):
        raise ValueError("shape mismatch")
    u = np.zeros((len(blevels), p ** d), dtype=np.float64)
    r = lib.oracle_box_fgt_boxes(d, n, _ptr(levels, ctypes.c_int32), _ptr(coords, ctypes.c_int32),
                                 p, float(delta), int(bool(periodic)), float(rcut),
                                 _ptr(sigma, ctypes.c_double), len(blevels),
                                 _ptr(blevels, ctypes.c_int32), _ptr(bcoords, ctypes.c_int32),
                                 _ptr(u, ctypes.c_double), int(nthreads))
    if r < 0:
        raise RuntimeError(f"oracle_box_fgt_boxes failed ({r})")
    return u


def oracle_interp(levels, coords, p: int, values, x, chunk: int = 65536):
    """The piecewise polynomial given by ``values[nleaves, p**d]`` at the
    tensor Gauss-Legendre nodes of each leaf (degree p-1 per axis, Eq.
    (papprox)), evaluated at the points ``x[npts, d]`` of [-1/2, 1/2]^d.

    Each point is located in the leaf that contains it (a point on a shared
    face goes to the leaf on its upper side, the top face of the unit box to
    the last leaf); the leaf's Legendre coefficients come from a Vandermonde
    solve on the nodes, and the polynomial is summed at the point's local
    coordinates."""
    from numpy.polynomial import legendre as npleg
    levels = np.asarray(levels, dtype=np.int64)
    coords = np.asarray(coords, dtype=np.int64)
    values = np.asarray(values, dtype=np.float64)
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, d = coords.shape
    eta = gauss_legendre(p)[0]
    Vinv = np.linalg.inv(npleg.legvander(eta, p - 1))
    # locate: for every level present, the cell of each point and a lookup of
    # (cell) among the leaves of that level
    leaf = np.full(len(x), -1, dtype=np.int64)
    for l in np.unique(levels):
        sel = np.where(levels == l)[0]
        nb = 1 << int(l)
        cell = np.clip(np.floor((x + 0.5) * nb).astype(np.int64), 0, nb - 1)
        key = np.zeros(len(x), dtype=np.int64)
        lkey = np.zeros(len(sel), dtype=np.int64)
        for a in range(d):
            key = key * nb + cell[:, a]
            lkey = lkey * nb + coords[sel, a]
        order = np.argsort(lkey)
        pos = np.clip(np.searchsorted(lkey[order], key), 0, len(sel) - 1)
        hit = lkey[order][pos] == key
        leaf[hit] = sel[order][pos[hit]]
    if np.any(leaf < 0):
        raise ValueError("a point lies outside the leaves")
    out = np.empty(len(x))
    for s in range(0, len(x), chunk):
        xs, ls = x[s:s + chunk], leaf[s:s + chunk]
        L = 2.0 ** -levels[ls]
        lo = -0.5 + coords[ls] * L[:, None]
        t = 2.0 * (xs - lo) / L[:, None] - 1.0
        c = values[ls].reshape((len(ls),) + (p,) * d)        # [m, i_d, ..., i_1]
        for ax in range(1, d + 1):
            c = np.moveaxis(np.tensordot(Vinv, c, axes=([1], [ax])), 0, ax)
        # contract axis d first (array axis 1), then d-1, ..., 1
        for a in range(d - 1, -1, -1):
            P = npleg.legvander(t[:, a], p - 1)              # [m, p]
            c = np.einsum("mn,mn...->m...", P, c)
        out[s:s + chunk] = c
    return out


def oracle_point(sources, charges, targets, delta: float, cut: float | None = None,
                 nthreads: int = 0, return_pairs: bool = False):
    """The discrete Gauss transform (Eq. (pgt)) summed directly:
    u_i = sum_j exp(-|x_i - y_j|^2/delta) q_j for sources ``[n, d]`` and
    targets ``[m, d]`` in [-1/2, 1/2]^d.  cut: sources farther than it along
    some axis are skipped (each skipped term is below exp(-cut^2/delta)|q_j|);
    default sqrt(delta ln 1e18); 0 sums every pair."""
    lib = _load()
    y = np.ascontiguousarray(sources, dtype=np.float64)
    q = np.ascontiguousarray(charges, dtype=np.float64).reshape(-1)
    x = np.ascontiguousarray(targets, dtype=np.float64)
    if y.ndim != 2 or x.ndim != 2 or y.shape[1] != x.shape[1] or len(q) != len(y):
        raise ValueError("sources [n, d], charges [n], targets [m, d]")
    if cut is None:
        cut = math.sqrt(delta * math.log(1e18))
    u = np.zeros(len(x))
    n = lib.oracle_point_fgt(y.shape[1], len(y), _ptr(y, ctypes.c_double), _ptr(q, ctypes.c_double),
                             len(x), _ptr(x, ctypes.c_double), float(delta), float(cut),
                             _ptr(u, ctypes.c_double), int(nthreads))
    if n < 0:
        raise RuntimeError(f"oracle_point_fgt failed ({n})")
    return (u, int(n)) if return_pairs else u


def threads_used() -> int:
    return int(_load().oracle_threads())


def gauss_legendre(n: int):
    lib = _load()
    x = np.zeros(n)
    w = np.zeros(n)
    lib.oracle_gauss_legendre(n, _ptr(x, ctypes.c_double), _ptr(w, ctypes.c_double))
    return x, w
