"""Seeded synthetic inputs for the continuous (box) Gauss transform.

This module builds inputs only.  It holds none of the transform's arithmetic:
no plane waves, no Gaussian integrals, no tables.  It

* builds a level-restricted adaptive tree that resolves a density
  (the refinement test of Algorithm 3 of the paper, Eq. (funerr)), followed by
  2:1 balancing with corner adjacency (Definition treedefs: leaves that share a
  boundary point differ by at most one level);
* samples densities at the tensor-product Gauss-Legendre nodes of every leaf,
  with the node multi-index (i_1..i_d) stored at i_1 + p*i_2 + p^2*i_3;
* draws the random parameters of the synthetic workloads from a seeded numpy
  PCG64 generator.

Gauss-Legendre nodes come from numpy's own rule, so neither the oracle nor the
GPU path shares code with this module: both receive its arrays as inputs.

A tree is a pair of integer arrays: ``levels[nleaves]`` and
``coords[nleaves, d]``; leaf ``i`` is the box of side ``2**-levels[i]`` whose
lower corner is ``-1/2 + coords[i] * 2**-levels[i]`` on every axis.
"""

from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np
from numpy.polynomial import legendre as npleg

# ----------------------------------------------------------------------------
# geometry of leaves and nodes


def gl_nodes(p: int) -> np.ndarray:
    """Ascending Gauss-Legendre nodes on [-1, 1] (numpy's rule)."""
    return npleg.leggauss(p)[0]


def leaf_centers(levels: np.ndarray, coords: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Centers ``[n, d]`` and side lengths ``[n]`` of the leaves."""
    L = np.ldexp(1.0, -np.asarray(levels, dtype=np.int64).astype(np.int32))
    c = -0.5 + (np.asarray(coords, dtype=np.float64) + 0.5) * L[:, None]
    return c, L


def node_offsets(p: int, d: int) -> np.ndarray:
    """Reference-box node coordinates ``[p**d, d]`` in [-1,1]^d, axis 1 fastest."""
    eta = gl_nodes(p)
    f = np.arange(p ** d)
    return np.stack([eta[(f // p ** a) % p] for a in range(d)], axis=-1)


def leaf_points(levels, coords, p: int) -> np.ndarray:
    """Physical node coordinates of every leaf, ``[n, p**d, d]``."""
    c, L = leaf_centers(levels, coords)
    off = node_offsets(p, c.shape[1])
    return c[:, None, :] + 0.5 * L[:, None, None] * off[None, :, :]


def sample(levels, coords, p: int, func, chunk: int = 4096) -> np.ndarray:
    """Density values at the nodes of every leaf, ``[n, p**d]`` float64."""
    n = len(levels)
    d = np.asarray(coords).shape[1]
    out = np.empty((n, p ** d), dtype=np.float64)
    for s in range(0, n, chunk):
        pts = leaf_points(levels[s:s + chunk], coords[s:s + chunk], p)
        out[s:s + chunk] = func(pts)
    return out


# ----------------------------------------------------------------------------
# densities


@dataclasses.dataclass
class GaussianSum:
    """sigma(x) = sum_i a_i exp(-|x - c_i|^2 / w_i^2)  (w is a length)."""

    centers: np.ndarray  # [n, d]
    widths: np.ndarray   # [n]
    amps: np.ndarray     # [n]
    periodic: bool = False  # if True, the blobs are periodized over Z^d

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        d = x.shape[-1]
        out = np.zeros(x.shape[:-1])
        shifts = [np.zeros(d)]
        if self.periodic:
            shifts = [np.array(s, dtype=np.float64)
                      for s in itertools.product((-1, 0, 1), repeat=d)]
        for c, w, a in zip(self.centers, self.widths, self.amps):
            for sh in shifts:
                r2 = np.sum((x - (c + sh)) ** 2, axis=-1)
                out += a * np.exp(-r2 / (w * w))
        return out

    def l2norm(self) -> float:
        """(integral over R^d of sigma^2)^(1/2); the blobs sit well inside B."""
        d = self.centers.shape[1]
        s = 0.0
        for i in range(len(self.amps)):
            for j in range(len(self.amps)):
                wi2, wj2 = self.widths[i] ** 2, self.widths[j] ** 2
                r2 = float(np.sum((self.centers[i] - self.centers[j]) ** 2))
                s += (self.amps[i] * self.amps[j]
                      * (math.pi * wi2 * wj2 / (wi2 + wj2)) ** (d / 2)
                      * math.exp(-r2 / (wi2 + wj2)))
        return math.sqrt(max(s, 1e-300))


@dataclasses.dataclass
class SinCosProduct:
    """The periodic density of Eq. (sigmap): sin on odd axes, cos on even
    axes, all at frequency nu (the paper's n_p in that equation)."""

    nu: int
    d: int

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        out = np.ones(x.shape[:-1])
        for a in range(self.d):
            f = np.sin if a % 2 == 0 else np.cos
            out = out * f(2.0 * math.pi * self.nu * x[..., a])
        return out

    def l2norm(self) -> float:
        return 0.5 ** (self.d / 2)


class Constant:
    def __init__(self, value: float = 1.0):
        self.value = value

    def __call__(self, x):
        return np.full(np.asarray(x).shape[:-1], self.value)

    def l2norm(self) -> float:
        return abs(self.value)


# ----------------------------------------------------------------------------
# trees


def uniform_tree(d: int, level: int) -> tuple[np.ndarray, np.ndarray]:
    n = 2 ** level
    grid = np.stack(np.meshgrid(*([np.arange(n)] * d), indexing="ij"), -1)
    coords = grid.reshape(-1, d)[:, ::-1].copy()  # axis 1 fastest in leaf order
    levels = np.full(len(coords), level, dtype=np.int32)
    return levels, coords.astype(np.int32)


def _tail_mask(p: int, d: int) -> np.ndarray:
    """Multi-indices alpha (reference order [a_d,...,a_1]) of the l2 tail
    ||alpha||_2 >= p used by Eq. (funerr); the last shell when d == 1."""
    idx = np.stack(np.meshgrid(*([np.arange(p)] * d), indexing="ij"), -1)
    n2 = np.sqrt(np.sum(idx.astype(np.float64) ** 2, axis=-1))
    if d == 1:
        return idx[..., 0] >= p - 2
    return n2 >= p


def _coefficients(vals: np.ndarray, p: int, d: int) -> np.ndarray:
    """Legendre coefficients of the interpolant on each box: ``vals[nb, p**d]``
    -> ``[nb, p, ..., p]`` (numpy's Vandermonde solve, axis by axis)."""
    eta = gl_nodes(p)
    Vinv = np.linalg.inv(npleg.legvander(eta, p - 1))  # coef = Vinv @ values
    t = vals.reshape((vals.shape[0],) + (p,) * d)      # [nb, i_d, ..., i_1]
    for ax in range(1, d + 1):
        t = np.moveaxis(np.tensordot(Vinv, t, axes=([1], [ax])), 0, ax)
    return t


def resolve_tree(func, d: int, p: int, eps: float, norm: float | None = None,
                 max_level: int = 12, min_level: int = 0,
                 periodic: bool = False, chunk: int = 2048, max_leaves: int | None = None):
    """Adaptive tree that resolves ``func`` (Algorithm 3): a box is split when
    the RMS of its Legendre tail exceeds eps*||sigma||_2, then the tree is
    2:1 balanced.  Returns (levels, coords), or None if the tree before
    balancing would exceed ``max_leaves``."""
    sampler = sample
    if isinstance(func, GaussianSum) and not func.periodic:
        sampler = sample_separable
    if norm is None:
        norm = func.l2norm()
    thr = eps * norm
    mask = _tail_mask(p, d)
    leaves_l, leaves_c = [], []
    boxes = uniform_tree(d, min_level)[1]
    level = min_level
    while len(boxes):
        split = np.zeros(len(boxes), dtype=bool)
        if level < max_level:
            for s in range(0, len(boxes), chunk):
                b = boxes[s:s + chunk]
                vals = sampler(np.full(len(b), level), b, p, func)
                coef = _coefficients(vals, p, d)
                e = np.sqrt(np.mean(coef[:, mask] ** 2, axis=1))
                split[s:s + chunk] = e > thr
        keep = boxes[~split]
        leaves_l.append(np.full(len(keep), level, dtype=np.int32))
        leaves_c.append(keep)
        parents = boxes[split]
        kids = [2 * parents + np.array(o, dtype=np.int32)
                for o in itertools.product((0, 1), repeat=d)]
        boxes = np.concatenate(kids, 0) if len(parents) else np.zeros((0, d), np.int32)
        level += 1
        if max_leaves is not None and sum(len(c) for c in leaves_c) + len(boxes) > max_leaves:
            return None
    levels = np.concatenate(leaves_l)
    coords = np.concatenate(leaves_c, 0).astype(np.int32)
    return balance_fast(levels, coords, periodic=periodic)


def balance(levels, coords, periodic: bool = False):
    """2:1 balance with corner adjacency: split coarse leaves until every pair
    of leaves that share a boundary point differs by at most one level."""
    d = np.asarray(coords).shape[1]
    leaf = {(int(l), tuple(int(v) for v in c)) for l, c in zip(levels, coords)}
    dirs = [np.array(o) for o in itertools.product((-1, 0, 1), repeat=d) if any(o)]
    maxl = max(l for l, _ in leaf)

    def covering(l, q):
        for ll in range(l, -1, -1):
            key = (ll, tuple(v >> (l - ll) for v in q))
            if key in leaf:
                return key
        return None

    for l in range(maxl, 1, -1):
        work = [c for (ll, c) in leaf if ll == l]
        for c in work:
            n = 1 << l
            for o in dirs:
                q = np.array(c) + o
                if periodic:
                    q %= n
                elif np.any(q < 0) or np.any(q >= n):
                    continue
                q = tuple(int(v) for v in q)
                while True:
                    key = covering(l, q)
                    if key is None or key[0] >= l - 1:
                        break
                    kl, kc = key
                    leaf.discard(key)
                    for b in itertools.product((0, 1), repeat=d):
                        leaf.add((kl + 1, tuple(2 * kc[a] + b[a] for a in range(d))))
    items = sorted(leaf)
    lv = np.array([l for l, _ in items], dtype=np.int32)
    cs = np.array([c for _, c in items], dtype=np.int32).reshape(-1, d)
    return lv, cs


def is_balanced(levels, coords, periodic: bool = False) -> bool:
    lv2, _ = balance(levels, coords, periodic)
    return len(lv2) == len(levels)


# ----------------------------------------------------------------------------
# workloads


@dataclasses.dataclass
class Problem:
    name: str
    d: int
    p: int
    delta: float
    tol: float
    periodic: bool
    levels: np.ndarray
    coords: np.ndarray
    sigma: np.ndarray
    density: object

    @property
    def npoints(self) -> int:
        return int(self.sigma.size)


def _blobs(rng, n, d, lo, hi, wlo, whi, log_widths):
    centers = rng.uniform(lo, hi, size=(n, d))
    if log_widths:
        widths = 10.0 ** rng.uniform(math.log10(wlo), math.log10(whi), size=n)
    else:
        widths = rng.uniform(wlo, whi, size=n)
    amps = rng.uniform(-1.0, 1.0, size=n)
    return centers, widths, amps


def point_sphere(seed: int = 0, n: int = 3_400_000, radius: float = 0.35):
    """Point workload after the paper's 3D point-transform experiment (points
    on a surface, so that the tree must refine): n points uniform on the
    sphere of the given radius about the box center, charges U(-1,1); the
    points are both the sources and the targets.  Returns (points, charges)."""
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, 1.0, (n, 3))
    x = radius * x / np.linalg.norm(x, axis=1)[:, None]
    return x, rng.uniform(-1.0, 1.0, n)


def small_2d(seed: int = 0) -> Problem:
    """2D free space, uniform level-3 tree (64 leaves) on [-1/2,1/2]^2, p=8
    (4096 points), delta=1e-3, four Gaussians with centers U[-0.3,0.3]^2,
    widths U[0.01,0.05], amplitudes U(-1,1); tol 1e-6."""
    rng = np.random.default_rng(seed)
    dens = GaussianSum(*_blobs(rng, 4, 2, -0.3, 0.3, 1e-2, 5e-2, False))
    lv, cs = uniform_tree(2, 3)
    return Problem("2d-uniform-l3-p8", 2, 8, 1e-3, 1e-6, False, lv, cs,
                   sample(lv, cs, 8, dens), dens)


def adaptive_3d_density(seed: int = 0, nblobs: int = 8, wrap_blobs: bool = False) -> GaussianSum:
    """The density of the 3D workload: 8 Gaussians with widths log-uniform in
    [1e-3,1e-2], amplitudes U(-1,1) and centers U[-0.4,0.4]^3, or U[-0.5,0.5]^3
    periodized over Z^3 when wrap_blobs."""
    rng = np.random.default_rng(seed)
    lo, hi = (-0.5, 0.5) if wrap_blobs else (-0.4, 0.4)
    return GaussianSum(*_blobs(rng, nblobs, 3, lo, hi, 1e-3, 1e-2, True), periodic=wrap_blobs)


def adaptive_3d(seed: int = 0, periodic: bool = False, eps: float = 1e-9,
                max_level: int = 7, delta: float = 1e-4, tol: float = 1e-10,
                nblobs: int = 8, wrap_blobs: bool = False) -> Problem:
    """3D adaptive tree, p=16, resolving sigma = sum of 8 Gaussians (widths
    log-uniform in [1e-3,1e-2], centers U[-0.4,0.4]^3, amplitudes U(-1,1)) to
    a Legendre-tail RMS of eps*||sigma||_2, levels capped at max_level."""
    dens = adaptive_3d_density(seed, nblobs, wrap_blobs)
    lv, cs = resolve_tree(dens, 3, 16, eps, max_level=max_level, periodic=periodic)
    name = f"3d-adaptive-p16-{'periodic' if periodic else 'free'}"
    return Problem(name, 3, 16, delta, tol, periodic, lv, cs,
                   sample(lv, cs, 16, dens), dens)


def random_problem(rng, d: int, p: int, delta: float, tol: float, max_level: int,
                   nblobs: int, periodic: bool = False, eps: float = 1e-9,
                   min_level: int = 0) -> Problem:
    """A Gaussian-sum density as in the small 2D workload (centers
    U[-0.3,0.3]^d, widths U[0.01,0.05], amplitudes U(-1,1)) resolved on an
    adaptive tree capped at max_level."""
    dens = GaussianSum(*_blobs(rng, nblobs, d, -0.3, 0.3, 1e-2, 5e-2, False))
    lv, cs = resolve_tree(dens, d, p, eps, max_level=max_level,
                          min_level=min_level, periodic=periodic)
    return Problem(f"{d}d-adaptive-p{p}", d, p, delta, tol, periodic, lv, cs,
                   sample(lv, cs, p, dens), dens)


def point_refined_tree(d: int, point, max_level: int, periodic: bool = False):
    """Tree refined around one point down to max_level, then 2:1 balanced:
    a small mixed-level tree for tests."""
    point = np.asarray(point, dtype=np.float64)
    leaves = []
    boxes = [(0, (0,) * d)]
    while boxes:
        l, c = boxes.pop()
        L = 2.0 ** -l
        lo = -0.5 + np.array(c) * L
        inside = np.all(point >= lo) and np.all(point < lo + L)
        if inside and l < max_level:
            for o in itertools.product((0, 1), repeat=d):
                boxes.append((l + 1, tuple(2 * c[a] + o[a] for a in range(d))))
        else:
            leaves.append((l, c))
    lv = np.array([l for l, _ in leaves], dtype=np.int32)
    cs = np.array([c for _, c in leaves], dtype=np.int32).reshape(-1, d)
    return balance(lv, cs, periodic=periodic)


# ----------------------------------------------------------------------------
# trees of a requested size (serving workload)


def _box_center_distance(levels_l: int, coords: np.ndarray, centers: np.ndarray,
                         periodic: bool) -> np.ndarray:
    """Euclidean distance from each box (all at one level) to its nearest
    center; 0 for boxes that contain a center."""
    L = 2.0 ** -levels_l
    mid = -0.5 + (coords + 0.5) * L
    diff = np.abs(mid[:, None, :] - centers[None, :, :])
    if periodic:
        diff = np.minimum(diff, 1.0 - diff)
    gap = np.maximum(diff - 0.5 * L, 0.0)
    return np.sqrt(np.sum(gap * gap, axis=-1)).min(axis=1)


def graded_tree(d: int, centers, lmax: int, r0: float, periodic: bool = False):
    """Tree graded around `centers`: a box at level l < lmax is split while
    its distance to the nearest center is below r0 (2^(lmax-l) - 1), so the
    leaf side grows about linearly with the distance.  With
    r0 >= 2 sqrt(d) 2^-lmax neighboring leaves differ by at most one level;
    the result is passed through `balance` only if it is not."""
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, d)
    boxes = np.zeros((1, d), dtype=np.int64)
    lv, cs = [], []
    for l in range(lmax + 1):
        if l == lmax:
            split = np.zeros(len(boxes), dtype=bool)
        else:
            split = _box_center_distance(l, boxes, centers, periodic) < r0 * (2.0 ** (lmax - l) - 1.0)
        keep = boxes[~split]
        lv.append(np.full(len(keep), l, dtype=np.int32))
        cs.append(keep)
        par = boxes[split]
        if len(par) == 0:
            break
        boxes = np.concatenate([2 * par + np.array(o, dtype=np.int64)
                                for o in itertools.product((0, 1), repeat=d)], 0)
    return np.concatenate(lv), np.concatenate(cs, 0).astype(np.int32)


def sized_tree(d: int, centers, nleaves: int, periodic: bool = False):
    """A 2:1-balanced graded tree (`graded_tree`, then `balance_fast`) with
    about `nleaves` leaves: for finest levels around the smallest whose
    uniform tree has enough leaves, r0 is found by bisection (the leaf count
    grows with r0); the closest wins."""
    nleaves = max(1, int(nleaves))
    l0 = 0
    while 2 ** (d * l0) < nleaves:
        l0 += 1
    if l0 == 0:
        return uniform_tree(d, 0)
    best = None
    for lmax in (l0 - 1, l0, l0 + 1):
        if lmax < 1:
            continue
        lo, hi = math.log(0.25 * 2.0 ** -lmax), math.log(4.0)
        for _ in range(30):
            mid = 0.5 * (lo + hi)
            lv, cs = graded_tree(d, centers, lmax, math.exp(mid), periodic)
            if best is None or abs(len(lv) - nleaves) < abs(len(best[0]) - nleaves):
                best = (lv, cs)
            if len(lv) < nleaves:
                lo = mid
            else:
                hi = mid
            if abs(len(lv) - nleaves) <= 0.02 * nleaves:
                break
        if abs(len(best[0]) - nleaves) <= 0.02 * nleaves:
            break
    return balance_fast(*best, periodic)


def sample_separable(levels, coords, p: int, dens: GaussianSum, chunk: int = 8192) -> np.ndarray:
    """`sample` for a free-space Gaussian sum, built from per-axis factors
    (each blob is a product of 1D Gaussians): the same values up to rounding,
    much faster for large trees."""
    levels = np.asarray(levels)
    coords = np.asarray(coords)
    n, d = coords.shape
    eta = gl_nodes(p)
    out = np.empty((n, p ** d), dtype=np.float64)
    for s in range(0, n, chunk):
        c, L = leaf_centers(levels[s:s + chunk], coords[s:s + chunk])
        x = c[:, :, None] + 0.5 * L[:, None, None] * eta[None, None, :]  # [m, d, p]
        # per-axis factors f[m, axis, i, b] of every blob b
        f = np.exp(-((x[:, :, :, None] - dens.centers.T[None, :, None, :]) ** 2)
                   / (dens.widths[None, None, None, :] ** 2))
        a = np.asarray(dens.amps, dtype=np.float64)
        if d == 1:
            acc = f[:, 0] @ a
        elif d == 2:
            acc = np.einsum("mib,mjb->mij", f[:, 1] * a, f[:, 0])
        else:
            g = (f[:, 2, :, None, :] * f[:, 1, None, :, :] * a).reshape(len(c), p * p, -1)
            acc = np.einsum("mib,mjb->mij", g, f[:, 0])
        out[s:s + chunk] = acc.reshape(len(c), -1)
    return out


@dataclasses.dataclass
class RequestType:
    key: int
    d: int
    p: int
    delta: float
    tol: float
    precision: str
    levels: np.ndarray
    coords: np.ndarray
    sigma: np.ndarray

    @property
    def npoints(self) -> int:
        return int(self.sigma.size)


def serve_request_types(seed: int, ntypes: int, log10_n=(4.0, 8.0), log10_delta=(-6.0, -2.0),
                        tols=(1e-3, 1e-6, 1e-10), ps=(8, 16), fp32_min_tol: float = 1e-3):
    """Request types of the serving workload: d ~ U{2,3}, grid points N with
    log10 N ~ U[log10_n], log10 delta ~ U[log10_delta], tol ~ U{tols},
    p ~ U{ps}; a graded tree with about N / p^d leaves around 2-16 Gaussian
    blobs drawn as in the small 2D workload (centers U[-0.3,0.3]^d, widths
    U[0.01,0.05], amplitudes U(-1,1)), which also give sigma.  Precision is
    FP32 for tol >= fp32_min_tol, else FP64."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(ntypes):
        d = int(rng.integers(2, 4))
        n = 10.0 ** rng.uniform(*log10_n)
        delta = float(10.0 ** rng.uniform(*log10_delta))
        tol = float(tols[int(rng.integers(0, len(tols)))])
        p = int(ps[int(rng.integers(0, len(ps)))])
        nb = int(rng.integers(2, 17))
        dens = GaussianSum(*_blobs(rng, nb, d, -0.3, 0.3, 1e-2, 5e-2, False))
        lv, cs = sized_tree(d, dens.centers, round(n / p ** d))
        lv, cs = balance_fast(lv, cs)
        out.append(RequestType(k, d, p, delta, tol, "fp32" if tol >= fp32_min_tol else "fp64",
                               lv, cs, sample_separable(lv, cs, p, dens)))
    return out


def _coarse_neighbors(levels, coords, periodic: bool = False) -> np.ndarray:
    """Indices of leaves that violate 2:1 balance (corner adjacency) by being
    at least two levels coarser than a leaf they touch; vectorized, for trees
    that tile the box.  If leaves A (coarser) and B touch, B's whole face,
    edge or corner on that contact lies in A's boundary, so the finest-grid
    cell just outside B in that direction (at B's lower corner along the other
    axes) lies in A: for every leaf and each of the 3^d - 1 directions, the
    leaf covering that cell is found and reported if it is too coarse."""
    levels = np.asarray(levels, dtype=np.int64)
    coords = np.asarray(coords, dtype=np.int64)
    n, d = coords.shape
    lmax = int(levels.max())
    side = 1 << lmax

    def keys(lv, cs):
        k = lv.copy()
        for ax in range(d):
            k = k * side + cs[:, ax]
        return k

    key = keys(levels, coords)
    order = np.argsort(key)
    table = key[order]

    def lookup(lv, cs):
        k = keys(lv, cs)
        i = np.minimum(np.searchsorted(table, k), n - 1)
        return np.where(table[i] == k, order[i], -1)

    sh = lmax - levels
    base = coords << sh[:, None]
    step = (np.int64(1) << sh)[:, None]
    bad = []
    for o in itertools.product((-1, 0, 1), repeat=d):
        if not any(o):
            continue
        o = np.array(o, dtype=np.int64)
        q = base + np.where(o > 0, step, np.where(o < 0, -1, 0))
        if periodic:
            q %= side
            sel = np.arange(n)
        else:
            sel = np.nonzero(np.all((q >= 0) & (q < side), axis=1))[0]
        found = np.zeros(len(sel), dtype=bool)
        for dl in (-1, 0, 1):
            ll = levels[sel] + dl
            okl = (ll >= 0) & (ll <= lmax)
            llc = np.clip(ll, 0, lmax)
            found |= okl & (lookup(llc, q[sel] >> (lmax - llc)[:, None]) >= 0)
        miss = sel[~found]
        qm = q[miss]
        for ll in range(lmax - 2, -1, -1):  # the covering leaf is coarser still
            lv = np.full(len(miss), ll, dtype=np.int64)
            hit = lookup(lv, qm >> (lmax - ll))
            ok = (hit >= 0) & (ll <= levels[miss] - 2)
            bad.append(hit[ok])
    return np.unique(np.concatenate(bad)) if bad else np.zeros(0, dtype=np.int64)


def is_balanced_fast(levels, coords, periodic: bool = False) -> bool:
    """Vectorized equivalent of `is_balanced` for trees that tile the box."""
    return len(_coarse_neighbors(levels, coords, periodic)) == 0


def balance_fast(levels, coords, periodic: bool = False):
    """Vectorized equivalent of `balance`: split every leaf that is two or
    more levels coarser than a leaf it touches, until none is."""
    levels = np.asarray(levels, dtype=np.int32)
    coords = np.asarray(coords, dtype=np.int32)
    d = coords.shape[1]
    kids_off = np.array(list(itertools.product((0, 1), repeat=d)), dtype=np.int32)
    while True:
        bad = _coarse_neighbors(levels, coords, periodic)
        if len(bad) == 0:
            break
        keep = np.ones(len(levels), dtype=bool)
        keep[bad] = False
        kl = np.repeat(levels[bad] + 1, len(kids_off))
        kc = (2 * coords[bad][:, None, :] + kids_off[None, :, :]).reshape(-1, d)
        levels = np.concatenate([levels[keep], kl]).astype(np.int32)
        coords = np.concatenate([coords[keep], kc], 0).astype(np.int32)
    idx = np.lexsort(tuple(coords[:, a] for a in range(d - 1, -1, -1)) + (levels,))
    return levels[idx], coords[idx]

def _batch_tree(args):
    """Parameters and tree of transform k of the batched workload."""
    seed, k, max_points, eps, tols, fp32_min_tol, one_thread = args
    if one_thread:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            return _batch_tree((seed, k, max_points, eps, tols, fp32_min_tol, False))
    rng = np.random.default_rng((seed, k))
    d = int(rng.integers(2, 4))
    delta = float(10.0 ** rng.uniform(-6.0, -2.0))
    depth = int(rng.integers(3, 10))
    p = int((8, 16)[int(rng.integers(0, 2))])
    nb = int(rng.integers(2, 17))
    tol = float(tols[int(rng.integers(0, len(tols)))])
    dens = GaussianSum(*_blobs(rng, nb, d, -0.3, 0.3, 1e-2, 5e-2, False))
    cap = max(1, max_points // p ** d)
    while True:
        t = resolve_tree(dens, d, p, eps, max_level=depth, max_leaves=cap)
        if t is not None and len(t[0]) <= cap:
            break
        depth -= 1
    return k, d, p, delta, tol, "fp32" if tol >= fp32_min_tol else "fp64", t[0], t[1], dens


def batch_problems(seed: int, n: int = 512, max_points: int = 1 << 21, eps: float = 1e-9,
                   tols=(1e-3, 1e-6, 1e-10), fp32_min_tol: float = 1e-6, workers: int = 1):
    """The batched workload: n independent transforms, each with d ~ U{2,3},
    log10 delta ~ U[-6,-2], a depth cap ~ U{3..9} on the Algorithm 3 tree that
    resolves sigma to eps*||sigma||_2, p ~ U{8,16}, sigma a sum of 2-16
    Gaussians as in the small 2D workload (centers U[-0.3,0.3]^d, widths
    U[0.01,0.05], amplitudes U(-1,1)), tol ~ U{tols}; FP32 when
    tol >= fp32_min_tol, else FP64.  A transform over max_points grid points
    has its depth cap lowered until it fits.  Transform k draws from its own
    generator (seed, k), so the result does not depend on `workers`: processes
    forked to build the trees (fork them before the process uses a GPU)."""
    jobs = [(seed, k, max_points, eps, tuple(tols), fp32_min_tol, True) for k in range(n)]
    if workers <= 1:
        trees = [_batch_tree(j) for j in jobs]
    else:
        import multiprocessing
        with multiprocessing.get_context("fork").Pool(workers) as pool:
            trees = pool.map(_batch_tree, jobs, chunksize=2)
    return [RequestType(k, d, p, delta, tol, prec, lv, cs, sample_separable(lv, cs, p, dens))
            for k, d, p, delta, tol, prec, lv, cs, dens in trees]
