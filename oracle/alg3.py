"""Algorithm 3 (resolving a density on a level-restricted adaptive tree), plain
numpy, box by box.

TEST INFRASTRUCTURE.  Only ``tests/`` may use this module.  It shares no code
with the GPU path or with the input generator and imports neither.

Steps, in the paper's order (Section 4, Algorithm 3):

1. Level by level from the starting level, every box B_i of the level is
   sampled at its k^d tensor Gauss-Legendre nodes.
2. The Legendre coefficients c_alpha of the interpolant are computed by the
   quadrature formula of Eq. (val2poleq), one axis at a time:
   c_n = (2n + 1)/2 * sum_j w_j P_n(eta_j) f_j.
3. The error e(B_i) of Eq. (funerr) is the root mean square of the c_alpha in
   the tail ||alpha||_2 >= k.  For d = 1 that set is empty; the reading taken
   for d = 1 is the last two coefficients, alpha >= k - 2.
4. B_i is split into its 2^d children when e(B_i) > eps * ||sigma||_2
   (boxes at the deepest allowed level are kept as leaves).
5. The leaves are then refined until the tree is level-restricted: two leaves
   that share a boundary point (corner adjacency; across the periodic wrap if
   asked) differ by at most one level.  A leaf that is two or more levels
   coarser than a leaf it touches is split, until none is.

The norm ||sigma||_2 is an input: ``gaussian_sum_norm`` gives the reading
used for sums of Gaussians, (integral over R^d of sigma^2)^(1/2) in closed
form.
"""

from __future__ import annotations

import itertools
import math

import numpy as np
from numpy.polynomial import legendre as npleg


# ---------------------------------------------------------------------------
# densities


def gaussian_sum(centers, widths, amps, periodic: bool = False):
    """sigma(x) = sum_i a_i exp(-|x - c_i|^2 / w_i^2), the blobs repeated over
    the 3^d nearest unit shifts when periodic.  Returns a callable on [..., d]."""
    centers = np.asarray(centers, dtype=np.float64)
    widths = np.asarray(widths, dtype=np.float64)
    amps = np.asarray(amps, dtype=np.float64)
    d = centers.shape[1]
    shifts = list(itertools.product((-1, 0, 1), repeat=d)) if periodic else [(0,) * d]

    def f(x):
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[:-1])
        for c, w, a in zip(centers, widths, amps):
            for s in shifts:
                diff = x - (c + np.asarray(s, dtype=np.float64))
                out += a * np.exp(-np.sum(diff * diff, axis=-1) / (w * w))
        return out

    return f


def gaussian_sum_norm(centers, widths, amps) -> float:
    """(integral over R^d of sigma^2)^(1/2) for sigma = sum_i a_i g_i: the
    integral of g_i g_j factorizes per axis into a Gaussian integral,
    int exp(-(x-a)^2/p - (x-b)^2/q) dx = sqrt(pi p q/(p+q)) exp(-(a-b)^2/(p+q))."""
    centers = np.asarray(centers, dtype=np.float64)
    d = centers.shape[1]
    total = 0.0
    for i in range(len(amps)):
        for j in range(len(amps)):
            pi_, qj = widths[i] ** 2, widths[j] ** 2
            term = amps[i] * amps[j]
            for a in range(d):
                term *= math.sqrt(math.pi * pi_ * qj / (pi_ + qj)) * \
                    math.exp(-(centers[i][a] - centers[j][a]) ** 2 / (pi_ + qj))
            total += term
    return math.sqrt(total)


# ---------------------------------------------------------------------------
# one box


def box_nodes(level: int, coord, k: int) -> np.ndarray:
    """The k^d Gauss-Legendre nodes of the box (level, coord) of [-1/2, 1/2]^d,
    node (i_1, ..., i_d) at row i_1 + k i_2 + k^2 i_3 (axis 1 fastest)."""
    eta, _ = npleg.leggauss(k)
    side = 0.5 ** level
    d = len(coord)
    axes = [-0.5 + (coord[a] + 0.5) * side + 0.5 * side * eta for a in range(d)]
    # grids indexed [i_d, ..., i_1]; flattening in C order puts i_1 fastest
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    return np.stack([g.reshape(-1) for g in grids[::-1]], axis=-1)


def coefficients(values: np.ndarray, k: int, d: int) -> np.ndarray:
    """c[alpha_d, ..., alpha_1] of the tensor Legendre interpolant through the
    node values (Eq. (val2poleq) along each axis)."""
    eta, w = npleg.leggauss(k)
    # Q[n, j] = (2n+1)/2 w_j P_n(eta_j)
    P = npleg.legvander(eta, k - 1).T  # [n, j] = P_n(eta_j)
    Q = (2.0 * np.arange(k) + 1.0)[:, None] / 2.0 * P * w[None, :]
    t = np.asarray(values, dtype=np.float64).reshape((k,) * d)  # [i_d, ..., i_1]
    for ax in range(d):
        t = np.moveaxis(np.tensordot(Q, t, axes=([1], [ax])), 0, ax)
    return t


def tail_indices(k: int, d: int) -> np.ndarray:
    """Boolean mask over [alpha_d, ..., alpha_1] of the tail in Eq. (funerr)."""
    idx = np.indices((k,) * d)
    if d == 1:
        return idx[0] >= k - 2
    return np.sum(idx.astype(np.int64) ** 2, axis=0) >= k * k


def tail_error(values: np.ndarray, k: int, d: int) -> float:
    """e(B) of Eq. (funerr) from the node values of one box."""
    c = coefficients(values, k, d)
    m = tail_indices(k, d)
    return math.sqrt(float(np.mean(c[m] ** 2)))


# ---------------------------------------------------------------------------
# the tree


def _touch_neighbors(level: int, coord, periodic: bool):
    """Boxes of the same level that share a boundary point with (level, coord)."""
    n = 1 << level
    d = len(coord)
    for off in itertools.product((-1, 0, 1), repeat=d):
        if not any(off):
            continue
        q = [coord[a] + off[a] for a in range(d)]
        if periodic:
            q = [v % n for v in q]
        elif any(v < 0 or v >= n for v in q):
            continue
        yield tuple(q)


def _leaf_covering(leaves: set, level: int, coord):
    """The leaf that contains the box (level, coord), or None if the box is
    split further."""
    for l in range(level, -1, -1):
        key = (l, tuple(v >> (level - l) for v in coord))
        if key in leaves:
            return key
    return None


def balance(leaves: set, periodic: bool = False) -> set:
    """Step 5: split every leaf two or more levels coarser than a leaf it
    touches, until none is."""
    leaves = set(leaves)
    changed = True
    while changed:
        changed = False
        for (l, c) in sorted(leaves, key=lambda t: -t[0]):
            if (l, c) not in leaves:
                continue
            for q in _touch_neighbors(l, c, periodic):
                cov = _leaf_covering(leaves, l, q)
                if cov is not None and cov[0] < l - 1:
                    leaves.discard(cov)
                    cl, cc = cov
                    for o in itertools.product((0, 1), repeat=len(cc)):
                        leaves.add((cl + 1, tuple(2 * cc[a] + o[a] for a in range(len(cc)))))
                    changed = True
    return leaves


def resolve(sigma, d: int, k: int, eps: float, norm: float, min_level: int = 0,
            max_level: int = 12, periodic: bool = False):
    """Steps 1-5.  Returns (levels, coords) sorted by (level, coords); and the
    list of (level, coord, e) of every box examined."""
    thr = eps * norm
    boxes = [tuple(c) for c in itertools.product(range(1 << min_level), repeat=d)]
    level = min_level
    leaves = set()
    examined = []
    while boxes:
        nxt = []
        for c in boxes:
            if level >= max_level:
                leaves.add((level, c))
                continue
            e = tail_error(sigma(box_nodes(level, c, k)), k, d)
            examined.append((level, c, e))
            if e > thr:
                for o in itertools.product((0, 1), repeat=d):
                    nxt.append(tuple(2 * c[a] + o[a] for a in range(d)))
            else:
                leaves.add((level, c))
        boxes = nxt
        level += 1
    leaves = sorted(balance(leaves, periodic))
    levels = np.array([l for l, _ in leaves], dtype=np.int32)
    coords = np.array([c for _, c in leaves], dtype=np.int32).reshape(len(leaves), d)
    return levels, coords, examined


def is_balanced(levels, coords, periodic: bool = False) -> bool:
    """Every pair of leaves that share a boundary point differs by at most one
    level (all pairs, from the boxes' extents)."""
    levels = np.asarray(levels, dtype=np.int64)
    coords = np.asarray(coords, dtype=np.int64)
    side = 0.5 ** levels.astype(np.float64)
    lo = -0.5 + coords * side[:, None]
    hi = lo + side[:, None]
    shifts = (-1.0, 0.0, 1.0) if periodic else (0.0,)
    for i in range(len(levels)):
        far = np.abs(levels - levels[i]) > 1
        if not far.any():
            continue
        touch = np.ones(len(levels), dtype=bool)
        for a in range(coords.shape[1]):
            ok = np.zeros(len(levels), dtype=bool)
            for s in shifts:
                ok |= (lo[i, a] <= hi[:, a] + s + 1e-15) & (lo[:, a] + s <= hi[i, a] + 1e-15)
            touch &= ok
        if (touch & far).any():
            return False
    return True
