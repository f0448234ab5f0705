"""Test-only numpy walk of a host plan's lists and tables.

It applies the stages of Algorithm 4 exactly as the plan describes them
(formation into cutoff boxes, translations along the P-lists, evaluation,
near field along the D-lists) with numpy einsum, so the host plan -- lists,
f-flags, table entries, signs of the translations -- can be checked against
the oracle on a CPU.  It is not part of the product path: the product runs
only in the HIP kernels.
"""

from __future__ import annotations

import numpy as np

from paper_2305_07165_amd import api


def _contract(mats, t):
    """Apply mats[a] (rows out, cols in) along axis a of tensor t whose array
    axes are [i_d, ..., i_1] (axis 1 fastest)."""
    d = len(mats)
    for a, m in enumerate(mats):
        ax = d - 1 - a
        t = np.moveaxis(np.tensordot(m, t, axes=([1], [ax])), 0, ax)
    return t


def _along(m, t, a, d):
    """Apply matrix m (rows out, cols in) along axis a (0-based, axis 1 = a 0)
    of a tensor stored [i_d, ..., i_1]."""
    ax = d - 1 - a
    return np.moveaxis(np.tensordot(m, t, axes=([1], [ax])), 0, ax)


def _rot_matrix(nrs, rot, dir_):
    """Rotation of every stored (cos, sin) pair (2m, 2m+1) by dir * k_m L_c;
    mode 0 (the constant and its zero slot) is left alone."""
    R = np.zeros((nrs, nrs))
    R[0, 0] = R[1, 1] = 1.0
    for m in range(1, nrs // 2):
        c, s = rot[m]
        s = s * dir_
        if dir_ == 0:
            c, s = 1.0, 0.0
        i, j = 2 * m, 2 * m + 1
        R[i, i], R[i, j], R[j, i], R[j, j] = c, -s, s, c
    return R


def run(plan: api.Plan, sigma: np.ndarray, grouped: bool = False) -> np.ndarray:
    """u of the plan's stages.  grouped (d = 3 only): formation and evaluation
    walk the plan's planes and rows the way the device kernels do -- each
    leaf's axis-2 table, then once per row the axis-1 table, then once per
    plane the axis-3 table (and the reverse for evaluation) -- instead of
    applying all tables per leaf."""
    info = plan.info()
    d, p, nr = info["dim"], info["p"], info["nr_stored"]  # stored modes: (2m, 2m+1) = mode m
    M = nr // 2
    F = plan.array("F").reshape(-1, nr, p)
    E = plan.array("E").reshape(-1, p, nr)
    V = plan.array("V").reshape(-1, p, p)
    rot = plan.array("rot").reshape(M, 2)
    pw_start = plan.array("pw_start")
    pwleaf_id = plan.array("pwleaf_id")
    pwleaf_tab = plan.array("pwleaf_tab").reshape(-1, d)
    plist_start = plan.array("plist_start")
    plist_src = plan.array("plist_src")
    plist_dir = plan.array("plist_dir")
    near_tgt = plan.array("near_tgt")
    near_haspw = plan.array("near_haspw")
    near_start = plan.array("near_start")
    near_src = plan.array("near_src")
    near_tab = plan.array("near_tab").reshape(-1, d)
    nA = len(pw_start) - 1
    u = np.zeros_like(sigma)
    shp = (p,) * d
    phi = np.zeros((nA,) + (nr,) * d)
    if grouped:
        assert d == 3
        plane_start = plan.array("plane_start")
        plane_tab = plan.array("plane_tab").reshape(-1, 3)
        plane_row = plan.array("plane_row")
        row_start = plan.array("row_start")
        row_tab = plan.array("row_tab")
        for A in range(nA):
            for P in range(plane_start[A], plane_start[A + 1]):
                Y = np.zeros((p, nr, nr))
                for rw in range(plane_row[P], plane_row[P + 1]):
                    X = np.zeros((p, nr, p))
                    for s in range(row_start[rw], row_start[rw + 1]):
                        X += _along(F[pwleaf_tab[s, 1]], sigma[pwleaf_id[s]].reshape(shp), 1, 3)
                    Y += _along(F[row_tab[rw]], X, 0, 3)
                phi[A] += _along(F[plane_tab[P, 2]], Y, 2, 3)
    else:
        for A in range(nA):
            for s in range(pw_start[A], pw_start[A + 1]):
                mats = [F[pwleaf_tab[s, a]] for a in range(d)]
                phi[A] += _contract(mats, sigma[pwleaf_id[s]].reshape(shp))
    psi = np.zeros_like(phi)
    for A in range(nA):
        for q in range(plist_start[A], plist_start[A + 1]):
            code = int(plist_dir[q])
            mats = []
            for a in range(d):
                mats.append(_rot_matrix(nr, rot, code % 3 - 1))
                code //= 3
            psi[A] += _contract(mats, phi[plist_src[q]])
    haspw = np.zeros(len(sigma), dtype=bool)
    if grouped:
        for A in range(nA):
            for P in range(plane_start[A], plane_start[A + 1]):
                Z = _along(E[plane_tab[P, 2]], psi[A], 2, 3)
                for rw in range(plane_row[P], plane_row[P + 1]):
                    W = _along(E[row_tab[rw]], Z, 0, 3)
                    for s in range(row_start[rw], row_start[rw + 1]):
                        u[pwleaf_id[s]] = _along(E[pwleaf_tab[s, 1]], W, 1, 3).reshape(-1)
                        haspw[pwleaf_id[s]] = True
    else:
        for A in range(nA):
            for s in range(pw_start[A], pw_start[A + 1]):
                mats = [E[pwleaf_tab[s, a]] for a in range(d)]
                u[pwleaf_id[s]] = _contract(mats, psi[A]).reshape(-1)
                haspw[pwleaf_id[s]] = True
    for t in range(len(near_tgt)):
        T = near_tgt[t]
        assert bool(near_haspw[t]) == bool(haspw[T])
        acc = np.zeros(shp)
        for q in range(near_start[t], near_start[t + 1]):
            mats = [V[near_tab[q, a]] for a in range(d)]
            acc += _contract(mats, sigma[near_src[q]].reshape(shp))
        u[T] = u[T] + acc.reshape(-1) if haspw[T] else acc.reshape(-1)
    return u
