"""Pins of the oracle's Algorithm 3 (oracle/alg3.py) against facts fixed by
the mathematics, not by the code (CPU).

* Eq. (val2poleq) is exact for polynomials of degree < k, so a product of
  Legendre polynomials has one known coefficient, on the root and on every
  child (a degree-n Legendre polynomial restricted to a half box has leading
  Legendre coefficient 2^-n in the child's own variable).
* The tail of Eq. (funerr) for k = 8, d = 2 is the set of alpha in [0,7]^2 with
  alpha_1^2 + alpha_2^2 >= 64; by hand: (7,4), (7,5), (7,6), (7,7), (6,6),
  (6,7), (5,7), (4,7), eight indices; for k = 5: (3,4), (4,3), (4,4).
* The norm of a Gaussian sum in closed form against numerical integration.
* A level-restricted refinement is balanced, refines its input, and cannot
  merge any family it created without becoming unbalanced.
* On the torus, shifting the density by half the box shifts the tree.
"""

import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import integrate

from oracle import alg3


def _legendre_product(a1, a2):
    """sigma(x) = P_a1(2 x_1) P_a2(2 x_2) on [-1/2, 1/2]^2."""
    def f(x):
        x = np.asarray(x)
        return npleg.legval(2 * x[..., 0], [0] * a1 + [1]) * npleg.legval(2 * x[..., 1], [0] * a2 + [1])
    return f


def test_coefficients_of_a_legendre_product_on_the_root():
    k = 8
    vals = _legendre_product(7, 4)(alg3.box_nodes(0, (0, 0), k))
    c = alg3.coefficients(vals, k, 2)  # [alpha_2, alpha_1]
    want = np.zeros((k, k))
    want[4, 7] = 1.0
    assert np.max(np.abs(c - want)) < 1e-13


def test_tail_has_the_eight_hand_counted_indices():
    m = alg3.tail_indices(8, 2)
    got = {(int(a1), int(a2)) for a2, a1 in zip(*np.nonzero(m))}
    assert got == {(7, 4), (7, 5), (7, 6), (7, 7), (6, 6), (6, 7), (5, 7), (4, 7)}
    # k = 5: 3^2 + 4^2 = 5^2 sits on the boundary of the tail and belongs to it
    m = alg3.tail_indices(5, 2)
    got = {(int(a1), int(a2)) for a2, a1 in zip(*np.nonzero(m))}
    assert got == {(3, 4), (4, 3), (4, 4)}


def test_tail_error_of_a_legendre_product_on_root_and_children():
    # (7,4) is in the tail, and on a child every other tail coefficient of
    # P_7 x P_4 is zero (degree 4 along axis 2): e = 2^(-11 l) / sqrt(8) at level l
    k, f = 8, _legendre_product(7, 4)
    for level, coord in ((0, (0, 0)), (1, (0, 1)), (1, (1, 0)), (2, (3, 1)), (2, (0, 2))):
        e = alg3.tail_error(f(alg3.box_nodes(level, coord, k)), k, 2)
        want = 2.0 ** (-11 * level) / math.sqrt(8)
        assert abs(e - want) < 1e-12 * want + 1e-16, (level, coord, e, want)


@pytest.mark.parametrize("eps,depth", [(3e-3, 1), (1e-4, 2)])
def test_legendre_product_resolves_to_the_predicted_uniform_depth(eps, depth):
    # ||sigma||_2 = (1/15 * 1/9)^(1/2); level l splits iff 2^(-11 l)/sqrt(8) > eps ||sigma||_2.
    # eps = 3e-3 separates the RMS over the tail from its sum (level 1 kept);
    # eps = 1e-4 stops at level 2
    norm = math.sqrt(1.0 / 135.0)
    lv, cs, _ = alg3.resolve(_legendre_product(7, 4), 2, 8, eps, norm, max_level=8)
    assert set(lv.tolist()) == {depth}
    assert len(lv) == 4 ** depth


def test_polynomial_outside_the_tail_never_splits():
    # P_5 x P_5: every coefficient of it on every box has alpha <= (5,5),
    # 25 + 25 < 64, so the tail is empty at any depth
    lv, cs, ex = alg3.resolve(_legendre_product(5, 5), 2, 8, 1e-14, 1.0, max_level=6)
    assert len(lv) == 1 and lv[0] == 0
    assert ex[0][2] < 1e-15


def test_one_dimensional_tail_reading():
    # d = 1: the last two coefficients.  P_7(2x) on the root: e = (1/2)^(1/2);
    # P_5(2x) has none there, and none on any child
    f7 = lambda x: npleg.legval(2 * np.asarray(x)[..., 0], [0] * 7 + [1])
    f5 = lambda x: npleg.legval(2 * np.asarray(x)[..., 0], [0] * 5 + [1])
    e7 = alg3.tail_error(f7(alg3.box_nodes(0, (0,), 8)), 8, 1)
    assert abs(e7 - math.sqrt(0.5)) < 1e-13
    lv, _, _ = alg3.resolve(f5, 1, 8, 1e-14, 1.0, max_level=6)
    assert len(lv) == 1


def test_gaussian_sum_norm_against_quadrature():
    c = np.array([[0.1, -0.2], [-0.15, 0.05], [0.3, 0.3]])
    w = np.array([0.05, 0.08, 0.03])
    a = np.array([1.0, -0.7, 0.4])
    f = alg3.gaussian_sum(c, w, a)
    val, _ = integrate.dblquad(lambda y, x: f(np.array([x, y])) ** 2, -1.0, 1.0, -1.0, 1.0,
                               epsabs=1e-14, epsrel=1e-12)
    assert abs(alg3.gaussian_sum_norm(c, w, a) - math.sqrt(val)) < 1e-10 * math.sqrt(val)


def _point_refined(d, point, level):
    leaves = {(0, (0,) * d)}
    for l in range(level):
        key = alg3._leaf_covering(leaves, l, tuple(int((point[a] + 0.5) * 2 ** l) for a in range(d)))
        leaves.discard(key)
        for o in np.ndindex(*(2,) * d):
            leaves.add((key[0] + 1, tuple(2 * key[1][a] + o[a] for a in range(d))))
    return leaves


@pytest.mark.parametrize("d,periodic", [(2, False), (2, True), (3, False)])
def test_balance_is_balanced_refining_and_minimal(d, periodic):
    src = _point_refined(d, [0.49] + [0.1] * (d - 1), 6 if d == 2 else 4)
    out = alg3.balance(src, periodic)
    lv = np.array([l for l, _ in sorted(out)])
    cs = np.array([c for _, c in sorted(out)])
    assert alg3.is_balanced(lv, cs, periodic)
    assert not alg3.is_balanced(np.array([l for l, _ in sorted(src)]),
                                np.array([c for _, c in sorted(src)]), periodic)
    # refines: every input leaf is an output leaf or split into output leaves
    for (l, c) in out:
        assert alg3._leaf_covering(src, l, c) is not None
    # minimal: no family created by the balance can be merged back
    parents = {}
    for (l, c) in out:
        if l > 0:
            parents.setdefault((l - 1, tuple(v >> 1 for v in c)), []).append((l, c))
    for par, kids in parents.items():
        if len(kids) != 2 ** d or par in src or any((l, c) in src for (l, c) in kids):
            continue
        if alg3._leaf_covering(src, *par) is None:
            continue  # the family comes from the input's own splits
        merged = (out - set(kids)) | {par}
        ml = np.array([l for l, _ in sorted(merged)])
        mc = np.array([c for _, c in sorted(merged)])
        assert not alg3.is_balanced(ml, mc, periodic), par


def test_periodic_tree_follows_a_half_box_shift():
    c = np.array([[0.46, -0.2], [-0.1, 0.48]])
    w = np.array([0.02, 0.03])
    a = np.array([1.0, -0.6])
    norm = alg3.gaussian_sum_norm(c, w, a)
    lv, cs, _ = alg3.resolve(alg3.gaussian_sum(c, w, a, periodic=True), 2, 8, 1e-8, norm,
                             min_level=1, max_level=8, periodic=True)
    shifted = (c + 0.5 + 0.5) % 1.0 - 0.5  # centers moved by +1/2 on both axes, wrapped
    lv2, cs2, _ = alg3.resolve(alg3.gaussian_sum(shifted, w, a, periodic=True), 2, 8, 1e-8, norm,
                               min_level=1, max_level=8, periodic=True)
    moved = {(int(l), tuple(int((v + (1 << (l - 1))) % (1 << l)) for v in cc)) for l, cc in zip(lv, cs)}
    assert moved == set(zip(lv2.tolist(), map(tuple, cs2.tolist())))
    assert alg3.is_balanced(lv, cs, True)
    assert len(lv) > 40  # the blobs across the boundary are refined
