"""Pins of the oracle's point transform (Eq. (pgt): u_i = sum_j G(x_i - y_j) q_j)
against facts fixed by the mathematics (CPU).

* Poisson summation: a uniform lattice of unit charges with spacing h sums, at
  a target far from the lattice's edge, to (sqrt(pi delta)/h)^d up to
  exp(-pi^2 delta / h^2) per axis (1e-43 here): a wrong scale in the exponent
  or a dropped axis changes the value.
* Separability: charges q = a(y_1) b(y_2) c(y_3) on a tensor grid give u(x) as
  the product of three 1D sums.
* Brute force on tiny inputs; translation, permutation and linearity.
* The cell-list cutoff: the skipped terms stay below exp(-cut^2/delta) sum|q|.
"""

import math

import numpy as np
import pytest

import oracle


def _lattice(d, h):
    t = -0.5 + h * (np.arange(int(round(1 / h))) + 0.5)
    g = np.meshgrid(*([t] * d), indexing="ij")
    return np.stack([x.reshape(-1) for x in g], -1)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_lattice_sum_is_the_poisson_value(d):
    h, delta = 1.0 / 40 if d == 3 else 1.0 / 100, 1e-3 if d < 3 else 4e-3
    y = _lattice(d, h)
    q = np.ones(len(y))
    rng = np.random.default_rng(d)
    x = rng.uniform(-0.1, 0.1, (50, d))  # > 0.35 from the edge: exp(-0.35^2/delta) < 1e-13
    u = oracle.oracle_point(y, q, x, delta)
    want = (math.sqrt(math.pi * delta) / h) ** d
    assert np.max(np.abs(u / want - 1.0)) < 1e-12


def test_separable_charges_give_a_product_of_1d_sums():
    rng = np.random.default_rng(3)
    delta = 2e-3
    t = [np.sort(rng.uniform(-0.5, 0.5, n)) for n in (7, 9, 11)]
    w = [rng.uniform(-1, 1, len(ti)) for ti in t]
    g = np.meshgrid(*t, indexing="ij")
    y = np.stack([x.reshape(-1) for x in g], -1)
    q = np.einsum("i,j,k->ijk", *w).reshape(-1)
    x = rng.uniform(-0.5, 0.5, (40, 3))
    u = oracle.oracle_point(y, q, x, delta, cut=0)
    one = [np.exp(-(x[:, a, None] - t[a][None, :]) ** 2 / delta) @ w[a] for a in range(3)]
    want = one[0] * one[1] * one[2]
    assert np.max(np.abs(u - want)) < 1e-13 * np.max(np.abs(want)) + 1e-300


def test_brute_force_on_tiny_inputs():
    rng = np.random.default_rng(5)
    y, x = rng.uniform(-0.5, 0.5, (13, 2)), rng.uniform(-0.5, 0.5, (17, 2))
    q = rng.uniform(-1, 1, 13)
    delta = 0.05
    want = np.array([sum(math.exp(-((xi[0] - yj[0]) ** 2 + (xi[1] - yj[1]) ** 2) / delta) * qj
                         for yj, qj in zip(y, q)) for xi in x])
    for cut in (0.0, None):
        assert np.max(np.abs(oracle.oracle_point(y, q, x, delta, cut=cut) - want)) < 1e-14


def test_invariants():
    rng = np.random.default_rng(7)
    y, x = rng.uniform(-0.3, 0.3, (400, 3)), rng.uniform(-0.3, 0.3, (300, 3))
    q, q2 = rng.uniform(-1, 1, 400), rng.uniform(-1, 1, 400)
    delta = 1e-3
    u = oracle.oracle_point(y, q, x, delta)
    shift = np.array([0.13, -0.17, 0.05])
    assert np.allclose(oracle.oracle_point(y + shift, q, x + shift, delta), u, rtol=0, atol=1e-13)
    perm = rng.permutation(400)
    assert np.allclose(oracle.oracle_point(y[perm], q[perm], x, delta), u, rtol=0, atol=1e-13)
    lin = oracle.oracle_point(y, 2 * q - 3 * q2, x, delta)
    assert np.allclose(lin, 2 * u - 3 * oracle.oracle_point(y, q2, x, delta), rtol=0, atol=1e-12)


def test_cutoff_skips_only_negligible_terms():
    rng = np.random.default_rng(9)
    y, x = rng.uniform(-0.5, 0.5, (5000, 3)), rng.uniform(-0.5, 0.5, (500, 3))
    q = rng.uniform(-1, 1, 5000)
    delta = 1e-3
    full, nfull = oracle.oracle_point(y, q, x, delta, cut=0, return_pairs=True)
    for cut in (math.sqrt(delta * math.log(1e18)), 0.1):
        cutv, n = oracle.oracle_point(y, q, x, delta, cut=cut, return_pairs=True)
        assert n < nfull
        assert np.max(np.abs(cutv - full)) <= math.exp(-cut * cut / delta) * np.sum(np.abs(q)) + 1e-15
