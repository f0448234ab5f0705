"""Pins of the CPU oracle against facts fixed outside its own code.

Each check is chosen so that a plausible mistake in the oracle fails it:
* closed forms (sigma = 1, Gaussian blobs, the sin/cos eigenfunction) catch a
  wrong kernel scale, a dropped leaf, a wrong image sum or a sign error in an
  offset;
* brute-force nested quadrature on tiny trees with random samples catches a
  wrong interpolant (val->pol matrix, transposed or mis-scaled);
* a separable polynomial density with different factors per axis catches a
  transposed axis in the tensor contraction;
* reflection / permutation / linearity / periodic shift are invariants of the
  exact transform.
"""

import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import integrate

import closed_forms as cf
import oracle
from paper_2305_07165_amd import synth


def _run(lv, cs, p, delta, dens, periodic=False):
    sig = synth.sample(lv, cs, p, dens)
    u = oracle.oracle_u(lv, cs, p, delta, sig, periodic=periodic)
    x = synth.leaf_points(lv, cs, p)
    return u, x, sig


def test_gauss_legendre_rule():
    for n in (1, 2, 5, 8, 16, 20):
        x, w = oracle.gauss_legendre(n)
        xn, wn = npleg.leggauss(n)
        assert np.max(np.abs(x - xn)) < 1e-15
        assert np.max(np.abs(w - wn)) < 2e-15
        # exact for degree 2n-1
        assert abs(np.sum(w * x ** (2 * n - 2)) - 2.0 / (2 * n - 1)) < 1e-14


@pytest.mark.parametrize("d,delta,p", [(1, 3e-3, 7), (2, 1e-3, 8), (2, 2e-2, 5), (3, 4e-3, 5)])
def test_constant_free(d, delta, p):
    lv, cs = synth.point_refined_tree(d, [0.131] * d, 4 if d < 3 else 3)
    u, x, _ = _run(lv, cs, p, delta, synth.Constant(1.0))
    ref = cf.const_free(x, delta)
    assert cf.rel_l2(u, ref) < 1e-13
    assert np.max(np.abs(u - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,delta", [(1, 1e-2), (1, 0.5), (2, 5e-3), (2, 8e-2), (3, 1e-2), (3, 0.1)])
def test_constant_periodic(d, delta):
    lv, cs = synth.point_refined_tree(d, [0.49] * d, 3, periodic=True)
    u, x, _ = _run(lv, cs, 4, delta, synth.Constant(1.0), periodic=True)
    assert np.max(np.abs(u / (math.pi * delta) ** (d / 2) - 1.0)) < 1e-13


def test_blob_free_2d_resolved():
    dens = synth.GaussianSum(np.array([[0.11, -0.17], [-0.2, 0.05]]),
                             np.array([0.05, 0.08]), np.array([0.7, -0.4]))
    lv, cs = synth.resolve_tree(dens, 2, 12, 1e-13, max_level=7)
    delta = 2e-3
    u, x, _ = _run(lv, cs, 12, delta, dens)
    ref = cf.gaussian_sum_free(x, delta, dens)
    assert cf.rel_l2(u, ref) < 1e-11


def test_blob_free_3d_resolved():
    dens = synth.GaussianSum(np.array([[0.1, -0.12, 0.05]]), np.array([0.09]),
                             np.array([1.0]))
    lv, cs = synth.resolve_tree(dens, 3, 10, 1e-10, max_level=4)
    delta = 5e-3
    u, x, _ = _run(lv, cs, 10, delta, dens)
    ref = cf.gaussian_sum_free(x, delta, dens)
    assert cf.rel_l2(u, ref) < 1e-8


def test_blob_periodized_periodic_2d():
    dens = synth.GaussianSum(np.array([[0.45, -0.48], [-0.1, 0.2]]),
                             np.array([0.06, 0.07]), np.array([1.0, -0.5]),
                             periodic=True)
    lv, cs = synth.resolve_tree(dens, 2, 12, 1e-13, max_level=6, periodic=True)
    delta = 4e-3
    u, x, _ = _run(lv, cs, 12, delta, dens, periodic=True)
    ref = cf.gaussian_sum_periodized(x, delta, dens)
    assert cf.rel_l2(u, ref) < 1e-11


@pytest.mark.parametrize("d,nu,delta", [(2, 2, 3e-3), (3, 1, 2e-2), (2, 1, 0.1), (1, 3, 0.05)])
def test_sincos_eigenfunction_periodic(d, nu, delta):
    lv, cs = synth.uniform_tree(d, 2)
    p = 14 if d == 2 else 10
    dens = synth.SinCosProduct(nu, d)
    u, x, _ = _run(lv, cs, p, delta, dens, periodic=True)
    ref = cf.sincos_periodic(x, delta, nu)
    assert cf.rel_l2(u, ref) < (1e-12 if d == 2 else 1e-9)


def _interp(vals, p, lo, L):
    """Tensor Legendre interpolant on one 2D leaf via numpy (independent)."""
    eta = npleg.leggauss(p)[0]
    V = npleg.legvander(eta, p - 1)
    c = np.linalg.solve(V, np.linalg.solve(V, vals.reshape(p, p)).T).T  # [n2, n1]

    def f(y1, y2):
        t1 = 2 * (y1 - lo[0]) / L - 1
        t2 = 2 * (y2 - lo[1]) / L - 1
        return float(npleg.legval2d(t2, t1, c))
    return f


def test_bruteforce_tiny_2d():
    # 7 leaves: three at level 1, four at level 2 in the remaining quadrant
    lv = np.array([1, 1, 1, 2, 2, 2, 2], dtype=np.int32)
    cs = np.array([[1, 0], [0, 1], [1, 1], [0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.int32)
    p, delta = 3, 0.05
    rng = np.random.default_rng(3)
    sig = rng.normal(size=(7, p * p))
    targets = np.array([3, 1])
    u = oracle.oracle_u(lv, cs, p, delta, sig, targets=targets)
    x = synth.leaf_points(lv, cs, p)
    cen, L = synth.leaf_centers(lv, cs)
    fs = [_interp(sig[s], p, cen[s] - L[s] / 2, L[s]) for s in range(7)]
    for ti, t in enumerate(targets):
        for node in (0, 4, 7):
            xt = x[t, node]
            tot = 0.0
            for s in range(7):
                lo = cen[s] - L[s] / 2
                val, _ = integrate.dblquad(
                    lambda y2, y1: math.exp(-((xt[0] - y1) ** 2 + (xt[1] - y2) ** 2) / delta)
                    * fs[s](y1, y2),
                    lo[0], lo[0] + L[s], lo[1], lo[1] + L[s], epsabs=1e-13, epsrel=1e-12)
                tot += val
            assert abs(u[ti, node] - tot) < 1e-10 * max(1.0, abs(tot))


def test_separable_polynomial_2d():
    p, delta = 6, 4e-3
    rng = np.random.default_rng(7)
    cf1 = rng.normal(size=p)       # degree p-1 in x1
    cf2 = rng.normal(size=p - 2)   # degree p-3 in x2 (different factor per axis)

    def dens(x):
        return npleg.legval(2 * x[..., 0], cf1) * npleg.legval(2 * x[..., 1], cf2)

    lv, cs = synth.point_refined_tree(2, [-0.3, 0.22], 4)
    sig = synth.sample(lv, cs, p, dens)
    u = oracle.oracle_u(lv, cs, p, delta, sig)
    x = synth.leaf_points(lv, cs, p)

    def u1d(xv, coef):
        v, _ = integrate.quad(lambda y: math.exp(-(xv - y) ** 2 / delta)
                              * npleg.legval(2 * y, coef), -0.5, 0.5,
                              points=[xv], epsabs=1e-14, epsrel=1e-13, limit=200)
        return v
    pick = rng.choice(x.shape[0] * x.shape[1], 40, replace=False)
    for f in pick:
        lf, nf = divmod(int(f), x.shape[1])
        xt = x[lf, nf]
        ref = u1d(xt[0], cf1) * u1d(xt[1], cf2)
        assert abs(u[lf, nf] - ref) < 1e-12 * max(1.0, np.max(np.abs(u)))


def _reflect_axis(lv, cs, sig, p, d, axis):
    cs2 = cs.copy()
    cs2[:, axis] = (1 << lv) - 1 - cs[:, axis]
    s = sig.reshape((-1,) + (p,) * d)
    s = np.flip(s, axis=d - axis)  # array axes are [i_d,...,i_1]
    return cs2, s.reshape(len(lv), -1)


@pytest.mark.parametrize("periodic", [False, True])
def test_invariants_3d(periodic):
    d, p, delta = 3, 4, 6e-3
    lv, cs = synth.point_refined_tree(d, [0.2, -0.31, 0.07], 3, periodic=periodic)
    rng = np.random.default_rng(11)
    sig = rng.normal(size=(len(lv), p ** d))
    u = oracle.oracle_u(lv, cs, p, delta, sig, periodic=periodic)
    # reflection of axis 2
    cs2, sig2 = _reflect_axis(lv, cs, sig, p, d, 1)
    u2 = oracle.oracle_u(lv, cs2, p, delta, sig2, periodic=periodic)
    _, u2b = _reflect_axis(lv, cs2, u2, p, d, 1)
    assert np.max(np.abs(u2b - u)) < 1e-14 * np.max(np.abs(u)) * 10
    # permutation of axes 1 and 3
    cs3 = cs[:, ::-1].copy()
    sig3 = sig.reshape(-1, p, p, p).transpose(0, 3, 2, 1).reshape(len(lv), -1)
    u3 = oracle.oracle_u(lv, cs3, p, delta, sig3, periodic=periodic)
    u3b = u3.reshape(-1, p, p, p).transpose(0, 3, 2, 1).reshape(len(lv), -1)
    assert np.max(np.abs(u3b - u)) < 1e-13 * np.max(np.abs(u))
    # linearity
    sb = rng.normal(size=sig.shape)
    ub = oracle.oracle_u(lv, cs, p, delta, sb, periodic=periodic)
    uab = oracle.oracle_u(lv, cs, p, delta, 2.0 * sig - 3.0 * sb, periodic=periodic)
    assert np.max(np.abs(uab - (2.0 * u - 3.0 * ub))) < 1e-13 * np.max(np.abs(uab))


def test_periodic_shift_2d():
    d, p, delta = 2, 5, 5e-3
    lv, cs = synth.uniform_tree(d, 3)
    rng = np.random.default_rng(5)
    sig = rng.normal(size=(len(lv), p ** d))
    u = oracle.oracle_u(lv, cs, p, delta, sig, periodic=True)
    # shift every leaf by 3 boxes along axis 1 and 5 along axis 2 (wrapping)
    cs2 = cs.copy()
    cs2[:, 0] = (cs[:, 0] + 3) % 8
    cs2[:, 1] = (cs[:, 1] + 5) % 8
    u2 = oracle.oracle_u(lv, cs2, p, delta, sig, periodic=True)
    assert np.max(np.abs(u2 - u)) < 1e-14 * np.max(np.abs(u)) * 10
    # the same shift is not an invariant in free space (sanity of the image sum)
    uf = oracle.oracle_u(lv, cs, p, delta, sig)
    uf2 = oracle.oracle_u(lv, cs2, p, delta, sig)
    assert np.max(np.abs(uf2 - uf)) > 1e-6 * np.max(np.abs(uf))


# ---------------------------------------------------------------------------
# targets that are not leaves of the source tree (output trees, Section 4.2)


def _random_boxes(rng, d, n, lmin, lmax):
    bl = rng.integers(lmin, lmax + 1, n).astype(np.int32)
    bc = np.stack([rng.integers(0, 1 << int(l), d) for l in bl]).astype(np.int32)
    return bl, bc


def test_boxes_equal_leaves_when_targets_are_leaves():
    dens = synth.GaussianSum(np.array([[0.11, -0.17]]), np.array([0.05]), np.array([1.0]))
    lv, cs = synth.resolve_tree(dens, 2, 6, 1e-8, max_level=6)
    sig = synth.sample(lv, cs, 6, dens)
    a = oracle.oracle_u(lv, cs, 6, 2e-3, sig)
    b = oracle.oracle_u_boxes(lv, cs, 6, 2e-3, sig, lv, cs)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("d,periodic", [(1, False), (2, False), (3, False), (2, True)])
def test_boxes_constant_closed_form(d, periodic):
    """sigma = 1 at boxes finer and coarser than the leaves they overlap."""
    rng = np.random.default_rng(7 + d)
    lv, cs = synth.point_refined_tree(d, [0.131] * d, 4 if d < 3 else 3, periodic=periodic)
    p, delta = 5, 4e-3
    bl, bc = _random_boxes(rng, d, 40 if d < 3 else 12, 0, 7 if d < 3 else 5)
    sig = np.ones((len(lv), p ** d))
    u = oracle.oracle_u_boxes(lv, cs, p, delta, sig, bl, bc, periodic=periodic)
    x = synth.leaf_points(bl, bc, p)
    ref = cf.const_periodic(x, delta) if periodic else cf.const_free(x, delta)
    assert np.max(np.abs(u - ref)) < 1e-13 * np.max(np.abs(ref))


def test_boxes_blob_closed_form_2d():
    dens = synth.GaussianSum(np.array([[0.11, -0.17], [-0.2, 0.05]]),
                             np.array([0.05, 0.08]), np.array([0.7, -0.4]))
    lv, cs = synth.resolve_tree(dens, 2, 12, 1e-13, max_level=7)
    rng = np.random.default_rng(3)
    bl, bc = _random_boxes(rng, 2, 60, 2, 9)
    delta = 2e-3
    sig = synth.sample(lv, cs, 12, dens)
    u = oracle.oracle_u_boxes(lv, cs, 12, delta, sig, bl, bc)
    ref = cf.gaussian_sum_free(synth.leaf_points(bl, bc, 12), delta, dens)
    assert cf.rel_l2(u, ref) < 1e-11


@pytest.mark.parametrize("d", [1, 2, 3])
def test_interp_reproduces_nodes_and_polynomials(d):
    """At a leaf's own nodes the interpolant returns the values; a polynomial
    of degree < p per axis is reproduced exactly anywhere (numpy polyval)."""
    rng = np.random.default_rng(20 + d)
    lv, cs = synth.point_refined_tree(d, [0.31] * d, 4 if d < 3 else 3)
    p = 5
    coefs = [rng.normal(size=p) for _ in range(d)]

    def f(x):
        return np.prod([np.polynomial.polynomial.polyval(x[..., a], coefs[a]) for a in range(d)], 0)

    xn = synth.leaf_points(lv, cs, p)                     # [n, p^d, d]
    vals = f(xn)
    got = oracle.oracle_interp(lv, cs, p, vals, xn.reshape(-1, d))
    assert np.max(np.abs(got - vals.ravel())) < 1e-12 * np.max(np.abs(vals))
    x = rng.uniform(-0.5, 0.5, (2000, d))
    x[:3] = 0.5                                           # the top corner
    x[3:6] = -0.5
    assert np.max(np.abs(oracle.oracle_interp(lv, cs, p, vals, x) - f(x))) < 1e-12 * np.max(np.abs(vals))
