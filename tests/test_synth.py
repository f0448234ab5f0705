"""CPU tests of the seeded input generators (host logic, no transform
arithmetic): tree validity and balance, the vectorized balance against the
reference one, the separable sampler against direct sampling, and the
batched / served workload recipes."""

import itertools

import numpy as np
import pytest

from paper_2305_07165_amd import api, synth


def _tiles(lv, cs):
    """True if the leaves tile [0,1)^d exactly (volumes add up, no overlap)."""
    d = cs.shape[1]
    vol = np.sum(2.0 ** (-d * lv.astype(np.float64)))
    keys = {(int(l), tuple(int(v) for v in c)) for l, c in zip(lv, cs)}
    if len(keys) != len(lv):
        return False
    # no leaf contains another leaf's lower corner at a finer level
    for l, c in keys:
        for ll in range(l):
            if (ll, tuple(v >> (l - ll) for v in c)) in keys:
                return False
    return abs(vol - 1.0) < 1e-12


def _raw_refined(d, pts, maxl):
    """A tree refined around points, not balanced."""
    leaves, boxes = [], [(0, (0,) * d)]
    while boxes:
        l, c = boxes.pop()
        L = 2.0 ** -l
        lo = -0.5 + np.array(c) * L
        inside = any(np.all(pt >= lo) and np.all(pt < lo + L) for pt in pts)
        if inside and l < maxl:
            for o in itertools.product((0, 1), repeat=d):
                boxes.append((l + 1, tuple(2 * c[a] + o[a] for a in range(d))))
        else:
            leaves.append((l, c))
    return (np.array([l for l, _ in leaves], np.int32),
            np.array([c for _, c in leaves], np.int32).reshape(-1, d))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_balance_fast_equals_reference_balance(d):
    rng = np.random.default_rng(10 + d)
    for _ in range(12):
        pts = rng.uniform(-0.5, 0.5, (int(rng.integers(1, 4)), d))
        lv, cs = _raw_refined(d, pts, int(rng.integers(2, 7 if d < 3 else 5)))
        for periodic in (False, True):
            a = synth.balance(lv, cs, periodic)
            b = synth.balance_fast(lv, cs, periodic)
            assert set(zip(a[0].tolist(), map(tuple, a[1].tolist()))) == \
                set(zip(b[0].tolist(), map(tuple, b[1].tolist())))
            assert synth.is_balanced_fast(*b, periodic)
            assert synth.is_balanced_fast(lv, cs, periodic) == synth.is_balanced(lv, cs, periodic)


@pytest.mark.parametrize("d,p", [(1, 5), (2, 8), (3, 4)])
def test_separable_sampler_equals_direct(d, p):
    rng = np.random.default_rng(4)
    dens = synth.GaussianSum(rng.uniform(-0.3, 0.3, (5, d)), rng.uniform(0.01, 0.05, 5),
                             rng.uniform(-1, 1, 5))
    lv, cs = synth.sized_tree(d, dens.centers, 200)
    a = synth.sample(lv, cs, p, dens)
    b = synth.sample_separable(lv, cs, p, dens)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))


@pytest.mark.parametrize("d,target", [(2, 300), (2, 5000), (3, 200), (3, 3000)])
def test_sized_tree_is_a_balanced_tiling_near_the_size(d, target):
    rng = np.random.default_rng(target)
    lv, cs = synth.sized_tree(d, rng.uniform(-0.3, 0.3, (4, d)), target)
    assert _tiles(lv, cs) if len(lv) < 4000 else True
    assert synth.is_balanced_fast(lv, cs)
    assert 0.7 * target <= len(lv) <= 1.4 * target


def test_serve_request_types_follow_the_recipe():
    types = synth.serve_request_types(3, 6, log10_n=(3.5, 5.0))
    for t in types:
        assert t.d in (2, 3) and t.p in (8, 16) and t.tol in (1e-3, 1e-6, 1e-10)
        assert 1e-6 <= t.delta <= 1e-2
        assert t.precision == ("fp32" if t.tol >= 1e-3 else "fp64")
        assert t.sigma.shape == (len(t.levels), t.p ** t.d)
        assert synth.is_balanced_fast(t.levels, t.coords)
        # the host plan accepts the tree
        api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, host_only=True).close()


def test_batch_problems_are_independent_of_workers_and_capped():
    a = synth.batch_problems(1, 6, max_points=1 << 15)
    b = synth.batch_problems(1, 6, max_points=1 << 15, workers=2)
    for x, y in zip(a, b):
        assert np.array_equal(x.levels, y.levels) and np.array_equal(x.sigma, y.sigma)
        assert x.npoints <= 1 << 15
        assert x.precision == ("fp32" if x.tol >= 1e-6 else "fp64")
        assert synth.is_balanced_fast(x.levels, x.coords)
