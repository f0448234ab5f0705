"""GPU tests of Algorithm 3 on the device (include/fgt_density.h).

The device resolves a Gaussian-sum density level by level (samples at the
box nodes, Legendre-tail estimate, split above eps*||sigma||_2) and balances
the tree.  The oracle's Algorithm 3 (oracle/alg3.py: box by box in numpy,
pinned on the CPU by Legendre-product densities with known tails, the
hand-counted tail sets, a quadrature of the norm and balance properties)
must produce the same set of leaves, and sigma on them must agree to
rounding with the density evaluated at the oracle's own nodes.  A split
decision is a floating-point comparison taken on both sides in FP64 (with
different summation orders); every case asserts that no examined box lies
within 1e-9 of the threshold, so the trees must be identical.
"""

import time

import numpy as np
import pytest

import closed_forms as cf
from oracle import alg3
from paper_2305_07165_amd import api, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-density] {msg}", flush=True)


def _leafset(lv, cs):
    return set(zip(np.asarray(lv).tolist(), map(tuple, np.asarray(cs).tolist())))


CASES = [
    # name, d, p, eps, periodic, max_level, min_level, density builder
    ("1d", 1, 9, 1e-12, False, 14, 0,
     lambda: synth.GaussianSum(np.array([[0.13], [-0.31]]), np.array([0.004, 0.02]), np.array([1.0, -0.5]))),
    ("2d-small", 2, 8, 1e-10, False, 10, 0,
     lambda: synth.small_2d(3).density),
    ("2d-periodic", 2, 8, 1e-10, True, 9, 2,
     lambda: synth.GaussianSum(np.array([[0.47, -0.3], [-0.2, 0.49]]), np.array([0.01, 0.02]),
                               np.array([1.0, -0.7]), periodic=True)),
    ("3d-bench-density", 3, 16, 1e-9, False, 7, 0,
     lambda: synth.GaussianSum(*synth._blobs(np.random.default_rng(0), 8, 3, -0.4, 0.4, 1e-3, 1e-2, True))),
]


@pytest.mark.parametrize("name,d,p,eps,periodic,maxl,minl,make", CASES, ids=[c[0] for c in CASES])
def test_resolve_matches_the_oracle_algorithm_3(name, d, p, eps, periodic, maxl, minl, make):
    dens = make()
    norm = alg3.gaussian_sum_norm(dens.centers, dens.widths, dens.amps)
    t0 = time.time()
    lv_o, cs_o, examined = alg3.resolve(alg3.gaussian_sum(dens.centers, dens.widths, dens.amps, periodic),
                                        d, p, eps, norm, min_level=minl, max_level=maxl, periodic=periodic)
    t_oracle = time.time() - t0
    margin = min(abs(e - eps * norm) / (eps * norm) for _, _, e in examined)
    torch.cuda.synchronize()
    t0 = time.time()
    lv, cs, sig, info = api.resolve_gaussians(dens.centers, dens.widths, dens.amps, p, eps,
                                              periodic=dens.periodic, min_level=minl, max_level=maxl)
    torch.cuda.synchronize()
    t_dev = time.time() - t0
    _say(f"{name}: {info['nleaves']} leaves (oracle {len(lv_o)}), boxes sampled {info['boxes_sampled']} "
         f"(oracle {len(examined)}), device {1e3 * t_dev:.1f} ms, oracle {1e3 * t_oracle:.1f} ms, "
         f"closest box to the threshold {margin:.2e} of it")
    assert margin > 1e-9
    # the device's closed-form norm, then the same threshold on both sides
    assert abs(info["norm"] - norm) <= 1e-13 * norm
    assert _leafset(lv, cs) == _leafset(lv_o, cs_o)
    assert alg3.is_balanced(lv, cs, periodic)
    f = alg3.gaussian_sum(dens.centers, dens.widths, dens.amps, periodic)
    ref = np.stack([f(alg3.box_nodes(int(l), tuple(int(v) for v in c), p)) for l, c in zip(lv, cs)])
    got = sig.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"{name}: sigma max rel diff {err:.2e}")
    assert err < 1e-14


def test_sample_gaussians_on_a_given_tree():
    dens = synth.GaussianSum(np.array([[0.1, -0.2, 0.05]]), np.array([0.05]), np.array([0.8]), periodic=True)
    lv, cs = synth.point_refined_tree(3, [0.49, -0.2, 0.1], 4, periodic=True)
    got = api.sample_gaussians(dens.centers, dens.widths, dens.amps, lv, cs, 6, periodic=True).cpu().numpy()
    f = alg3.gaussian_sum(dens.centers, dens.widths, dens.amps, periodic=True)
    ref = np.stack([f(alg3.box_nodes(int(l), tuple(int(v) for v in c), 6)) for l, c in zip(lv, cs)])
    assert np.max(np.abs(got - ref)) < 1e-14 * np.max(np.abs(ref))


def test_resolved_tree_runs_the_transform():
    """The device-built input feeds fgt_plan / fgt_execute directly."""
    dens = synth.small_2d(1).density
    lv, cs, sig, info = api.resolve_gaussians(dens.centers, dens.widths, dens.amps, 8, 1e-10, max_level=9)
    u = api.Plan(lv, cs, 8, 1e-3, 1e-8).execute(sig)
    x = synth.leaf_points(lv, cs, 8)
    ref = cf.gaussian_sum_free(x, 1e-3, dens)
    err = cf.rel_l2(u.cpu().numpy(), ref)
    _say(f"transform of the device-built input vs closed form: {err:.2e}")
    assert err < 1e-8


def test_resolve_errors():
    c, w, a = np.array([[0.0, 0.0]]), np.array([0.1]), np.array([1.0])
    with pytest.raises(api.FgtError):
        api.resolve_gaussians(c, np.array([0.0]), a, 8, 1e-8)          # width 0
    with pytest.raises(api.FgtError):
        api.resolve_gaussians(c, w, a, 8, 1e-8, min_level=3, max_level=2)
    with pytest.raises(api.FgtError):
        api.resolve_gaussians(c, w, a, 8, 1e-14, max_level=12, max_leaves=4)
