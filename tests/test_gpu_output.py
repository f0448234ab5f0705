"""GPU tests of the output trees (include/fgt_output.h; Section 4.2,
Algorithms 5 and 6) and of point evaluation.

Bars: u on the output leaves equals the FP64 oracle's transform of the input
density evaluated at those boxes (a sample of them, always including the
largest |u|) within the transform's tol; the output tree is a 2:1 balanced
tiling; refinement leaves no leaf above the error threshold except at the
depth limit; point evaluation equals the oracle's numpy interpolant.  The
worked example of Section 4.2 is reproduced in kind: interpolating u from the
input tree loses digits that the output tree recovers.
"""

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_2305_07165_amd import api, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-output] {msg}", flush=True)


def _tiles(lv, cs):
    d = cs.shape[1]
    vol = np.sum(2.0 ** (-d * lv.astype(np.float64)))
    keys = {(int(l), tuple(int(v) for v in c)) for l, c in zip(lv, cs)}
    return len(keys) == len(lv) and abs(vol - 1.0) < 1e-12


def _tail_errors(u, p, d):
    """Eq. (funerr) per leaf in numpy (test-side, independent of the kernels)."""
    from numpy.polynomial import legendre as npleg
    eta = oracle.gauss_legendre(p)[0]
    Vinv = np.linalg.inv(npleg.legvander(eta, p - 1))
    c = u.reshape((u.shape[0],) + (p,) * d)
    for ax in range(1, d + 1):
        c = np.moveaxis(np.tensordot(Vinv, c, axes=([1], [ax])), 0, ax)
    idx = np.stack(np.meshgrid(*([np.arange(p)] * d), indexing="ij"), -1)
    mask = (idx[..., 0] >= p - 2) if d == 1 else (np.sum(idx ** 2, -1) >= p * p)
    return np.sqrt(np.mean(c[:, mask] ** 2, axis=1))


def _sample_boxes(u, n, seed):
    rng = np.random.default_rng(seed)
    top = np.argsort(-np.max(np.abs(u), axis=1))[:16]
    rest = rng.choice(len(u), size=min(n, len(u)), replace=False)
    return np.unique(np.r_[top, rest])


def _check_parity(lv0, cs0, sig0, p, delta, tol, out, periodic, seed, n=120):
    u = out.u.cpu().numpy()
    idx = _sample_boxes(u, n, seed)
    uo = oracle.oracle_u_boxes(lv0, cs0, p, delta, sig0, out.levels[idx], out.coords[idx],
                               periodic=periodic)
    err = cf.rel_l2(u[idx], uo)
    _say(f"  u on {len(idx)} output leaves vs oracle: rel_l2={err:.2e} (tol {tol})")
    assert err < tol
    return err


def _two_peaks(alpha=1e-4):
    """sigma = exp(-|x-x1|^2/alpha) + exp(-|x-x2|^2/alpha); the peaks' positions
    are not given in the paper (any two interior points off the dyadic grid).
    Trees of it start at level 3 so that the nodes see the peaks."""
    w = np.sqrt(alpha)
    return synth.GaussianSum(np.array([[-0.1873, 0.1062], [0.2291, -0.1517]]),
                             np.array([w, w]), np.array([1.0, 1.0]))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_interp_matches_oracle(d):
    p = {1: 9, 2: 8, 3: 5}[d]
    dens = synth.GaussianSum(np.array([[0.13, -0.2, 0.07][:d]]), np.array([0.05]), np.array([1.0]))
    lv, cs = synth.resolve_tree(dens, d, p, 1e-8, max_level={1: 9, 2: 7, 3: 4}[d])
    rng = np.random.default_rng(d)
    vals = rng.normal(size=(len(lv), p ** d))
    x = rng.uniform(-0.5, 0.5, (20000, d))
    # faces, corners and the top of the unit box
    x[:200] = np.round(x[:200] * 64) / 64
    x[200:210] = 0.5
    x[210:220] = -0.5
    ref = oracle.oracle_interp(lv, cs, p, vals, x)
    got = api.interp(lv, cs, p, torch.from_numpy(vals).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(vals))
    _say(f"interp d={d} p={p} leaves={len(lv)}: max rel diff {err:.2e}")
    assert err < 1e-12
    # at the leaves' own nodes the interpolant returns the values
    xn = synth.leaf_points(lv, cs, p).reshape(-1, d)
    got = api.interp(lv, cs, p, torch.from_numpy(vals).cuda(), torch.from_numpy(xn).cuda()).cpu().numpy()
    assert np.max(np.abs(got - vals.ravel())) < 1e-12 * np.max(np.abs(vals))


def test_refine_only_3d_every_leaf_resolved():
    dens = synth.GaussianSum(np.array([[0.1, -0.12, 0.05]]), np.array([0.03]), np.array([1.0]))
    p, delta, tol = 6, 2e-3, 1e-8
    lv, cs = synth.resolve_tree(dens, 3, p, 1e-8, max_level=5)
    sig = synth.sample(lv, cs, p, dens)
    out = api.OutputTree(lv, cs, p, delta, tol, torch.from_numpy(sig).cuda(), coarsen=False)
    info = out.info
    _say(f"3d refine-only: {info}")
    assert _tiles(out.levels, out.coords) and synth.is_balanced_fast(out.levels, out.coords)
    assert info["deleted_coarsen"] == 0 and info["added_balance"] == 0
    assert info["nboxes"] == info["nboxes_in"] + info["added_refine"] + info["added_refine_balance"]
    e = _tail_errors(out.u.cpu().numpy(), p, 3)
    at_limit = out.levels >= lv.max()
    assert np.all((e <= info["threshold"] * (1 + 1e-6)) | at_limit)
    _check_parity(lv, cs, sig, p, delta, tol, out, False, 3, n=60)


def test_coarsen_only_2d_merges_an_over_resolved_tree():
    """A uniform level-6 tree under a smooth density: u is over-resolved and
    coarsening merges most of the tree; merged leaves carry the children's
    interpolant, which still matches the transform."""
    dens = synth.GaussianSum(np.array([[0.05, -0.1]]), np.array([0.2]), np.array([1.0]))
    p, delta, tol = 8, 1e-2, 1e-8
    lv, cs = synth.uniform_tree(2, 6)
    sig = synth.sample(lv, cs, p, dens)
    out = api.OutputTree(lv, cs, p, delta, tol, torch.from_numpy(sig).cuda(), refine=False)
    info = out.info
    _say(f"2d coarsen-only: {info}")
    assert info["passes"] == 1 and info["added_refine"] == 0
    assert info["nleaves"] < info["nleaves_in"] // 4
    assert _tiles(out.levels, out.coords) and synth.is_balanced_fast(out.levels, out.coords)
    assert info["nboxes"] == info["nboxes_in"] - info["deleted_coarsen"] + info["added_balance"]
    _check_parity(lv, cs, sig, p, delta, tol, out, False, 4)


@pytest.mark.parametrize("periodic", [False, True])
def test_refine_and_coarsen_2d(periodic):
    if periodic:
        dens = synth.GaussianSum(np.array([[0.47, -0.3], [-0.2, 0.49]]), np.array([0.01, 0.01]),
                                 np.array([1.0, -0.7]), periodic=True)
    else:
        dens = _two_peaks()
    p, delta, tol = 8, 4e-3, 1e-10
    lv, cs = synth.resolve_tree(dens, 2, p, 1e-10, max_level=10, min_level=3, periodic=periodic)
    sig = synth.sample(lv, cs, p, dens)
    out = api.OutputTree(lv, cs, p, delta, tol, torch.from_numpy(sig).cuda(), periodic=periodic)
    info = out.info
    _say(f"2d refine+coarsen periodic={periodic}: {info}")
    assert info["passes"] >= 2 and info["added_refine"] > 0 and info["deleted_coarsen"] > 0
    assert _tiles(out.levels, out.coords)
    assert synth.is_balanced_fast(out.levels, out.coords, periodic)
    assert info["nboxes"] == (info["nboxes_in"] + info["added_refine"] + info["added_refine_balance"]
                              - info["deleted_coarsen"] + info["added_balance"])
    _check_parity(lv, cs, sig, p, delta, tol, out, periodic, 5)


def test_section_4_2_example():
    """Two peaks with alpha = 1e-4, delta = 4e-3, k = 8, eps = 1e-12, u at 4M
    equispaced points (Section 4.2): interpolation from the input tree loses
    digits; the refined and coarsened output tree recovers them."""
    dens = _two_peaks()
    p, delta, eps = 8, 4e-3, 1e-12
    lv, cs = synth.resolve_tree(dens, 2, p, eps, max_level=12, min_level=3)
    sig = synth.sample(lv, cs, p, dens)
    s = torch.from_numpy(sig).cuda()
    u0 = api.Plan(lv, cs, p, delta, eps).execute(s)
    out = api.OutputTree(lv, cs, p, delta, eps, s)
    info = out.info
    g = (np.arange(2000) + 0.5) / 2000 - 0.5
    X = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    ref = cf.gaussian_sum_free(X, delta, dens)
    xt = torch.from_numpy(X).cuda()
    e0 = cf.rel_l2(api.interp(lv, cs, p, u0, xt).cpu().numpy(), ref)
    e1 = cf.rel_l2(out.interp(xt).cpu().numpy(), ref)
    _say(f"section 4.2: input tree {len(lv)} leaves / {info['nboxes_in']} boxes, interp error {e0:.2e}; "
         f"output tree {info['nleaves']} leaves / {info['nboxes']} boxes, interp error {e1:.2e}; "
         f"+{info['added_refine']} refine (+{info['added_refine_balance']} balance) "
         f"-{info['deleted_coarsen']} coarsen +{info['added_balance']} rebalance, passes {info['passes']}")
    assert e1 < 1e-10
    assert e0 > 100 * e1


def test_output_errors():
    lv, cs = synth.uniform_tree(2, 2)
    sig = torch.zeros((len(lv), 16), dtype=torch.float64, device="cuda")
    with pytest.raises(api.FgtError):
        api.OutputTree(lv, cs, 4, 1e-3, 1e-6, sig, eps=2.0)
    with pytest.raises(api.FgtError):
        api.OutputTree(lv[1:], cs[1:], 4, 1e-3, 1e-6, sig[1:])   # not a tiling
    with pytest.raises(api.FgtError):
        api.fgt_output_resolve(lv, cs, 4, 1e-3, 1e-6, None)
    # a zero density resolves to a zero potential on a coarsened tree
    out = api.OutputTree(lv, cs, 4, 1e-3, 1e-6, sig)
    assert torch.count_nonzero(out.u) == 0 and out.info["nleaves"] <= len(lv)
