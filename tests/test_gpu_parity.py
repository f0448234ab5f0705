"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: relative l2 error over all returned nodes below the requested tol
(the accuracy the method promises, Theorem 1 applied in Algorithm 4), and the
largest pointwise error below tol times the largest |u|.  For FP64 plans the
device result must also equal the test-only numpy walk of the same host plan
to rounding (1e-12 relative): the kernels implement exactly the stages the
plan describes.  The full-size cases compare every node of the benchmark tree.
"""

import numpy as np
import pytest

import closed_forms as cf
import host_exec
import oracle
from paper_2305_07165_amd import api, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


def _run(lv, cs, p, delta, tol, sig, periodic=False, precision="fp64", force_lc=-1,
         eps_internal=0.0):
    pl = api.Plan(lv, cs, p, delta, tol, periodic=periodic, precision=precision,
                  force_lc=force_lc, eps_internal=eps_internal)
    s = torch.from_numpy(np.ascontiguousarray(sig)).cuda()
    u = pl.execute(s)
    torch.cuda.synchronize()
    pl.sync()
    return u.cpu().numpy(), pl


def _adaptive_2d(periodic=False, p=8, widths=(0.01, 0.03), maxl=8):
    c = [[0.46, -0.17], [-0.2, 0.49]] if periodic else [[0.11, -0.17], [-0.2, 0.05]]
    dens = synth.GaussianSum(np.array(c), np.array(widths), np.array([0.7, -0.4]),
                             periodic=periodic)
    lv, cs = synth.resolve_tree(dens, 2, p, 1e-10, max_level=maxl, periodic=periodic)
    return lv, cs, synth.sample(lv, cs, p, dens)


def _adaptive_3d(periodic=False, p=6, maxl=5):
    dens = synth.GaussianSum(np.array([[0.1, -0.12, 0.05], [-0.3, 0.2, 0.1]]),
                             np.array([0.02, 0.05]), np.array([1.0, -0.6]))
    lv, cs = synth.resolve_tree(dens, 3, p, 1e-8, max_level=maxl, periodic=periodic)
    return lv, cs, synth.sample(lv, cs, p, dens)


def _adaptive_1d_periodic():
    dens = synth.GaussianSum(np.array([[0.47]]), np.array([0.01]), np.array([1.0]), periodic=True)
    lv, cs = synth.resolve_tree(dens, 1, 9, 1e-12, max_level=9, periodic=True)
    return lv, cs, synth.sample(lv, cs, 9, dens)


CASES = [
    # name, builder, p, delta, tol, periodic, force_lc
    ("2d-uniform-direct", lambda: (synth.small_2d(0).levels, synth.small_2d(0).coords, synth.small_2d(0).sigma), 8, 1e-3, 1e-6, False, -1),
    ("2d-uniform-pw-lc2", lambda: (synth.small_2d(0).levels, synth.small_2d(0).coords, synth.small_2d(0).sigma), 8, 1e-3, 1e-6, False, 2),
    ("2d-uniform-pw-lc1", lambda: (synth.small_2d(0).levels, synth.small_2d(0).coords, synth.small_2d(0).sigma), 8, 1e-3, 1e-6, False, 1),
    ("2d-adaptive-free-1e-6", lambda: _adaptive_2d(False), 8, 1e-3, 1e-6, False, -1),
    ("2d-adaptive-free-1e-10", lambda: _adaptive_2d(False), 8, 1e-4, 1e-10, False, -1),
    ("2d-adaptive-periodic-1e-6", lambda: _adaptive_2d(True), 8, 1e-3, 1e-6, True, -1),
    ("2d-adaptive-periodic-1e-10", lambda: _adaptive_2d(True), 8, 1e-4, 1e-10, True, -1),
    ("2d-adaptive-p5-ragged", lambda: _adaptive_2d(False, p=5, widths=(0.02, 0.04), maxl=7), 5, 2e-3, 1e-8, False, -1),
    ("2d-adaptive-p16", lambda: _adaptive_2d(False, p=16, widths=(0.01, 0.03), maxl=7), 16, 1e-3, 1e-10, False, -1),
    ("3d-adaptive-free-p6", lambda: _adaptive_3d(False), 6, 1e-3, 1e-6, False, -1),
    ("3d-adaptive-periodic-p6", lambda: _adaptive_3d(True), 6, 1e-3, 1e-6, True, -1),
    ("3d-adaptive-free-p6-1e-10", lambda: _adaptive_3d(False), 6, 1e-3, 1e-10, False, -1),
    ("3d-adaptive-free-p16", lambda: _adaptive_3d(False, p=16, maxl=4), 16, 1e-3, 1e-10, False, -1),
    # periodic with cutoff level <= 1: the root Fourier series (automatic or forced)
    ("2d-periodic-fourier", lambda: _adaptive_2d(True), 8, 0.05, 1e-6, True, -1),
    ("2d-periodic-fourier-forced", lambda: _adaptive_2d(True), 8, 2e-3, 1e-8, True, 0),
    ("3d-periodic-fourier", lambda: _adaptive_3d(True, maxl=4), 6, 0.02, 1e-6, True, -1),
    ("3d-periodic-fourier-forced", lambda: _adaptive_3d(True), 6, 4e-3, 1e-6, True, 1),
    ("1d-periodic-fourier", lambda: _adaptive_1d_periodic(), 9, 0.2, 1e-10, True, -1),
    ("1d-adaptive", lambda: (lambda t: (t[0], t[1], synth.sample(t[0], t[1], 9, synth.GaussianSum(np.array([[0.13]]), np.array([0.01]), np.array([1.0])))))(synth.resolve_tree(synth.GaussianSum(np.array([[0.13]]), np.array([0.01]), np.array([1.0])), 1, 9, 1e-12, max_level=9)), 9, 1e-4, 1e-10, False, -1),
]


@pytest.mark.parametrize("name,build,p,delta,tol,periodic,force_lc", CASES, ids=[c[0] for c in CASES])
def test_parity_fp64(name, build, p, delta, tol, periodic, force_lc):
    lv, cs, sig = build()
    _say(f"{name}: nleaves={len(lv)} p={p} delta={delta} tol={tol} periodic={periodic} force_lc={force_lc}")
    uo = oracle.oracle_u(lv, cs, p, delta, sig, periodic=periodic)
    ug, pl = _run(lv, cs, p, delta, tol, sig, periodic=periodic, force_lc=force_lc)
    info = pl.info()
    err, emax = cf.rel_l2(ug, uo), cf.max_rel(ug, uo)
    _say(f"{name}: lc={info['lc']} nr={info['nr']} pwleaves={info['n_pwleaf']} near={info['n_near_pair']} "
         f"rel_l2={err:.3e} max_rel={emax:.3e}")
    assert np.all(np.isfinite(ug))
    assert err < tol
    assert emax < tol
    hp = api.Plan(lv, cs, p, delta, tol, periodic=periodic, force_lc=force_lc, host_only=True)
    uh = host_exec.run(hp, sig)
    assert cf.rel_l2(ug, uh) < 1e-12


@pytest.mark.parametrize("tol", [1e-3, 1e-6])
@pytest.mark.parametrize("shape", ["2d", "3d"])
def test_parity_fp32(shape, tol):
    if shape == "2d":
        lv, cs, sig = _adaptive_2d(False)
        p, delta = 8, 1e-3
    else:
        lv, cs, sig = _adaptive_3d(False)
        p, delta = 6, 1e-3
    _say(f"fp32 {shape} tol={tol}")
    uo = oracle.oracle_u(lv, cs, p, delta, sig)
    ug, _ = _run(lv, cs, p, delta, tol, sig, precision="fp32")
    err, emax = cf.rel_l2(ug, uo), cf.max_rel(ug, uo)
    _say(f"fp32 {shape} tol={tol}: rel_l2={err:.3e} max_rel={emax:.3e}")
    assert err < tol
    assert emax < tol


@pytest.mark.parametrize("tol", [1e-3, 1e-4])
@pytest.mark.parametrize("shape", ["2d", "3d"])
def test_parity_bf16x3(shape, tol):
    """Split bf16 products carry about 1e-5 relative error each; fgt_plan
    accepts them from tol 1e-4 (the smallest tol they meet), and below it
    refuses the plan."""
    if shape == "2d":
        lv, cs, sig = _adaptive_2d(False)
        p, delta = 8, 1e-3
    else:
        lv, cs, sig = _adaptive_3d(False)
        p, delta = 6, 1e-3
    uo = oracle.oracle_u(lv, cs, p, delta, sig)
    ug, _ = _run(lv, cs, p, delta, tol, sig, precision="bf16x3")
    assert np.all(np.isfinite(ug))
    err, emax = cf.rel_l2(ug, uo), cf.max_rel(ug, uo)
    _say(f"bf16x3 {shape} tol={tol}: rel_l2={err:.3e} max_rel={emax:.3e}")
    assert err < tol
    assert emax < tol
    with pytest.raises(api.FgtError) as ei:
        api.Plan(lv, cs, p, delta, 1e-6, precision="bf16x3")
    assert ei.value.code == api.FGT_ERR_UNSUPPORTED


def test_bf16x3_rejected_in_1d():
    lv = np.array([1, 1], dtype=np.int32)
    cs = np.array([[0], [1]], dtype=np.int32)
    with pytest.raises(api.FgtError):
        api.Plan(lv, cs, 8, 1e-3, 1e-3, precision="bf16x3")


def test_deterministic_and_reusable():
    lv, cs, sig = _adaptive_2d(False)
    pl = api.Plan(lv, cs, 8, 1e-3, 1e-6)
    s = torch.from_numpy(sig).cuda()
    u1 = pl.execute(s).clone()
    u2 = pl.execute(s)
    s2 = 2.0 * s
    u3 = pl.execute(s2)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    assert torch.allclose(u3, 2.0 * u1, rtol=1e-13, atol=0)


def test_single_leaf_root():
    lv = np.array([0], dtype=np.int32)
    cs = np.zeros((1, 2), dtype=np.int32)
    sig = np.ones((1, 64))
    uo = oracle.oracle_u(lv, cs, 8, 0.02, sig)
    ug, _ = _run(lv, cs, 8, 0.02, 1e-8, sig)
    assert cf.rel_l2(ug, uo) < 1e-8
    x = synth.leaf_points(lv, cs, 8)
    assert cf.rel_l2(ug, cf.const_free(x, 0.02)) < 1e-8
    # periodic, large delta: the root Fourier series; sigma = 1 gives (pi delta)^(d/2)
    ug, pl = _run(lv, cs, 8, 0.1, 1e-10, sig, periodic=True)
    assert pl.info()["fourier"] == 1
    assert np.max(np.abs(ug / (np.pi * 0.1) - 1.0)) < 1e-10


def test_errors_surface():
    lv = np.array([1, 1, 1, 2, 2, 2, 2, 2], dtype=np.int32)  # not a tiling
    cs = np.array([[1, 0], [0, 1], [1, 1], [0, 0], [1, 0], [0, 1], [1, 1], [1, 1]], dtype=np.int32)
    with pytest.raises(api.FgtError):
        api.Plan(lv, cs, 4, 1e-3, 1e-6)


# ---------------------------------------------------------------------------
# full size: the benchmark's 3D adaptive tree (2,661 leaves, N = 10,899,456;
# periodic variant 3,613 leaves, N = 14,798,848) in the launch configuration
# bench.py times, compared with the oracle at every node of every leaf.  The
# oracle of one (tree, delta) is computed once and shared by the cases.

_FULL = {}
_ORACLE = {}


def _full(periodic):
    if periodic not in _FULL:
        _FULL[periodic] = synth.adaptive_3d(0, periodic=periodic, wrap_blobs=periodic)
    return _FULL[periodic]


def _full_oracle(periodic, delta):
    key = (periodic, delta)
    if key not in _ORACLE:
        pr = _full(periodic)
        _ORACLE[key] = oracle.oracle_u(pr.levels, pr.coords, pr.p, delta, pr.sigma, periodic=periodic)
    return _ORACLE[key]


@pytest.mark.parametrize("periodic,tol,precision", [(False, 1e-6, "fp64"), (False, 1e-10, "fp64"),
                                                     (False, 1e-6, "fp32"), (True, 1e-6, "fp64"),
                                                     (True, 1e-10, "fp64")])
def test_full_size_3d_whole_tree(periodic, tol, precision):
    pr = _full(periodic)
    _say(f"full-size periodic={periodic} tol={tol} {precision}: N={pr.npoints} leaves={len(pr.levels)}")
    uo = _full_oracle(periodic, pr.delta)
    ug, pl = _run(pr.levels, pr.coords, pr.p, pr.delta, tol, pr.sigma, periodic=periodic,
                  precision=precision)
    err, emax = cf.rel_l2(ug, uo), cf.max_rel(ug, uo)
    _say(f"full-size: lc={pl.info()['lc']} nr={pl.info()['nr']} rel_l2={err:.3e} max_rel={emax:.3e}")
    assert np.all(np.isfinite(ug))
    assert err < tol
    assert emax < tol


# the precision workload: the same tree at delta = 1e-3 and 1e-5, FP32 and
# split bf16 products at every tol fgt_plan accepts for them (FP32 from 1e-6,
# BF16x3 from 1e-4), against the oracle at every node
@pytest.mark.parametrize("delta,tol,precision", [(1e-3, 1e-3, "fp32"), (1e-3, 1e-6, "fp32"),
                                                 (1e-5, 1e-3, "fp32"), (1e-5, 1e-6, "fp32"),
                                                 (1e-3, 1e-3, "bf16x3"), (1e-5, 1e-3, "bf16x3"),
                                                 (1e-3, 1e-4, "bf16x3"), (1e-5, 1e-4, "bf16x3")])
def test_full_size_3d_precision(delta, tol, precision):
    pr = _full(False)
    _say(f"precision delta={delta} tol={tol} {precision}: whole tree")
    uo = _full_oracle(False, delta)
    ug, pl = _run(pr.levels, pr.coords, pr.p, delta, tol, pr.sigma, precision=precision)
    err, emax = cf.rel_l2(ug, uo), cf.max_rel(ug, uo)
    _say(f"precision: lc={pl.info()['lc']} nr={pl.info()['nr']} rel_l2={err:.3e} max_rel={emax:.3e}")
    assert np.all(np.isfinite(ug))
    assert err < tol
    assert emax < tol
