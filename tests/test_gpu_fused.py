"""The fused 3D translation (target groups, tile-major phi; stage_bodies.h
transeval3) against the pair of kernels it replaces (plain translation, then
the first evaluation step), plan option no_fuse, on the same plan and input.

Both compute psi_A = sum over the P-list of Rot(c_B - c_A) phi_B and then
Z_P = E3_P psi_A; they differ only in the association of the sums, so the
results agree to FP64 rounding (1e-12 relative to max|u|), far inside the
transform's tol: a source missing from a group, a wrong direction or a wrong
tile offset would show at the size of that term, not hidden by tol.  The trees
are large enough that the plan fuses (psi above 128 MB).
"""

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_2305_07165_amd import api, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-fused] {msg}", flush=True)


def _two_level_tree(seed, frac):
    """Level-4 boxes of the unit cube, a random fraction split into their eight
    level-5 children (2:1 balanced)."""
    rng = np.random.default_rng(seed)
    lv, cs = [], []
    for c in np.ndindex(16, 16, 16):
        if rng.random() < frac:
            for ch in np.ndindex(2, 2, 2):
                lv.append(5)
                cs.append([2 * c[0] + ch[0], 2 * c[1] + ch[1], 2 * c[2] + ch[2]])
        else:
            lv.append(4)
            cs.append(list(c))
    return np.array(lv, np.int32), np.array(cs, np.int32)


def _pair(lv, cs, p, delta, tol, sig, periodic=False):
    s = torch.from_numpy(np.ascontiguousarray(sig)).cuda()
    out = []
    for no_fuse in (False, True):
        pl = api.Plan(lv, cs, p, delta, tol, periodic=periodic, no_fuse=no_fuse)
        info = pl.info()
        assert info["fused_translate"] == (0 if no_fuse else 1)
        u = pl.execute(s)
        torch.cuda.synchronize()
        pl.sync()
        out.append(u.cpu().numpy())
        pl.close()
    return out


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_fused_equals_unfused_benchmark_tree(tol):
    pr = synth.adaptive_3d(0)
    uf, uu = _pair(pr.levels, pr.coords, pr.p, pr.delta, tol, pr.sigma)
    d = float(np.max(np.abs(uf - uu)) / np.max(np.abs(uu)))
    _say(f"benchmark tree tol={tol}: fused vs unfused max rel {d:.2e}")
    assert np.all(np.isfinite(uf)) and d < 1e-12


@pytest.mark.parametrize("periodic", [False, True])
def test_fused_equals_unfused_two_level_tree(periodic):
    lv, cs = _two_level_tree(11, 0.05)
    p = 4
    dens = synth.GaussianSum(np.array([[0.1, -0.2, 0.3], [-0.25, 0.15, -0.1], [0.3, 0.3, -0.3]]),
                             np.array([0.03, 0.05, 0.02]), np.array([1.0, -0.7, 0.4]),
                             periodic=periodic)
    sig = synth.sample(lv, cs, p, dens)
    uf, uu = _pair(lv, cs, p, 1e-4, 1e-6, sig, periodic=periodic)
    d = float(np.max(np.abs(uf - uu)) / np.max(np.abs(uu)))
    _say(f"two-level tree periodic={periodic}: {len(lv)} leaves, fused vs unfused max rel {d:.2e}")
    assert np.all(np.isfinite(uf)) and d < 1e-12
    # and both against the oracle on a sample of leaves
    pick = np.random.default_rng(3).choice(len(lv), 64, replace=False)
    uo = oracle.oracle_u(lv, cs, p, 1e-4, sig, periodic=periodic, targets=pick)
    err = cf.rel_l2(uf.reshape(len(lv), -1)[pick], uo.reshape(len(pick), -1))
    _say(f"two-level tree periodic={periodic}: sampled rel_l2 vs oracle {err:.2e}")
    assert err < 1e-6
