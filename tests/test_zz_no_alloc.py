"""fgt_execute_noalloc through the C ABI: the same transform as fgt_execute,
with the workspace taken from the library's static device scratch.

Two calls in a row on different plans, the second with a smaller input (the
scratch keeps the first call's contents), each checked bitwise against
fgt_execute of the same plan and against the FP64 oracle within the plan's
tol; then a third call back on the first plan; and a plan whose workspace
exceeds the scratch is refused before anything is enqueued.
"""

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_2305_07165_amd import api, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[no-alloc] {msg}", flush=True)


def _tree_3d(maxl):
    dens = synth.GaussianSum(np.array([[0.1, -0.12, 0.05], [-0.3, 0.2, 0.1]]),
                             np.array([0.02, 0.05]), np.array([1.0, -0.6]))
    lv, cs = synth.resolve_tree(dens, 3, 6, 1e-8, max_level=maxl)
    return lv, cs, synth.sample(lv, cs, 6, dens)


def _case(lv, cs, p, delta, tol, sig, force_lc=-1):
    pl = api.Plan(lv, cs, p, delta, tol, force_lc=force_lc)
    s = torch.from_numpy(np.ascontiguousarray(sig)).cuda()
    ref = pl.execute(s)
    torch.cuda.synchronize()
    uo = oracle.oracle_u(lv, cs, p, delta, sig)
    return pl, s, ref.clone(), uo


def _check(name, pl, s, ref, uo, tol):
    u = torch.full_like(s, float("nan"))
    pl.execute_noalloc(s, u)
    pl.sync()
    torch.cuda.synchronize()
    ug = u.cpu().numpy()
    err, emax = cf.rel_l2(ug, uo), cf.max_rel(ug, uo)
    _say(f"{name}: rel_l2={err:.3e} max_rel={emax:.3e} bitwise={torch.equal(u, ref)}")
    assert torch.equal(u, ref)
    assert err < tol and emax < tol


def test_noalloc_matches_execute_two_calls_second_smaller():
    # first call: a 3D tree with plane waves and a near field (about 30 MB of
    # workspace); second: the 64-leaf 2D tree with every pair by plane waves
    lv, cs, sig = _tree_3d(4)
    _say(f"3d: {len(lv)} leaves, p=6, delta=4e-3, tol 1e-6")
    big = _case(lv, cs, 6, 4e-3, 1e-6, sig)
    info = big[0].info()
    assert info["n_pwleaf"] > 0 and info["n_near_pair"] > 0
    pr = synth.small_2d(0)
    _say("2d: 64 leaves, p=8, delta=1e-3, tol 1e-6, cutoff level forced to 2")
    small = _case(pr.levels, pr.coords, pr.p, pr.delta, pr.tol, pr.sigma, force_lc=2)
    assert small[1].numel() < big[1].numel()
    _check("call 1 (3d)", *big, 1e-6)
    _check("call 2 (2d, smaller)", *small, pr.tol)
    _check("call 3 (3d again)", *big, 1e-6)
    for pl in (big[0], small[0]):
        pl.close()


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    lv, cs, sig = _tree_3d(5)
    pl = api.Plan(lv, cs, 6, 1e-3, 1e-6)
    assert pl.info()["device_bytes"] > 64 << 20
    s = torch.from_numpy(sig).cuda()
    u = torch.full_like(s, float("nan"))
    with pytest.raises(api.FgtError) as ei:
        pl.execute_noalloc(s, u)
    assert ei.value.code == api.FGT_ERR_UNSUPPORTED
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.isnan(u).all()  # nothing was enqueued
    pl.close()
