"""GPU parity of the point transform with proxy grids (include/fgt_point.h)
against the oracle's direct sum of Eq. (pgt).

Bar: relative l2 error below tol over every target (or over a sampled set of
targets at the largest size, each computed by the oracle one by one), and the
largest error below tol times the largest |u|.  Cases mix clustered and
uniform points so that dense cutoff boxes (plane waves through proxy grids)
and sparse ones (direct) meet; the extremes are all-direct (n_s above every
box count), no sources, and no targets.
"""

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_2305_07165_amd import api, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-point] {msg}", flush=True)


def _clusters(d, n, rng, k=4, w=0.03):
    c = rng.uniform(-0.35, 0.35, (k, d))
    x = c[rng.integers(0, k, n)] + rng.normal(0, w, (n, d))
    return np.clip(x, -0.5, 0.5)


def _points(d, nsrc, ntgt, seed):
    rng = np.random.default_rng(seed)
    src = np.concatenate([_clusters(d, nsrc // 2, rng), rng.uniform(-0.5, 0.5, (nsrc - nsrc // 2, d))])
    tgt = np.concatenate([_clusters(d, ntgt // 2, rng), rng.uniform(-0.5, 0.5, (ntgt - ntgt // 2, d))])
    q = rng.uniform(-1, 1, nsrc)
    return src, tgt, q


CASES = [
    # name, d, nsrc, ntgt, delta, tol, p, ns, seed
    ("2d-mixed-1e-6", 2, 6000, 5000, 1e-3, 1e-6, 12, 20, 0),
    ("2d-mixed-p16-1e-6", 2, 6000, 5000, 1e-3, 1e-6, 16, 20, 1),
    ("2d-small-delta", 2, 8000, 4000, 1e-4, 1e-6, 16, 10, 2),
    ("2d-1e-10", 2, 5000, 5000, 1e-3, 1e-10, 16, 20, 3),
    ("3d-mixed-1e-6", 3, 20000, 8000, 2e-3, 1e-6, 16, 40, 4),
    ("3d-p10-1e-3", 3, 20000, 8000, 2e-3, 1e-3, 10, 40, 5),
    ("3d-small-delta", 3, 30000, 6000, 3e-4, 1e-6, 16, 30, 6),
    ("3d-all-direct", 3, 5000, 3000, 2e-3, 1e-6, 16, 100000, 7),
]


@pytest.mark.parametrize("name,d,nsrc,ntgt,delta,tol,p,ns,seed", CASES, ids=[c[0] for c in CASES])
def test_point_parity(name, d, nsrc, ntgt, delta, tol, p, ns, seed):
    src, tgt, q = _points(d, nsrc, ntgt, seed)
    pl = api.PointPlan(src, tgt, delta, tol, p=p, ns=ns)
    info = pl.info()
    _say(f"{name}: lc={info['lc']} lp={info['lp']} leaves={info['nleaves']} dense={info['ndense']} "
         f"pwboxes={info['npwbox']} proxies={info['nproxy']} translations={info['nplist']} "
         f"direct terms={info['ndirect_terms']}")
    u = pl.execute(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    ug = u.cpu().numpy()
    uo = oracle.oracle_point(src, q, tgt, delta)
    err, emax = cf.rel_l2(ug, uo), cf.max_rel(ug, uo)
    _say(f"{name}: rel_l2={err:.3e} max_rel={emax:.3e}")
    assert np.all(np.isfinite(ug))
    assert err < tol and emax < tol
    if name != "3d-all-direct":
        assert info["ndense"] > 0 and info["nplist"] > 0
    else:
        assert info["nproxy"] == 0
    # deterministic and linear
    u2 = pl.execute(torch.from_numpy(2.0 * q).cuda())
    u1 = pl.execute(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    assert torch.equal(u1, u)
    assert torch.allclose(u2, 2.0 * u1, rtol=1e-13, atol=0)
    pl.close()


def test_point_large_sampled():
    """The paper's first 3D point workload shape: 1,000,000 points on a sphere
    (each a source and a target), delta = 0.01, tol 1e-6; 2,000 targets
    checked one by one against the oracle's direct sum over every source."""
    x, q = synth.point_sphere(5, 1_000_000)
    pl = api.PointPlan(x, x, 0.01, 1e-6, p=16, ns=64)
    info = pl.info()
    _say(f"sphere: lc={info['lc']} lp={info['lp']} dense={info['ndense']} proxies={info['nproxy']} "
         f"direct terms={info['ndirect_terms']}")
    u = pl.execute(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    ug = u.cpu().numpy()
    pick = np.random.default_rng(12).choice(len(x), 2000, replace=False)
    uo = oracle.oracle_point(x, q, x[pick], 0.01)
    err = float(np.linalg.norm(ug[pick] - uo) / np.linalg.norm(uo))
    emax = float(np.max(np.abs(ug[pick] - uo)) / np.max(np.abs(uo)))
    _say(f"sphere: sampled rel_l2={err:.3e} max_rel={emax:.3e}")
    assert err < 1e-6 and emax < 1e-6
    pl.close()


def test_point_degenerate_inputs():
    rng = np.random.default_rng(13)
    x = rng.uniform(-0.5, 0.5, (100, 2))
    # no sources: u = 0
    pl = api.PointPlan(np.zeros((0, 2)), x, 1e-3, 1e-6, p=12, ns=4)
    u = pl.execute(torch.zeros(0, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.count_nonzero(u).item() == 0
    pl.close()
    # no targets: nothing to write
    pl = api.PointPlan(x, np.zeros((0, 2)), 1e-3, 1e-6, p=12, ns=4)
    u = pl.execute(torch.from_numpy(rng.uniform(-1, 1, 100)).cuda())
    torch.cuda.synchronize()
    assert u.numel() == 0
    pl.close()
    # a single source and target on the box's corner
    s = np.array([[0.5, 0.5]])
    t = np.array([[0.5, 0.49]])
    pl = api.PointPlan(s, t, 1e-3, 1e-10, p=12, ns=1)
    u = pl.execute(torch.ones(1, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert abs(u[0] - np.exp(-1e-4 / 1e-3)) < 1e-12
    pl.close()
