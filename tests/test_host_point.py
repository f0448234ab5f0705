"""Host plan of the point transform (include/fgt_point.h), without a GPU.

Algorithm 1's tree: leaves tile the box, leaves above the cutoff level hold at
most n_s sources and n_s targets, the tree is level-restricted and a dense
cutoff-level leaf has no coarse neighbor.  Lists: every source-target pair
whose Gaussian is not negligible (closer than the cutoff-box side on every
axis) is summed exactly once -- by plane waves (target in a plane-wave box,
source in one of its dense colleagues) or directly (source leaf in the
target leaf's D-list) -- and no pair twice.  Proxy grids: every source of a
dense box and every target of a plane-wave box lies in the proxy box whose
point range holds it.
"""

import math

import numpy as np
import pytest

from paper_2305_07165_amd import api


def _clusters(d, n, rng, k=4, w=0.03):
    c = rng.uniform(-0.35, 0.35, (k, d))
    x = c[rng.integers(0, k, n)] + rng.normal(0, w, (n, d))
    return np.clip(x, -0.5, 0.5)


def _plan(d, ns, delta, tol, seed, p=12, nsrc=3000, ntgt=2500):
    rng = np.random.default_rng(seed)
    src = np.concatenate([_clusters(d, nsrc // 2, rng), rng.uniform(-0.5, 0.5, (nsrc - nsrc // 2, d))])
    tgt = np.concatenate([_clusters(d, ntgt // 2, rng), rng.uniform(-0.5, 0.5, (ntgt - ntgt // 2, d))])
    pl = api.PointPlan(src, tgt, delta, tol, p=p, ns=ns, host_only=True)
    return pl, src, tgt


def _boxes_touch(l1, c1, l2, c2):
    lo1, hi1 = c1 * 2.0 ** -l1, (c1 + 1) * 2.0 ** -l1
    lo2, hi2 = c2 * 2.0 ** -l2, (c2 + 1) * 2.0 ** -l2
    return bool(np.all((lo1 <= hi2 + 1e-15) & (lo2 <= hi1 + 1e-15)))


@pytest.mark.parametrize("d,ns,delta,seed", [(2, 20, 1e-3, 0), (3, 30, 2e-3, 1), (2, 5, 1e-4, 2), (3, 400, 1e-3, 3)])
def test_tree_lists_and_proxies(d, ns, delta, seed):
    tol = 1e-6
    pl, src, tgt = _plan(d, ns, delta, tol, seed)
    info = pl.info()
    lc, lp = info["lc"], info["lp"]
    lv = pl.array("leaf_level")
    cs = pl.array("leaf_coord").reshape(-1, d)
    dense = pl.array("leaf_dense").astype(bool)
    nleaf = len(lv)
    # tiling
    assert abs(np.sum(2.0 ** (-d * lv.astype(float))) - 1.0) < 1e-12
    assert lv.max() <= lc
    # points by leaf
    sperm, tperm = pl.array("src_perm"), pl.array("tgt_perm")
    ss, ts = pl.array("leaf_src_start"), pl.array("leaf_tgt_start")
    assert sorted(sperm) == list(range(len(src))) and sorted(tperm) == list(range(len(tgt)))
    sleaf = np.empty(len(src), int)
    tleaf = np.empty(len(tgt), int)
    for i in range(nleaf):
        sleaf[sperm[ss[i]:ss[i + 1]]] = i
        tleaf[tperm[ts[i]:ts[i + 1]]] = i
    for pts, leaf in ((src, sleaf), (tgt, tleaf)):
        cell = np.floor((pts + 0.5) * 2.0 ** lv[leaf][:, None]).astype(int)
        cell = np.minimum(cell, 2 ** lv[leaf][:, None] - 1)
        assert np.all(cell == cs[leaf])
    nsrc_leaf, ntgt_leaf = np.diff(ss), np.diff(ts)
    coarse = lv < lc
    assert np.all(nsrc_leaf[coarse] <= ns) and np.all(ntgt_leaf[coarse] <= ns)
    assert np.all(dense == ((lv == lc) & ((nsrc_leaf > ns) | (ntgt_leaf > ns))))
    # level restriction; no coarse neighbor of a dense leaf
    for i in range(nleaf):
        for j in range(i + 1, nleaf):
            if abs(int(lv[i]) - int(lv[j])) >= 1 and _boxes_touch(lv[i], cs[i], lv[j], cs[j]):
                assert abs(int(lv[i]) - int(lv[j])) == 1
                assert not dense[i] and not dense[j]
    # pairs: plane waves or direct, exactly once for every pair that matters
    pws, pwleaf = pl.array("pw_start"), pl.array("pwleaf_id")
    pst, psrc = pl.array("plist_start"), pl.array("plist_src")
    pxc = pl.array("px_coord").reshape(-1, d)
    # the leaf of every plane-wave box (a cutoff-level leaf holding its proxy boxes)
    box_leaf = []
    for a in range(len(pws) - 1):
        c = pxc[pwleaf[pws[a]]] >> (lp - lc)
        box_leaf.append(int(np.where((lv == lc) & np.all(cs == c, axis=1))[0][0]))
    box_leaf = np.array(box_leaf, int)
    leaf_box = {int(L): a for a, L in enumerate(box_leaf)}
    pw_pairs = set()
    for a in range(len(box_leaf)):
        for b in psrc[pst[a]:pst[a + 1]]:
            assert dense[box_leaf[b]]
            pw_pairs.add((int(box_leaf[a]), int(box_leaf[b])))
    dt, dst_, dsrc = pl.array("dl_tgt"), pl.array("dl_start"), pl.array("dl_src")
    hp = pl.array("dl_haspw")
    direct_pairs = set()
    for k in range(len(dt)):
        assert bool(hp[k]) == (int(dt[k]) in leaf_box)
        for S in dsrc[dst_[k]:dst_[k + 1]]:
            direct_pairs.add((int(dt[k]), int(S)))
    assert not (pw_pairs & direct_pairs)
    side = 2.0 ** -lc
    rng = np.random.default_rng(seed + 10)
    ti = rng.choice(len(tgt), min(400, len(tgt)), replace=False)
    for i in ti:
        near = np.where(np.all(np.abs(src - tgt[i]) < side, axis=1))[0]
        T = tleaf[i]
        for j in near:
            S = sleaf[j]
            by_pw = (int(T), int(S)) in pw_pairs
            by_direct = (int(T), int(S)) in direct_pairs
            assert by_pw != by_direct, (i, j, T, S)
    # proxy boxes hold their points
    psr, ptr = pl.array("px_src_start").reshape(-1, 2), pl.array("px_tgt_start").reshape(-1, 2)
    for x in range(len(pxc)):
        for (r0, r1), pts, perm in ((psr[x], src, sperm), (ptr[x], tgt, tperm)):
            if r1 > r0:
                cell = np.minimum(np.floor((pts[perm[r0:r1]] + 0.5) * 2 ** lp).astype(int), 2 ** lp - 1)
                assert np.all(cell == pxc[x])
    for a, L in enumerate(box_leaf):
        covered = sum(ptr[x][1] - ptr[x][0] for x in pwleaf[pws[a]:pws[a + 1]])
        assert covered == ntgt_leaf[L]
        if dense[L]:
            covered = sum(psr[x][1] - psr[x][0] for x in pwleaf[pws[a]:pws[a + 1]])
            assert covered == nsrc_leaf[L]
    assert info["proxy_err"] <= tol / (10 * d)


def test_proxy_level_deepens_with_tol_and_with_fewer_nodes():
    rng = np.random.default_rng(4)
    pts = rng.uniform(-0.5, 0.5, (500, 3))
    lp = {}
    for tol, p in ((1e-3, 16), (1e-6, 16), (1e-10, 16), (1e-6, 8)):
        pl = api.PointPlan(pts, pts, 1e-3, tol, p=p, ns=10, host_only=True)
        lp[(tol, p)] = pl.info()["lp"] - pl.info()["lc"]
    assert lp[(1e-3, 16)] <= lp[(1e-6, 16)] <= lp[(1e-10, 16)]
    assert lp[(1e-6, 8)] > lp[(1e-6, 16)]


def test_point_plan_errors():
    x = np.zeros((4, 3))
    with pytest.raises(api.FgtError):
        api.PointPlan(x + 0.6, x, 1e-3, 1e-6, host_only=True)  # outside the box
    with pytest.raises(api.FgtError):
        api.PointPlan(x, x, -1.0, 1e-6, host_only=True)
    with pytest.raises(api.FgtError):
        api.PointPlan(x, x, 1e-3, 1e-6, p=2, host_only=True)
    with pytest.raises(ValueError):
        api.PointPlan(np.zeros((4, 2)), x, 1e-3, 1e-6, host_only=True)
