"""CPU tests of the host side of the C ABI: parameters, tables and lists.

No device is touched: plans are built with host_only=1 and inspected through
fgt_plan_array.  Expected values come from the paper's Tables 1 and 2
(tests/golden), from the paper's closed forms for the Gaussian-Legendre
integrals, from independent scipy quadrature, and from the oracle.
"""

import ctypes
import math
import os
import re

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import integrate
from scipy.special import erf

import closed_forms as cf
import host_exec
import oracle
from paper_2305_07165_amd import _lib, api, synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _golden(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


def _plan(lv, cs, p, delta, tol, **kw):
    return api.Plan(lv, cs, p, delta, tol, host_only=True, **kw)


# ---------------------------------------------------------------------------
# the library and its declared symbols


def test_library_exports_every_declared_symbol():
    declared = set()
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            header = open(os.path.join(ROOT, "include", name)).read()
            # function declarations: a name followed by "(" outside comments
            code = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
            declared |= set(re.findall(r"\b(fgt_[a-z_]+)\s*\(", code))
    assert "fgt_server_submit" in declared
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert declared == set(_lib.EXPORTED)


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library the transform raises; there is no fallback."""
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(HERE, "no_such_dir", "libfgt.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    lv, cs = synth.uniform_tree(2, 1)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        api.Plan(lv, cs, 4, 1e-2, 1e-6, host_only=True)


def test_product_package_does_not_use_the_oracle():
    """The oracle is test infrastructure: nothing in the package imports,
    loads or links it."""
    pkg = os.path.join(ROOT, "paper_2305_07165_amd")
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle)|oracle\.c|liboracle|oracle/", re.M)
    hits = []
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                if pat.search(open(os.path.join(dirpath, f), errors="replace").read()):
                    hits.append(f)
    assert not hits, hits


# ---------------------------------------------------------------------------
# Theorem 1 and Tables 1-2


def test_table1_plane_wave_counts():
    for eps, d0, n2, n3, n4 in _golden("table1.txt"):
        assert round(math.sqrt(math.log(3.0 / eps)), 2) == pytest.approx(d0, abs=1e-9)
        assert [api.fgt_pw_terms(eps, r) for r in (2.0, 3.0, 4.0)] == [n2, n3, n4]


def test_table2_periodic_terms():
    epss = [1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12]
    for row in _golden("table2.txt"):
        delta, counts = row[0], row[1:]
        assert [api.fgt_periodic_terms(e, delta) for e in epss] == counts


def test_table2_through_the_periodic_plan():
    """A periodic plan with cutoff level <= 1 uses n_p Fourier terms per side
    (Table 2): 2 n_p + 1 real modes, one root box, one translation (the
    identity) and no near field.  The automatic cutoff level reaches that
    route for large deltas; a forced level 0 reaches it for any."""
    lv, cs = synth.uniform_tree(2, 2)
    epss = [1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12]
    for row in _golden("table2.txt"):
        delta, counts = row[0], row[1:]
        for eps, n_p in zip(epss, counts):
            for flc in (0, -1):
                info = _plan(lv, cs, 4, delta, eps, periodic=True, force_lc=flc).info()
                if flc == -1 and info["fourier"] == 0:
                    assert info["lc"] >= 2  # the image-layer form
                    continue
                assert info["fourier"] == 1 and info["lc"] == 0
                assert info["nr"] == 2 * n_p + 1 and info["nf"] == 2 * (n_p + 1)
                assert info["n_pwbox"] == 1 and info["n_plist"] == 1
                assert info["n_near_target"] == 0 and info["n_pwleaf"] == len(lv)
                assert info["h"] == pytest.approx(2 * math.pi * math.sqrt(delta), rel=1e-15)
    # free space with the same deltas keeps Theorem 1's modes
    assert _plan(lv, cs, 4, 0.1, 1e-6).info()["fourier"] == 0


def test_fourier_modes_bound_the_image_sum():
    """The plan's Fourier modes (weights of Theorem 1 at h = 2 pi sqrt(delta))
    reproduce the image sum of the periodic kernel (Eq. (gper_kernel)) to eps
    on a whole period; the two agree by Poisson summation."""
    lv, cs = synth.uniform_tree(1, 3)
    for delta in (0.3, 0.1, 1e-2, 1e-3):
        for eps in (1e-2, 1e-6, 1e-12):
            info = _plan(lv, cs, 4, delta, eps, periodic=True, force_lc=0).info()
            h, M = info["h"], (info["nr"] + 1) // 2
            x = np.linspace(-1.0, 1.0, 4001)
            j = np.arange(-40, 41)
            img = np.sum(np.exp(-(x[:, None] - j[None, :]) ** 2 / delta), 1)
            m = np.arange(1, M)
            w = h / (2 * math.sqrt(math.pi)) * np.exp(-(m * h) ** 2 / 4)
            ser = h / (2 * math.sqrt(math.pi)) + 2 * np.cos(np.outer(x, m * h / math.sqrt(delta))) @ w
            assert np.max(np.abs(ser - img)) <= eps


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10])
@pytest.mark.parametrize("delta", [1e-3, 3e-4, 1e-4])
def test_theorem1_bound_with_plan_modes(tol, delta):
    """The plan's modes (symmetric truncation |m| <= M-1, real form) keep the
    Theorem 1 bound |G(x) - PW(x)| <= eps for |x| <= R sqrt(delta)."""
    lv, cs = synth.uniform_tree(2, 5)
    info = _plan(lv, cs, 4, delta, tol).info()
    eps, h, R, M = info["eps"], info["h"], info["R"], (info["nr"] + 1) // 2
    assert info["nf"] == 2 * M
    x = np.linspace(-R, R, 20001)  # units of sqrt(delta)
    m = np.arange(1, M)
    w0 = h / (2 * math.sqrt(math.pi))
    pw = w0 + 2 * w0 * np.sum(np.exp(-(m[:, None] * h) ** 2 / 4) * np.cos(np.outer(m * h, x)), 0)
    err = np.max(np.abs(np.exp(-x * x) - pw))
    assert err <= eps
    # cutoff level: boxes of side >= D0 sqrt(delta), the finest such level
    L = 2.0 ** -info["lc"]
    assert L >= info["D0"] * math.sqrt(delta) > L / 2
    assert 2 * info["D0"] <= R < 4 * info["D0"] + 1e-12


# ---------------------------------------------------------------------------
# near-field tables


def _paper_J(nmax, t, lam):
    """J^paper_n(t), n < nmax, from the closed forms for n <= 3 and the
    five-term recurrence (Eq. (Jnrecurrence)), with the factor lambda that the
    printed closed forms omit restored by the caller (J = lambda * J^paper)."""
    a, b = (-1 - t) / lam, (1 - t) / lam
    d1 = lam * (math.exp(-b * b) - math.exp(-a * a))
    d2 = lam * (math.exp(-b * b) + math.exp(-a * a))
    J = [0.0] * max(nmax, 4)
    J[0] = 0.5 * math.sqrt(math.pi) * (erf(b) - erf(a))
    J[1] = -0.5 * d1 + t * J[0]
    J[2] = 0.75 * (-d2 - t * d1 + (lam ** 2 - 2.0 / 3 + 2 * t * t) * J[0])
    J[3] = 0.625 * (-d1 + 2 * t * (4 * J[2] - J[0]) / 3 - (0.4 - 4 * lam ** 2) * J[1])
    for n in range(2, nmax - 2):
        J[n + 2] = ((2 * n + 3) / (n + 2)) * (
            t * (J[n + 1] - J[n - 1]) + (n - 1) / (2 * n - 1) * J[n - 2]
            + (2 * n + 1) * (lam ** 2 / 2 + 1.0 / ((2 * n + 3) * (2 * n - 1))) * J[n])
    return np.array(J[:nmax])


_REL = {0: -1.0, 1: 0.0, 2: 1.0, 3: -0.75, 4: -0.25, 5: 0.25, 6: 0.75,
        7: -1.5, 8: -0.5, 9: 0.5, 10: 1.5}


def _near_tables(p, delta, lv, cs):
    pl = _plan(lv, cs, p, delta, 1e-10)
    V = pl.array("V").reshape(-1, p, p)
    meta = pl.array("vtab_meta").reshape(2, -1)
    return V, meta


def test_near_tables_match_paper_closed_forms():
    """sum_j V[i][j] P_n(eta_j) = (L/2) lambda J^paper_n(t_i) with
    lambda = 2 sqrt(delta)/L (the garbled lambda = 2 delta/L read as
    2 sqrt(delta)/L, and the printed closed forms multiplied by lambda)."""
    p, delta = 8, 1e-6
    lv, cs = synth.point_refined_tree(2, [0.3, -0.2], 3)  # leaves at levels 1..3, all direct
    V, meta = _near_tables(p, delta, lv, cs)
    eta = npleg.leggauss(p)[0]
    Pn = np.stack([npleg.legval(eta, np.eye(p)[n]) for n in range(p)], 1)  # [j][n]
    checked = 0
    for tid in range(V.shape[0]):
        lev, ty = int(meta[0, tid]), int(meta[1, tid])
        LS = 2.0 ** -lev
        LT = LS if ty < 3 else (LS / 2 if ty < 7 else 2 * LS)
        lam = 2 * math.sqrt(delta) / LS
        if lam > 1.0 / 16:
            continue  # the recurrence is only stable for small lambda
        tpot = V[tid] @ Pn
        for i in range(p):
            xi = _REL[ty] * LS + 0.5 * LT * eta[i]
            ref = 0.5 * LS * lam * _paper_J(p, 2 * xi / LS, lam)
            assert np.max(np.abs(tpot[i] - ref)) < 1e-14 * math.sqrt(math.pi * delta)
        checked += 1
    assert checked >= 5


def test_near_tables_match_quadrature():
    p, delta = 6, 2e-3
    lv, cs = synth.point_refined_tree(2, [0.1, 0.1], 3)
    V, meta = _near_tables(p, delta, lv, cs)
    eta = npleg.leggauss(p)[0]

    def lagrange(j, t):
        return np.prod([(t - eta[m]) / (eta[j] - eta[m]) for m in range(p) if m != j])

    for tid in range(V.shape[0]):
        lev, ty = int(meta[0, tid]), int(meta[1, tid])
        LS = 2.0 ** -lev
        LT = LS if ty < 3 else (LS / 2 if ty < 7 else 2 * LS)
        for i in (0, p // 2, p - 1):
            xi = _REL[ty] * LS + 0.5 * LT * eta[i]
            for j in (0, p - 1):
                ref, _ = integrate.quad(
                    lambda y: math.exp(-(xi - y) ** 2 / delta) * lagrange(j, 2 * y / LS),
                    -LS / 2, LS / 2, points=[min(max(xi, -LS / 2), LS / 2)],
                    epsabs=1e-15, epsrel=1e-13, limit=200)
                assert abs(V[tid, i, j] - ref) < 1e-13


# ---------------------------------------------------------------------------
# formation / evaluation tables and the rotations


def test_form_eval_tables_reproduce_the_1d_kernel():
    """E_T F_S (same cutoff box) and E_T' Rot F_S (colleague box) give the 1D
    integral int_S G(x_i - y) l_j(y) dy to the plane-wave tolerance."""
    p, delta, tol = 8, 1e-3, 1e-8
    lv, cs = synth.uniform_tree(1, 4)  # 1D, level-4 leaves
    pl = _plan(lv, cs, p, delta, tol, force_lc=2)
    info = pl.info()
    nr, M = info["nr_stored"], (info["nr"] + 1) // 2
    assert nr == 2 * M
    F = pl.array("F").reshape(-1, nr, p)
    E = pl.array("E").reshape(-1, p, nr)
    # the stored zero slot of mode 0
    assert np.all(F[:, 1, :] == 0.0) and np.all(E[:, :, 1] == 0.0)
    rot = pl.array("rot").reshape(M, 2)
    meta = pl.array("ftab_meta").reshape(2, -1)
    tid = {(int(meta[0, k]), int(meta[1, k])): k for k in range(meta.shape[1])}
    eta = npleg.leggauss(p)[0]
    L, Lc = 2.0 ** -4, 2.0 ** -2
    Vinv = np.linalg.inv(npleg.legvander(eta, p - 1))

    def exact(xt, pos_s, box_shift):
        cS = -Lc / 2 + L * (pos_s + 0.5)  # relative to its cutoff box center
        out = np.zeros((p, p))
        for j in range(p):
            coef = Vinv[:, j]
            for i in range(p):
                val, _ = integrate.quad(
                    lambda y: math.exp(-(xt[i] - y) ** 2 / delta)
                    * npleg.legval(2 * (y - cS) / L, coef),
                    cS - L / 2, cS + L / 2, epsabs=1e-15, epsrel=1e-13)
                out[i, j] = val
        return out

    def R(dir_):
        Rm = np.eye(nr)
        for m in range(1, M):
            c, s = rot[m]
            s *= dir_
            Rm[2 * m:2 * m + 2, 2 * m:2 * m + 2] = [[c, -s], [s, c]]
        return Rm

    for pos_s, pos_t in ((0, 1), (3, 0), (2, 2)):
        FS, ET = F[tid[(4, pos_s)]], E[tid[(4, pos_t)]]
        xt = -Lc / 2 + L * (pos_t + 0.5) + 0.5 * L * eta  # target nodes, same box
        assert np.max(np.abs(ET @ FS - exact(xt, pos_s, 0))) < 10 * info["eps"]
        # target in the colleague box to the right: psi_A' = Rot(c_A - c_A') phi_A,
        # dir = A - A' = -1 along the axis
        assert np.max(np.abs(ET @ R(-1) @ FS - exact(xt + Lc, pos_s, 0))) < 10 * info["eps"]


# ---------------------------------------------------------------------------
# validation


def _code(fn):
    with pytest.raises(api.FgtError) as ei:
        fn()
    return ei.value.code


def test_validation_errors():
    lv, cs = synth.uniform_tree(2, 2)
    ok = dict(p=4, delta=1e-3, tol=1e-6)
    mk = lambda lv_, cs_, **kw: _plan(lv_, cs_, kw.pop("p", 4), kw.pop("delta", 1e-3),
                                      kw.pop("tol", 1e-6), **kw)
    assert _code(lambda: mk(lv, cs, tol=0.1)) == _lib.FGT_ERR_INVALID_ARG
    assert _code(lambda: mk(lv, cs, p=0)) == _lib.FGT_ERR_INVALID_ARG
    assert _code(lambda: mk(lv, cs, p=17)) == _lib.FGT_ERR_INVALID_ARG
    assert _code(lambda: mk(lv, cs, delta=0.0)) == _lib.FGT_ERR_INVALID_ARG
    assert _code(lambda: mk(lv, cs, force_lc=9)) == _lib.FGT_ERR_INVALID_ARG
    # gap: drop a leaf
    assert _code(lambda: mk(lv[1:], cs[1:])) == _lib.FGT_ERR_NOT_TILING
    # duplicate
    assert _code(lambda: mk(np.r_[lv, lv[:1]], np.r_[cs, cs[:1]])) == _lib.FGT_ERR_NOT_TILING
    # overlap: a leaf and its parent
    lv2 = np.r_[lv, [1]].astype(np.int32)
    cs2 = np.r_[cs, [[0, 0]]].astype(np.int32)
    assert _code(lambda: mk(lv2, cs2)) == _lib.FGT_ERR_NOT_TILING
    # out of range coordinate
    cs3 = cs.copy()
    cs3[0, 0] = 4
    assert _code(lambda: mk(lv, cs3)) == _lib.FGT_ERR_NOT_TILING
    # unbalanced: level-3 leaf (3,3) shares the corner (0,0) with the level-1 leaf (1,1)
    lvu = [1, 1, 1] + [2] * 3 + [3] * 4
    csu = [[1, 0], [0, 1], [1, 1], [0, 0], [1, 0], [0, 1], [2, 2], [3, 2], [2, 3], [3, 3]]
    assert _code(lambda: mk(np.array(lvu, np.int32), np.array(csu, np.int32))) == _lib.FGT_ERR_NOT_BALANCED
    # periodic with a cutoff level <= 1 runs the root Fourier series; forced onto a
    # small delta it would need more than 128 real modes
    assert mk(lv, cs, delta=0.05, periodic=True).info()["fourier"] == 1
    assert _code(lambda: mk(lv, cs, delta=1e-5, periodic=True, force_lc=0)) == _lib.FGT_ERR_UNSUPPORTED
    # reduced precision only where its rounding stays below tol: FP32 from
    # tol 1e-6, split bf16 products from tol 1e-4 (FP64 everywhere)
    assert _code(lambda: mk(lv, cs, tol=1e-7, precision="fp32")) == _lib.FGT_ERR_UNSUPPORTED
    assert _code(lambda: mk(lv, cs, tol=1e-10, precision="fp32")) == _lib.FGT_ERR_UNSUPPORTED
    assert mk(lv, cs, tol=1e-6, precision="fp32").info()["precision"] == _lib.FGT_FP32
    assert _code(lambda: mk(lv, cs, tol=1e-6, precision="bf16x3")) == _lib.FGT_ERR_UNSUPPORTED
    assert _code(lambda: mk(lv, cs, tol=5e-5, precision="bf16x3")) == _lib.FGT_ERR_UNSUPPORTED
    assert mk(lv, cs, tol=1e-4, precision="bf16x3").info()["precision"] == _lib.FGT_BF16X3
    assert mk(lv, cs, tol=1e-10, precision="fp64").info()["precision"] == _lib.FGT_FP64
    # a valid plan works
    assert mk(lv, cs).info()["nleaves"] == 16
    assert ok


# ---------------------------------------------------------------------------
# f-flags, P-lists and D-lists on a hand-drawn tree


def test_fflags_plists_dlists_small_tree():
    # uniform level-2 2D tree with box (1,1) refined to level 3, cutoff forced to 2
    lv, cs = synth.uniform_tree(2, 2)
    keep = ~((cs[:, 0] == 1) & (cs[:, 1] == 1))
    kids = np.array([[2, 2], [3, 2], [2, 3], [3, 3]], dtype=np.int32)
    lv = np.r_[lv[keep], [3] * 4].astype(np.int32)
    cs = np.r_[cs[keep], kids].astype(np.int32)
    pl = _plan(lv, cs, 4, 1e-3, 1e-6, force_lc=2)
    isleaf = pl.array("pwbox_isleaf")
    # f = 1: the refined box and its 8 colleagues (all interior neighbors of (1,1))
    assert len(isleaf) == 9 and isleaf.sum() == 8
    st, src = pl.array("plist_start"), pl.array("plist_src")
    nonleaf = int(np.where(isleaf == 0)[0][0])
    for a in range(9):
        got = set(src[st[a]:st[a + 1]].tolist())
        if a == nonleaf:
            assert got == set(range(9))      # every colleague with f = 1, itself included
        else:
            assert got == {nonleaf}          # leaf-leaf pairs are direct
    # leaves at level 3 have no near list; the 15 level-2 leaves gather directly
    tg = pl.array("near_tgt")
    assert sorted(lv[tg].tolist()) == [2] * 15
    assert pl.array("near_haspw").sum() == 8
    # every PW leaf maps to exactly one box
    assert len(pl.array("pwleaf_id")) == 8 + 4


# ---------------------------------------------------------------------------
# the host plan, walked in numpy, against the oracle


@pytest.mark.parametrize("d,delta,tol,flc", [(1, 0.2, 1e-10, -1), (2, 0.05, 1e-6, -1),
                                             (2, 2e-3, 1e-8, 1), (3, 0.02, 1e-6, -1)])
def test_fourier_route_matches_oracle(d, delta, tol, flc):
    """Periodic transforms with cutoff level <= 1 (the root Fourier series)
    against the oracle's image sums, on adaptive trees near the boundary."""
    c = {1: [[0.47]], 2: [[0.46, -0.17], [-0.2, 0.49]], 3: [[0.45, -0.12, 0.05]]}[d]
    dens = synth.GaussianSum(np.array(c), np.array([0.02, 0.04][:len(c)]),
                             np.array([1.0, -0.5][:len(c)]), periodic=True)
    p = {1: 8, 2: 8, 3: 5}[d]
    lv, cs = synth.resolve_tree(dens, d, p, 1e-9, max_level={1: 8, 2: 6, 3: 3}[d], periodic=True)
    sig = synth.sample(lv, cs, p, dens)
    pl = _plan(lv, cs, p, delta, tol, periodic=True, force_lc=flc)
    assert pl.info()["fourier"] == 1
    uo = oracle.oracle_u(lv, cs, p, delta, sig, periodic=True)
    assert cf.rel_l2(host_exec.run(pl, sig), uo) < tol
    if d == 3:
        assert cf.rel_l2(host_exec.run(pl, sig, grouped=True), uo) < tol


@pytest.mark.parametrize("case", ["2d-pw", "2d-adaptive", "2d-periodic", "3d"])
def test_host_plan_matches_oracle(case):
    if case == "2d-pw":
        pr = synth.small_2d(0)
        lv, cs, sig, p, delta, tol, per, flc = pr.levels, pr.coords, pr.sigma, 8, 1e-3, 1e-6, False, 2
    elif case in ("2d-adaptive", "2d-periodic"):
        per = case == "2d-periodic"
        c = [[0.46, -0.17], [-0.2, 0.49]] if per else [[0.11, -0.17], [-0.2, 0.05]]
        dens = synth.GaussianSum(np.array(c), np.array([0.01, 0.03]), np.array([0.7, -0.4]),
                                 periodic=per)
        lv, cs = synth.resolve_tree(dens, 2, 8, 1e-10, max_level=7, periodic=per)
        sig = synth.sample(lv, cs, 8, dens)
        p, delta, tol, flc = 8, 1e-4, 1e-10, -1
    else:
        dens = synth.GaussianSum(np.array([[0.1, -0.12, 0.05]]), np.array([0.03]), np.array([1.0]))
        lv, cs = synth.resolve_tree(dens, 3, 5, 1e-7, max_level=4)
        sig = synth.sample(lv, cs, 5, dens)
        p, delta, tol, per, flc = 5, 1e-3, 1e-6, False, -1
    uo = oracle.oracle_u(lv, cs, p, delta, sig, periodic=per)
    uh = host_exec.run(_plan(lv, cs, p, delta, tol, periodic=per, force_lc=flc), sig)
    assert cf.rel_l2(uh, uo) < tol


# ---------------------------------------------------------------------------
# d = 3 planes and rows: the grouping the device formation/evaluation uses


def _tree_3d_deep():
    """A 3D tree whose leaves sit up to three levels below the cutoff level
    (wide Gaussian, fine tree), so that planes and rows hold many leaves."""
    dens = synth.GaussianSum(np.array([[0.1, -0.12, 0.05], [-0.2, 0.15, -0.1]]),
                             np.array([0.03, 0.05]), np.array([1.0, -0.5]))
    lv, cs = synth.resolve_tree(dens, 3, 4, 1e-6, max_level=5)
    return lv, cs, synth.sample(lv, cs, 4, dens)


def test_planes_and_rows_partition_the_pw_leaves():
    lv, cs, _ = _tree_3d_deep()
    pl = _plan(lv, cs, 4, 5e-2, 1e-6)
    info = pl.info()
    pw_start, tab = pl.array("pw_start"), pl.array("pwleaf_tab").reshape(-1, 3)
    ps, pt = pl.array("plane_start"), pl.array("plane_tab").reshape(-1, 3)
    pr, rs, rt = pl.array("plane_row"), pl.array("row_start"), pl.array("row_tab")
    meta = pl.array("ftab_meta").reshape(2, -1)  # level, position of each table
    pid = pl.array("pwleaf_id")
    assert len(ps) == len(pw_start) and ps[0] == 0 and pr[0] == 0 and rs[0] == 0
    assert rs[-1] == len(pid) and pr[-1] == len(rt) and ps[-1] == len(pr) - 1
    assert len(pr) - 1 < len(rt) < len(pid)  # the tree does group leaves
    for A in range(len(pw_start) - 1):
        # the planes of box A cover exactly its pw leaves, in order
        assert rs[pr[ps[A]]] == pw_start[A] and rs[pr[ps[A + 1]]] == pw_start[A + 1]
        keys = set()
        for P in range(ps[A], ps[A + 1]):
            keys.add(int(pt[P, 2]))
            for r in range(pr[P], pr[P + 1]):
                leaves = range(rs[r], rs[r + 1])
                assert len(leaves) > 0
                assert all(tab[s, 2] == pt[P, 2] for s in leaves)   # one axis-3 table
                assert all(tab[s, 0] == rt[r] for s in leaves)      # one axis-1 table
                assert all(lv[pid[s]] == meta[0, pt[P, 2]] for s in leaves)  # one level
        assert len(keys) == ps[A + 1] - ps[A]  # planes of a box are distinct
    assert info["lc"] < lv.max() - 1
    # dispatch order of the per-plane stages: a permutation, most work first
    order = pl.array("plane_order")
    assert sorted(order) == list(range(len(pr) - 1))
    work = [(rs[pr[P + 1]] - rs[pr[P]]) + 3 * (pr[P + 1] - pr[P]) for P in order]
    assert all(a >= b for a, b in zip(work, work[1:]))


def test_grouped_walk_equals_per_leaf_walk():
    lv, cs, sig = _tree_3d_deep()
    for delta, tol in ((5e-2, 1e-6), (1e-2, 1e-10)):
        pl = _plan(lv, cs, 4, delta, tol)
        a = host_exec.run(pl, sig)
        b = host_exec.run(pl, sig, grouped=True)
        assert cf.rel_l2(b, a) < 1e-13
    uo = oracle.oracle_u(lv, cs, 4, 5e-2, sig)
    assert cf.rel_l2(host_exec.run(_plan(lv, cs, 4, 5e-2, 1e-6), sig, grouped=True), uo) < 1e-6


# ---------------------------------------------------------------------------
# 2:1 rebalancing of the output trees (host logic of include/fgt_output.h)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_tree_balance_matches_the_input_generator(d):
    """fgt_tree_balance (C++) against the input generator's plain balance
    (Python), on unbalanced trees refined around random points."""
    import itertools
    rng = np.random.default_rng(40 + d)
    for _ in range(8):
        pts = rng.uniform(-0.5, 0.5, (int(rng.integers(1, 4)), d))
        maxl = int(rng.integers(3, 8 if d < 3 else 5))
        leaves, boxes = [], [(0, (0,) * d)]
        while boxes:
            l, c = boxes.pop()
            lo = -0.5 + np.array(c) * 2.0 ** -l
            inside = any(np.all(pt >= lo) and np.all(pt < lo + 2.0 ** -l) for pt in pts)
            if inside and l < maxl:
                for o in itertools.product((0, 1), repeat=d):
                    boxes.append((l + 1, tuple(2 * c[a] + o[a] for a in range(d))))
            else:
                leaves.append((l, c))
        lv = np.array([l for l, _ in leaves], np.int32)
        cs = np.array([c for _, c in leaves], np.int32).reshape(-1, d)
        for periodic in (False, True):
            a = synth.balance(lv, cs, periodic)
            b = api.fgt_tree_balance(lv, cs, periodic)
            assert set(zip(a[0].tolist(), map(tuple, a[1].tolist()))) == \
                set(zip(b[0].tolist(), map(tuple, b[1].tolist())))
            # Morton order of the lower corners
            lmax = int(b[0].max())
            key = [sum(((int(c[a]) << (lmax - int(l))) >> bit & 1) << (bit * d + a)
                       for bit in range(lmax) for a in range(d)) for l, c in zip(*b)]
            assert key == sorted(key)
    # an already balanced tree is returned unchanged
    lv, cs = synth.uniform_tree(d, 2)
    b = api.fgt_tree_balance(lv, cs)
    assert len(b[0]) == len(lv)


def test_tree_entry_points_validate_arguments_before_any_device_call():
    """The output-tree, density and interpolation entry points reject bad
    arguments on the host (no device is touched, so this runs on a CPU)."""
    L = _lib.lib()
    lv, cs = synth.uniform_tree(2, 2)
    tree, keep = api._tree(lv, cs)
    out = ctypes.c_void_p()
    oo = _lib.fgt_output_opts_t(0.0, 1, 1, 0)
    # NULL sigma, p out of range, eps out of range
    assert L.fgt_output_resolve(ctypes.byref(tree), 4, 1e-3, 1e-6, 0, None, ctypes.byref(oo), None,
                                ctypes.byref(out)) == _lib.FGT_ERR_INVALID_ARG
    assert L.fgt_output_resolve(ctypes.byref(tree), 0, 1e-3, 1e-6, 0, None, ctypes.byref(oo), 8,
                                ctypes.byref(out)) == _lib.FGT_ERR_INVALID_ARG
    bad = _lib.fgt_output_opts_t(1.5, 1, 1, 0)
    assert L.fgt_output_resolve(ctypes.byref(tree), 4, 1e-3, 1e-6, 0, None, ctypes.byref(bad), 8,
                                ctypes.byref(out)) == _lib.FGT_ERR_INVALID_ARG
    # a coordinate outside its level's range
    cs2 = cs.copy()
    cs2[0, 0] = 9
    tree2, keep2 = api._tree(lv, cs2)
    assert L.fgt_interp(ctypes.byref(tree2), 4, 8, 1, 8, 8, None) == _lib.FGT_ERR_NOT_TILING
    assert L.fgt_interp(ctypes.byref(tree), 4, 8, -1, 8, 8, None) == _lib.FGT_ERR_INVALID_ARG
    assert L.fgt_interp(ctypes.byref(tree), 4, 8, 0, None, None, None) == _lib.FGT_OK  # nothing to do
    assert L.fgt_tree_balance(ctypes.byref(tree), 7, None, None, 0) == _lib.FGT_ERR_INVALID_ARG
    # gaussians: zero width, eps, level range
    g, gk = api._gaussians(np.array([[0.0, 0.0]]), np.array([0.0]), np.array([1.0]), False)
    assert L.fgt_resolve_gaussians(ctypes.byref(g), 8, 1e-8, None, ctypes.byref(out)) == _lib.FGT_ERR_INVALID_ARG
    g, gk = api._gaussians(np.array([[0.0, 0.0]]), np.array([0.1]), np.array([1.0]), False)
    assert L.fgt_resolve_gaussians(ctypes.byref(g), 8, 0.0, None, ctypes.byref(out)) == _lib.FGT_ERR_INVALID_ARG
    o = _lib.fgt_resolve_opts_t(5, 3, 0, 0.0, None)
    assert L.fgt_resolve_gaussians(ctypes.byref(g), 8, 1e-8, ctypes.byref(o), ctypes.byref(out)) == \
        _lib.FGT_ERR_INVALID_ARG
    assert L.fgt_sample_gaussians(ctypes.byref(g), ctypes.byref(tree), 8, None, None) == _lib.FGT_ERR_INVALID_ARG
    assert out.value is None
    del keep, keep2, gk


# ---------------------------------------------------------------------------
# target groups of the fused 3D translation (fgt_host.h te_*)


def _two_level_tree(seed, frac):
    """Level-4 boxes of the unit cube, a random fraction of them split into
    their eight level-5 children (always 2:1 balanced)."""
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


@pytest.mark.parametrize("frac,periodic", [(0.05, False), (0.05, True), (1.0, False)])
def test_fused_translation_groups(frac, periodic):
    lv, cs = _two_level_tree(7, frac)
    pl = _plan(lv, cs, 4, 1e-4, 1e-6, periodic=periodic)
    info = pl.info()
    assert info["fused_translate"] == 1 and info["lc"] == 4
    lc = info["lc"]
    pws, pid = pl.array("pw_start"), pl.array("pwleaf_id")
    nA = len(pws) - 1
    bc = np.array([cs[pid[pws[a]]] >> (lv[pid[pws[a]]] - lc) for a in range(nA)])
    ps, src, code = pl.array("plist_start"), pl.array("plist_src"), pl.array("plist_dir")
    ts = pl.array("te_start")
    G = len(pl.array("te_mem")) // (len(ts) - 1)  # member slots per group
    mem = pl.array("te_mem").reshape(-1, G)
    tsrc, tdir = pl.array("te_src"), pl.array("te_dir").view(np.uint32).reshape(-1, (G + 3) // 4)
    assert len(ts) == len(mem) + 1 and ts[0] == 0 and ts[-1] == len(tsrc) == len(tdir)
    # every P-list sorted by (source box, code)
    for A in range(nA):
        pairs = list(zip(src[ps[A]:ps[A + 1]].tolist(), code[ps[A]:ps[A + 1]].tolist()))
        assert pairs == sorted(pairs)
    seen = np.zeros(nA, int)
    sizes = []
    for g in range(len(mem)):
        members = [int(m) for m in mem[g] if m >= 0]
        assert members == [int(m) for m in mem[g][:len(members)]]  # filled from slot 0
        sizes.append(len(members))
        seen[members] += 1
        # siblings: one parent at level lc - 1, one position along axis 3
        assert len({(*(bc[m][:2] >> 1), bc[m][2]) for m in members}) == 1
        es = range(ts[g], ts[g + 1])
        assert [int(tsrc[e]) for e in es] == sorted(int(tsrc[e]) for e in es)
        for t in range(G):
            got = []
            for e in es:
                c = int(tdir[e][t // 4] >> (8 * (t % 4))) & 0xFF
                if c != 0xFF:
                    assert t < len(members)
                    got.append((int(tsrc[e]), c))
            if t < len(members):
                A = members[t]
                # the member meets exactly its P-list, in its order
                assert got == list(zip(src[ps[A]:ps[A + 1]].tolist(), code[ps[A]:ps[A + 1]].tolist()))
        # every entry serves some member, and its members share the axis-3
        # part of their codes (the kernel turns the source along axis 3 once)
        for e in es:
            codes = [int(tdir[e][t // 4] >> (8 * (t % 4))) & 0xFF for t in range(G)]
            present = [c for c in codes if c != 0xFF]
            assert present and len({c // 9 for c in present}) == 1
    assert np.all(seen == 1)
    # groups share sources: fewer entries than P-list pairs
    assert len(tsrc) < len(src)
    # workgroups: every (group, tile) once; tile t runs on XCD t % 8 except
    # the tiles past the last multiple of 8
    wg = pl.array("te_wg").reshape(-1, 2)
    ntile = int(wg[:, 1].max()) + 1
    assert len(wg) % 8 == 0
    live = wg[wg[:, 0] >= 0]
    assert len(live) == len(mem) * ntile
    assert len({(int(a), int(b)) for a, b in live}) == len(live)
    fixed = ntile // 8 * 8
    for b, (g, t) in enumerate(wg):
        if g >= 0 and t < fixed:
            assert b % 8 == t % 8
    if frac == 1.0:
        assert set(sizes) == {G}
    else:
        assert min(sizes) < 8


@pytest.mark.parametrize("frac,periodic", [(0.05, False), (0.3, True)])
def test_near_target_order(frac, periodic):
    """Near targets: every target once with its own list; the targets of XCD x
    (positions b with b % 8 == x) are the x-th of eight equal-count runs of the
    targets in Morton order; the last 64 of a run go most sources first."""
    lv, cs = _two_level_tree(3, frac)
    pl = _plan(lv, cs, 4, 1e-4, 1e-6, periodic=periodic)
    tg, st = pl.array("near_tgt"), pl.array("near_start")
    nt = len(tg)
    assert nt > 8 * 64 and len(set(tg.tolist())) == nt and st[0] == 0
    lmax = int(lv.max())

    def morton(T):
        v = 0
        for a in range(3):
            c = int(cs[T][a]) << (lmax - int(lv[T]))
            for b in range(21):
                v |= ((c >> b) & 1) << (3 * b + a)
        return v

    mk = sorted((morton(T), T) for T in tg.tolist())
    base, extra = divmod(nt, 8)
    at = 0
    for x in range(8):
        n_x = base + (1 if x < extra else 0)
        run = tg[x::8]
        assert len(run) == n_x
        assert {T for _, T in mk[at:at + n_x]} == set(run.tolist())
        at += n_x
        ns = [int(st[b + 1] - st[b]) for b in range(x, nt, 8)]
        tail = ns[max(0, n_x - 64):]
        assert tail == sorted(tail, reverse=True)
