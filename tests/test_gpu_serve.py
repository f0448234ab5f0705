"""GPU tests of the request loop (include/fgt_serve.h).

The serving bar: a request's result is the same alone and in a mix of
concurrent requests.  The design makes it bitwise: every request runs the
plan's kernels, in the same order, on a workspace of its own, and every
reduction is a fixed-order gather.  The tests also check a few request types
against the FP64 oracle within their tol, memory-budget eviction, host-memory
requests and error reporting.
"""

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_2305_07165_amd import api, serving, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-serve] {msg}", flush=True)


_TYPES = {}


def _types():
    if not _TYPES:
        _TYPES["t"] = synth.serve_request_types(11, 8, log10_n=(3.5, 6.0))
    return _TYPES["t"]


def _alone(types):
    out = []
    for t in types:
        pl = api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, precision=t.precision)
        u = pl.execute(torch.from_numpy(t.sigma).cuda())
        torch.cuda.synchronize()
        out.append(u.cpu())
        pl.close()
    return out


def test_predicted_device_bytes_bound_the_resident_plan():
    for t in _types()[:4]:
        hp = api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, precision=t.precision, host_only=True)
        dp = api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, precision=t.precision)
        pred, real = hp.info()["device_bytes"], dp.info()["device_bytes"]
        _say(f"type {t.key}: predicted {pred} resident {real}")
        assert real <= pred <= real + 4096
        dp.close()
        hp.close()


def test_alone_vs_mix_bitwise():
    types = _types()
    for t in types:
        _say(f"type {t.key}: d={t.d} p={t.p} leaves={len(t.levels)} N={t.npoints} "
             f"delta={t.delta:.2e} tol={t.tol} {t.precision}")
    ref = _alone(types)
    pool = serving.Pool(types)
    rng = np.random.default_rng(5)
    kinds = rng.integers(0, len(types), 64)
    with api.Server(nslots=4, nbuilders=2) as srv:
        live = {}
        for i, k in enumerate(kinds):
            k = int(k)
            u = torch.full_like(pool.sigma[k], float("nan"))
            live[serving._submit(srv, pool, k, u)] = (k, u)
            if i % 16 == 15:  # later requests arrive while earlier ones run
                for c in srv.poll():
                    assert c["status"] == 0
        done = srv.drain()
        st = srv.stats()
        _say(f"stats {st}")
        assert st["completed"] == len(kinds) and st["failed"] == 0
        assert st["plans_built"] == len(set(kinds.tolist()))
        assert st["peak_resident_bytes"] <= st["budget_bytes"]
    torch.cuda.synchronize()
    ids = set()
    for rid, (k, u) in live.items():
        assert torch.equal(u.cpu(), ref[k]), f"request {rid} (type {k}) differs from its result alone"
        ids.add(rid)
    assert len(ids) == len(kinds)


def test_served_results_match_oracle():
    types = [t for t in _types() if t.npoints <= 300_000][:3]
    assert types
    pool = serving.Pool(types)
    with api.Server(nslots=2) as srv:
        us = []
        for k in range(len(types)):
            u = pool.take_u(k)
            serving._submit(srv, pool, k, u)
            us.append(u)
        done = srv.drain()
        assert all(c["status"] == 0 for c in done)
    for t, u in zip(types, us):
        tg = np.unique(np.linspace(0, len(t.levels) - 1, 12).astype(np.int64))
        uo = oracle.oracle_u(t.levels, t.coords, t.p, t.delta, t.sigma, targets=tg)
        err = cf.rel_l2(u.cpu().numpy()[tg], uo)
        _say(f"type {t.key} vs oracle on {len(tg)} leaves: rel_l2={err:.2e} tol={t.tol}")
        assert err < t.tol


def test_budget_eviction_keeps_results():
    types = _types()[:5]
    ref = _alone(types)
    need = []
    for t in types:
        hp = api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, precision=t.precision, host_only=True)
        need.append(hp.info()["device_bytes"])
        hp.close()
    budget = int(max(need) * 1.2)
    pool = serving.Pool(types)
    rng = np.random.default_rng(9)
    kinds = rng.integers(0, len(types), 30)
    with api.Server(nslots=3, hbm_budget=budget) as srv:
        live = {}
        for k in kinds:
            k = int(k)
            u = torch.empty_like(pool.sigma[k])
            live[serving._submit(srv, pool, k, u)] = (k, u)
        done = srv.drain()
        st = srv.stats()
    _say(f"budget {budget}: {st}")
    assert all(c["status"] == 0 for c in done)
    assert st["plans_evicted"] > 0
    assert st["peak_resident_bytes"] <= budget
    for rid, (k, u) in live.items():
        assert torch.equal(u.cpu(), ref[k])


def test_host_memory_requests():
    types = _types()[:3]
    ref = _alone(types)
    with api.Server(nslots=2) as srv:
        outs = []
        for t in types:
            s = torch.from_numpy(t.sigma).pin_memory()
            u = torch.empty_like(s).pin_memory()
            srv.submit(t.key, s, u, t.p, t.delta, t.tol, precision=t.precision,
                       levels=t.levels, coords=t.coords, host_io=True)
            outs.append(u)
        done = srv.drain()
    assert all(c["status"] == 0 for c in done)
    for u, r in zip(outs, ref):
        assert torch.equal(u, r)


def test_errors_are_reported():
    t = _types()[0]
    s = torch.from_numpy(t.sigma).cuda()
    u = torch.empty_like(s)
    with api.Server(nslots=1, hbm_budget=1024) as srv:
        # a type that cannot fit the budget completes with FGT_ERR_OOM
        srv.submit(1, s, u, t.p, t.delta, t.tol, precision=t.precision,
                   levels=t.levels, coords=t.coords)
        # a key reused with other parameters is refused at submit
        with pytest.raises(api.FgtError):
            srv.submit(1, s, u, t.p, t.delta * 2, t.tol, precision=t.precision)
        # a tree that is not a tiling fails in planning, reported on completion
        lv = np.array([1, 1, 1], dtype=np.int32)
        cs = np.array([[0, 0], [1, 0], [0, 1]], dtype=np.int32)
        s2 = torch.zeros((3, 16), dtype=torch.float64, device="cuda")
        srv.submit(2, s2, torch.empty_like(s2), 4, 1e-3, 1e-6, levels=lv, coords=cs)
        done = {c["key"]: c for c in srv.drain()}
    assert done[1]["status"] == -4
    assert done[2]["status"] == -2
