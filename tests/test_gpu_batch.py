"""GPU tests of batched execution (include/fgt_batch.h).

A batch runs the same kernel bodies as fgt_execute, so every transform's
result must equal its result alone bitwise, in graph replay and direct mode,
under every schedule the autotuner tries, and after rebinding.  Two
transforms are also checked against the FP64 oracle within their tol.
"""

import time

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_2305_07165_amd import api, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-batch] {msg}", flush=True)


_CACHE = {}


def _problems():
    if "p" not in _CACHE:
        probs = synth.batch_problems(3, 20, max_points=1 << 17)
        # a periodic 2D transform and a 1D transform (run with their own launches)
        dens = synth.GaussianSum(np.array([[0.46, -0.17], [-0.2, 0.49]]), np.array([0.01, 0.03]),
                                 np.array([0.7, -0.4]), periodic=True)
        lv, cs = synth.resolve_tree(dens, 2, 8, 1e-10, max_level=6, periodic=True)
        probs.append(synth.RequestType(100, 2, 8, 1e-3, 1e-6, "fp64", lv, cs,
                                       synth.sample(lv, cs, 8, dens)))
        d1 = synth.GaussianSum(np.array([[0.13]]), np.array([0.01]), np.array([1.0]))
        lv, cs = synth.resolve_tree(d1, 1, 9, 1e-12, max_level=9)
        probs.append(synth.RequestType(101, 1, 9, 1e-4, 1e-10, "fp64", lv, cs, synth.sample(lv, cs, 9, d1)))
        _CACHE["p"] = probs
    return _CACHE["p"]


def _periodic(t):
    return t.key == 100


def _plans(probs):
    return [api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, periodic=_periodic(t), precision=t.precision)
            for t in probs]


def _alone(plans, sig):
    out = []
    for pl, s in zip(plans, sig):
        out.append(pl.execute(s).clone())
    torch.cuda.synchronize()
    return out


def test_batch_equals_alone_graph_and_direct():
    probs = _problems()
    for t in probs:
        _say(f"job {t.key}: d={t.d} p={t.p} leaves={len(t.levels)} N={t.npoints} delta={t.delta:.1e} "
             f"tol={t.tol} {t.precision}")
    plans = _plans(probs)
    sig = [torch.from_numpy(t.sigma).cuda() for t in probs]
    ref = _alone(plans, sig)
    for use_graph in (True, False):
        b = api.Batch(plans, use_graph=use_graph)
        us = [torch.full_like(s, float("nan")) for s in sig]
        b.bind(sig, us)
        info = b.info()
        _say(f"graph={use_graph} info {info}")
        assert info["njobs"] == len(probs) and info["nsingle"] == 1
        for rep in range(3):
            b.execute()
            torch.cuda.synchronize()
            for i, (u, r) in enumerate(zip(us, ref)):
                assert torch.equal(u, r), f"rep {rep} job {i} differs from its result alone"
            # eager work between replays; results must not depend on it
            for u in us:
                u.fill_(float("nan"))
            torch.cuda.synchronize()
        b.close()


@pytest.mark.skip(reason="persistent batched launches did not finish their first execution within three "
                         "minutes on the device, twice (acquire-polled waits, then relaxed-polled waits with "
                         "one acquire); the cause is not established, so fgt_batch_create refuses the option "
                         "and this case stays off the GPU")
def test_batch_persistent_equals_alone():
    """One persistent launch per kernel class (every stage of every transform
    of the class behind a work queue): bitwise the results alone, in graph
    replay and direct mode, repeatedly, with eager work between executions;
    no bounded wait runs out."""
    probs = _problems()
    # add a split-bf16 transform: its class keeps the per-stage launches
    t0 = probs[0]
    extra = synth.RequestType(102, t0.d, t0.p, t0.delta, 1e-3, "bf16x3", t0.levels, t0.coords, t0.sigma)
    probs = probs + [extra]
    plans = _plans(probs)
    sig = [torch.from_numpy(t.sigma).cuda() for t in probs]
    ref = _alone(plans, sig)
    for use_graph in (True, False):
        b = api.Batch(plans, use_graph=use_graph, persistent=True)
        us = [torch.full_like(s, float("nan")) for s in sig]
        b.bind(sig, us)
        info = b.info()
        _say(f"persistent graph={use_graph} info {info}")
        assert 0 < info["persistent"] < info["nclasses"]
        for rep in range(3):
            t0 = time.perf_counter()
            b.execute()
            torch.cuda.synchronize()
            _say(f"persistent graph={use_graph} rep {rep}: {1e3 * (time.perf_counter() - t0):.1f} ms")
            for i, (u, r) in enumerate(zip(us, ref)):
                assert torch.equal(u, r), f"rep {rep} job {i} differs from its result alone"
            for u in us:
                u.fill_(float("nan"))
            torch.cuda.synchronize()
        assert b.info()["persistent_error"] == 0
        b.close()


def test_batch_persistent_is_refused():
    probs = _problems()[:2]
    plans = _plans(probs)
    with pytest.raises(api.FgtError) as ei:
        api.Batch(plans, persistent=True)
    assert ei.value.code == api.FGT_ERR_UNSUPPORTED


def test_batch_rebind_and_tuner_off():
    probs = _problems()
    plans = _plans(probs)
    sig = [torch.from_numpy(t.sigma).cuda() for t in probs]
    ref = _alone(plans, sig)
    b = api.Batch(plans)
    us = [torch.empty_like(s) for s in sig]
    b.bind(sig, us)
    b.execute()
    torch.cuda.synchronize()
    # the schedule autotuner is switched off: it refuses without touching the device
    with pytest.raises(api.FgtError) as ei:
        b.tune(reps=2)
    assert ei.value.code == api.FGT_ERR_UNSUPPORTED
    assert b.info()["tuned_ms"] == 0
    # new outputs and doubled inputs: linear, and still exact per job
    sig2 = [2.0 * s for s in sig]
    us2 = [torch.full_like(s, float("nan")) for s in sig]
    b.bind(sig2, us2)
    b.execute()
    torch.cuda.synchronize()
    ref2 = _alone(plans, sig2)
    for u, r in zip(us2, ref2):
        assert torch.equal(u, r)
    b.close()


@pytest.mark.skip(reason="the schedule autotuner aborted inside fgt_batch_tune (SIGABRT, no GPU fault "
                         "reported) in this test, and a later version crashed a benchmark run (SIGSEGV) "
                         "on 512 transforms; the cause is not established, so fgt_batch_tune is switched "
                         "off and this case stays off the GPU")
def test_batch_graph_replays_after_repeated_tuning():
    """Tuning leaves any of 1, 2 or 4 streams (a fork/join in the graph); the
    replays after each tuning, with eager work between them, stay exact."""
    probs = _problems()
    plans = _plans(probs)
    sig = [torch.from_numpy(t.sigma).cuda() for t in probs]
    ref = _alone(plans, sig)
    b = api.Batch(plans, nstreams=4)
    us = [torch.full_like(s, float("nan")) for s in sig]
    b.bind(sig, us)
    picked = []
    for rnd in range(3):
        b.tune(reps=1)
        picked.append(b.info()["nstreams"])
        for rep in range(2):
            b.execute()
            torch.cuda.synchronize()
            for i, (u, r) in enumerate(zip(us, ref)):
                assert torch.equal(u, r), f"tuning {rnd} replay {rep} job {i} differs from its result alone"
            for u in us:
                u.fill_(float("nan"))
            torch.cuda.synchronize()
    _say(f"streams picked by three tunings: {picked}")
    b.close()


def test_batch_matches_oracle():
    probs = [t for t in _problems() if t.d == 2 and t.npoints <= 40_000][:2]
    assert probs
    plans = _plans(probs)
    sig = [torch.from_numpy(t.sigma).cuda() for t in probs]
    us = [torch.empty_like(s) for s in sig]
    b = api.Batch(plans)
    b.bind(sig, us)
    b.execute()
    torch.cuda.synchronize()
    for t, u in zip(probs, us):
        uo = oracle.oracle_u(t.levels, t.coords, t.p, t.delta, t.sigma, periodic=_periodic(t))
        err = cf.rel_l2(u.cpu().numpy(), uo)
        _say(f"job {t.key} vs oracle: rel_l2={err:.2e} tol={t.tol}")
        assert err < t.tol
    b.close()


def test_batch_alternative_tile_equals_alone():
    """Every d = 3 class on the alternative box-formation tile (two slabs per
    wave): the same columns and sums, so results stay bitwise equal."""
    dens = synth.GaussianSum(np.array([[0.1, -0.12, 0.05], [-0.3, 0.2, 0.1]]),
                             np.array([0.02, 0.05]), np.array([1.0, -0.6]))
    lv, cs = synth.resolve_tree(dens, 3, 6, 1e-8, max_level=5)
    probs = [synth.RequestType(200, 3, 6, 1e-3, 1e-6, "fp64", lv, cs, synth.sample(lv, cs, 6, dens)),
             synth.RequestType(201, 3, 6, 1e-3, 1e-3, "fp32", lv, cs, synth.sample(lv, cs, 6, dens))]
    probs += [t for t in _problems() if t.d == 3][:4] + [_problems()[-1]]
    plans = _plans(probs)
    assert plans[0].info()["n_pwleaf"] > 0
    sig = [torch.from_numpy(t.sigma).cuda() for t in probs]
    ref = _alone(plans, sig)
    b = api.Batch(plans, form_tile=1)
    us = [torch.full_like(s, float("nan")) for s in sig]
    b.bind(sig, us)
    info = b.info()
    _say(f"alternative tile: {info}")
    assert info["tile_alt_classes"] > 0
    b.execute()
    torch.cuda.synchronize()
    for u, r in zip(us, ref):
        assert torch.equal(u, r)
    b.close()
    with pytest.raises(api.FgtError):
        api.Batch(plans, form_tile=2)


def test_batch_rejects_host_only_plans():
    t = _problems()[0]
    hp = api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, host_only=True)
    with pytest.raises(api.FgtError):
        api.Batch([hp])


def test_batch_with_a_fused_plan_equals_alone():
    """A large 3D plan whose translation runs fused with the first evaluation
    step (fgt_info_t.fused_translate) batched with a small 2D plan: the fused
    batched kernel must reproduce the plan's own result bitwise."""
    pr = synth.adaptive_3d(0)
    small = _problems()[0]
    plans = [api.Plan(pr.levels, pr.coords, pr.p, pr.delta, 1e-6),
             api.Plan(small.levels, small.coords, small.p, small.delta, small.tol, precision=small.precision)]
    assert plans[0].info()["fused_translate"] == 1
    sig = [torch.from_numpy(pr.sigma).cuda(), torch.from_numpy(small.sigma).cuda()]
    ref = _alone(plans, sig)
    for use_graph in (True, False):
        b = api.Batch(plans, use_graph=use_graph)
        us = [torch.full_like(s, float("nan")) for s in sig]
        b.bind(sig, us)
        b.execute()
        torch.cuda.synchronize()
        _say(f"fused batch graph={use_graph}: {b.info()}")
        for i, (u, r) in enumerate(zip(us, ref)):
            assert torch.equal(u, r), f"job {i} differs from its result alone"
        b.close()
