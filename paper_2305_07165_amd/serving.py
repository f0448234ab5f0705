"""Load generator for the request loop (include/fgt_serve.h).

Drives a ``Server`` with a pool of request types (``synth.serve_request_types``)
held on the device: sigma once per type, result buffers recycled per type.
Three measurements:

* ``sequential``: every request of a list run alone, one after another, with
  plain ``fgt_execute`` on one stream (plans built beforehand);
* ``closed_loop``: the same list submitted at once and drained (capacity);
* ``poisson``: arrivals with exponential gaps at a fixed rate; latency is
  arrival -> completion (the native completion time plus any lateness of the
  submit call behind its scheduled arrival).

No arithmetic of the transform happens here: every request runs in libfgt.so.
"""

from __future__ import annotations

import time

import numpy as np

from . import api


class Pool:
    """Request types with their sigma on the device and per-type free lists of
    result buffers."""

    def __init__(self, types, device="cuda"):
        import torch
        self.torch = torch
        self.types = list(types)
        self.sigma = [torch.from_numpy(t.sigma).to(device) for t in self.types]
        self.free = [[] for _ in self.types]
        self.device = device
        torch.cuda.synchronize()

    def take_u(self, k):
        if self.free[k]:
            return self.free[k].pop()
        return self.torch.empty_like(self.sigma[k])

    def give_u(self, k, u):
        self.free[k].append(u)


def _submit(server, pool, k, u):
    t = pool.types[k]
    return server.submit(t.key, pool.sigma[k], u, t.p, t.delta, t.tol, precision=t.precision,
                         levels=t.levels, coords=t.coords)


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def warm(server, pool):
    """One request of every type: builds and uploads every plan."""
    live = {}
    for k in range(len(pool.types)):
        u = pool.take_u(k)
        live[_submit(server, pool, k, u)] = (k, u)
    for c in server.drain():
        k, u = live.pop(c["id"])
        if c["status"] != 0:
            raise RuntimeError(f"request type {k} failed with status {c['status']}")
        pool.give_u(k, u)


def sequential(pool, kinds):
    """Every request alone with plain fgt_execute on one stream; plans are
    built before timing.  Returns (seconds, points)."""
    torch = pool.torch
    plans = {}
    for k in sorted(set(int(k) for k in kinds)):
        t = pool.types[k]
        plans[k] = api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, precision=t.precision)
    us = {k: pool.take_u(k) for k in plans}
    for k, pl in plans.items():
        pl.execute(pool.sigma[k], us[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pts = 0
    for k in kinds:
        k = int(k)
        plans[k].execute(pool.sigma[k], us[k])
        pts += pool.types[k].npoints
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for k, u in us.items():
        pool.give_u(k, u)
    for pl in plans.values():
        pl.close()
    return dt, pts


def closed_loop(server, pool, kinds):
    """All requests submitted at once, then drained.  Returns (seconds,
    points, completions)."""
    pool.torch.cuda.synchronize()
    live = {}
    t0 = time.perf_counter()
    for k in kinds:
        k = int(k)
        u = pool.take_u(k)
        live[_submit(server, pool, k, u)] = (k, u)
    done = server.drain()
    dt = time.perf_counter() - t0
    pts = 0
    for c in done:
        k, u = live.pop(c["id"])
        pool.give_u(k, u)
        if c["status"] != 0:
            raise RuntimeError(f"request {c['id']} failed with status {c['status']}")
        pts += c["npoints"]
    return dt, pts, done


def poisson(server, pool, kinds, qps, rng):
    """Poisson arrivals at `qps` requests/s.  Returns a summary dict."""
    gaps = rng.exponential(1.0 / qps, size=len(kinds))
    arrive = np.cumsum(gaps)
    live = {}
    late = {}
    lat = []
    pts = 0

    def collect(done):
        nonlocal pts
        for c in done:
            k, u = live.pop(c["id"])
            pool.give_u(k, u)
            if c["status"] != 0:
                raise RuntimeError(f"request {c['id']} failed with status {c['status']}")
            lat.append(late.pop(c["id"]) + c["total_ms"])
            pts += c["npoints"]

    pool.torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, k in enumerate(kinds):
        k = int(k)
        while True:
            now = time.perf_counter() - t0
            if now >= arrive[i]:
                break
            collect(server.poll())
            if arrive[i] - now > 2e-3:
                time.sleep(0.5e-3)
        u = pool.take_u(k)
        rid = _submit(server, pool, k, u)
        live[rid] = (k, u)
        late[rid] = 1e3 * (time.perf_counter() - t0 - arrive[i])
    collect(server.drain())
    dt = time.perf_counter() - t0
    return {"qps": float(qps), "requests": len(kinds), "seconds": dt,
            "achieved_qps": len(kinds) / dt, "points_per_s": pts / dt,
            "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "max_ms": float(max(lat))}
