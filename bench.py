"""Benchmark of the MI355X machine fast Gauss transform.

Headline workload (one "step" = one fgt_execute, every stage of Algorithm 4
over the whole tree): the 3D adaptive free-space transform with p = 16
Gauss-Legendre nodes per axis, delta = 1e-4, sigma a sum of 8 Gaussians
(widths log-uniform in [1e-3, 1e-2], centers U[-0.4,0.4]^3, amplitudes
U(-1,1), seed 0) resolved by the Legendre-tail test to 1e-9 ||sigma||_2 and
2:1 balanced: 2,661 leaves, N = 10,899,456 grid points, FP64 at tol = 1e-6.
Inputs are resident in HBM before the timed region.

The parent process never touches the GPU.  It runs every measurement in a
child process of its own (the headline first, then the small 2D workload,
the other tolerances and precisions, the periodic variant, the precision
form, the batched and the served forms), merges the children's JSON, records
the exit status of a child that fails (never retried), then runs the CPU
leg: the FP64 oracle over every leaf of each tree a child returned u for
(accuracy of every form, whole tree), timed on the headline tree as
cpu_baseline.  It prints ONE JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import shutil
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12   # dense FP64 matrix and vector, FLOP/s
PEAK_FP32 = 157.3e12  # dense FP32, FLOP/s
PEAK_HBM = 8.0e12     # bytes/s
STAGES = ("form_leaf", "form_box", "translate", "eval_box", "eval_leaf", "near")
CHILDREN = ("headline", "config0", "forms", "periodic", "precision", "batched", "served", "point")
METRIC = "grid points/s at tol=1e-6 (3D adaptive), FP64 vs mixed; p50/p99 latency"


def near_runs(plan) -> tuple:
    """(sources, (axis-3, axis-1) table runs, axis-3 table runs) summed over
    the near-field targets: the contraction counts of the near stage, which
    applies the axis-2 table per source, the axis-1 table once per run of
    sources sharing the axis-3 and axis-1 tables, and the axis-3 table once per
    run sharing the axis-3 table (d = 2: axis 1 per source, axis 2 per run)."""
    import numpy as np
    info = plan.info()
    d = info["dim"]
    st = plan.array("near_start")
    tab = plan.array("near_tab").reshape(-1, d)
    r_a = r_b = 0
    for t in range(len(st) - 1):
        q = tab[st[t]:st[t + 1]]
        if len(q) == 0:
            continue
        if d == 3:
            r_a += 1 + int(np.count_nonzero((q[1:, 2] != q[:-1, 2]) | (q[1:, 0] != q[:-1, 0])))
            r_b += 1 + int(np.count_nonzero(q[1:, 2] != q[:-1, 2]))
        else:
            r_a += 1 + int(np.count_nonzero(q[1:, 1] != q[:-1, 1]))
    return len(tab), r_a, r_b


def stage_work(info: dict, runs=None) -> dict:
    """Algorithmic flops and bytes per launch of every stage (real plane-wave
    basis, separable contractions, each 1D table applied once per group of
    leaves that shares it).  bytes are the HBM bytes the stage must move at
    minimum in this design.  runs: near_runs() of the plan (None: every near
    pair applies all d tables)."""
    d, p, nr = info["dim"], info["p"], info["nr"]
    nL, nA, nP, nN = info["n_pwleaf"], info["n_pwbox"], info["n_plist"], info["n_near_pair"]
    ts = 4 if info["precision"] == 1 else 8
    n2 = nr ** (d - 1)
    npts = info["npoints"]
    npw = nL * p ** d
    if d == 3:
        # axis 2 per leaf, axis 1 per row, axis 3 per plane (leaf groups that
        # share a 1D table); the intermediate holds one p x nr^2 block per plane
        nU = info["n_plane"]
        lead = 2.0 * nr * p ** 3 * nL + 2.0 * nr ** 2 * p ** 2 * info["n_row"]
        last = 2.0 * nr ** 3 * p * nU
    else:
        nU = nL
        lead = nL * sum(2.0 * nr ** a * p ** (d - a + 1) for a in range(1, d))
        last = nL * 2.0 * nr ** d * p
    tr_flops = (3.0 * d + 1) * nr ** d * nP
    if d == 3 and info["fused_translate"]:
        # the translation is fused with the first evaluation step: phi is read,
        # the plane intermediate written; psi never leaves the chip
        translate = {"flops": tr_flops + last, "bytes": ts * nA * nr ** d + ts * nU * p * n2}
        eval_box = {"flops": 0.0, "bytes": 0.0}
    else:
        translate = {"flops": tr_flops, "bytes": 2.0 * ts * nA * nr ** d}
        eval_box = {"flops": last, "bytes": ts * nA * nr ** d + ts * nU * p * n2}
    return {
        "form_leaf": {"flops": lead, "bytes": 8.0 * npw + ts * nU * p * n2},
        "form_box": {"flops": last, "bytes": ts * nU * p * n2 + ts * nA * nr ** d},
        "translate": translate,
        "eval_box": eval_box,
        "eval_leaf": {"flops": lead, "bytes": ts * nU * p * n2 + 8.0 * npw},
        # sigma of every distinct source once; u of every target written (and
        # read first where the plane-wave evaluation already wrote it)
        "near": {"flops": (2.0 * d * p ** (d + 1) * nN if runs is None else
                           2.0 * p ** (d + 1) * sum(runs)),
                 "bytes": 8.0 * p ** d * (info["n_near_source"] + info["n_near_target"]
                                          + info["n_near_haspw"])},
    }


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels_fast.hip", "kernels.h", "mfma.h", "stage_bodies.h", "translate.h",
              "plan.cpp"):
        with open(os.path.join(ROOT, "paper_2305_07165_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(stage: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this stage, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get("stages", {}).get(stage)
    if not rec or t.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def timed_steps(plan, s, u, steps, warmup, torch):
    for _ in range(warmup):
        plan.execute(s, u)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        plan.execute(s, u)
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = sorted(a.elapsed_time(b) for a, b in zip(starts, ends))
    return wall, per


def pct(sorted_ms, q):
    if not sorted_ms:
        return None
    i = min(len(sorted_ms) - 1, max(0, int(math.ceil(q / 100.0 * len(sorted_ms))) - 1))
    return sorted_ms[i]




# ---------------------------------------------------------------------------
# children: each runs one measurement on the GPU and returns a dict; arrays of
# u it wants checked against the oracle are saved under the run's scratch
# directory and listed in "arrays"


class Ctx:
    def __init__(self, args):
        self.args = args
        self.tmp = args.tmp

    def log(self, msg):
        print(f"[bench:{self.args.child}] {msg}", file=sys.stderr, flush=True)

    def save(self, name, arr):
        import numpy as np
        path = os.path.join(self.tmp, f"{self.args.child}-{name}.npy")
        np.save(path, np.ascontiguousarray(arr))
        return path


def _array(name, path, tree, delta, periodic, tol):
    return {"name": name, "path": path, "tree": tree, "delta": delta, "periodic": periodic, "tol": tol}


def child_headline(ctx):
    import torch

    from paper_2305_07165_amd import api, synth
    args = ctx.args
    t0 = time.perf_counter()
    pr = synth.adaptive_3d(args.seed)
    ctx.log(f"tree: {len(pr.levels)} leaves, N={pr.npoints}, generated in {time.perf_counter() - t0:.1f}s")
    s = torch.from_numpy(pr.sigma).to("cuda:0")
    u = torch.empty_like(s)
    tp = time.perf_counter()
    plan = api.Plan(pr.levels, pr.coords, pr.p, pr.delta, args.tol)
    plan_ms = 1e3 * (time.perf_counter() - tp)
    info = plan.info()
    ctx.log(f"plan: lc={info['lc']} nr={info['nr']} pw_boxes={info['n_pwbox']} pw_leaves={info['n_pwleaf']} "
            f"translations={info['n_plist']} near_pairs={info['n_near_pair']} plan_ms={plan_ms:.1f}")
    wall, per = timed_steps(plan, s, u, args.steps, args.warmup, torch)
    ms_step = 1e3 * wall / args.steps
    value = pr.npoints * args.steps / wall
    ctx.log(f"fp64 tol={args.tol:g}: {ms_step:.3f} ms/step, {value:.3e} pts/s")
    upath = ctx.save("u", u.cpu().numpy())
    # per-stage HIP-event durations on the plan's stream (profiled plan, same work)
    pplan = api.Plan(pr.levels, pr.coords, pr.p, pr.delta, args.tol, profile=True)
    for _ in range(args.warmup):
        pplan.execute(s, u)
    torch.cuda.synchronize()
    acc = {k: 0.0 for k in STAGES}
    for _ in range(args.steps):
        pplan.execute(s, u)
        pplan.sync()
        for k, v in pplan.stage_times().items():
            acc[k] += v
    stage_ms = {k: v / args.steps for k, v in acc.items()}
    pplan.close()
    work = stage_work(info, near_runs(plan))
    plan.close()
    dom = max(stage_ms, key=stage_ms.get)
    wd = work[dom]
    t_dom = stage_ms[dom] * 1e-3
    fl_rate, by_rate = wd["flops"] / t_dom, wd["bytes"] / t_dom
    if wd["flops"] / PEAK_FP64 >= wd["bytes"] / PEAK_HBM:
        # translations are vector arithmetic (rotations), the rest matrix-core products
        roof = {"bound": "alu" if dom == "translate" else "mfma", "achieved": fl_rate / 1e12,
                "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": fl_rate / PEAK_FP64}
    else:
        roof = {"bound": "hbm", "achieved": by_rate / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": by_rate / PEAK_HBM}
    roof.update({"kernel": dom, "traffic": load_traffic(dom), "mean_ms": stage_ms[dom],
                 "algorithmic_flops": wd["flops"], "algorithmic_bytes": wd["bytes"]})
    tstar = sum(max(work[k]["flops"] / PEAK_FP64, work[k]["bytes"] / PEAK_HBM) for k in STAGES)
    path = {"t_star_ms": 1e3 * tstar, "stage_ms": stage_ms,
            "frac": 1e3 * tstar / max(sum(stage_ms.values()), 1e-9)}
    ctx.log(f"stages: {json.dumps({k: round(v, 4) for k, v in stage_ms.items()})}")
    return {"value": value, "ms_per_step": ms_step, "p50_ms": pct(per, 50), "p99_ms": pct(per, 99),
            "roofline": roof, "path_roofline": path,
            "flops_per_point": sum(work[k]["flops"] for k in STAGES) / pr.npoints,
            "config": {"workload": "3d-adaptive-free p=16 delta=1e-4 8 Gaussians seed %d, tol %g"
                                   % (args.seed, args.tol),
                       "npoints": pr.npoints, "nleaves": int(len(pr.levels)), "tol": args.tol,
                       "lc": info["lc"], "nr": info["nr"], "plan_ms": plan_ms},
            "arrays": [_array("fp64_tol%g" % args.tol, upath, "adaptive_3d", pr.delta, False, args.tol)]}


def child_config0(ctx):
    """The small 2D workload (uniform level-3 tree, 64 leaves, p = 8, 4,096
    points, delta = 1e-3, tol 1e-6): launch-latency bound, so it reports the
    per-execute device time (HIP events, p50/p99 in microseconds), the host
    time per call, and points/s, on both routes: the automatic cutoff level
    (3: every pair direct) and the cutoff forced to 2 (every pair by plane
    waves)."""
    import torch

    from paper_2305_07165_amd import api, synth
    args = ctx.args
    pr = synth.small_2d(args.seed)
    s = torch.from_numpy(pr.sigma).to("cuda:0")
    steps, warm = max(200, 4 * args.steps), max(20, args.warmup)
    out = {"workload": "2d-uniform-l3 p=8 delta=1e-3 4 Gaussians seed %d, tol 1e-6" % args.seed,
           "npoints": pr.npoints, "arrays": []}
    for name, force_lc in (("auto", -1), ("forced_lc2", 2)):
        u = torch.empty_like(s)
        plan = api.Plan(pr.levels, pr.coords, pr.p, pr.delta, pr.tol, force_lc=force_lc)
        info = plan.info()
        wall, per = timed_steps(plan, s, u, steps, warm, torch)
        med = pct(per, 50)
        rec = {"lc": info["lc"], "nr": info["nr"], "n_near_pair": info["n_near_pair"],
               "n_pwleaf": info["n_pwleaf"], "steps": steps,
               "p50_us": 1e3 * med, "p99_us": 1e3 * pct(per, 99),
               "host_us_per_call": 1e6 * wall / steps,
               "points_per_s": pr.npoints / (med * 1e-3),
               "points_per_s_wall": pr.npoints * steps / wall}
        out[name] = rec
        out["arrays"].append(_array(f"config0_{name}", ctx.save(name, u.cpu().numpy()),
                                    "small_2d", pr.delta, False, pr.tol))
        plan.close()
        ctx.log(f"{name}: lc={info['lc']} p50 {rec['p50_us']:.1f} us p99 {rec['p99_us']:.1f} us, "
                f"{rec['points_per_s']:.3e} pts/s, host {rec['host_us_per_call']:.1f} us/call")
    return out


def child_forms(ctx):
    """The headline tree at tol 1e-10 (FP64) and at tol 1e-6 with FP32 products."""
    import torch

    from paper_2305_07165_amd import api, synth
    args = ctx.args
    pr = synth.adaptive_3d(args.seed)
    s = torch.from_numpy(pr.sigma).to("cuda:0")
    out = {"arrays": []}
    for name, tol, prec in (("fp64_tol1e-10", 1e-10, "fp64"), ("fp32_tol1e-6", 1e-6, "fp32")):
        fp = api.Plan(pr.levels, pr.coords, pr.p, pr.delta, tol, precision=prec)
        uf = torch.empty_like(s)
        fw, fper = timed_steps(fp, s, uf, args.steps, args.warmup, torch)
        fi = fp.info()
        out[name] = {"value": pr.npoints * args.steps / fw, "ms_per_step": 1e3 * fw / args.steps,
                     "p50_ms": pct(fper, 50), "p99_ms": pct(fper, 99), "tol": tol,
                     "dtype": "f64" if prec == "fp64" else "f32", "nr": fi["nr"], "lc": fi["lc"]}
        out["arrays"].append(_array(name, ctx.save(name, uf.cpu().numpy()), "adaptive_3d", pr.delta,
                                    False, tol))
        fp.close()
        ctx.log(f"{name}: {out[name]['ms_per_step']:.3f} ms/step")
    return out


def child_periodic(ctx):
    """The periodic variant of the 3D workload (blobs periodized over Z^3); its
    tree and samples are built on the device by Algorithm 3."""
    import torch

    from paper_2305_07165_amd import api, synth
    args = ctx.args
    dens = synth.adaptive_3d_density(args.seed, wrap_blobs=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lvp, csp, sp, _ = api.resolve_gaussians(dens.centers, dens.widths, dens.amps, 16, 1e-9,
                                           periodic=True, max_level=7)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    tree = {"levels": ctx.save("levels", lvp), "coords": ctx.save("coords", csp),
            "sigma": ctx.save("sigma", sp.cpu().numpy()), "p": 16}
    up = torch.empty_like(sp)
    npp = int(sp.numel())
    out = {"arrays": []}
    for tol in (1e-6, 1e-10):
        pp = api.Plan(lvp, csp, 16, 1e-4, tol, periodic=True)
        pw, pper = timed_steps(pp, sp, up, args.steps, args.warmup, torch)
        pi = pp.info()
        name = f"periodic_fp64_tol{tol:g}"
        out[name] = {"value": npp * args.steps / pw, "ms_per_step": 1e3 * pw / args.steps,
                     "p50_ms": pct(pper, 50), "p99_ms": pct(pper, 99), "tol": tol, "dtype": "f64",
                     "npoints": npp, "nleaves": int(len(lvp)), "lc": pi["lc"], "nr": pi["nr"],
                     "tree_ms_device": 1e3 * tg}
        out["arrays"].append(_array(name, ctx.save(name, up.cpu().numpy()), tree, 1e-4, True, tol))
        pp.close()
        ctx.log(f"periodic tol={tol:g}: {len(lvp)} leaves (built on the device in {1e3 * tg:.1f} ms), "
                f"{1e3 * pw / args.steps:.3f} ms/step, {npp * args.steps / pw:.3e} pts/s")
    return out


def child_precision(ctx):
    """The headline tree at delta in {1e-3, 1e-5}: FP32 and split-bf16 products
    at tol 1e-3 and 1e-6 (and 1e-4, the smallest tol split bf16 is accepted
    at), timed beside FP64 at tol 1e-6 on the same delta.  A precision fgt_plan
    refuses at a tol is recorded as refused."""
    import torch

    from paper_2305_07165_amd import api, synth
    args = ctx.args
    steps = min(args.steps, 20)
    pr = synth.adaptive_3d(args.seed)
    s = torch.from_numpy(pr.sigma).to("cuda:0")
    u = torch.empty_like(s)
    out = {"arrays": []}
    for delta in (1e-3, 1e-5):
        key = f"delta_{delta:g}"

        def run(tol, prec):
            pl = api.Plan(pr.levels, pr.coords, pr.p, delta, tol, precision=prec)
            wall, per = timed_steps(pl, s, u, steps, args.warmup, torch)
            info = pl.info()
            pl.close()
            name = f"{key}_{prec}_tol{tol:g}"
            out["arrays"].append(_array(name, ctx.save(name, u.cpu().numpy()), "adaptive_3d", delta,
                                        False, tol))
            return 1e3 * wall / steps, info

        ms64, i64 = run(1e-6, "fp64")
        rec = {"delta": delta, "fp64_tol1e-6": {"ms": ms64, "points_per_s": pr.npoints / (ms64 * 1e-3),
                                                "lc": i64["lc"], "nr": i64["nr"]}}
        for prec, tol in (("fp32", 1e-3), ("fp32", 1e-6), ("bf16x3", 1e-3), ("bf16x3", 1e-4),
                          ("bf16x3", 1e-6)):
            name = f"{prec}_tol{tol:g}"
            try:
                ms, info = run(tol, prec)
            except api.FgtError as e:
                rec[name] = {"refused": str(e)}
                continue
            rec[name] = {"ms": ms, "points_per_s": pr.npoints / (ms * 1e-3), "nr": info["nr"],
                         "speedup_vs_fp64_tol1e-6": ms64 / ms}
        ctx.log(f"precision delta={delta:g}: fp64 1e-6 {ms64:.3f} ms; " + "; ".join(
            f"{k} " + (f"{v['ms']:.3f} ms" if "ms" in v else "refused") for k, v in rec.items()
            if isinstance(v, dict) and k != "fp64_tol1e-6"))
        out[key] = rec
    return out


def child_batched(ctx):
    """The batched workload (synth.batch_problems): every transform in its own
    precision (FP32 when tol >= 1e-6, else FP64) in one batch (per-class
    launches captured in one HIP graph on one stream), against the same
    transforms run one after another with plain fgt_execute, in their own
    precision and all in FP64."""
    from paper_2305_07165_amd import synth
    args = ctx.args
    t0 = time.perf_counter()
    # generated before the process touches the GPU (tree building forks workers)
    probs = synth.batch_problems(args.seed + 200, args.batch_size, workers=min(16, os.cpu_count() or 1))
    ctx.log(f"{len(probs)} transforms, generated in {time.perf_counter() - t0:.1f}s")
    import torch

    from paper_2305_07165_amd import api
    steps = 3
    npts = sum(t.npoints for t in probs)
    sig = [torch.from_numpy(t.sigma).cuda() for t in probs]

    def seq(prec_of, no_fuse=False):
        plans = [api.Plan(t.levels, t.coords, t.p, t.delta, t.tol, precision=prec_of(t), no_fuse=no_fuse)
                 for t in probs]
        us = [torch.empty_like(s) for s in sig]
        for pl, s_, u_ in zip(plans, sig, us):
            pl.execute(s_, u_)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for pl, s_, u_ in zip(plans, sig, us):
                pl.execute(s_, u_)
        torch.cuda.synchronize()
        return plans, us, (time.perf_counter() - t0) / steps

    plans64, _, dt64 = seq(lambda t: "fp64")
    for pl in plans64:
        pl.close()
    del plans64
    plans, us_seq, dtmix = seq(lambda t: t.precision)
    ctx.log(f"{npts} points; sequential fp64 {1e3 * dt64:.2f} ms, sequential mixed {1e3 * dtmix:.2f} ms")
    b = api.Batch(plans)
    us = [torch.empty_like(s) for s in sig]
    b.bind(sig, us)
    b.execute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.execute()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    same = all(torch.equal(a, c) for a, c in zip(us, us_seq))
    info = b.info()
    ctx.log(f"{1e3 * dt:.2f} ms per batch ({npts / dt:.3e} pts/s), {info['nclasses']} classes, "
            f"{info['nlaunches']} launches, bitwise equal to sequential: {same}")
    b.close()
    for pl in plans:
        pl.close()
    return {"value": npts / dt, "unit": "grid points/s", "ms_per_batch": 1e3 * dt, "transforms": len(probs),
            "npoints": npts, "sequential_fp64_ms": 1e3 * dt64, "sequential_same_precision_ms": 1e3 * dtmix,
            "speedup_vs_sequential_fp64": dt64 / dt, "speedup_vs_sequential_same_precision": dtmix / dt,
            "bitwise_equal_to_sequential": same, "schedule": "per-class launches, one stream, one HIP graph",
            "persistent": "switched off: one persistent launch per kernel class did not finish on the device",
            "nclasses": info["nclasses"], "nlaunches": info["nlaunches"],
            "precisions": {"fp32": sum(t.precision == "fp32" for t in probs),
                           "fp64": sum(t.precision == "fp64" for t in probs)}}


def child_served(ctx):
    """The serving workload: a pool of request types (d ~ U{2,3}, N log-uniform
    in [1e4, 1e8], delta log-uniform in [1e-6, 1e-2], tol ~ U{1e-3, 1e-6,
    1e-10}, p ~ U{8, 16}), requests drawn uniformly from the pool.  Reports
    sequential plain execution, the server's closed-loop capacity, and Poisson
    arrivals at 30/60/90% of that capacity (latency arrival -> done)."""
    import numpy as np

    from paper_2305_07165_amd import api, serving, synth
    args = ctx.args
    seed, nreq = args.seed + 100, args.serve_requests
    t0 = time.perf_counter()
    types = synth.serve_request_types(seed, 12)
    ctx.log(f"{len(types)} request types, {sum(t.npoints for t in types)} points in all, "
            f"generated in {time.perf_counter() - t0:.1f}s")
    pool = serving.Pool(types)
    rng = np.random.default_rng(seed + 1)
    kinds = rng.integers(0, len(types), nreq)
    out = {"pool": [{"d": t.d, "p": t.p, "npoints": t.npoints, "delta": t.delta, "tol": t.tol,
                     "precision": t.precision} for t in types], "requests": int(nreq)}
    seq_s, seq_pts = serving.sequential(pool, kinds)
    out["sequential_points_per_s"] = seq_pts / seq_s
    with api.Server(nslots=4, nbuilders=4) as srv:
        tw = time.perf_counter()
        serving.warm(srv, pool)
        out["warm_s"] = time.perf_counter() - tw
        cl_s, cl_pts, done = serving.closed_loop(srv, pool, kinds)
        cap = nreq / cl_s
        out.update({"value": cl_pts / cl_s, "unit": "grid points/s", "capacity_rps": cap,
                    "speedup_vs_sequential": (cl_pts / cl_s) / (seq_pts / seq_s),
                    "closed_loop_p50_ms": float(np.percentile([c["total_ms"] for c in done], 50)),
                    "closed_loop_p99_ms": float(np.percentile([c["total_ms"] for c in done], 99))})
        ctx.log(f"closed loop: {cap:.1f} req/s, {cl_pts / cl_s:.3e} pts/s "
                f"(sequential {seq_pts / seq_s:.3e} pts/s)")
        out["poisson"] = []
        for frac in (0.3, 0.6, 0.9):
            r = serving.poisson(srv, pool, kinds, frac * cap, np.random.default_rng(seed + 2))
            r["load"] = frac
            out["poisson"].append(r)
            ctx.log(f"poisson {frac:.0%}: p50 {r['p50_ms']:.2f} ms p99 {r['p99_ms']:.2f} ms "
                    f"{r['points_per_s']:.3e} pts/s")
        out["server_stats"] = srv.stats()
    return out


def child_point(ctx):
    """The point transform with proxy grids (fgt_point.h) on the paper's 3D
    point workload shape (points on a surface, delta = 0.007 with N = 3.4e6):
    3,400,000 points uniform on the sphere of radius 0.35 (synth.point_sphere,
    seed + 300), each a source and a target, tol 1e-6, p = 16, n_s = 64.
    Reports sources + targets per second of execute (plan time apart) and
    saves 1,000 sampled targets for the oracle."""
    import numpy as np
    import torch

    from paper_2305_07165_amd import api, synth
    args = ctx.args
    x, q = synth.point_sphere(args.seed + 300)
    delta, tol = 0.007, 1e-6
    tp = time.perf_counter()
    pl = api.PointPlan(x, x, delta, tol, p=16, ns=64)
    plan_ms = 1e3 * (time.perf_counter() - tp)
    info = pl.info()
    qd = torch.from_numpy(q).cuda()
    u = torch.empty(len(x), dtype=torch.float64, device="cuda")
    steps = max(5, args.steps // 2)
    for _ in range(args.warmup):
        pl.execute(qd, u)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        pl.execute(qd, u)
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = sorted(a.elapsed_time(b) for a, b in zip(starts, ends))
    pl.close()
    pick = np.random.default_rng(args.seed + 301).choice(len(x), 1000, replace=False)
    ms = 1e3 * wall / steps
    npts = 2 * len(x)
    ctx.log(f"{len(x)} points on a sphere: lc={info['lc']} lp={info['lp']} dense={info['ndense']} "
            f"proxies={info['nproxy']} direct terms={info['ndirect_terms']}; {ms:.3f} ms/execute, "
            f"{npts / (ms * 1e-3):.3e} points/s, plan {plan_ms:.0f} ms")
    arrays = {"src": ctx.save("src", x), "q": ctx.save("q", q), "tgt": ctx.save("tgt", x[pick]),
              "u": ctx.save("u", u.cpu().numpy()[pick])}
    return {"value": npts / (ms * 1e-3), "unit": "source+target points/s", "ms_per_execute": ms,
            "p50_ms": pct(per, 50), "p99_ms": pct(per, 99), "plan_ms": plan_ms, "delta": delta, "tol": tol,
            "workload": "3d points on a sphere (r = 0.35), 3.4e6 sources = targets, delta=0.007, tol 1e-6, "
                        "p=16, n_s=64, seed %d" % (args.seed + 300),
            "info": {k: info[k] for k in ("lc", "lp", "ndense", "npwbox", "nproxy", "nplist",
                                          "ndirect_terms", "proxy_err")},
            "point_arrays": arrays}


# ---------------------------------------------------------------------------
# parent: children in order, then the CPU leg


CHILD_TIMEOUT_S = {"headline": 300, "config0": 120, "forms": 180, "periodic": 180, "precision": 240, "point": 180,
                   "batched": 300, "served": 300}


def run_child(name, args, log):
    cmd = [sys.executable, os.path.abspath(__file__), "--child", name, "--tmp", args.tmp,
           "--steps", str(args.steps), "--warmup", str(args.warmup), "--seed", str(args.seed),
           "--tol", repr(args.tol), "--batch-size", str(args.batch_size),
           "--serve-requests", str(args.serve_requests)]
    t0 = time.perf_counter()
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=None, text=True,
                           timeout=CHILD_TIMEOUT_S[name])
        rc, text = r.returncode, r.stdout
    except subprocess.TimeoutExpired as e:
        rc, text = 124, (e.stdout or b"").decode() if isinstance(e.stdout, bytes) else (e.stdout or "")
    dt = time.perf_counter() - t0
    res = None
    for line in reversed(text.strip().splitlines()):
        if line.startswith("{"):
            try:
                res = json.loads(line)
            except ValueError:
                res = None
            break
    if rc != 0 or res is None:
        log(f"child {name} failed: rc={rc} after {dt:.1f}s")
        return {"rc": rc, "seconds": dt, "error": "exit status %d" % rc}
    log(f"child {name} done in {dt:.1f}s")
    res["rc"], res["seconds"] = 0, dt
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(results, args, log):
    """The oracle over every leaf of each (tree, delta, boundary) that a child
    returned u for: rel-l2 and max-abs errors of every form, and the oracle's
    own time on the headline tree (cpu_baseline)."""
    import numpy as np

    import oracle
    from paper_2305_07165_amd import synth
    groups = {}
    for cname, res in results.items():
        for a in res.get("arrays", []):
            tk = json.dumps(a["tree"], sort_keys=True)
            groups.setdefault((tk, a["delta"], a["periodic"]), []).append((cname, a))
    trees = {}
    acc = {}
    cpu = None
    for (tk, delta, periodic), items in groups.items():
        tree = json.loads(tk)
        if tree not in ("adaptive_3d", "small_2d") and not isinstance(tree, dict):
            continue
        if tk not in trees:
            if tree == "adaptive_3d":
                pr = synth.adaptive_3d(args.seed)
                trees[tk] = (pr.levels, pr.coords, pr.p, pr.sigma)
            elif tree == "small_2d":
                pr = synth.small_2d(args.seed)
                trees[tk] = (pr.levels, pr.coords, pr.p, pr.sigma)
            else:
                trees[tk] = (np.load(tree["levels"]), np.load(tree["coords"]), tree["p"],
                             np.load(tree["sigma"]))
        lv, cs, p, sig = trees[tk]
        t0 = time.perf_counter()
        uo = oracle.oracle_u(lv, cs, p, delta, sig, periodic=periodic)
        dt = time.perf_counter() - t0
        log(f"oracle: {len(lv)} leaves, delta={delta:g}, periodic={periodic}: {dt:.1f}s")
        if tree == "adaptive_3d" and delta == 1e-4 and not periodic:
            nt = len(lv)
            cpu = {"value": nt * p ** 3 / dt, "unit": "grid points/s", "cores": oracle.threads_used(),
                   "cpu_model": cpu_model(), "kind": "oracle",
                   "sample": f"all {nt} leaves ({nt * p ** 3} grid points) of the headline tree, every "
                             f"source leaf within r_cut, FP64, {dt:.1f} s"}
        nrm, mx = float(np.linalg.norm(uo)), float(np.max(np.abs(uo)))
        for cname, a in items:
            ug = np.load(a["path"])
            e = {"rel_l2": float(np.linalg.norm(ug - uo) / nrm),
                 "max_abs_rel": float(np.max(np.abs(ug - uo)) / mx), "tol": a["tol"],
                 "nodes_compared": int(ug.size)}
            e["meets_tol"] = e["rel_l2"] < a["tol"] and e["max_abs_rel"] < a["tol"]
            acc[a["name"]] = e
            os.remove(a["path"])
    pa = results.get("point", {}).get("point_arrays")
    if pa:
        src, q, tgt, ug = (np.load(pa[k]) for k in ("src", "q", "tgt", "u"))
        t0 = time.perf_counter()
        uo = oracle.oracle_point(src, q, tgt, results["point"]["delta"])
        log(f"oracle: point transform at {len(tgt)} sampled targets: {time.perf_counter() - t0:.1f}s")
        acc["point"] = {"rel_l2": float(np.linalg.norm(ug - uo) / np.linalg.norm(uo)),
                        "max_abs_rel": float(np.max(np.abs(ug - uo)) / np.max(np.abs(uo))), "tol": 1e-6,
                        "nodes_compared": int(len(tgt)), "sampled": True}
        acc["point"]["meets_tol"] = acc["point"]["rel_l2"] < 1e-6 and acc["point"]["max_abs_rel"] < 1e-6
        for k in pa.values():
            os.remove(k)
    return acc, cpu


def attach_accuracy(forms, acc):
    """Puts each array's error next to the timing it belongs to."""
    for name, e in acc.items():
        if name in forms and isinstance(forms[name], dict):
            forms[name]["accuracy"] = e
    prec = forms.get("precision", {})
    for key, rec in prec.items():
        if not isinstance(rec, dict) or not key.startswith("delta_"):
            continue
        for k, v in rec.items():
            a = acc.get(f"{key}_{k}")
            if isinstance(v, dict) and a:
                v["accuracy"] = a
    if "point" in forms and "point" in acc:
        forms["point"]["accuracy"] = acc["point"]
    c0 = forms.get("config0", {})
    for k in ("auto", "forced_lc2"):
        if k in c0 and f"config0_{k}" in acc:
            c0[k]["accuracy"] = acc[f"config0_{k}"]


def parent(args):
    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    skip = set()
    if args.no_forms:
        skip |= {"forms", "periodic", "precision", "batched", "served", "point"}
    if args.no_batch:
        skip.add("batched")
    if args.no_serve:
        skip.add("served")
    args.tmp = tempfile.mkdtemp(prefix="fgt_bench_")
    results = {}
    try:
        for name in CHILDREN:
            if name in skip:
                continue
            log(f"child {name}")
            results[name] = run_child(name, args, log)
        acc, cpu = ({}, None)
        if args.cpu_leaves != 0:
            acc, cpu = cpu_leg(results, args, log)
    finally:
        shutil.rmtree(args.tmp, ignore_errors=True)
    head = results.get("headline", {})
    forms = {}
    for name in ("forms", "periodic"):
        for k, v in results.get(name, {}).items():
            if isinstance(v, dict) and "ms_per_step" in v:
                if head.get("value"):
                    v["speedup_vs_fp64_tol1e-6"] = v["value"] / head["value"]
                forms[k] = v
    for name in ("config0", "precision", "batched", "served", "point"):
        if name in results:
            forms[name] = {k: v for k, v in results[name].items() if k not in ("arrays", "point_arrays")}
    attach_accuracy(forms, acc)
    for name in ("forms", "periodic"):
        if name in results and results[name].get("rc"):
            forms[name + "_error"] = {"rc": results[name]["rc"]}
    hacc = acc.get("fp64_tol%g" % args.tol)
    out = {
        "metric": METRIC, "value": head.get("value"), "unit": "grid points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head.get("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": head.get("config", {"workload": "3d-adaptive-free p=16 delta=1e-4 8 Gaussians seed %d, "
                                                  "tol %g" % (args.seed, args.tol)}),
        "p50_ms": head.get("p50_ms"), "p99_ms": head.get("p99_ms"),
        "roofline": head.get("roofline"), "path_roofline": head.get("path_roofline"),
        "cpu_baseline": cpu,
        "accuracy": hacc,
        "accuracy_rel_l2": {k: v["rel_l2"] for k, v in acc.items()},
        "forms": forms,
        "flops_per_point": head.get("flops_per_point"),
        "children": {k: {"rc": v.get("rc"), "seconds": v.get("seconds")} for k, v in results.items()},
        # the paper's own figures for this method, on other hardware: context, not a target
        "paper_context": {"value_range": [1e6, 7e6], "unit": "grid points/s", "d": 3,
                          "hardware": "1 thread of an Intel i9-10885H at 2.40 GHz, Fortran, no SIMD",
                          "workload": "adaptive tensor Legendre grids, k = 16, several tolerances"},
    }
    print(json.dumps(out), flush=True)
    return 0 if head.get("rc") == 0 else 1


def profile_only(args):
    """warmup + steps of the headline plan in this process (for rocprofv3)."""
    import torch

    from paper_2305_07165_amd import api, synth
    pr = synth.adaptive_3d(args.seed)
    s = torch.from_numpy(pr.sigma).to("cuda:0")
    u = torch.empty_like(s)
    plan = api.Plan(pr.levels, pr.coords, pr.p, pr.delta, args.tol)
    timed_steps(plan, s, u, args.steps, args.warmup, torch)
    if args.calib_copy:
        # a plain device copy of known size: 1 GiB read + 1 GiB written, to
        # scale the FETCH_SIZE / WRITE_SIZE counters
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    plan.close()
    print("[bench] profile-only run done", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cpu-leaves", type=int, default=-1,
                    help="0 = skip the CPU leg (oracle accuracy and cpu_baseline); else every leaf")
    ap.add_argument("--no-forms", action="store_true", help="headline and the small 2D workload only")
    ap.add_argument("--no-serve", action="store_true", help="skip the served form")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched form")
    ap.add_argument("--batch-size", type=int, default=512)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup+steps of the headline plan only, in this process (for rocprofv3)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="with --profile-only: also run a 1 GiB device copy (counter scale)")
    ap.add_argument("--child", choices=CHILDREN, help=argparse.SUPPRESS)
    ap.add_argument("--tmp", help=argparse.SUPPRESS)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the transform runs on one GPU only; there is no multi-GPU run "
              "(it would shard by cutoff-level subtrees with a one-box halo of sigma).",
              file=sys.stderr)
        sys.exit(2)
    if args.profile_only:
        profile_only(args)
        return
    if args.child:
        ctx = Ctx(args)
        res = globals()["child_" + args.child](ctx)
        print(json.dumps(res), flush=True)
        return
    sys.exit(parent(args))


if __name__ == "__main__":
    main()
