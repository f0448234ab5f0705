"""Python binding of the C ABI (include/*.h), argument marshalling only.

Functions carry the C names (``fgt_plan``, ``fgt_execute``, ...).  ``Plan`` is
a small owner object on top of them.  sigma/u are torch tensors on the GPU
(or anything with ``data_ptr()``); no arithmetic of the transform happens here.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (FGT_BF16X3, FGT_ERR_UNSUPPORTED, FGT_FP32, FGT_FP64, FGT_FREE, FGT_PERIODIC,  # noqa: F401
                   FgtError, check)

_PRECISION = {"fp64": FGT_FP64, "fp32": FGT_FP32, "bf16x3": FGT_BF16X3}


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _tree(levels, coords):
    """(fgt_tree_t, the arrays it points to) for host leaf arrays."""
    levels = np.ascontiguousarray(levels, dtype=np.int32)
    coords = np.ascontiguousarray(coords, dtype=np.int32)
    if coords.ndim != 2 or coords.shape[0] != levels.shape[0]:
        raise ValueError("coords must be [nleaves, dim] matching levels")
    tree = _lib.fgt_tree_t(coords.shape[1], levels.shape[0],
                           levels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           coords.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return tree, (levels, coords)


def fgt_plan(levels, coords, p: int, delta: float, tol: float, bc: int = FGT_FREE,
             precision: int = FGT_FP64, eps_internal: float = 0.0, force_lc: int = -1,
             stream: int = 0, profile: bool = False, host_only: bool = False,
             own_stream: bool = False, no_fuse: bool = False) -> int:
    """Plans a transform; returns the opaque plan handle (an int)."""
    L = _lib.lib()
    levels = np.ascontiguousarray(levels, dtype=np.int32)
    coords = np.ascontiguousarray(coords, dtype=np.int32)
    if coords.ndim != 2 or coords.shape[0] != levels.shape[0]:
        raise ValueError("coords must be [nleaves, dim] matching levels")
    tree = _lib.fgt_tree_t(coords.shape[1], levels.shape[0],
                           levels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           coords.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    opts = _lib.fgt_opts_t(int(precision), float(eps_internal), int(force_lc),
                           ctypes.c_void_p(int(stream) or None), int(bool(own_stream)),
                           int(bool(profile)), int(bool(host_only)), int(bool(no_fuse)))
    h = ctypes.c_void_p()
    check(L.fgt_plan(ctypes.byref(tree), int(p), float(delta), float(tol), int(bc),
                     ctypes.byref(opts), ctypes.byref(h)), "fgt_plan")
    return h.value


def fgt_execute(plan: int, sigma, u) -> None:
    check(_lib.lib().fgt_execute(plan, _ptr(sigma), _ptr(u)), "fgt_execute")


def fgt_execute_noalloc(plan: int, sigma, u) -> None:
    check(_lib.lib().fgt_execute_noalloc(plan, _ptr(sigma), _ptr(u)), "fgt_execute_noalloc")


def fgt_sync(plan: int) -> None:
    check(_lib.lib().fgt_sync(plan), "fgt_sync")


def fgt_plan_info(plan: int) -> dict:
    info = _lib.fgt_info_t()
    check(_lib.lib().fgt_plan_info(plan, ctypes.byref(info)), "fgt_plan_info")
    return info.as_dict()


STAGES = ("form_leaf", "form_box", "translate", "eval_box", "eval_leaf", "near")


def fgt_stage_times(plan: int) -> dict:
    ms = (ctypes.c_double * 6)()
    n = check(_lib.lib().fgt_stage_times(plan, ms, 6), "fgt_stage_times")
    return {STAGES[i]: ms[i] for i in range(n)}


def fgt_destroy(plan: int) -> None:
    if plan:
        _lib.lib().fgt_destroy(plan)


def fgt_strerror(code: int) -> str:
    return _lib.lib().fgt_strerror(code).decode()


def fgt_pw_terms(eps: float, r_over_d0: float) -> int:
    return check(_lib.lib().fgt_pw_terms(eps, r_over_d0), "fgt_pw_terms")


def fgt_periodic_terms(eps: float, delta: float) -> int:
    return check(_lib.lib().fgt_periodic_terms(eps, delta), "fgt_periodic_terms")


_DOUBLE_ARRAYS = {"F", "E", "V", "rot"}


def fgt_plan_array(plan: int, name: str) -> np.ndarray:
    L = _lib.lib()
    n = check(L.fgt_plan_array(plan, name.encode(), None, 0), "fgt_plan_array")
    dt = np.float64 if name in _DOUBLE_ARRAYS else np.int32
    out = np.zeros(n, dtype=dt)
    if n:
        check(L.fgt_plan_array(plan, name.encode(), out.ctypes.data, n), "fgt_plan_array")
    return out


class Plan:
    """Owns one plan.  ``execute(sigma)`` returns u (a new tensor like sigma).

    By default the plan runs on torch's current stream of the current device,
    so it is ordered with the torch work that produces sigma and consumes u.
    """

    def __init__(self, levels, coords, p: int, delta: float, tol: float,
                 periodic: bool = False, precision: str = "fp64", eps_internal: float = 0.0,
                 force_lc: int = -1, stream=None, profile: bool = False,
                 host_only: bool = False, own_stream: bool = False, no_fuse: bool = False):
        if stream is None and not host_only and not own_stream:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self.p = int(p)
        self.dim = int(np.asarray(coords).shape[1])
        self.nleaves = int(np.asarray(levels).shape[0])
        self.handle = 0
        self.handle = fgt_plan(levels, coords, p, delta, tol,
                               FGT_PERIODIC if periodic else FGT_FREE,
                               _PRECISION[precision], eps_internal, force_lc,
                               int(stream or 0), profile, host_only, own_stream, no_fuse)

    def execute(self, sigma, u=None):
        if u is None:
            import torch
            u = torch.empty_like(sigma)
        self._check_io(sigma, u)
        fgt_execute(self.handle, sigma, u)
        return u

    def _check_io(self, sigma, u):
        expect = (self.nleaves, self.p ** self.dim)
        for name, t in (("sigma", sigma), ("u", u)):
            if hasattr(t, "shape"):
                if tuple(t.shape) != expect:
                    raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {expect}")
                if str(getattr(t, "dtype", "torch.float64")) != "torch.float64":
                    raise ValueError(f"{name} must be float64")
                if hasattr(t, "is_cuda") and not t.is_cuda:
                    raise ValueError(f"{name} must be a device tensor")
                if hasattr(t, "is_contiguous") and not t.is_contiguous():
                    raise ValueError(f"{name} must be contiguous")

    def execute_noalloc(self, sigma, u):
        """fgt_execute_noalloc: the workspace comes from the library's static
        device scratch; u must be given (nothing is allocated)."""
        self._check_io(sigma, u)
        fgt_execute_noalloc(self.handle, sigma, u)
        return u

    def sync(self):
        fgt_sync(self.handle)

    def info(self) -> dict:
        return fgt_plan_info(self.handle)

    def stage_times(self) -> dict:
        return fgt_stage_times(self.handle)

    def array(self, name: str) -> np.ndarray:
        return fgt_plan_array(self.handle, name)

    def close(self):
        if self.handle:
            fgt_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# request loop (include/fgt_serve.h)


def fgt_server_create(nslots: int = 0, nbuilders: int = 0, hbm_budget: int = 0) -> int:
    opts = _lib.fgt_server_opts_t(int(nslots), int(nbuilders), int(hbm_budget))
    h = ctypes.c_void_p()
    check(_lib.lib().fgt_server_create(ctypes.byref(opts), ctypes.byref(h)), "fgt_server_create")
    return h.value


def fgt_server_submit(server: int, key: int, sigma, u, p: int, delta: float, tol: float,
                      bc: int = FGT_FREE, precision: int = FGT_FP64, levels=None, coords=None,
                      host_io: bool = False) -> int:
    """Queues one request; returns its id.  levels/coords are needed for the
    first request of a key only."""
    tree_p = None
    keep = None
    if levels is not None:
        levels = np.ascontiguousarray(levels, dtype=np.int32)
        coords = np.ascontiguousarray(coords, dtype=np.int32)
        if coords.ndim != 2 or coords.shape[0] != levels.shape[0]:
            raise ValueError("coords must be [nleaves, dim] matching levels")
        keep = _lib.fgt_tree_t(coords.shape[1], levels.shape[0],
                               levels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               coords.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        tree_p = ctypes.pointer(keep)
    req = _lib.fgt_request_t(int(key), tree_p, int(p), float(delta), float(tol), int(bc),
                             int(precision), ctypes.c_void_p(_ptr(sigma) or None),
                             ctypes.c_void_p(_ptr(u) or None), int(bool(host_io)))
    rid = ctypes.c_int64()
    check(_lib.lib().fgt_server_submit(server, ctypes.byref(req), ctypes.byref(rid)),
          "fgt_server_submit")
    return rid.value


def fgt_server_poll(server: int, max_n: int = 256) -> list:
    buf = (_lib.fgt_completion_t * max_n)()
    n = ctypes.c_int32()
    check(_lib.lib().fgt_server_poll(server, buf, max_n, ctypes.byref(n)), "fgt_server_poll")
    return [buf[i].as_dict() for i in range(n.value)]


def fgt_server_wait(server: int, timeout_ms: float = -1.0, max_n: int = 256) -> list:
    buf = (_lib.fgt_completion_t * max_n)()
    n = ctypes.c_int32()
    check(_lib.lib().fgt_server_wait(server, buf, max_n, ctypes.byref(n), float(timeout_ms)),
          "fgt_server_wait")
    return [buf[i].as_dict() for i in range(n.value)]


def fgt_server_drain(server: int) -> None:
    check(_lib.lib().fgt_server_drain(server), "fgt_server_drain")


def fgt_server_stats(server: int) -> dict:
    st = _lib.fgt_server_stats_t()
    check(_lib.lib().fgt_server_stats(server, ctypes.byref(st)), "fgt_server_stats")
    return st.as_dict()


def fgt_server_destroy(server: int) -> None:
    check(_lib.lib().fgt_server_destroy(server), "fgt_server_destroy")


class Server:
    """Owns one request loop.  Holds a reference to every request's sigma and
    u until its completion has been collected, so their memory stays valid."""

    def __init__(self, nslots: int = 4, nbuilders: int = 2, hbm_budget: int = 0):
        self.handle = 0
        self.handle = fgt_server_create(nslots, nbuilders, hbm_budget)
        self._live = {}

    def submit(self, key: int, sigma, u, p: int, delta: float, tol: float,
               periodic: bool = False, precision: str = "fp64", levels=None, coords=None,
               host_io: bool = False) -> int:
        rid = fgt_server_submit(self.handle, key, sigma, u, p, delta, tol,
                                FGT_PERIODIC if periodic else FGT_FREE, _PRECISION[precision],
                                levels, coords, host_io)
        self._live[rid] = (sigma, u)
        return rid

    def _collect(self, done: list) -> list:
        for c in done:
            self._live.pop(c["id"], None)
        return done

    def poll(self) -> list:
        return self._collect(fgt_server_poll(self.handle))

    def wait(self, timeout_ms: float = -1.0) -> list:
        return self._collect(fgt_server_wait(self.handle, timeout_ms))

    def drain(self) -> list:
        fgt_server_drain(self.handle)
        out = []
        while True:
            got = self.poll()
            if not got:
                return out
            out += got

    def stats(self) -> dict:
        return fgt_server_stats(self.handle)

    def close(self):
        if self.handle:
            fgt_server_destroy(self.handle)
            self.handle = 0
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# many transforms per launch (include/fgt_batch.h)


def fgt_batch_create(plans, stream: int = 0, use_graph: bool = True, nstreams: int = 1,
                     class_major: bool = False, form_tile: int = 0, persistent: bool = False) -> int:
    handles = (ctypes.c_void_p * len(plans))(*[int(p) for p in plans])
    opts = _lib.fgt_batch_opts_t(ctypes.c_void_p(int(stream) or None), int(bool(use_graph)),
                                 int(nstreams), int(bool(class_major)), int(form_tile),
                                 int(bool(persistent)))
    h = ctypes.c_void_p()
    check(_lib.lib().fgt_batch_create(handles, len(plans), ctypes.byref(opts), ctypes.byref(h)),
          "fgt_batch_create")
    return h.value


def fgt_batch_bind(batch: int, sigmas, us) -> None:
    n = len(sigmas)
    sp = (ctypes.c_void_p * n)(*[_ptr(x) for x in sigmas])
    up = (ctypes.c_void_p * n)(*[_ptr(x) for x in us])
    check(_lib.lib().fgt_batch_bind(batch, sp, up), "fgt_batch_bind")


def fgt_batch_execute(batch: int) -> None:
    check(_lib.lib().fgt_batch_execute(batch), "fgt_batch_execute")


def fgt_batch_tune(batch: int, reps: int = 5) -> float:
    ms = ctypes.c_double()
    check(_lib.lib().fgt_batch_tune(batch, int(reps), ctypes.byref(ms)), "fgt_batch_tune")
    return ms.value


def fgt_batch_info(batch: int) -> dict:
    info = _lib.fgt_batch_info_t()
    check(_lib.lib().fgt_batch_info(batch, ctypes.byref(info)), "fgt_batch_info")
    return info.as_dict()


def fgt_batch_destroy(batch: int) -> None:
    check(_lib.lib().fgt_batch_destroy(batch), "fgt_batch_destroy")


class Batch:
    """Owns one batch over existing ``Plan`` objects (kept alive here).  By
    default it runs on torch's current stream."""

    def __init__(self, plans, stream=None, use_graph: bool = True, nstreams: int = 1,
                 class_major: bool = False, form_tile: int = 0, persistent: bool = False):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self.plans = list(plans)
        self.handle = 0
        self.handle = fgt_batch_create([p.handle for p in self.plans], int(stream or 0),
                                       use_graph, nstreams, class_major, form_tile, persistent)
        self._bound = None

    def bind(self, sigmas, us):
        if len(sigmas) != len(self.plans) or len(us) != len(self.plans):
            raise ValueError("one sigma and one u per plan")
        for pl, s_, u_ in zip(self.plans, sigmas, us):
            expect = (pl.nleaves, pl.p ** pl.dim)
            for t in (s_, u_):
                if tuple(t.shape) != expect or str(t.dtype) != "torch.float64" or not t.is_cuda \
                        or not t.is_contiguous():
                    raise ValueError(f"sigma/u must be contiguous float64 device tensors of shape {expect}")
        fgt_batch_bind(self.handle, sigmas, us)
        self._bound = (list(sigmas), list(us))

    def execute(self):
        fgt_batch_execute(self.handle)

    def tune(self, reps: int = 5) -> float:
        return fgt_batch_tune(self.handle, reps)

    def info(self) -> dict:
        return fgt_batch_info(self.handle)

    def close(self):
        if self.handle:
            fgt_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# output trees (include/fgt_output.h)


def fgt_output_resolve(levels, coords, p: int, delta: float, tol: float, sigma,
                       bc: int = FGT_FREE, precision: int = FGT_FP64, stream: int = 0,
                       eps: float = 0.0, refine: bool = True, coarsen: bool = True,
                       max_passes: int = 0, force_lc: int = -1) -> int:
    """Runs the transform and resolves u on an output tree; returns the handle."""
    L = _lib.lib()
    tree, keep = _tree(levels, coords)
    opts = _lib.fgt_opts_t(int(precision), 0.0, int(force_lc), ctypes.c_void_p(int(stream) or None),
                           0, 0, 0, 0)
    oo = _lib.fgt_output_opts_t(float(eps), int(bool(refine)), int(bool(coarsen)), int(max_passes))
    h = ctypes.c_void_p()
    check(L.fgt_output_resolve(ctypes.byref(tree), int(p), float(delta), float(tol), int(bc),
                               ctypes.byref(opts), ctypes.byref(oo), _ptr(sigma), ctypes.byref(h)),
          "fgt_output_resolve")
    del keep
    return h.value


def fgt_output_info(out: int) -> dict:
    info = _lib.fgt_output_info_t()
    check(_lib.lib().fgt_output_info(out, ctypes.byref(info)), "fgt_output_info")
    return info.as_dict()


def fgt_output_tree(out: int):
    info = fgt_output_info(out)
    n, d = info["nleaves"], info["dim"]
    lv = np.zeros(n, dtype=np.int32)
    cs = np.zeros((n, d), dtype=np.int32)
    check(_lib.lib().fgt_output_tree(out, lv.ctypes.data, cs.ctypes.data), "fgt_output_tree")
    return lv, cs


def fgt_output_values(out: int, u) -> None:
    check(_lib.lib().fgt_output_values(out, _ptr(u)), "fgt_output_values")


def fgt_output_destroy(out: int) -> None:
    if out:
        _lib.lib().fgt_output_destroy(out)


def fgt_interp(levels, coords, p: int, u, x, out, stream: int = 0) -> None:
    """out[i] = the tree's piecewise polynomial (values u) at x[i]; device arrays."""
    tree, keep = _tree(levels, coords)
    npts = int(x.shape[0]) if hasattr(x, "shape") else 0
    check(_lib.lib().fgt_interp(ctypes.byref(tree), int(p), _ptr(u), npts, _ptr(x), _ptr(out),
                                int(stream) or None), "fgt_interp")
    del keep


def fgt_tree_balance(levels, coords, periodic: bool = False):
    """The 2:1 balanced tree (host arrays), leaves in Morton order."""
    L = _lib.lib()
    tree, keep = _tree(levels, coords)
    bc = FGT_PERIODIC if periodic else FGT_FREE
    n = check(L.fgt_tree_balance(ctypes.byref(tree), bc, None, None, 0), "fgt_tree_balance")
    d = keep[1].shape[1]
    lv = np.zeros(n, dtype=np.int32)
    cs = np.zeros((n, d), dtype=np.int32)
    check(L.fgt_tree_balance(ctypes.byref(tree), bc, lv.ctypes.data, cs.ctypes.data, n),
          "fgt_tree_balance")
    return lv, cs


class PointPlan:
    """The point Gauss transform with proxy grids (include/fgt_point.h):
    sources [n, d] and targets [m, d] on the host at planning time; execute
    takes the charges [n] and returns u [m] as float64 device tensors."""

    def __init__(self, sources, targets, delta: float, tol: float, p: int = 16, ns: int = 64,
                 host_only: bool = False, stream=None):
        self.handle = 0
        src = np.ascontiguousarray(sources, dtype=np.float64)
        tgt = np.ascontiguousarray(targets, dtype=np.float64)
        if src.ndim != 2 or tgt.ndim != 2 or src.shape[1] != tgt.shape[1]:
            raise ValueError("sources [n, d] and targets [m, d]")
        self.dim, self.nsrc, self.ntgt = src.shape[1], src.shape[0], tgt.shape[0]
        if stream is None and not host_only:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        o = _lib.fgt_point_opts_t(int(p), int(ns), int(bool(host_only)), ctypes.c_void_p(int(stream or 0) or None))
        h = ctypes.c_void_p()
        check(_lib.lib().fgt_point_plan(self.dim, self.nsrc, src.ctypes.data, self.ntgt, tgt.ctypes.data,
                                        float(delta), float(tol), ctypes.byref(o), ctypes.byref(h)),
              "fgt_point_plan")
        self.handle = h.value

    def execute(self, q, u=None):
        if u is None:
            import torch
            u = torch.empty(self.ntgt, dtype=torch.float64, device=q.device)
        for name, t, n in (("q", q, self.nsrc), ("u", u, self.ntgt)):
            if tuple(t.shape) != (n,) or str(t.dtype) != "torch.float64" or not t.is_cuda:
                raise ValueError(f"{name} must be a float64 device tensor of shape ({n},)")
        check(_lib.lib().fgt_point_execute(self.handle, _ptr(q), _ptr(u)), "fgt_point_execute")
        return u

    def info(self) -> dict:
        info = _lib.fgt_point_info_t()
        check(_lib.lib().fgt_point_info(self.handle, ctypes.byref(info)), "fgt_point_info")
        return info.as_dict()

    def array(self, name: str) -> np.ndarray:
        L = _lib.lib()
        n = check(L.fgt_point_array(self.handle, name.encode(), None, 0), "fgt_point_array")
        out = np.zeros(n, dtype=np.int32)
        if n:
            L.fgt_point_array(self.handle, name.encode(), out.ctypes.data, n)
        return out

    def close(self):
        if self.handle:
            _lib.lib().fgt_point_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class OutputTree:
    """u resolved on its own adaptive tree (Section 4.2).  ``levels``,
    ``coords`` and ``u`` (a tensor on sigma's device) are filled on
    construction; ``info`` holds the box counts and error figures."""

    def __init__(self, levels, coords, p: int, delta: float, tol: float, sigma,
                 periodic: bool = False, precision: str = "fp64", eps: float = 0.0,
                 refine: bool = True, coarsen: bool = True, max_passes: int = 0,
                 force_lc: int = -1, stream=None):
        import torch
        n, d = np.asarray(coords).reshape(len(levels), -1).shape
        if tuple(sigma.shape) != (n, int(p) ** d) or sigma.dtype != torch.float64 or not sigma.is_cuda:
            raise ValueError(f"sigma must be a float64 device tensor of shape {(n, int(p) ** d)}")
        sigma = sigma.contiguous()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = fgt_output_resolve(levels, coords, p, delta, tol, sigma,
                               FGT_PERIODIC if periodic else FGT_FREE, _PRECISION[precision],
                               stream, eps, refine, coarsen, max_passes, force_lc)
        try:
            self.info = fgt_output_info(h)
            self.levels, self.coords = fgt_output_tree(h)
            self.p = int(p)
            self.u = torch.empty((len(self.levels), self.p ** self.coords.shape[1]),
                                 dtype=torch.float64, device=sigma.device)
            fgt_output_values(h, self.u)
        finally:
            fgt_output_destroy(h)

    def interp(self, x):
        """u at the points x (a [npts, dim] float64 tensor on the device)."""
        return interp(self.levels, self.coords, self.p, self.u, x)


def interp(levels, coords, p: int, u, x):
    """The tree's piecewise polynomial (values u) at the points x; returns a
    new tensor on x's device."""
    import torch
    n, d = np.asarray(coords).reshape(len(levels), -1).shape
    if x.dim() != 2 or x.shape[1] != d or x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError(f"x must be a float64 device tensor of shape [npts, {d}]")
    if u.numel() != n * int(p) ** d or u.dtype != torch.float64 or not u.is_cuda:
        raise ValueError(f"u must be a float64 device tensor of {n} x {int(p) ** d} values")
    x = x.contiguous()
    out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    fgt_interp(levels, coords, p, u.contiguous(), x, out, torch.cuda.current_stream().cuda_stream)
    return out


# ---------------------------------------------------------------------------
# input trees on the device (include/fgt_density.h)


def _gaussians(centers, widths, amps, periodic: bool):
    c = np.ascontiguousarray(np.atleast_2d(centers), dtype=np.float64)
    w = np.ascontiguousarray(widths, dtype=np.float64).ravel()
    a = np.ascontiguousarray(amps, dtype=np.float64).ravel()
    if c.shape[0] != len(w) or len(w) != len(a):
        raise ValueError("centers [n, dim], widths [n] and amps [n] must agree")
    dp = ctypes.POINTER(ctypes.c_double)
    g = _lib.fgt_gaussians_t(c.shape[1], c.shape[0], c.ctypes.data_as(dp), w.ctypes.data_as(dp),
                             a.ctypes.data_as(dp), int(bool(periodic)))
    return g, (c, w, a)


def resolve_gaussians(centers, widths, amps, p: int, eps: float, periodic: bool = False,
                      min_level: int = 0, max_level: int = 12, max_leaves: int = 0,
                      norm: float = 0.0, stream=None):
    """Algorithm 3 on the device for sigma = sum_i a_i exp(-|x - c_i|^2/w_i^2):
    returns (levels, coords, sigma, info) with sigma a float64 tensor on the
    current device."""
    import torch
    L = _lib.lib()
    g, keep = _gaussians(centers, widths, amps, periodic)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    o = _lib.fgt_resolve_opts_t(int(min_level), int(max_level), int(max_leaves), float(norm),
                                ctypes.c_void_p(int(stream) or None))
    h = ctypes.c_void_p()
    check(L.fgt_resolve_gaussians(ctypes.byref(g), int(p), float(eps), ctypes.byref(o), ctypes.byref(h)),
          "fgt_resolve_gaussians")
    try:
        info = _lib.fgt_density_info_t()
        check(L.fgt_density_info(h, ctypes.byref(info)), "fgt_density_info")
        info = info.as_dict()
        n, d = info["nleaves"], info["dim"]
        lv = np.zeros(n, dtype=np.int32)
        cs = np.zeros((n, d), dtype=np.int32)
        check(L.fgt_density_tree(h, lv.ctypes.data, cs.ctypes.data), "fgt_density_tree")
        sig = torch.empty((n, int(p) ** d), dtype=torch.float64, device="cuda")
        check(L.fgt_density_values(h, _ptr(sig)), "fgt_density_values")
    finally:
        L.fgt_density_destroy(h)
    del keep
    return lv, cs, sig, info


def sample_gaussians(centers, widths, amps, levels, coords, p: int, periodic: bool = False):
    """sigma at the nodes of the leaves (a new float64 tensor on the device)."""
    import torch
    g, keep = _gaussians(centers, widths, amps, periodic)
    tree, tkeep = _tree(levels, coords)
    sig = torch.empty((len(tkeep[0]), int(p) ** tkeep[1].shape[1]), dtype=torch.float64, device="cuda")
    check(_lib.lib().fgt_sample_gaussians(ctypes.byref(g), ctypes.byref(tree), int(p), _ptr(sig),
                                          torch.cuda.current_stream().cuda_stream),
          "fgt_sample_gaussians")
    del keep, tkeep
    return sig
