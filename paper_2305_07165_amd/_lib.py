"""ctypes declarations of the C ABI in include/*.h (argument marshalling only).

Every step of the transform runs in libfgt.so's HIP kernels; there is no CPU
fallback.  If the library is missing this module raises on first use.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfgt.so")

FGT_OK = 0
FGT_ERR_INVALID_ARG = -1
FGT_ERR_NOT_TILING = -2
FGT_ERR_NOT_BALANCED = -3
FGT_ERR_OOM = -4
FGT_ERR_UNSUPPORTED = -5
FGT_ERR_HIP = -6
FGT_FREE = 0
FGT_PERIODIC = 1
FGT_FP64 = 0
FGT_FP32 = 1
FGT_BF16X3 = 2

EXPORTED = ["fgt_plan", "fgt_execute", "fgt_execute_noalloc", "fgt_sync", "fgt_plan_info", "fgt_stage_times",
            "fgt_destroy", "fgt_strerror", "fgt_last_error", "fgt_pw_terms",
            "fgt_periodic_terms", "fgt_plan_array",
            "fgt_server_create", "fgt_server_submit", "fgt_server_poll", "fgt_server_wait",
            "fgt_server_drain", "fgt_server_stats", "fgt_server_destroy",
            "fgt_batch_create", "fgt_batch_bind", "fgt_batch_execute", "fgt_batch_tune",
            "fgt_batch_info", "fgt_batch_destroy",
            "fgt_output_resolve", "fgt_output_info", "fgt_output_tree", "fgt_output_values",
            "fgt_output_destroy", "fgt_interp", "fgt_tree_balance",
            "fgt_resolve_gaussians", "fgt_density_info", "fgt_density_tree", "fgt_density_values",
            "fgt_density_destroy", "fgt_sample_gaussians",
            "fgt_point_plan", "fgt_point_execute", "fgt_point_info", "fgt_point_array",
            "fgt_point_destroy"]


class fgt_tree_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nleaves", ctypes.c_int64),
                ("level", ctypes.POINTER(ctypes.c_int32)),
                ("coord", ctypes.POINTER(ctypes.c_int32))]


class fgt_opts_t(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("eps_internal", ctypes.c_double),
                ("force_lc", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("own_stream", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("host_only", ctypes.c_int32), ("no_fuse", ctypes.c_int32)]


class fgt_info_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("p", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("lc", ctypes.c_int32),
                ("lmin", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("nf", ctypes.c_int32), ("nr", ctypes.c_int32),
                ("delta", ctypes.c_double), ("tol", ctypes.c_double), ("eps", ctypes.c_double),
                ("D0", ctypes.c_double), ("R", ctypes.c_double), ("h", ctypes.c_double),
                ("nleaves", ctypes.c_int64), ("npoints", ctypes.c_int64),
                ("n_pwbox", ctypes.c_int64), ("n_pwleaf", ctypes.c_int64),
                ("n_plist", ctypes.c_int64), ("n_near_target", ctypes.c_int64),
                ("n_near_pair", ctypes.c_int64),
                ("flops_form", ctypes.c_double), ("flops_eval", ctypes.c_double),
                ("flops_translate", ctypes.c_double), ("flops_near", ctypes.c_double),
                ("bytes_min", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("n_plane", ctypes.c_int64), ("n_row", ctypes.c_int64),
                ("n_near_source", ctypes.c_int64), ("n_near_haspw", ctypes.c_int64),
                ("fused_translate", ctypes.c_int32), ("fourier", ctypes.c_int32),
                ("nr_stored", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class fgt_server_opts_t(ctypes.Structure):
    _fields_ = [("nslots", ctypes.c_int32), ("nbuilders", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64)]


class fgt_request_t(ctypes.Structure):
    _fields_ = [("key", ctypes.c_int64), ("tree", ctypes.POINTER(fgt_tree_t)),
                ("p", ctypes.c_int32), ("delta", ctypes.c_double), ("tol", ctypes.c_double),
                ("bc", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("sigma", ctypes.c_void_p), ("u", ctypes.c_void_p), ("host_io", ctypes.c_int32)]


class fgt_completion_t(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("key", ctypes.c_int64), ("status", ctypes.c_int32),
                ("cache_hit", ctypes.c_int32), ("npoints", ctypes.c_int64),
                ("queue_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("device_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class fgt_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("plans_built", ctypes.c_int64),
                ("plans_uploaded", ctypes.c_int64), ("plans_evicted", ctypes.c_int64),
                ("workspaces_added", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("peak_resident_bytes", ctypes.c_int64), ("budget_bytes", ctypes.c_int64),
                ("nslots", ctypes.c_int32), ("running", ctypes.c_int32),
                ("waiting", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class fgt_batch_opts_t(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("use_graph", ctypes.c_int32),
                ("nstreams", ctypes.c_int32), ("class_major", ctypes.c_int32),
                ("form_tile", ctypes.c_int32), ("persistent", ctypes.c_int32)]


class fgt_batch_info_t(ctypes.Structure):
    _fields_ = [("njobs", ctypes.c_int64), ("npoints", ctypes.c_int64),
                ("nclasses", ctypes.c_int32), ("nsingle", ctypes.c_int32),
                ("nlaunches", ctypes.c_int32), ("nstreams", ctypes.c_int32),
                ("class_major", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("tuned_ms", ctypes.c_double), ("tile_alt_classes", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("persistent_error", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class fgt_output_opts_t(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("refine", ctypes.c_int32),
                ("coarsen", ctypes.c_int32), ("max_passes", ctypes.c_int32)]


class fgt_output_info_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("p", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("nleaves_in", ctypes.c_int64), ("nleaves", ctypes.c_int64),
                ("nboxes_in", ctypes.c_int64), ("nboxes", ctypes.c_int64),
                ("added_refine", ctypes.c_int64), ("added_refine_balance", ctypes.c_int64),
                ("deleted_coarsen", ctypes.c_int64), ("added_balance", ctypes.c_int64),
                ("u_l2", ctypes.c_double), ("threshold", ctypes.c_double),
                ("max_leaf_error", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class fgt_gaussians_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int64),
                ("centers", ctypes.POINTER(ctypes.c_double)),
                ("widths", ctypes.POINTER(ctypes.c_double)),
                ("amps", ctypes.POINTER(ctypes.c_double)), ("periodic", ctypes.c_int32)]


class fgt_point_opts_t(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("ns", ctypes.c_int32), ("host_only", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class fgt_point_info_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("p", ctypes.c_int32), ("ns", ctypes.c_int32),
                ("lc", ctypes.c_int32), ("lp", ctypes.c_int32), ("nr", ctypes.c_int32),
                ("nsrc", ctypes.c_int64), ("ntgt", ctypes.c_int64), ("nleaves", ctypes.c_int64),
                ("ndense", ctypes.c_int64), ("npwbox", ctypes.c_int64), ("nproxy", ctypes.c_int64),
                ("nplist", ctypes.c_int64), ("ndirect_terms", ctypes.c_int64),
                ("delta", ctypes.c_double), ("tol", ctypes.c_double), ("proxy_err", ctypes.c_double),
                ("device_bytes", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class fgt_resolve_opts_t(ctypes.Structure):
    _fields_ = [("min_level", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("max_leaves", ctypes.c_int64), ("norm", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class fgt_density_info_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("p", ctypes.c_int32), ("nleaves", ctypes.c_int64),
                ("nleaves_unbalanced", ctypes.c_int64), ("boxes_sampled", ctypes.c_int64),
                ("lmin", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("norm", ctypes.c_double), ("threshold", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """The loaded libfgt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the transform has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.fgt_plan.restype = ctypes.c_int
        L.fgt_plan.argtypes = [ctypes.POINTER(fgt_tree_t), ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.POINTER(fgt_opts_t),
                               ctypes.POINTER(vp)]
        L.fgt_execute.restype = ctypes.c_int
        L.fgt_execute.argtypes = [vp, vp, vp]
        L.fgt_execute_noalloc.restype = ctypes.c_int
        L.fgt_execute_noalloc.argtypes = [vp, vp, vp]
        L.fgt_sync.restype = ctypes.c_int
        L.fgt_sync.argtypes = [vp]
        L.fgt_plan_info.restype = ctypes.c_int
        L.fgt_plan_info.argtypes = [vp, ctypes.POINTER(fgt_info_t)]
        L.fgt_stage_times.restype = ctypes.c_int
        L.fgt_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        L.fgt_destroy.restype = None
        L.fgt_destroy.argtypes = [vp]
        L.fgt_strerror.restype = ctypes.c_char_p
        L.fgt_strerror.argtypes = [ctypes.c_int]
        L.fgt_last_error.restype = ctypes.c_char_p
        L.fgt_last_error.argtypes = []
        L.fgt_pw_terms.restype = ctypes.c_int
        L.fgt_pw_terms.argtypes = [ctypes.c_double, ctypes.c_double]
        L.fgt_periodic_terms.restype = ctypes.c_int
        L.fgt_periodic_terms.argtypes = [ctypes.c_double, ctypes.c_double]
        L.fgt_plan_array.restype = ctypes.c_int64
        L.fgt_plan_array.argtypes = [vp, ctypes.c_char_p, vp, ctypes.c_int64]
        L.fgt_server_create.restype = ctypes.c_int
        L.fgt_server_create.argtypes = [ctypes.POINTER(fgt_server_opts_t), ctypes.POINTER(vp)]
        L.fgt_server_submit.restype = ctypes.c_int
        L.fgt_server_submit.argtypes = [vp, ctypes.POINTER(fgt_request_t),
                                        ctypes.POINTER(ctypes.c_int64)]
        for name in ("fgt_server_poll", "fgt_server_wait"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [vp, ctypes.POINTER(fgt_completion_t), ctypes.c_int32,
                          ctypes.POINTER(ctypes.c_int32)] + ([ctypes.c_double] if name.endswith("wait") else [])
        L.fgt_server_drain.restype = ctypes.c_int
        L.fgt_server_drain.argtypes = [vp]
        L.fgt_server_stats.restype = ctypes.c_int
        L.fgt_server_stats.argtypes = [vp, ctypes.POINTER(fgt_server_stats_t)]
        L.fgt_server_destroy.restype = ctypes.c_int
        L.fgt_server_destroy.argtypes = [vp]
        L.fgt_batch_create.restype = ctypes.c_int
        L.fgt_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int64,
                                       ctypes.POINTER(fgt_batch_opts_t), ctypes.POINTER(vp)]
        L.fgt_batch_bind.restype = ctypes.c_int
        L.fgt_batch_bind.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.fgt_batch_execute.restype = ctypes.c_int
        L.fgt_batch_execute.argtypes = [vp]
        L.fgt_batch_tune.restype = ctypes.c_int
        L.fgt_batch_tune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.fgt_batch_info.restype = ctypes.c_int
        L.fgt_batch_info.argtypes = [vp, ctypes.POINTER(fgt_batch_info_t)]
        L.fgt_batch_destroy.restype = ctypes.c_int
        L.fgt_batch_destroy.argtypes = [vp]
        L.fgt_output_resolve.restype = ctypes.c_int
        L.fgt_output_resolve.argtypes = [ctypes.POINTER(fgt_tree_t), ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.POINTER(fgt_opts_t),
                                         ctypes.POINTER(fgt_output_opts_t), vp, ctypes.POINTER(vp)]
        L.fgt_output_info.restype = ctypes.c_int
        L.fgt_output_info.argtypes = [vp, ctypes.POINTER(fgt_output_info_t)]
        L.fgt_output_tree.restype = ctypes.c_int
        L.fgt_output_tree.argtypes = [vp, vp, vp]
        L.fgt_output_values.restype = ctypes.c_int
        L.fgt_output_values.argtypes = [vp, vp]
        L.fgt_output_destroy.restype = None
        L.fgt_output_destroy.argtypes = [vp]
        L.fgt_interp.restype = ctypes.c_int
        L.fgt_interp.argtypes = [ctypes.POINTER(fgt_tree_t), ctypes.c_int, vp, ctypes.c_int64, vp, vp, vp]
        L.fgt_point_plan.restype = ctypes.c_int
        L.fgt_point_plan.argtypes = [ctypes.c_int, ctypes.c_int64, vp, ctypes.c_int64, vp, ctypes.c_double,
                                     ctypes.c_double, ctypes.POINTER(fgt_point_opts_t), ctypes.POINTER(vp)]
        L.fgt_point_execute.restype = ctypes.c_int
        L.fgt_point_execute.argtypes = [vp, vp, vp]
        L.fgt_point_info.restype = ctypes.c_int
        L.fgt_point_info.argtypes = [vp, ctypes.POINTER(fgt_point_info_t)]
        L.fgt_point_array.restype = ctypes.c_int64
        L.fgt_point_array.argtypes = [vp, ctypes.c_char_p, vp, ctypes.c_int64]
        L.fgt_point_destroy.restype = None
        L.fgt_point_destroy.argtypes = [vp]
        L.fgt_tree_balance.restype = ctypes.c_int64
        L.fgt_tree_balance.argtypes = [ctypes.POINTER(fgt_tree_t), ctypes.c_int, vp, vp, ctypes.c_int64]
        L.fgt_resolve_gaussians.restype = ctypes.c_int
        L.fgt_resolve_gaussians.argtypes = [ctypes.POINTER(fgt_gaussians_t), ctypes.c_int, ctypes.c_double,
                                            ctypes.POINTER(fgt_resolve_opts_t), ctypes.POINTER(vp)]
        L.fgt_density_info.restype = ctypes.c_int
        L.fgt_density_info.argtypes = [vp, ctypes.POINTER(fgt_density_info_t)]
        L.fgt_density_tree.restype = ctypes.c_int
        L.fgt_density_tree.argtypes = [vp, vp, vp]
        L.fgt_density_values.restype = ctypes.c_int
        L.fgt_density_values.argtypes = [vp, vp]
        L.fgt_density_destroy.restype = None
        L.fgt_density_destroy.argtypes = [vp]
        L.fgt_sample_gaussians.restype = ctypes.c_int
        L.fgt_sample_gaussians.argtypes = [ctypes.POINTER(fgt_gaussians_t), ctypes.POINTER(fgt_tree_t),
                                           ctypes.c_int, vp, vp]
        _lib = L
    return _lib


class FgtError(RuntimeError):
    def __init__(self, code: int, what: str):
        L = lib()
        detail = L.fgt_last_error().decode()
        super().__init__(f"{what}: {L.fgt_strerror(code).decode()} ({code}): {detail}")
        self.code = code


def check(code: int, what: str) -> int:
    if code < 0:
        raise FgtError(code, what)
    return code
