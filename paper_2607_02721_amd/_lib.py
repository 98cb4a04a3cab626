"""ctypes binding of libgscoreset.so (include/gs_coreset.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  There is no fallback: if the library cannot be loaded, every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgscoreset.so")

GS_OK = 0
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of memory",
                4: "no positive sensitivity", 5: "invalid data", 6: "device error"}
EXPORTED = ["gs_sensitivity", "gs_sample_coreset", "gs_render_objective", "gs_default_params",
            "gs_release_workspace", "gs_last_error", "gs_status_string", "gs_mlp_param_count",
            "gs_mlp_init", "gs_features", "gs_feature_stats", "gs_mlp_forward", "gs_mlp_train_step",
            "gs_plan_create", "gs_plan_set_config", "gs_plan_tune", "gs_plan_get_info",
            "gs_plan_sensitivity", "gs_plan_status", "gs_plan_destroy", "gs_proposal_mixture",
            "gs_log_targets", "gs_measure_peaks", "gs_knn", "gs_coreset_error", "gs_mlp_gradient",
            "gs_sample_coreset_noalloc", "gs_set_allocator", "gs_region_bound", "gs_tune_tile"]

OBJ_FULL, OBJ_FIXED, OBJ_TRUE = 0, 1, 2
MLP_BF16, MLP_FP32 = 0, 1
FLAG_COUNT_PAIRS = 1
AGG_RAY, AGG_TILE, AGG_IMAGE, AGG_SCENE = 0, 1, 2, 3
QUERY_RGBSUM, QUERY_NOCOLOR, QUERY_L2, QUERY_CHANNEL = 0, 1, 2, 3
ATTR_F32, ATTR_MIXED16 = 0, 1


class GsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("format", C.c_int32),
                ("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class Views(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("world_to_cam", C.c_void_p),
                ("intrinsics", C.c_void_p), ("size", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("footprint_sigma", C.c_float), ("dilation", C.c_float), ("z_near", C.c_float),
                ("share_floor", C.c_float), ("query_mode", C.c_int32),
                ("max_views_per_chunk", C.c_int32), ("flags", C.c_int32), ("ray_mask", C.c_void_p),
                ("aggregate", C.c_int32), ("ambiguous_rays", C.c_void_p),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_projected", C.c_int64), ("n_entries", C.c_int64), ("n_pairs", C.c_int64),
                ("n_live_pairs", C.c_int64), ("n_lane_pairs", C.c_int64), ("n_rays_positive", C.c_int64),
                ("n_invalid_gaussians", C.c_int64), ("total_sensitivity", C.c_double),
                ("ms_project", C.c_double), ("ms_sort", C.c_double), ("ms_bin", C.c_double),
                ("ms_pass1", C.c_double), ("ms_pass2", C.c_double), ("ms_emit", C.c_double),
                ("n_bins", C.c_int64), ("sort_passes", C.c_int32), ("pad0", C.c_int32),
                ("n_ambiguous_keys", C.c_int64), ("n_ambiguous_pairs", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanConfig(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("xcd_remap", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("n_scenes", C.c_int32), ("n_groups", C.c_int32), ("config", PlanConfig),
                ("graph_captured", C.c_int32), ("device_bytes", C.c_int64),
                ("list_capacity", C.c_int64), ("compact_bytes", C.c_int64), ("n_launches", C.c_int32),
                ("n_compact_launches", C.c_int32), ("n_sort3_scenes", C.c_int32), ("pad", C.c_int32)]


class Peaks(C.Structure):
    _fields_ = [("copy_bytes_per_s", C.c_double), ("fma_per_s", C.c_double), ("exp_per_s", C.c_double),
                ("mfma_bf16_flop_per_s", C.c_double)]


class RegionReport(C.Structure):
    _fields_ = [("L_full", C.c_double), ("L_w", C.c_double), ("A_min", C.c_double), ("eps_0", C.c_double),
                ("rho", C.c_double), ("eps_reg", C.c_double), ("max_err", C.c_double), ("n_pixels", C.c_int64),
                ("n_net", C.c_int32), ("pad", C.c_int32)]


class RenderDiag(C.Structure):
    _fields_ = [("n_invalid_pairs", C.c_int64), ("gamma_max", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing; build it with paper_2607_02721_amd/build.py")
        try:
            # share torch's HIP runtime: loading it first makes the library's
            # libamdhip64 dependency resolve to the copy torch already holds
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(path)
        P = C.c_void_p
        lib.gs_sensitivity.argtypes = [P, P, P, P, P, P]
        lib.gs_sensitivity.restype = C.c_int
        lib.gs_sample_coreset.argtypes = [P, C.c_int64, C.c_int64, C.c_uint64, P, P, P, P]
        lib.gs_sample_coreset.restype = C.c_int
        lib.gs_sample_coreset_noalloc.argtypes = [P, C.c_int64, C.c_int64, C.c_uint64, P, P, P, P]
        lib.gs_sample_coreset_noalloc.restype = C.c_int
        lib.gs_render_objective.argtypes = [P, P, P, P, C.c_int32, P, P, P, P]
        lib.gs_render_objective.restype = C.c_int
        lib.gs_default_params.argtypes = [P]
        lib.gs_default_params.restype = None
        lib.gs_release_workspace.argtypes = []
        lib.gs_release_workspace.restype = C.c_int
        lib.gs_last_error.argtypes = []
        lib.gs_last_error.restype = C.c_char_p
        lib.gs_status_string.argtypes = [C.c_int]
        lib.gs_status_string.restype = C.c_char_p
        lib.gs_mlp_param_count.argtypes = []
        lib.gs_mlp_param_count.restype = C.c_int64
        lib.gs_mlp_init.argtypes = [P, C.c_uint64, P]
        lib.gs_features.argtypes = [P, P, P]
        lib.gs_knn.argtypes = [P, P, P, P]
        lib.gs_region_bound.argtypes = [P, C.c_int32, C.c_double, C.c_double, P, P, C.c_int64, C.c_float, P, P, P]
        lib.gs_region_bound.restype = C.c_int
        lib.gs_set_allocator.argtypes = [P, P, P]
        lib.gs_set_allocator.restype = C.c_int
        lib.gs_mlp_gradient.argtypes = [P, P, P, P, C.c_int64, C.c_int32, P, P, P]
        lib.gs_coreset_error.argtypes = [P, C.c_int32, P, P]
        lib.gs_feature_stats.argtypes = [P, C.c_int64, P, P]
        lib.gs_mlp_forward.argtypes = [P, P, P, C.c_int64, P, P]
        lib.gs_mlp_train_step.argtypes = [P, P, C.c_int64, C.c_float, P, P, P, C.c_int64, P, P, P]
        lib.gs_plan_create.argtypes = [P, P, C.c_int32, P, P, P]
        lib.gs_plan_set_config.argtypes = [P, P]
        lib.gs_plan_tune.argtypes = [P, P, C.c_int32, P, P, P]
        lib.gs_tune_tile.argtypes = [P, P, P, C.c_int32, P, P, P, P, P]
        lib.gs_tune_tile.restype = C.c_int
        lib.gs_plan_get_info.argtypes = [P, P]
        lib.gs_plan_sensitivity.argtypes = [P, P, P]
        lib.gs_plan_status.argtypes = [P, P]
        lib.gs_proposal_mixture.argtypes = [P, C.c_int64, C.c_float, P, P]
        lib.gs_log_targets.argtypes = [P, C.c_int64, C.c_float, P, P]
        lib.gs_measure_peaks.argtypes = [P, P]
        lib.gs_plan_destroy.argtypes = [P]
        lib.gs_plan_destroy.restype = None
        for f in (lib.gs_mlp_init, lib.gs_features, lib.gs_knn, lib.gs_coreset_error, lib.gs_mlp_gradient, lib.gs_feature_stats, lib.gs_mlp_forward,
                  lib.gs_mlp_train_step, lib.gs_plan_create, lib.gs_plan_set_config, lib.gs_plan_tune,
                  lib.gs_plan_get_info, lib.gs_plan_sensitivity, lib.gs_plan_status, lib.gs_proposal_mixture,
                  lib.gs_log_targets, lib.gs_measure_peaks):
            f.restype = C.c_int
        _lib = lib
    return _lib


def check(status):
    if status != GS_OK:
        raise GsError(status, load().gs_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    load().gs_default_params(C.byref(p))
    for k, v in kw.items():
        if k in ("ray_mask", "ambiguous_rays"):
            setattr(p, k, v)
        else:
            setattr(p, k, v)
    return p


class HostViews:
    """Keeps the float64/int32 camera arrays alive and exposes the C struct."""

    def __init__(self, world_to_cam, intrinsics, size):
        self.w2c = np.ascontiguousarray(world_to_cam, np.float64).reshape(-1, 12)
        self.intr = np.ascontiguousarray(intrinsics, np.float64).reshape(-1, 4)
        self.size = np.ascontiguousarray(size, np.int32).reshape(-1, 2)
        self.c = Views(self.size.shape[0], self.w2c.ctypes.data, self.intr.ctypes.data,
                       self.size.ctypes.data)

    @property
    def n_rays(self):
        return int(np.sum(self.size[:, 0].astype(np.int64) * self.size[:, 1]))
