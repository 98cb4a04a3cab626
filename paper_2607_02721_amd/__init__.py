"""MI355X-native sensitivity pass and sensitivity sampler for coreset pruning
of 3D Gaussian Splatting scenes (Mousa & Maalouf, "Provable Pruning for
Efficient 3D Gaussian Splatting via Coresets").

Python surface over the C ABI in include/gs_coreset.h.  The functions here
only marshal arguments: torch provides device memory and the current stream,
and all computation runs in the library's HIP kernels for gfx950.

    scene = DeviceScene.from_arrays(mean, log_scale, quat, opacity, sh, sh_degree)
    s, st = sensitivity(scene, views)                  # Algorithm 1, steps 1-3
    counts, w, support = sample_coreset(s, m, seed)    # Algorithm 1, steps 3-5
    out = render_objective(scene, views, w)            # A, A^th_w, A_w
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (AGG_IMAGE, AGG_RAY, AGG_SCENE, AGG_TILE, ATTR_F32, ATTR_MIXED16, GsError, OBJ_FIXED,
                   OBJ_FULL, OBJ_TRUE, QUERY_CHANNEL, QUERY_L2, QUERY_NOCOLOR, QUERY_RGBSUM, load)

__all__ = ["DeviceScene", "sensitivity", "sample_coreset", "render_objective", "GsError",
           "OBJ_FULL", "OBJ_FIXED", "OBJ_TRUE", "QUERY_RGBSUM", "QUERY_NOCOLOR", "QUERY_L2", "QUERY_CHANNEL", "ATTR_F32",
           "ATTR_MIXED16", "AGG_RAY", "AGG_TILE", "AGG_IMAGE", "AGG_SCENE", "load", "release_workspace",
           "Plan", "measure_peaks", "coreset_error", "use_torch_allocator", "region_bound", "tune_tile"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceScene:
    """SoA scene planes resident in device memory (torch tensors).

    format ATTR_F32: float32 planes.  ATTR_MIXED16: bfloat16 mean, log_scale
    and sh; float16 quat and opacity."""

    def __init__(self, mean, log_scale, quat, opacity, sh, sh_degree, fmt=ATTR_F32):
        self.mean, self.log_scale, self.quat, self.opacity, self.sh = mean, log_scale, quat, opacity, sh
        self.sh_degree = int(sh_degree)
        self.format = int(fmt)
        self.n = int(opacity.shape[0])
        for t in (mean, log_scale, quat, opacity, sh):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("scene planes must be contiguous device tensors")

    @classmethod
    def from_arrays(cls, mean, log_scale, quat, opacity, sh, sh_degree, device="cuda",
                    fmt=ATTR_F32):
        torch = _torch()
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        planes = [f(mean), f(log_scale), f(quat), f(opacity), f(sh)]
        if fmt == ATTR_MIXED16:
            planes = [planes[0].to(torch.bfloat16), planes[1].to(torch.bfloat16),
                      planes[2].to(torch.float16), planes[3].to(torch.float16),
                      planes[4].to(torch.bfloat16)]
        return cls(*[p.contiguous() for p in planes], sh_degree, fmt)

    @classmethod
    def from_scene(cls, scene, device="cuda", fmt=ATTR_F32):
        """From any object with mean/log_scale/quat/opacity/sh arrays and sh_degree."""
        return cls.from_arrays(scene.mean, scene.log_scale, scene.quat, scene.opacity, scene.sh,
                               scene.sh_degree, device, fmt)

    def c_struct(self):
        return _lib.Scene(self.n, self.sh_degree, self.format, self.mean.data_ptr(),
                          self.log_scale.data_ptr(), self.quat.data_ptr(), self.opacity.data_ptr(),
                          self.sh.data_ptr())

    def attribute_bytes(self):
        return sum(t.numel() * t.element_size()
                   for t in (self.mean, self.log_scale, self.quat, self.opacity, self.sh))


def _views(views):
    if isinstance(views, _lib.HostViews):
        return views
    return _lib.HostViews(views.world_to_cam, views.intrinsics, views.size)


def _params(footprint_sigma, dilation, z_near, share_floor, query_mode, ray_mask,
            max_views_per_chunk, flags=0, aggregate=AGG_RAY, ambiguous_rays=None, tile=(16, 16)):
    p = _lib.default_params()
    if isinstance(tile, str):
        if tile != "auto":
            raise ValueError("tile is (width, height) or 'auto'")
        tile = (0, 0)
    p.tile_w, p.tile_h = int(tile[0]), int(tile[1])
    p.flags = flags
    p.aggregate = aggregate
    p.footprint_sigma = footprint_sigma
    p.dilation = dilation
    p.z_near = z_near
    p.share_floor = share_floor
    p.query_mode = query_mode
    p.max_views_per_chunk = max_views_per_chunk
    if ray_mask is not None:
        if not ray_mask.is_cuda or ray_mask.dtype.itemsize != 4:
            raise ValueError("ray_mask must be a device tensor of 32-bit words")
        p.ray_mask = ray_mask.data_ptr()
    if ambiguous_rays is not None:
        if not ambiguous_rays.is_cuda or ambiguous_rays.dtype.itemsize != 4:
            raise ValueError("ambiguous_rays must be a device tensor of 32-bit words")
        p.ambiguous_rays = ambiguous_rays.data_ptr()
    return p


def sensitivity(scene: DeviceScene, views, *, footprint_sigma=3.0, dilation=0.3, z_near=0.2,
                share_floor=1e-12, query_mode=QUERY_RGBSUM, ray_mask=None,
                max_views_per_chunk=0, stats=False, count_pairs=False, aggregate=AGG_RAY, out=None,
                ambiguous_rays=None, tile=(16, 16), stream=None):
    """Per-Gaussian sensitivities (float32 device tensor [n]) for queries of
    the given granularity (AGG_RAY, AGG_TILE, AGG_IMAGE, AGG_SCENE); with
    stats=True also a dict of counters and per-stage device milliseconds
    (pair counters need count_pairs=True, which can also OR the rays holding
    a pair within 1e-5 r^2 of the cutoff into the device bitset
    `ambiguous_rays`).  `tile` is the binning tile (width, height), each 8,
    16 or 32 pixels, or "auto" for the shape `tune_tile` last chose for
    views and scenes of this size class: it changes the speed, not the
    result."""
    torch = _torch()
    lib = load()
    hv = _views(views)
    p = _params(footprint_sigma, dilation, z_near, share_floor, query_mode, ray_mask,
                max_views_per_chunk, _lib.FLAG_COUNT_PAIRS if count_pairs else 0, aggregate, ambiguous_rays,
                tile)
    if out is None:
        out = torch.empty(scene.n, dtype=torch.float32, device=scene.opacity.device)
    sc = scene.c_struct()
    st = _lib.Stats() if stats else None
    status = lib.gs_sensitivity(C.byref(sc), C.byref(hv.c), C.byref(p), C.c_void_p(out.data_ptr()),
                                C.byref(st) if st is not None else None, _stream_handle(stream))
    _lib.check(status)
    return out, (st.as_dict() if st is not None else None)


def tune_tile(scene: DeviceScene, views, *, reps=2, footprint_sigma=3.0, dilation=0.3, z_near=0.2,
              share_floor=1e-12, query_mode=QUERY_RGBSUM, aggregate=AGG_RAY, max_views_per_chunk=0,
              stream=None):
    """Fastest binning tile (w, h) for gs_sensitivity on this scene and these
    views (gs_tune_tile), and the mean ms per call of each shape as a dict
    {(w, h): ms} (shapes the views cannot take are left out)."""
    torch = _torch()
    hv = _views(views)
    p = _params(footprint_sigma, dilation, z_near, share_floor, query_mode, None, max_views_per_chunk,
                aggregate=aggregate)
    out = torch.empty(scene.n, dtype=torch.float32, device=scene.opacity.device)
    bw, bh = C.c_int32(), C.c_int32()
    ms = (C.c_float * 9)()
    sc = scene.c_struct()
    _lib.check(load().gs_tune_tile(C.byref(sc), C.byref(hv.c), C.byref(p), int(reps),
                                   C.c_void_p(out.data_ptr()), C.byref(bw), C.byref(bh), ms,
                                   _stream_handle(stream)))
    sides = (8, 16, 32)
    table = {(sides[k // 3], sides[k % 3]): float(ms[k]) for k in range(9) if ms[k] >= 0}
    return (bw.value, bh.value), table


class Plan:
    """Batched sensitivity pass over several scenes (gs_plan_* in the C ABI):
    capacities fixed at creation, the whole pass queued without host
    synchronisation and replayed as a HIP graph.  The scenes' attribute
    tensors must stay alive, at the same addresses, while the plan exists."""

    def __init__(self, scenes, views, *, footprint_sigma=3.0, dilation=0.3, z_near=0.2,
                 share_floor=1e-12, query_mode=QUERY_RGBSUM, tile=(16, 16), stream=None):
        if len(scenes) != len(views) or not scenes:
            raise ValueError("need one views set per scene")
        lib = load()
        self.scenes = list(scenes)
        self._hv = [_views(v) for v in views]
        sc = (_lib.Scene * len(scenes))(*[s.c_struct() for s in scenes])
        vw = (_lib.Views * len(scenes))(*[h.c for h in self._hv])
        p = _params(footprint_sigma, dilation, z_near, share_floor, query_mode, None, 0, tile=tile)
        h = C.c_void_p()
        _lib.check(lib.gs_plan_create(sc, vw, len(scenes), C.byref(p), C.byref(h), _stream_handle(stream)))
        self._h = h
        self._outs = None

    def _ptrs(self, outs):
        return (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])

    def outputs(self):
        """Output tensors reused across runs (one float32 [n] per scene)."""
        torch = _torch()
        if self._outs is None:
            self._outs = [torch.empty(s.n, dtype=torch.float32, device=s.opacity.device) for s in self.scenes]
        return self._outs

    def run(self, outs=None, stream=None):
        outs = self.outputs() if outs is None else outs
        _lib.check(load().gs_plan_sensitivity(self._h, self._ptrs(outs), _stream_handle(stream)))
        return outs

    def set_config(self, persistent: int, xcd_remap: int):
        cfg = _lib.PlanConfig(persistent, xcd_remap)
        _lib.check(load().gs_plan_set_config(self._h, C.byref(cfg)))

    def tune(self, reps=3, outs=None, stream=None):
        """Times the launch shapes on this plan, keeps the fastest; returns
        (best config dict, mean ms per run of {0,1}, {0,0}, {1,0})."""
        outs = self.outputs() if outs is None else outs
        best = _lib.PlanConfig()
        ms = (C.c_float * 3)()
        _lib.check(load().gs_plan_tune(self._h, self._ptrs(outs), int(reps), C.byref(best), ms,
                                       _stream_handle(stream)))
        return {"persistent": best.persistent, "xcd_remap": best.xcd_remap}, list(ms)

    def info(self):
        i = _lib.PlanInfo()
        _lib.check(load().gs_plan_get_info(self._h, C.byref(i)))
        return {"n_scenes": i.n_scenes, "n_groups": i.n_groups, "persistent": i.config.persistent,
                "xcd_remap": i.config.xcd_remap, "graph_captured": i.graph_captured,
                "device_bytes": i.device_bytes, "list_capacity": i.list_capacity,
                "compact_bytes": i.compact_bytes, "n_launches": i.n_launches,
                "n_compact_launches": i.n_compact_launches, "n_sort3_scenes": i.n_sort3_scenes}

    def status(self, stream=None):
        """Raises GsError if some run overflowed a scene's list capacity."""
        _lib.check(load().gs_plan_status(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().gs_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sample_coreset(sens, m: int, seed: int, stream=None, out=None, noalloc=False):
    """Counts (int32 view of uint32), float64 weights and support (int64 [1]).
    out: optional (counts, weights, support) tensors to write into.
    noalloc=True calls gs_sample_coreset_noalloc (same results, no device
    allocation by the library; n <= 2^23)."""
    torch = _torch()
    lib = load()
    if sens.dtype != torch.float32 or not sens.is_cuda or not sens.is_contiguous():
        raise ValueError("sens must be a contiguous float32 device tensor")
    n = sens.numel()
    if out is None:
        counts = torch.empty(n, dtype=torch.int32, device=sens.device)
        weights = torch.empty(n, dtype=torch.float64, device=sens.device)
        support = torch.empty(1, dtype=torch.int64, device=sens.device)
    else:
        counts, weights, support = out
    fn = lib.gs_sample_coreset_noalloc if noalloc else lib.gs_sample_coreset
    status = fn(C.c_void_p(sens.data_ptr()), n, int(m), C.c_uint64(seed & (2**64 - 1)),
                C.c_void_p(counts.data_ptr()), C.c_void_p(weights.data_ptr()),
                C.c_void_p(support.data_ptr()), _stream_handle(stream))
    _lib.check(status)
    return counts, weights, support


def render_objective(scene: DeviceScene, views, weights=None, objective=OBJ_FULL, *,
                     footprint_sigma=3.0, dilation=0.3, z_near=0.2, query_mode=QUERY_RGBSUM,
                     ray_mask=None, max_views_per_chunk=0, per_ray=True, per_view=True,
                     diag=True, tile=(16, 16), stream=None):
    """Objective of a weighted pruned scene: per-ray values (float32 [rays]),
    per-view sums of (A, A^th_w, A_w) (float64 [V, 3]) and diagnostics."""
    torch = _torch()
    lib = load()
    hv = _views(views)
    p = _params(footprint_sigma, dilation, z_near, 0.0, query_mode, ray_mask, max_views_per_chunk, tile=tile)
    dev = scene.opacity.device
    pr = torch.zeros(hv.n_rays, dtype=torch.float32, device=dev) if per_ray else None
    pv = torch.zeros((hv.size.shape[0], 3), dtype=torch.float64, device=dev) if per_view else None
    if weights is not None and (weights.dtype != torch.float64 or not weights.is_cuda):
        raise ValueError("weights must be a float64 device tensor")
    dg = _lib.RenderDiag() if diag else None
    sc = scene.c_struct()
    status = lib.gs_render_objective(
        C.byref(sc), C.byref(hv.c), C.byref(p),
        C.c_void_p(weights.data_ptr()) if weights is not None else None, int(objective),
        C.c_void_p(pr.data_ptr()) if pr is not None else None,
        C.c_void_p(pv.data_ptr()) if pv is not None else None,
        C.byref(dg) if dg is not None else None, _stream_handle(stream))
    _lib.check(status)
    out = {"per_ray": pr, "per_view": pv}
    if dg is not None:
        out["n_invalid_pairs"] = int(dg.n_invalid_pairs)
        out["gamma_max"] = float(dg.gamma_max)
    return out


def region_bound(world_to_cam, A, A_w, lam=1.0, rho_target=0.0, a_floor=1e-3, stream=None):
    """Theorem 4's bound over a region of sampled camera poses
    (gs_region_bound): world_to_cam [K][12] host array, A and A_w float32
    device tensors [K][pixels] of per-ray full and reduced renders.  Returns
    (report dict, representative flags as a bool array)."""
    torch = _torch()
    w = np.ascontiguousarray(np.asarray(world_to_cam, np.float64).reshape(-1, 12))
    K = w.shape[0]
    for t in (A, A_w):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() % K:
            raise ValueError("A and A_w must be contiguous float32 device tensors of K rows")
    net = np.zeros(K, np.int32)
    rep = _lib.RegionReport()
    _lib.check(load().gs_region_bound(w.ctypes.data, K, float(lam), float(rho_target), C.c_void_p(A.data_ptr()),
                                      C.c_void_p(A_w.data_ptr()), A.numel() // K, float(a_floor), net.ctypes.data,
                                      C.byref(rep), _stream_handle(stream)))
    return {k: getattr(rep, k) for k, _ in rep._fields_ if k != "pad"}, net.astype(bool)


def measure_peaks(stream=None):
    """Measured copy bandwidth, FP32 FMA, v_exp_f32 and BF16 MFMA rates (gs_measure_peaks)."""
    p = _lib.Peaks()
    _lib.check(load().gs_measure_peaks(C.byref(p), _stream_handle(stream)))
    return {k: getattr(p, k) for k, _ in p._fields_}


def release_workspace():
    _lib.check(load().gs_release_workspace())


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_allocator_refs = None   # keeps the registered callbacks alive


def use_torch_allocator(enable: bool = True):
    """Route the library's device memory (scratch arenas, plan buffers)
    through torch's caching allocator (gs_set_allocator), or back to
    hipMalloc / hipFree with enable=False.  Memory the library holds then
    shows in torch.cuda.memory_allocated() and returns to torch's cache."""
    global _allocator_refs
    torch = _torch()
    lib = load()
    if not enable:
        _lib.check(lib.gs_set_allocator(None, None, None))
        _allocator_refs = None
        return

    def alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
        except Exception:   # noqa: BLE001 - a failed allocation is reported as NULL
            return None

    def release(ctx, ptr, stream):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:   # noqa: BLE001
            pass

    refs = (_ALLOC_FN(alloc), _FREE_FN(release))
    _lib.check(lib.gs_set_allocator(C.cast(refs[0], C.c_void_p), C.cast(refs[1], C.c_void_p), None))
    _allocator_refs = refs


def coreset_error(per_view, reduced=False, stream=None):
    """E = max over views of |sum A^th_w - sum A| / sum A (per-image fixed
    objective), or with reduced=True the same with the reduced render A_w
    (gs_coreset_error on the per-view sums of render_objective)."""
    torch = _torch()
    pv = per_view
    if not (hasattr(pv, "is_cuda") and pv.is_cuda and pv.dtype == torch.float64 and pv.is_contiguous()):
        pv = torch.as_tensor(np.ascontiguousarray(np.asarray(pv if not hasattr(pv, "detach") else pv.cpu()),
                                                  np.float64)).cuda()
    out = torch.empty(2, dtype=torch.float64, device=pv.device)
    _lib.check(load().gs_coreset_error(C.c_void_p(pv.data_ptr()), int(pv.shape[0]), C.c_void_p(out.data_ptr()),
                                       _stream_handle(stream)))
    return float(out[1 if reduced else 0].item())
