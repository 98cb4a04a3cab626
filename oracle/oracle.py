"""Python face of the FP64 CPU oracle (``gs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark.  The product package never imports
this module; the two share no code.

Every function takes ``synth.Scene`` / ``synth.Views`` inputs (float32 SoA
scene, float64 cameras) and returns NumPy arrays.  See ``gs_oracle.c`` for the
paper passages each step follows and for the conventions the paper leaves open.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "libgs_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-pthread",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32),
                ("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class _Views(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("world_to_cam", C.c_void_p),
                ("intrinsics", C.c_void_p), ("size", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("footprint_sigma", C.c_double), ("dilation", C.c_double),
                ("z_near", C.c_double), ("share_floor", C.c_double),
                ("ambiguity_beta", C.c_double), ("query_mode", C.c_int32),
                ("n_threads", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = C.CDLL(_LIB)
        P = C.c_void_p
        _lib.ora_sensitivity.argtypes = [P, P, P, P, P, P, P, P]
        _lib.ora_sensitivity_agg.argtypes = [P, P, P, P, C.c_int32, P]
        _lib.ora_objective.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
        _lib.ora_objective_true_scale.argtypes = [P, P, P, P, P, P]
        _lib.ora_objective_true_scale.restype = C.c_int
        _lib.ora_sample.argtypes = [P, C.c_int64, C.c_int64, C.c_uint64, P, P, P, P]
        _lib.ora_philox4x32_10.argtypes = [P, P, P]
        _lib.ora_project.argtypes = [P] * 13
        _lib.ora_draw_target.argtypes = [P, C.c_uint64]
        _lib.ora_draw_target.restype = C.c_uint64
        _lib.ora_sh_basis.argtypes = [C.c_double, C.c_double, C.c_double, P]
        _lib.ora_knn.argtypes = [P, C.c_int64, C.c_int, C.c_int, P, P]
        _lib.ora_knn.restype = C.c_int
        for f in (_lib.ora_sensitivity, _lib.ora_sensitivity_agg, _lib.ora_objective, _lib.ora_sample):
            f.restype = C.c_int
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Keep:
    """Holds contiguous copies so the pointers stay valid during a call."""

    def __init__(self, scene, views, params):
        self.mean = np.ascontiguousarray(scene.mean, np.float32)
        self.log_scale = np.ascontiguousarray(scene.log_scale, np.float32)
        self.quat = np.ascontiguousarray(scene.quat, np.float32)
        self.opacity = np.ascontiguousarray(scene.opacity, np.float32)
        self.sh = np.ascontiguousarray(scene.sh, np.float32)
        self.w2c = np.ascontiguousarray(views.world_to_cam, np.float64)
        self.intr = np.ascontiguousarray(views.intrinsics, np.float64)
        self.size = np.ascontiguousarray(views.size, np.int32)
        self.s = _Scene(scene.n, scene.sh_degree, _ptr(self.mean), _ptr(self.log_scale),
                        _ptr(self.quat), _ptr(self.opacity), _ptr(self.sh))
        self.v = _Views(views.n_views, _ptr(self.w2c), _ptr(self.intr), _ptr(self.size))
        self.p = _Params(params.get("footprint_sigma", 3.0), params.get("dilation", 0.3),
                         params.get("z_near", 0.2), params.get("share_floor", 1e-12),
                         params.get("ambiguity_beta", 1e-5), params.get("query_mode", 0),
                         params.get("n_threads", os.cpu_count() or 1))


# query modes (gs_oracle.c: pair_contrib)
QUERY_RGBSUM, QUERY_NOCOLOR, QUERY_L2, QUERY_CHANNEL = 0, 1, 2, 3


def default_params(**kw):
    p = dict(footprint_sigma=3.0, dilation=0.3, z_near=0.2, share_floor=1e-12,
             ambiguity_beta=1e-5, query_mode=0, n_threads=os.cpu_count() or 1)
    p.update(kw)
    return p


def sensitivity(scene, views, params=None, ray_mask=None):
    """Sensitivities s[n] (float64), per-ray A[rays] ([rays, 3] for per-channel
    queries), per-ray ambiguity flags, and counters (pairs, live pairs, rays
    with a positive query).  ``ray_mask`` is a uint32 bitset over rays
    (view-major, row-major) or None for every ray."""
    lib = _load()
    params = params or default_params()
    k = _Keep(scene, views, params)
    n_rays = views.n_rays
    nq = 3 if params.get("query_mode", 0) == QUERY_CHANNEL else 1
    s = np.zeros(scene.n, np.float64)
    A = np.zeros(n_rays * nq, np.float64)
    flag = np.zeros(n_rays, np.uint8)
    cnt = np.zeros(3, np.int64)
    mask = None if ray_mask is None else np.ascontiguousarray(ray_mask, np.uint32)
    rc = lib.ora_sensitivity(C.byref(k.s), C.byref(k.v), C.byref(k.p), _ptr(mask),
                             _ptr(s), _ptr(A), _ptr(flag), _ptr(cnt))
    assert rc == 0
    if nq > 1:
        A = A.reshape(n_rays, nq)
    return {"s": s, "A": A, "flag": flag.astype(bool), "pairs": int(cnt[0]),
            "live_pairs": int(cnt[1]), "rays_positive": int(cnt[2])}


AGG_RAY, AGG_TILE, AGG_IMAGE, AGG_SCENE = 0, 1, 2, 3


def sensitivity_agg(scene, views, level, params=None, ray_mask=None):
    """Aggregated sensitivities s[n] (float64) for queries that are 16x16
    tiles (level 1), whole views (2) or the whole scene (3): the maximum over
    queries of a_i(Q) / A(Q) with both summed over the query's rays
    (Section 3.5).  Level 0 is the per-ray sensitivity."""
    if level == AGG_RAY:
        return sensitivity(scene, views, params, ray_mask)["s"]
    lib = _load()
    k = _Keep(scene, views, params or default_params())
    s = np.zeros(scene.n, np.float64)
    mask = None if ray_mask is None else np.ascontiguousarray(ray_mask, np.uint32)
    rc = lib.ora_sensitivity_agg(C.byref(k.s), C.byref(k.v), C.byref(k.p), _ptr(mask), int(level), _ptr(s))
    if rc == 2:
        raise ValueError("per-channel queries have no aggregated form")
    assert rc == 0
    return s


def objective(scene, views, weights, params=None, ray_mask=None):
    """Per-ray full A, fixed A^th_w and true A_w, per-view sums [V][3], count of
    pairs with w rho >= 1, and the largest log-transmittance gap."""
    lib = _load()
    k = _Keep(scene, views, params or default_params())
    n_rays = views.n_rays
    out = [np.zeros(n_rays, np.float64) for _ in range(3)]
    vs = np.zeros((views.n_views, 3), np.float64)
    inv = np.zeros(1, np.int64)
    gam = np.zeros(1, np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    mask = None if ray_mask is None else np.ascontiguousarray(ray_mask, np.uint32)
    rc = lib.ora_objective(C.byref(k.s), C.byref(k.v), C.byref(k.p), _ptr(mask), _ptr(w),
                           _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(vs), _ptr(inv), _ptr(gam))
    if rc == 2:
        raise ValueError("the objectives hold one query per ray (not per channel)")
    assert rc == 0
    return {"A": out[0], "A_fixed": out[1], "A_true": out[2], "view_sums": vs,
            "n_invalid": int(inv[0]), "gamma": float(gam[0])}


def objective_true_scale(scene, views, weights, params=None, ray_mask=None):
    """Per-ray rounding scale E of the true reduced render (test
    infrastructure): a relative error d in every rho moves A_w by at most
    d E to first order (see ora_objective_true_scale)."""
    lib = _load()
    k = _Keep(scene, views, params or default_params())
    E = np.zeros(views.n_rays, np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    mask = None if ray_mask is None else np.ascontiguousarray(ray_mask, np.uint32)
    rc = lib.ora_objective_true_scale(C.byref(k.s), C.byref(k.v), C.byref(k.p), _ptr(mask), _ptr(w), _ptr(E))
    if rc == 2:
        raise ValueError("the objectives hold one query per ray (not per channel)")
    assert rc == 0
    return E


def project(scene, views, params=None):
    """FP64 projection of every (view, Gaussian): dict of arrays shaped [V, n, ...]."""
    lib = _load()
    k = _Keep(scene, views, params or default_params())
    V, n = views.n_views, scene.n
    present = np.zeros(V * n, np.int32)
    z = np.zeros(V * n, np.float64)
    key = np.zeros(V * n, np.float32)
    amb = np.zeros(V * n, np.int32)
    mean2d = np.zeros((V * n, 2), np.float64)
    cov = np.zeros((V * n, 3), np.float64)
    conic = np.zeros((V * n, 3), np.float64)
    rgb = np.zeros((V * n, 3), np.float64)
    cbar = np.zeros(V * n, np.float64)
    rad = np.zeros((V * n, 2), np.float64)
    lib.ora_project(C.byref(k.s), C.byref(k.v), C.byref(k.p), _ptr(present), _ptr(z), _ptr(key),
                    _ptr(amb), _ptr(mean2d), _ptr(cov), _ptr(conic), _ptr(rgb), _ptr(cbar), _ptr(rad))
    r = lambda a, *t: a.reshape((V, n) + t)
    return {"present": r(present).astype(bool), "z": r(z), "key": r(key),
            "key_ambiguous": r(amb).astype(bool), "mean2d": r(mean2d, 2), "cov": r(cov, 3),
            "conic": r(conic, 3), "rgb": r(rgb, 3), "cbar": r(cbar), "radius": r(rad, 2)}


def sample(s_f32, m, seed):
    """Counts u32[n], weights f64[n], support, Q and status (0 ok, 4 if all s = 0,
    5 if some s is outside [0, 1 + 2^-10] or NaN: outputs zeroed)."""
    lib = _load()
    s = np.ascontiguousarray(s_f32, np.float32)
    n = s.shape[0]
    counts = np.zeros(n, np.uint32)
    w = np.zeros(n, np.float64)
    sup = np.zeros(1, np.int64)
    Q = np.zeros(1, np.uint64)
    rc = lib.ora_sample(_ptr(s), n, m, C.c_uint64(seed), _ptr(counts), _ptr(w), _ptr(sup), _ptr(Q))
    return {"counts": counts, "weights": w, "support": int(sup[0]), "Q": int(Q[0]), "status": rc}


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib.ora_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw_target(words, Q):
    """floor(u Q / 2^128) for u given as four little-endian 32-bit words."""
    lib = _load()
    x = np.ascontiguousarray(words, np.uint32)
    return int(lib.ora_draw_target(_ptr(x), C.c_uint64(Q)))


def sh_basis(d):
    lib = _load()
    Y = np.zeros(16, np.float64)
    lib.ora_sh_basis(float(d[0]), float(d[1]), float(d[2]), _ptr(Y))
    return Y


# --------------------------------------------------------------------------
# Features of the learned sampling proposal.  The paper has no learned part:
# these follow the feature definition the library documents (64 values per
# Gaussian), evaluated in FP64 from neighbour sets chosen in float32.
N_FEATURES = 64
KNN_K = 16


def knn(mean, k=KNN_K, n_threads=None):
    """k nearest other means of every Gaussian by brute force over all pairs:
    float32 squared distances ((dx dx + dy dy) + dz dz, each step rounded to
    float32), ordered by (distance, index).  mean: float32 [3][n].
    Returns (idx uint32 [n][k], 0xFFFFFFFF where fewer than k others exist;
    d2 float32 [n][k], +inf there)."""
    lib = _load()
    m = np.ascontiguousarray(mean, np.float32).reshape(3, -1)
    n = m.shape[1]
    idx = np.zeros((n, k), np.uint32)
    d2 = np.zeros((n, k), np.float32)
    rc = lib.ora_knn(_ptr(m), n, int(k), int(n_threads or os.cpu_count() or 1), _ptr(idx), _ptr(d2))
    assert rc == 0
    return idx, d2


def features(scene, k=KNN_K):
    """FP64 features [n][64] of the learned proposal, from the float32 scene:
      0-2 mean, 3-5 log-scale, 6-9 quaternion / |quaternion| with the sign
      that makes w >= 0 (w = 0 keeps the sign), 10 logit(alpha) with alpha
      first clamped in float32 to [1e-6, 1 - 1e-6], 11-58 the SH
      coefficients in plane order (zero past the scene's degree), and over
      the k nearest other means (``knn``): 59 log of their mean distance,
      60 log of the k-th distance d_k, 61 mean and 62 largest neighbour
      opacity, 63 log(sum of neighbour opacities / (4/3 pi d_k^3)); each
      logarithm's argument is first raised to at least 1e-12.  With no
      neighbour at all: 59 = 60 = 0, 61 = 62 = 0 and d_k = 1 in 63."""
    n = scene.n
    f = np.zeros((n, N_FEATURES), np.float64)
    mean = np.asarray(scene.mean, np.float32).reshape(3, n)
    f[:, 0:3] = mean.T
    f[:, 3:6] = np.asarray(scene.log_scale, np.float32).reshape(3, n).T
    q = np.asarray(scene.quat, np.float32).reshape(4, n).T.astype(np.float64)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    qn[q[:, 0] < 0] *= -1.0
    f[:, 6:10] = qn
    op = np.asarray(scene.opacity, np.float32).reshape(n)
    lo, hi = np.float32(1e-6), np.float32(1.0) - np.float32(1e-6)
    a = np.minimum(np.maximum(op, lo), hi).astype(np.float64)
    f[:, 10] = np.log(a / (1.0 - a))
    sh = np.asarray(scene.sh, np.float32).reshape(-1, n)
    nsh = min(sh.shape[0], 48)
    f[:, 11:11 + nsh] = sh[:nsh].T
    idx, d2 = knn(mean, k)
    valid = idx != np.uint32(0xFFFFFFFF)
    cnt = valid.sum(axis=1)
    dist = np.where(valid, np.sqrt(np.where(valid, d2, 0).astype(np.float64)), 0.0)
    nb_a = np.where(valid, op[np.where(valid, idx, 0)].astype(np.float64), 0.0)
    has = cnt > 0
    dk = np.ones(n)
    dk[has] = dist[has, cnt[has] - 1]
    tiny = 1e-12
    mean_d = np.where(has, dist.sum(axis=1) / np.maximum(cnt, 1), 1.0)
    f[:, 59] = np.log(np.maximum(mean_d, tiny))
    f[:, 60] = np.log(np.maximum(dk, tiny))
    f[:, 61] = np.where(has, nb_a.sum(axis=1) / np.maximum(cnt, 1), 0.0)
    f[:, 62] = nb_a.max(axis=1)
    vol = 4.0 / 3.0 * np.pi * dk ** 3
    f[:, 63] = np.log(np.maximum(nb_a.sum(axis=1), tiny) / np.maximum(vol, tiny))
    return f, idx, d2


# --------------------------------------------------------------------------
# Theorem 3 (finite-query rendered coreset): a fixed-objective guarantee eps_c
# and log-transmittance stability gamma give the rendered guarantee eps_r.
def eps_rendered(gamma, eps_c):
    """eps_r = max{1 - e^-gamma (1 - eps_c), e^gamma (1 + eps_c) - 1}."""
    g = np.asarray(gamma, np.float64)
    e = np.asarray(eps_c, np.float64)
    return np.maximum(1.0 - np.exp(-g) * (1.0 - e), np.exp(g) * (1.0 + e) - 1.0)
