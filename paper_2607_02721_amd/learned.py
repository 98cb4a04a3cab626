"""Learned sampling proposal: features -> MLP -> mixture proposal, judged by the
fixed coreset objective with the exact pass as fallback.

Sensitivity sampling (Algorithm 1, steps 4-5) stays unbiased for any
proposal p with p_i > 0 wherever a Gaussian can contribute (proof of
Theorem 2: E[Y_t] = 1 needs only that), so a predictor of s mixed with a
uniform floor can stand in for the exact pass; the per-view fixed objective
on held-out rays decides whether the draw is good enough, and the exact pass
takes over when it is not.

Every computation runs in the library's HIP kernels (gs_features,
gs_feature_stats, gs_mlp_*, gs_log_targets, gs_proposal_mixture,
gs_sample_coreset, gs_render_objective, gs_sensitivity); this module only
sequences them and holds the device buffers (training batches are gathered
by index with torch: data movement only).
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import _lib
from . import (DeviceScene, OBJ_FIXED, coreset_error, load, render_objective, sample_coreset,
               sensitivity, _stream_handle)

N_FEATURES = 64
# Targets are ln(max(s, 1e-6)): below that a Gaussian's share of the proposal
# is negligible, and the floor keeps never-contributing Gaussians from
# dominating the squared error.
LOG_FLOOR = 1e-6


def _torch():
    import torch
    return torch


def features(scene: DeviceScene, stream=None):
    """float32 device tensor [n, 64] of raw features (gs_features)."""
    torch = _torch()
    out = torch.empty((scene.n, N_FEATURES), dtype=torch.float32, device=scene.opacity.device)
    sc = scene.c_struct()
    _lib.check(load().gs_features(C.byref(sc), C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def knn(scene: DeviceScene, stream=None):
    """The 16 nearest other means of every Gaussian (gs_knn): (indices as an
    int32 view of uint32 [n, 16], float32 squared distances [n, 16])."""
    torch = _torch()
    idx = torch.empty((scene.n, 16), dtype=torch.int32, device=scene.opacity.device)
    d2 = torch.empty((scene.n, 16), dtype=torch.float32, device=scene.opacity.device)
    sc = scene.c_struct()
    _lib.check(load().gs_knn(C.byref(sc), C.c_void_p(idx.data_ptr()), C.c_void_p(d2.data_ptr()),
                             _stream_handle(stream)))
    return idx, d2


def feature_stats(feat, stream=None):
    torch = _torch()
    norm = torch.empty((2, N_FEATURES), dtype=torch.float32, device=feat.device)
    _lib.check(load().gs_feature_stats(C.c_void_p(feat.data_ptr()), feat.shape[0],
                                       C.c_void_p(norm.data_ptr()), _stream_handle(stream)))
    return norm


def log_targets(sens, stream=None):
    """ln(max(s, 1e-6)) as float32 device tensor [n] (gs_log_targets)."""
    torch = _torch()
    out = torch.empty_like(sens)
    _lib.check(load().gs_log_targets(C.c_void_p(sens.data_ptr()), sens.numel(), C.c_float(LOG_FLOOR),
                                     C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


class Proposal:
    """MLP 64 -> 256 -> 256 -> 256 -> 1 (SiLU) predicting ln s; parameters and
    Adam moments live in device memory."""

    def __init__(self, seed: int = 0, device="cuda"):
        torch = _torch()
        lib = load()
        self.P = int(lib.gs_mlp_param_count())
        self.params = torch.empty(self.P, dtype=torch.float32, device=device)
        self.adam = torch.zeros(2 * self.P, dtype=torch.float32, device=device)
        self.norm = None
        self.step = 0
        _lib.check(lib.gs_mlp_init(C.c_void_p(self.params.data_ptr()), C.c_uint64(seed),
                                   _stream_handle()))

    def set_norm(self, norm):
        self.norm = norm.contiguous()

    def train_step(self, feat, target, lr=1e-3, grad=None):
        """One Adam step on a batch (<= 65536 rows); returns the loss tensor [1]."""
        torch = _torch()
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        self.step += 1
        _lib.check(load().gs_mlp_train_step(
            C.c_void_p(self.params.data_ptr()), C.c_void_p(self.adam.data_ptr()), self.step,
            C.c_float(lr), C.c_void_p(feat.data_ptr()), C.c_void_p(self.norm.data_ptr()),
            C.c_void_p(target.data_ptr()), feat.shape[0], C.c_void_p(loss.data_ptr()),
            C.c_void_p(grad.data_ptr()) if grad is not None else None, _stream_handle()))
        return loss

    def gradient(self, feat, target, fp32=False):
        """Loss and gradient on a batch without updating (gs_mlp_gradient), in
        BF16 (the training arithmetic) or with fp32=True in FP32."""
        torch = _torch()
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        grad = torch.empty(self.P, dtype=torch.float32, device=feat.device)
        _lib.check(load().gs_mlp_gradient(
            C.c_void_p(self.params.data_ptr()), C.c_void_p(feat.data_ptr()), C.c_void_p(self.norm.data_ptr()),
            C.c_void_p(target.data_ptr()), feat.shape[0], _lib.MLP_FP32 if fp32 else _lib.MLP_BF16,
            C.c_void_p(loss.data_ptr()), C.c_void_p(grad.data_ptr()), _stream_handle()))
        return loss, grad

    def predict(self, feat):
        torch = _torch()
        out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        _lib.check(load().gs_mlp_forward(C.c_void_p(self.params.data_ptr()), C.c_void_p(feat.data_ptr()),
                                         C.c_void_p(self.norm.data_ptr()), feat.shape[0],
                                         C.c_void_p(out.data_ptr()), _stream_handle()))
        return out

    def fit(self, feats, targets, epochs=4, batch=16384, lr=1e-3, seed=0, log=None):
        """Adam over the concatenated training set, shuffled per epoch."""
        torch = _torch()
        X = torch.cat(feats) if isinstance(feats, (list, tuple)) else feats
        Y = torch.cat(targets) if isinstance(targets, (list, tuple)) else targets
        if self.norm is None:
            self.set_norm(feature_stats(X))
        g = torch.Generator(device="cpu").manual_seed(seed)
        losses = []
        n = X.shape[0]
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(X.device)
            tot = torch.zeros(1, dtype=torch.float64, device=X.device)
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                loss = self.train_step(X[idx].contiguous(), Y[idx].contiguous(), lr)
                tot += loss.double() * idx.numel()
            losses.append(float(tot.item()) / n)
            if log:
                log(f"epoch {ep}: loss {losses[-1]:.4f}")
        return losses


def mixture(log_s_hat, floor=0.1, stream=None):
    """Proposal p = (1 - floor) s_hat / sum(s_hat) + floor / n (gs_proposal_mixture),
    as float32 scores for gs_sample_coreset."""
    torch = _torch()
    p = torch.empty_like(log_s_hat)
    _lib.check(load().gs_proposal_mixture(C.c_void_p(log_s_hat.data_ptr()), log_s_hat.numel(), C.c_float(floor),
                                          C.c_void_p(p.data_ptr()), _stream_handle(stream)))
    return p


def sample_with_fallback(scene: DeviceScene, judge_views, m: int, seed: int, proposal: Proposal,
                         judge_mask, err_bound=0.01, exact_views=None, floor=0.1, feat=None):
    """Draw a weighted coreset from the learned mixture proposal; judge it by
    E (per-view fixed objective on the masked judge rays); if E exceeds the
    bound, run the exact sensitivity pass (on `exact_views`, default the judge
    views) and draw from it instead.  The result says which draw it returns
    ("fallback") and whether that draw meets the bound ("bound_met": False
    when the exact draw misses it too, since no draw of this m did)."""
    torch = _torch()
    t0 = time.perf_counter()
    if feat is None:
        feat = features(scene)
    scores = mixture(proposal.predict(feat), floor)
    _, w, _ = sample_coreset(scores, m, seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ob = render_objective(scene, judge_views, w, OBJ_FIXED, ray_mask=judge_mask, per_ray=False, diag=False)
    err = coreset_error(ob["per_view"])
    t2 = time.perf_counter()
    out = {"weights": w, "E_learned": err, "fallback": False, "bound_met": err <= err_bound,
           "ms_propose": (t1 - t0) * 1e3, "ms_judge": (t2 - t1) * 1e3}
    if err > err_bound:
        s, _ = sensitivity(scene, exact_views if exact_views is not None else judge_views)
        _, w2, _ = sample_coreset(s, m, seed)
        ob2 = render_objective(scene, judge_views, w2, OBJ_FIXED, ray_mask=judge_mask, per_ray=False,
                               diag=False)
        torch.cuda.synchronize()
        e2 = coreset_error(ob2["per_view"])
        out.update(weights=w2, fallback=True, E_exact=e2, bound_met=e2 <= err_bound,
                   ms_fallback=(time.perf_counter() - t2) * 1e3)
    return out
