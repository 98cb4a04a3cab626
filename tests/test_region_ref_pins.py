"""Pins of the oracle's compact-region extension (Section 3.4; appendix,
compact-region extension from representatives): the pose metric against
closed forms, the rho-net's covering property, the bound's constants on
inputs with known Lipschitz constants, and Theorem 4 on real renders of a
small scene (the bound must hold at every sampled query)."""
import math

import numpy as np
import pytest

import synth
from oracle import region


def _rot(axis, ang):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def _w2c(R, c):
    R = np.asarray(R, np.float64)
    return np.concatenate([R, (-R @ np.asarray(c, np.float64))[:, None]], 1).ravel()


def test_pose_distance_closed_forms():
    R0 = _rot([0.3, -1, 0.2], 0.7)
    a = _w2c(R0, [1.0, 2.0, 3.0])
    b = _w2c(R0, [1.0, 2.0 + 0.25, 3.0 - 0.5])
    assert abs(region.pose_distance(a, b, 2.0) - math.hypot(0.25, 0.5)) < 1e-14
    for ang in (1e-9, 1e-4, 0.3, 2.0, 3.1):
        c = _w2c(_rot([1, 2, -0.5], ang) @ R0, [1.0, 2.0, 3.0])
        assert abs(region.pose_distance(a, c, 1.5) - 1.5 * ang) <= 1e-13 * max(1.0, ang) + 1e-15 * ang
    rng = np.random.default_rng(0)
    P = [_w2c(_rot(rng.normal(size=3), rng.uniform(0, 3)), rng.normal(size=3)) for _ in range(6)]
    D = region.distance_matrix(P, 0.8)
    assert np.allclose(D, D.T) and np.all(np.diag(D) == 0)
    for i in range(6):
        for j in range(6):
            for k in range(6):
                assert D[i, k] <= D[i, j] + D[j, k] + 1e-12


def test_rho_net_covers_and_separates():
    rng = np.random.default_rng(1)
    pts = rng.uniform(0, 1, (200, 2))
    D = np.linalg.norm(pts[:, None] - pts[None], axis=2)
    for rho in (0.05, 0.1, 0.3):
        net, reach = region.rho_net(D, rho)
        assert reach <= rho
        assert np.all(np.min(D[:, net], axis=1) <= rho)
        sub = D[np.ix_(net, net)] + np.eye(len(net)) * 10
        assert sub.min() > rho           # every representative was farther than rho from the others
    # points on a line 0..10: greedy takes 0, then 10, then 5, ...
    x = np.arange(11.0)
    net, reach = region.rho_net(np.abs(x[:, None] - x[None]), 2.5)
    assert net[:3] == [0, 10, 5] and reach <= 2.5


def test_bound_constants_on_linear_renders():
    """A_k = a + b x_k and A_w = (1 + e) A_k along a line of poses: the
    Lipschitz estimates are exactly |b| and (1 + e)|b|, eps_0 = e, and the
    bound follows Theorem 4's formula."""
    x = np.linspace(0.0, 2.0, 9)
    D = np.abs(x[:, None] - x[None])
    a = np.array([1.0, 2.0, 0.5])
    b = np.array([0.3, -0.7, 0.1])
    A = a[None] + b[None] * x[:, None]
    e = 0.02
    Aw = (1 + e) * A
    net, reach = region.rho_net(D, 0.5)
    r = region.region_bound(A, Aw, D, net, np.ones(3, bool))
    assert abs(r["L_full"] - 0.7) < 1e-12 and abs(r["L_w"] - 0.7 * (1 + e)) < 1e-12
    assert abs(r["eps_0"] - e) < 1e-12 and abs(r["A_min"] - A.min()) < 1e-15
    want = e + ((1 + e) * 0.7 + 0.7 * (1 + e)) * r["rho"] / A.min()
    assert abs(r["eps_reg"] - want) < 1e-12
    assert r["max_err"] <= r["eps_reg"]
    rho_t = region.rho_for_target(0.1, e, 0.7, 0.7 * (1 + e), A.min())
    assert abs(e + ((1 + e) * 0.7 + 0.7 * (1 + e)) * rho_t / A.min() - 0.1) < 1e-12


def test_theorem4_holds_on_rendered_region(ora):
    """Poses around one camera of the tiny scene, weights of a coreset: with
    the constants estimated over the sampled poses, every sampled query
    (pose, pixel with A > 0 everywhere) satisfies |A - A_w| <= eps_reg A."""
    sc, vw, m, seed = synth.make_config("tiny")
    w2c = synth.make_pose_region(vw.world_to_cam[0], 24, 0.05, 0.03, seed=5)
    views = synth.Views(np.stack(w2c), np.repeat(vw.intrinsics[:1], 24, 0), np.repeat(vw.size[:1], 24, 0))
    r = ora.sensitivity(sc, vw)
    w = ora.sample(r["s"].astype(np.float32), 1500, seed)["weights"]
    ob = ora.objective(sc, views, w)
    P = int(vw.size[0, 0] * vw.size[0, 1])
    A = ob["A"].reshape(24, P)
    Aw = ob["A_true"].reshape(24, P)
    keep = np.all(A > 1e-3, axis=0)
    assert keep.sum() > 100
    D = region.distance_matrix(w2c, 1.0)
    net, reach = region.rho_net(D, 0.04)
    out = region.region_bound(A, Aw, D, net, keep)
    err = np.abs(A - Aw)[:, keep] / A[:, keep]
    print("[region]", {k: v for k, v in out.items() if k != "err_per_pose"}, len(net), flush=True)
    assert np.all(err <= out["eps_reg"] * (1 + 1e-12))
    assert out["eps_0"] <= out["max_err"] <= out["eps_reg"]
