"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test pins one part of the oracle to something other than itself: a
closed form, an invariant, a special case that reduces to a library routine,
published known-answer values, or brute force on tiny inputs.  A plausible
slip in the oracle (a dropped term, a sign, a transposed operand, a wrong
index) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import synth
from synth import (make_camera_set, make_cluster_scene, make_explicit_scene, make_orbit_views, make_tiny_scene,
                   make_tiny_views, pack_bits)

HERE = os.path.dirname(os.path.abspath(__file__))
ID_Q = (1.0, 0.0, 0.0, 0.0)


def _axis_camera(width=63, height=63, fov=60.0, dist=4.0):
    """One camera on the -x axis looking at the origin (optical axis = +x)."""
    return make_camera_set([(-dist, 0.0, 0.0)], [(0.0, 0.0, 0.0)], width, height, fov)


def _focal(width, fov):
    return (width / 2.0) / math.tan(math.radians(fov) / 2.0)


# --------------------------------------------------------------------------
# Philox4x32-10: published known-answer vectors (Salmon et al., SC 2011).
def test_philox_known_answers(ora):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = ora.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# --------------------------------------------------------------------------
# Spherical-harmonic colour basis: orthonormal on the sphere, and equal up to
# a per-function sign to the real combinations of scipy's complex harmonics.
def test_sh_basis_orthonormal_and_matches_scipy(ora):
    from scipy.special import sph_harm_y
    xg, wg = np.polynomial.legendre.leggauss(24)          # cos(theta) nodes
    nphi = 48
    phis = 2 * np.pi * (np.arange(nphi) + 0.5) / nphi
    G = np.zeros((16, 16))
    ref_sign = {}
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for ph in phis:
            d = (st * math.cos(ph), st * math.sin(ph), ct)
            Y = ora.sh_basis(d)
            G += np.outer(Y, Y) * w * (2 * np.pi / nphi)
            theta = math.acos(ct)
            for l in range(4):
                for m in range(-l, l + 1):
                    k = l * l + l + m
                    c = sph_harm_y(l, abs(m), theta, ph)
                    if m == 0:
                        ref = c.real
                    elif m > 0:
                        ref = math.sqrt(2) * c.real
                    else:
                        ref = math.sqrt(2) * c.imag
                    if abs(ref) > 1e-3:
                        sgn = np.sign(Y[k] / ref)
                        ref_sign.setdefault(k, sgn)
                        assert sgn == ref_sign[k]
                        assert abs(abs(Y[k]) - abs(ref)) < 1e-12
    assert np.allclose(G, np.eye(16), atol=1e-12)


# --------------------------------------------------------------------------
# Projection (local-affine / EWA): closed forms and a finite-difference Jacobian.
def test_projection_isotropic_on_axis_closed_form(ora):
    W = 63
    f = _focal(W, 60.0)
    sig, dist, delta = 0.05, 4.0, 0.3
    sc = make_explicit_scene([(0.0, 0.0, 0.0)], [math.log(sig)] * 3, ID_Q, 0.5)
    vw = _axis_camera(W, W, 60.0, dist)
    pr = ora.project(sc, vw, ora.default_params(dilation=delta))
    s = float(np.float32(sig))
    expect = (f * s / dist) ** 2 + delta
    assert pr["present"][0, 0]
    assert abs(pr["z"][0, 0] - dist) < 1e-12
    assert np.allclose(pr["mean2d"][0, 0], [W / 2, W / 2], atol=1e-12)
    assert np.allclose(pr["cov"][0, 0], [expect, 0.0, expect], rtol=1e-6, atol=1e-12)
    # conic is the inverse of the 2D covariance
    c = pr["conic"][0, 0]
    assert np.allclose(c, [1 / expect, 0.0, 1 / expect], rtol=1e-6)


def _pixel_map(vw, v, p):
    P = vw.world_to_cam[v].reshape(3, 4)
    fx, fy, cx, cy = vw.intrinsics[v]
    q = P[:, :3] @ p + P[:, 3]
    return np.array([fx * q[0] / q[2] + cx, fy * q[1] / q[2] + cy])


def test_projection_matches_numerical_jacobian_and_rotation(ora):
    """Sigma_2d - delta I must equal Jn Sigma Jn^T, with Jn the central-difference
    Jacobian of the world-to-pixel map and Sigma built with scipy's rotation."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(7)
    n = 12
    means = rng.uniform(-0.6, 0.6, (n, 3))
    ls = rng.normal(-2.5, 0.4, (n, 3))
    q = rng.standard_normal((n, 4))
    sc = make_explicit_scene(means, ls, q, 0.5)
    vw = make_camera_set([(2.5, 1.5, 1.0), (-1.0, 3.0, -0.5)], [(0.1, 0.0, 0.05)] * 2, 96, 72, 50.0)
    pr = ora.project(sc, vw, ora.default_params(dilation=0.0))
    for v in range(2):
        for i in range(n):
            mu = sc.mean[:, i].astype(np.float64)
            h = 1e-6
            Jn = np.zeros((2, 3))
            for k in range(3):
                e = np.zeros(3); e[k] = h
                Jn[:, k] = (_pixel_map(vw, v, mu + e) - _pixel_map(vw, v, mu - e)) / (2 * h)
            qq = sc.quat[:, i].astype(np.float64)
            R = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()  # scipy is (x,y,z,w)
            S = np.diag(np.exp(2 * sc.log_scale[:, i].astype(np.float64)))
            Sig = R @ S @ R.T
            ref = Jn @ Sig @ Jn.T
            got = pr["cov"][v, i]
            assert np.allclose(got, [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=2e-6, atol=1e-9)
            assert np.allclose(pr["mean2d"][v, i], _pixel_map(vw, v, mu), atol=1e-9)


def test_projection_quaternion_sign_and_norm_invariance(ora):
    rng = np.random.default_rng(3)
    means = rng.uniform(-0.5, 0.5, (5, 3))
    ls = rng.normal(-3, 0.5, (5, 3))
    q = rng.standard_normal((5, 4))
    vw = synth.make_tiny_views()
    a = ora.project(make_explicit_scene(means, ls, q, 0.5), vw)
    b = ora.project(make_explicit_scene(means, ls, -2.0 * q, 0.5), vw)
    assert np.allclose(a["cov"], b["cov"], rtol=1e-6)


def test_near_plane_culls(ora):
    sc = make_explicit_scene([(0.0, 0, 0), (-3.9, 0, 0), (-4.5, 0, 0)], [-3.0] * 3, ID_Q, 0.5)
    vw = _axis_camera()
    pr = ora.project(sc, vw, ora.default_params(z_near=0.2))
    assert pr["present"][0].tolist() == [True, False, False]


# --------------------------------------------------------------------------
# Kernel, cutoff and compositing.
def _single_gaussian_nocolor(ora, sig_px_target=2.0, alpha=0.7, W=31):
    f = _focal(W, 60.0)
    dist = 4.0
    sig3 = sig_px_target * dist / f
    sc = make_explicit_scene([(0.0, 0.0, 0.0)], [math.log(sig3)] * 3, ID_Q, alpha)
    vw = _axis_camera(W, W, 60.0, dist)
    return sc, vw


def test_single_gaussian_kernel_closed_form(ora):
    """Alone on every ray it covers: A = rho = alpha exp(-d^2/2) inside the
    r-ellipse (boundary included), 0 outside; its sensitivity is exactly 1."""
    alpha = 0.7
    sc, vw = _single_gaussian_nocolor(ora, 2.0, alpha)
    W = int(vw.size[0, 0])
    prm = ora.default_params(query_mode=1, dilation=0.3)
    r = ora.sensitivity(sc, vw, prm)
    pr = ora.project(sc, vw, prm)
    var = pr["cov"][0, 0, 0]
    assert abs(pr["cov"][0, 0, 1]) < 1e-12
    A = r["A"].reshape(W, W)
    ys, xs = np.mgrid[0:W, 0:W]
    d2 = ((xs + 0.5 - W / 2) ** 2 + (ys + 0.5 - W / 2) ** 2) / var
    inside = d2 <= 9.0 * (1 - 1e-9)
    outside = d2 > 9.0 * (1 + 1e-9)
    a32 = float(np.float32(alpha))
    assert np.allclose(A[inside], a32 * np.exp(-0.5 * d2[inside]), rtol=1e-12)
    assert np.all(A[outside] == 0.0)
    assert r["s"][0] == pytest.approx(1.0, abs=1e-15)


def _axis_stack(alphas, colours, depths, W=31):
    """Gaussians on the optical axis (they project onto the central pixel
    centre), at the given distances from the camera."""
    n = len(alphas)
    means = [(d - 4.0, 0.0, 0.0) for d in depths]
    sc = make_explicit_scene(means, [math.log(0.01)] * 3, ID_Q, alphas, colours)
    return sc, _axis_camera(W, W, 60.0, 4.0)


def _central_ray_mask(vw):
    W, H = int(vw.size[0, 0]), int(vw.size[0, 1])
    keep = np.zeros(vw.n_rays, bool)
    keep[(H // 2) * W + W // 2] = True
    return pack_bits(keep)


def test_telescoping_and_two_gaussian_closed_form(ora):
    """On the central ray k = 1, so rho_j = alpha_j.  Front-to-back compositing
    gives A = sum_j c_j a_j prod_{k<j}(1 - a_k); with colour 1 this telescopes
    to 1 - prod_j (1 - a_j); and the shares of a single ray sum to 1."""
    al = np.array([0.3, 0.55, 0.8, 0.25], np.float32).astype(np.float64)
    col = np.array([[0.2, 0.3, 0.1], [0.9, 0.1, 0.4], [0.5, 0.5, 0.5], [0.05, 0.6, 0.7]])
    depths = [3.5, 2.0, 4.2, 3.0]            # front-to-back order: 1, 3, 0, 2
    sc, vw = _axis_stack(al, col, depths)
    mask = _central_ray_mask(vw)
    order = np.argsort(depths)
    # nocolor
    r = ora.sensitivity(sc, vw, ora.default_params(query_mode=1), mask)
    A = r["A"][mask_index(vw)]
    assert A == pytest.approx(1 - np.prod(1 - al), rel=1e-13)
    # colour: closed form with the float32-rounded SH degree-0 colours
    pr = ora.project(sc, vw)
    cbar = pr["cbar"][0]
    T, Aref, a = 1.0, 0.0, np.zeros(4)
    for j in order:
        a[j] = cbar[j] * al[j] * T
        Aref += a[j]
        T *= 1 - al[j]
    r = ora.sensitivity(sc, vw, ora.default_params(query_mode=0), mask)
    assert r["A"][mask_index(vw)] == pytest.approx(Aref, rel=1e-13)
    assert np.allclose(r["s"], a / Aref, rtol=1e-12)
    assert r["s"].sum() == pytest.approx(1.0, rel=1e-13)
    # two Gaussians, equal colour: shares r1/(r1 + r2(1-r1)) and r2(1-r1)/(...)
    sc2, vw2 = _axis_stack(al[:2], [[0.4, 0.4, 0.4]] * 2, [2.0, 3.0])
    r2 = ora.sensitivity(sc2, vw2, ora.default_params(query_mode=0), _central_ray_mask(vw2))
    r1_, r2_ = al[0], al[1]
    den = r1_ + r2_ * (1 - r1_)
    assert np.allclose(r2["s"], [r1_ / den, r2_ * (1 - r1_) / den], rtol=1e-12)


def test_l2_closed_forms(ora):
    """L2 queries (Section 3.5): on the central ray (rho_j = alpha_j)
    A = sum_j (c_R^2 + c_G^2 + c_B^2)_j alpha_j^2 T_j^2; for n equal
    Gaussians of colour c this is the geometric series
    |c|^2 alpha^2 (1 - (1 - alpha)^(2n)) / (1 - (1 - alpha)^2)."""
    al = np.array([0.3, 0.55, 0.8, 0.25], np.float32).astype(np.float64)
    col = np.array([[0.2, 0.3, 0.1], [0.9, 0.1, 0.4], [0.5, 0.5, 0.5], [0.05, 0.6, 0.7]])
    depths = [3.5, 2.0, 4.2, 3.0]
    sc, vw = _axis_stack(al, col, depths)
    mask = _central_ray_mask(vw)
    rgb = ora.project(sc, vw)["rgb"][0]
    T, Aref, a = 1.0, 0.0, np.zeros(4)
    for j in np.argsort(depths):
        a[j] = (rgb[j] ** 2).sum() * al[j] ** 2 * T ** 2
        Aref += a[j]
        T *= 1 - al[j]
    r = ora.sensitivity(sc, vw, ora.default_params(query_mode=ora.QUERY_L2), mask)
    assert r["A"][mask_index(vw)] == pytest.approx(Aref, rel=1e-13)
    assert np.allclose(r["s"], a / Aref, rtol=1e-12)
    n, alpha = 5, float(np.float32(0.4))
    sc5, vw5 = _axis_stack([alpha] * n, [[0.3, 0.6, 0.2]] * n, [2.0 + 0.3 * k for k in range(n)])
    c2 = (ora.project(sc5, vw5)["rgb"][0, 0] ** 2).sum()
    r5 = ora.sensitivity(sc5, vw5, ora.default_params(query_mode=ora.QUERY_L2), _central_ray_mask(vw5))
    geo = c2 * alpha ** 2 * (1 - (1 - alpha) ** (2 * n)) / (1 - (1 - alpha) ** 2)
    assert r5["A"][mask_index(vw5)] == pytest.approx(geo, rel=1e-13)


def test_per_channel_queries(ora):
    """Per-channel queries (Algorithm 1: queries per camera, pixel and RGB
    channel): a Gaussian that is alone in its channel on a ray has share 1
    there however deep it sits, while its RGB-sum share is below 1; and since
    a pixel's RGB-sum share is a weighted mean (mediant) of its channel
    shares, s_channel >= s_rgbsum for every Gaussian."""
    sc, vw = _axis_stack([0.6, 0.5], [[1.0, -0.2, -0.2], [-0.2, -0.2, 0.8]], [2.0, 3.0])
    mask = _central_ray_mask(vw)
    ch = ora.sensitivity(sc, vw, ora.default_params(query_mode=ora.QUERY_CHANNEL), mask)
    assert np.allclose(ch["s"], 1.0, rtol=0, atol=1e-15)
    A = ch["A"][mask_index(vw)]
    rgb = ora.project(sc, vw)["rgb"][0]
    assert rgb[0, 1] == rgb[0, 2] == rgb[1, 0] == rgb[1, 1] == 0.0
    assert A == pytest.approx([rgb[0, 0] * 0.6, 0.0, rgb[1, 2] * 0.5 * 0.4], rel=1e-7)
    s0 = ora.sensitivity(sc, vw, ora.default_params(query_mode=0), mask)["s"]
    assert s0[1] < 0.5
    tsc, tvw, _, _ = synth.make_config("tiny")
    a = ora.sensitivity(tsc, tvw, ora.default_params(query_mode=0))["s"]
    b = ora.sensitivity(tsc, tvw, ora.default_params(query_mode=ora.QUERY_CHANNEL))["s"]
    assert np.all(b >= a * (1 - 1e-12))
    assert np.mean(b > a * (1 + 1e-6)) > 0.5
    with pytest.raises(ValueError):
        ora.sensitivity_agg(tsc, tvw, ora.AGG_TILE, ora.default_params(query_mode=ora.QUERY_CHANNEL))


def mask_index(vw):
    W, H = int(vw.size[0, 0]), int(vw.size[0, 1])
    return (H // 2) * W + W // 2


def test_isolation_construction_all_sensitivities_one(ora):
    """Theorem 1's construction: each query isolates one Gaussian, so every
    s_i = 1 and S = N."""
    N = 7
    ang = 2 * np.pi * np.arange(N) / N
    means = np.stack([20 * np.cos(ang), 20 * np.sin(ang), np.zeros(N)], axis=1)
    eyes = means + np.stack([2 * np.cos(ang), 2 * np.sin(ang), 0.3 * np.ones(N)], axis=1)
    sc = make_explicit_scene(means, [math.log(0.02)] * 3, ID_Q, 0.6,
                             np.random.default_rng(1).uniform(0.1, 1, (N, 3)))
    vw = make_camera_set(eyes, means, 16, 16, 40.0)
    r = ora.sensitivity(sc, vw)
    assert np.allclose(r["s"], 1.0, atol=1e-15)
    assert r["s"].sum() == pytest.approx(N)


def test_tiny_scene_bounds_and_single_ray_sum(ora):
    """s in [0,1]; 1 <= S <= min(|I+|, rays with A > 0); on one ray S = 1."""
    sc, vw, _, _ = synth.make_config("tiny")
    r = ora.sensitivity(sc, vw)
    s = r["s"]
    assert s.min() >= 0 and s.max() <= 1 + 1e-15
    S = s.sum()
    assert 1 <= S <= min((s > 0).sum(), r["rays_positive"]) + 1e-9
    # single-ray query sets: shares sum to one
    A_all = r["A"]
    for ray in np.flatnonzero(A_all > 0)[:: max(1, (A_all > 0).sum() // 7)][:7]:
        keep = np.zeros(vw.n_rays, bool)
        keep[ray] = True
        r1 = ora.sensitivity(sc, vw, None, pack_bits(keep))
        assert r1["s"].sum() == pytest.approx(1.0, rel=1e-12)
        assert r1["A"][ray] == pytest.approx(A_all[ray], rel=1e-15)


def test_equal_colour_equals_nocolor(ora):
    sc, vw, _, _ = synth.make_config("tiny")
    same = make_explicit_scene(sc.mean.T, sc.log_scale.T, sc.quat.T, sc.opacity, [[0.3, 0.2, 0.9]])
    a = ora.sensitivity(same, vw, ora.default_params(query_mode=0))["s"]
    b = ora.sensitivity(same, vw, ora.default_params(query_mode=1))["s"]
    assert np.allclose(a, b, rtol=1e-12, atol=1e-300)


def test_permutation_invariance(ora):
    sc, vw, _, _ = synth.make_config("tiny")
    perm = np.random.default_rng(5).permutation(sc.n)
    a = ora.sensitivity(sc, vw)
    b = ora.sensitivity(sc.subset(perm), vw)
    pr = ora.project(sc, vw)
    # permutation invariance holds where no two present Gaussians share an order key
    keys = pr["key"]
    tie = np.zeros(sc.n, bool)
    for v in range(vw.n_views):
        k = keys[v][pr["present"][v]]
        u, c = np.unique(k, return_counts=True)
        tie |= np.isin(keys[v], u[c > 1]) & pr["present"][v]
    assert tie.sum() < 5
    ok = ~tie
    assert np.array_equal(b["A"], a["A"]) or np.allclose(b["A"], a["A"], rtol=1e-12)
    assert np.allclose(b["s"][ok[perm]], a["s"][perm][ok[perm]], rtol=1e-12, atol=0)


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_rigid_motion_invariance(ora):
    """Moving scene and cameras by the same rigid motion changes nothing."""
    from scipy.spatial.transform import Rotation
    sc, vw, _, _ = synth.make_config("tiny")
    g = Rotation.from_rotvec([0.3, -0.5, 0.8])
    G = g.as_matrix()
    gq = g.as_quat()                      # x, y, z, w
    gq = np.array([gq[3], gq[0], gq[1], gq[2]])
    tr = np.array([0.25, -0.4, 0.1])
    means = (G @ sc.mean.astype(np.float64)).T + tr
    quats = np.stack([_quat_mul(gq, q) for q in sc.quat.T.astype(np.float64)])
    colours = (sc.sh[0].T.astype(np.float64) * synth.SH_C0) + 0.5
    moved = make_explicit_scene(means, sc.log_scale.T, quats, sc.opacity, colours)
    base = make_explicit_scene(sc.mean.T, sc.log_scale.T, sc.quat.T, sc.opacity, colours)
    w2c = []
    for v in range(vw.n_views):
        P = vw.world_to_cam[v].reshape(3, 4)
        R2 = P[:, :3] @ G.T
        t2 = P[:, 3] - R2 @ tr
        w2c.append(np.concatenate([R2, t2[:, None]], axis=1).reshape(12))
    vw2 = synth.Views(np.stack(w2c), vw.intrinsics.copy(), vw.size.copy())
    a = ora.sensitivity(base, vw)
    b = ora.sensitivity(moved, vw2)
    # float32 storage of the moved means perturbs positions by ~1e-7:
    # compare away from the cutoff and key ambiguities.
    ok = ~(a["flag"] | b["flag"])
    assert np.allclose(a["A"][ok], b["A"][ok], rtol=2e-5, atol=1e-9)
    big = a["s"] > 1e-3
    assert np.median(np.abs(a["s"][big] - b["s"][big]) / a["s"][big]) < 1e-5


def test_adding_views_never_lowers_sensitivity(ora):
    sc, vw, _, _ = synth.make_config("tiny")
    s2 = ora.sensitivity(sc, vw.subset([0, 1]))["s"]
    s4 = ora.sensitivity(sc, vw)["s"]
    assert np.all(s4 >= s2)


def _mp_ray_contributions(sc, vw, W, H, mode=0):
    """All (ray, Gaussian) pairs in 50-digit arithmetic, no bounding boxes, no
    sorting shortcuts: {(view, px, py): ([A_q], [(i, [a_q])])} over every
    ray, for the queries of `mode` (Section 3.5): one with c_R + c_G + c_B
    (0), with colour 1 (1), the L2 form sum_k c_k^2 rho^2 T^2 (2), or three
    with c_R, c_G, c_B (3)."""
    import mpmath as mp
    mp.mp.dps = 50
    n = sc.n
    out = {}
    for v in range(vw.n_views):
        P = [[mp.mpf(float(x)) for x in vw.world_to_cam[v][4 * k:4 * k + 4]] for k in range(3)]
        fx, fy, cx, cy = [mp.mpf(float(x)) for x in vw.intrinsics[v]]
        camc = [-(P[0][c] * P[0][3] + P[1][c] * P[1][3] + P[2][c] * P[2][3]) for c in range(3)]
        gs = []
        for i in range(n):
            mu = [mp.mpf(float(sc.mean[k, i])) for k in range(3)]
            p = [P[k][0] * mu[0] + P[k][1] * mu[1] + P[k][2] * mu[2] + P[k][3] for k in range(3)]
            x, y, z = p
            qw, qx, qy, qz = [mp.mpf(float(sc.quat[k, i])) for k in range(4)]
            nn = mp.sqrt(qw ** 2 + qx ** 2 + qy ** 2 + qz ** 2)
            qw, qx, qy, qz = qw / nn, qx / nn, qy / nn, qz / nn
            Rq = mp.matrix([[1 - 2 * (qy ** 2 + qz ** 2), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)],
                            [2 * (qx * qy + qw * qz), 1 - 2 * (qx ** 2 + qz ** 2), 2 * (qy * qz - qw * qx)],
                            [2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx ** 2 + qy ** 2)]])
            S = mp.diag([mp.e ** (2 * mp.mpf(float(sc.log_scale[k, i]))) for k in range(3)])
            Sig = Rq * S * Rq.T
            Rv = mp.matrix([[P[a][b] for b in range(3)] for a in range(3)])
            J = mp.matrix([[fx / z, 0, -fx * x / z ** 2], [0, fy / z, -fy * y / z ** 2]])
            C2 = J * Rv * Sig * Rv.T * J.T
            C2[0, 0] += mp.mpf("0.3"); C2[1, 1] += mp.mpf("0.3")
            inv = C2 ** -1
            m2 = (fx * x / z + cx, fy * y / z + cy)
            d = [mu[k] - camc[k] for k in range(3)]
            rgb = [max(mp.mpf(float(sc.sh[0, ch, i])) * mp.mpf(1) / (2 * mp.sqrt(mp.pi)) + mp.mpf("0.5"), 0)
                   for ch in range(3)]
            gs.append((np.float32(float(z)), i, inv, m2, mp.mpf(float(sc.opacity[i])), rgb))
        gs.sort(key=lambda t: (t[0], t[1]))
        for py in range(H):
            for px in range(W):
                u = (mp.mpf(px) + mp.mpf("0.5"), mp.mpf(py) + mp.mpf("0.5"))
                nq = 3 if mode == 3 else 1
                T, A, contrib = mp.mpf(1), [mp.mpf(0)] * nq, []
                for (_, i, inv, m2, al, rgb) in gs:
                    dx, dy = u[0] - m2[0], u[1] - m2[1]
                    d2 = inv[0, 0] * dx * dx + 2 * inv[0, 1] * dx * dy + inv[1, 1] * dy * dy
                    if d2 > 9:
                        continue
                    rho = al * mp.e ** (-d2 / 2)
                    if mode == 0:
                        a = [(rgb[0] + rgb[1] + rgb[2]) * rho * T]
                    elif mode == 1:
                        a = [rho * T]
                    elif mode == 2:
                        a = [sum(c * c * rho * rho * T * T for c in rgb)]
                    else:
                        a = [c * rho * T for c in rgb]
                    contrib.append((i, a))
                    A = [x + y for x, y in zip(A, a)]
                    T *= 1 - rho
                out[(v, px, py)] = (A, contrib)
    return out


def _bruteforce_scene(n, W, H, seed):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-0.15, 0.15, (n, 3))
    ls = rng.normal(-2.6, 0.2, (n, 3))
    q = rng.standard_normal((n, 4))
    op = rng.uniform(0.2, 0.9, n)
    col = rng.uniform(0, 1, (n, 3))
    sc = make_explicit_scene(means, ls, q, op, col)
    vw = make_camera_set([(2.0, 0.5, 0.4), (-0.3, -2.0, 0.6)], [(0, 0, 0)] * 2, W, H, 40.0)
    return sc, vw


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_bruteforce_mpmath_tiny(ora, mode):
    """The oracle's per-ray sensitivities and query objectives agree with
    50-digit brute force to ~1e-13 for every query mode: RGB sum, nocolor,
    L2 and per channel (Section 3.5; Algorithm 1's channel queries)."""
    import mpmath as mp
    n, W, H = 6, 10, 8
    sc, vw = _bruteforce_scene(n, W, H, 11)
    r = ora.sensitivity(sc, vw, ora.default_params(dilation=0.3, query_mode=mode))
    rays = _mp_ray_contributions(sc, vw, W, H, mode)
    s_ref = [mp.mpf(0)] * n
    for (A, contrib) in rays.values():
        for q, Aq in enumerate(A):
            if Aq > 0:
                for i, a in contrib:
                    s_ref[i] = max(s_ref[i], a[q] / Aq)
    ref = np.array([float(x) for x in s_ref])
    assert (ref > 0).sum() >= 4
    assert np.allclose(r["s"], ref, rtol=1e-12, atol=1e-300)
    A_ref = np.array([[float(x) for x in rays[(v, px, py)][0]]
                      for v in range(vw.n_views) for py in range(H) for px in range(W)])
    A_got = r["A"].reshape(A_ref.shape)
    assert np.allclose(A_got, A_ref, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("mode", [0, 2])
def test_bruteforce_mpmath_aggregated(ora, mode):
    """Per-tile (16x16, ragged at the edges), per-image and per-scene
    sensitivities (Section 3.5): a_i and A summed over each query's rays in
    50-digit arithmetic, then the maximum over queries of their ratio (for
    the L1 and the L2 contributions)."""
    import mpmath as mp
    n, W, H = 6, 20, 18              # 2 x 2 tiles per view, the right and bottom ones ragged
    sc, vw = _bruteforce_scene(n, W, H, 12)
    rays = {k: (A[0], [(i, a[0]) for i, a in c]) for k, (A, c) in _mp_ray_contributions(sc, vw, W, H, mode).items()}
    keys = {1: lambda v, px, py: (v, px // 16, py // 16), 2: lambda v, px, py: v, 3: lambda v, px, py: 0}
    for level in (1, 2, 3):
        num, den = {}, {}
        for (v, px, py), (A, contrib) in rays.items():
            k = keys[level](v, px, py)
            den[k] = den.get(k, mp.mpf(0)) + A
            for i, a in contrib:
                num[(k, i)] = num.get((k, i), mp.mpf(0)) + a
        s_ref = [mp.mpf(0)] * n
        for (k, i), a in num.items():
            if den[k] > 0:
                s_ref[i] = max(s_ref[i], a / den[k])
        ref = np.array([float(x) for x in s_ref])
        got = ora.sensitivity_agg(sc, vw, level, ora.default_params(dilation=0.3, query_mode=mode))
        assert (ref > 0).sum() >= 4, level
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-300), (level, got, ref)


def test_aggregated_invariants(ora):
    """Per-scene S = 1 (the contributions of all Gaussians to a query sum to
    its objective); coarser queries average finer ones with weights A, so
    s_scene <= s_image <= s_tile <= s_ray elementwise; 1 <= S <= number of
    queries with A > 0."""
    for sc, vw in ((make_tiny_scene(2000, 0), make_tiny_views()),
                   (make_cluster_scene(6000, 7, 3), make_orbit_views(3, 17, 200, 136))):
        r = ora.sensitivity(sc, vw)
        s = [r["s"]] + [ora.sensitivity_agg(sc, vw, L) for L in (1, 2, 3)]
        assert abs(s[3].sum() - 1.0) < 1e-12
        for fine, coarse in zip(s[:-1], s[1:]):
            assert np.all(coarse <= fine * (1 + 1e-12) + 1e-300)
        A = r["A"]
        n_tiles_pos, n_views_pos, base = 0, 0, 0
        for v in range(vw.n_views):
            W, H = vw.size[v]
            img = A[base:base + W * H].reshape(H, W)
            base += W * H
            n_views_pos += img.sum() > 0
            for ty in range(0, H, 16):
                for tx in range(0, W, 16):
                    n_tiles_pos += img[ty:ty + 16, tx:tx + 16].sum() > 0
        assert 1.0 - 1e-12 <= s[2].sum() <= n_views_pos
        assert 1.0 - 1e-12 <= s[1].sum() <= n_tiles_pos


# --------------------------------------------------------------------------
# Sampler (Algorithm 1 steps 3-5; proof of Theorem 2).
def test_sampler_bookkeeping_and_zero_support(ora):
    rng = np.random.default_rng(2)
    s = rng.uniform(0, 1, 1000).astype(np.float32)
    s[::7] = 0
    r = ora.sample(s, 5000, 123)
    assert r["status"] == 0
    assert r["counts"].sum() == 5000
    assert r["support"] == (r["counts"] > 0).sum() <= 5000
    assert np.all(r["counts"][s == 0] == 0)
    assert np.all((r["weights"] > 0) == (r["counts"] > 0))
    q = np.ceil(s.astype(np.float64) * 2.0 ** 40)
    assert r["Q"] == int(q.sum())
    bad = ora.sample(np.zeros(10, np.float32), 5, 0)
    assert bad["status"] == 4 and bad["support"] == 0
    # a sensitivity is a largest share, so it lies in [0, 1] up to the float32
    # rounding of the share; anything past 1 + 2^-10 could let Q overflow 64
    # bits and is rejected
    for v in (np.float32(1.001), np.float32(2.0 ** 30), np.nan, np.inf, np.float32(-1e-30)):
        x = s.copy()
        x[5] = v
        r = ora.sample(x, 10, 0)
        assert r["status"] == 5 and r["support"] == 0 and not r["counts"].any() and not r["weights"].any()
    for v in (np.nextafter(np.float32(1), np.float32(2)), np.float32(1 + 2.0 ** -10)):
        x = s.copy()
        x[5] = v
        r = ora.sample(x, 10, 0)
        assert r["status"] == 0 and r["Q"] == int(np.ceil(np.asarray(x, np.float64) * 2.0 ** 40).sum())
    ones = np.ones(4096, np.float32)
    r = ora.sample(ones, 100, 0)
    assert r["status"] == 0 and r["Q"] == 4096 * 2 ** 40


def test_sampler_draws_match_bigint_definition(ora):
    """Targets floor(u Q / 2^128) with Python integers and a sorted search."""
    rng = np.random.default_rng(4)
    s = rng.uniform(0, 1, 257).astype(np.float32)
    s[3] = 0
    m, seed = 300, 0x1234_5678_9ABC_DEF0
    q = [int(math.ceil(float(x) * 2.0 ** 40)) for x in s]
    C = np.cumsum(np.array(q, dtype=object))
    Q = int(C[-1])
    counts = np.zeros(len(s), np.int64)
    for t in range(m):
        x = ora.philox4x32_10([t & 0xFFFFFFFF, t >> 32, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        u = int(x[0]) | (int(x[1]) << 32) | (int(x[2]) << 64) | (int(x[3]) << 96)
        target = (u * Q) >> 128
        i = next(k for k in range(len(s)) if C[k] > target)
        counts[i] += 1
    r = ora.sample(s, m, seed)
    assert np.array_equal(r["counts"].astype(np.int64), counts)
    nz = counts > 0
    w = np.array([counts[i] * float(Q) / (m * float(q[i])) if nz[i] else 0.0 for i in range(len(s))])
    assert np.array_equal(r["weights"], w)


def test_sampler_goodness_of_fit(ora):
    from scipy.stats import chisquare
    s = np.array([0.05, 0.1, 0.2, 0.4, 0.8, 1.0, 0.0, 0.3], np.float32)
    m = 200_000
    r = ora.sample(s, m, 99)
    p = np.ceil(s.astype(np.float64) * 2.0 ** 40)
    p /= p.sum()
    nz = p > 0
    stat = chisquare(r["counts"][nz], m * p[nz])
    assert stat.pvalue > 1e-4


def test_unbiased_fixed_objective_over_seeds(ora):
    """E[A^th_w(q)] = A(q) for every ray (proof of Theorem 2): the per-ray
    means over K seeds sit within a few standard errors of A."""
    sc, vw, _, _ = synth.make_config("tiny")
    vw1 = vw.subset([0])
    r = ora.sensitivity(sc, vw1)
    s = r["s"].astype(np.float32)
    K, m = 64, 150
    rays = np.flatnonzero(r["A"] > 0)
    acc = np.zeros((K, rays.size))
    for k in range(K):
        w = ora.sample(s, m, 1000 + k)["weights"]
        acc[k] = ora.objective(sc, vw1, w)["A_fixed"][rays]
    A = r["A"][rays]
    mean = acc.mean(0)
    se = acc.std(0, ddof=1) / math.sqrt(K)
    z = (mean - A) / np.maximum(se, 1e-30)
    assert np.mean(np.abs(z) < 3) > 0.97
    assert abs(np.mean(z)) < 0.2


def test_zero_variance_when_sensitivity_is_proportional_to_contribution(ora):
    """With one query and s_i = a_i / A, every draw gives A^th_w = A."""
    sc, vw, _, _ = synth.make_config("tiny")
    vw1 = vw.subset([0])
    r = ora.sensitivity(sc, vw1)
    ray = int(np.argmax(r["A"]))
    keep = np.zeros(vw1.n_rays, bool)
    keep[ray] = True
    mask = pack_bits(keep)
    r1 = ora.sensitivity(sc, vw1, None, mask)
    s = r1["s"].astype(np.float32)
    for seed in range(3):
        w = ora.sample(s, 40, seed)["weights"]
        ob = ora.objective(sc, vw1, w, None, mask)
        assert ob["A_fixed"][ray] == pytest.approx(ob["A"][ray], rel=1e-5)


def test_per_scene_sensitivities_give_zero_variance(ora):
    """With per-scene sensitivities (Section 3.5) the sampling probabilities
    are a_i(Q) / A(Q) for the single query Q holding every ray, so every draw
    reproduces the scene's total objective: sum over all rays of A^th_w equals
    sum of A, up to the 2^-40 quantisation of the probabilities; per-ray
    sensitivities do not have this property."""
    sc, vw, _, _ = synth.make_config("tiny")
    s_scene = ora.sensitivity_agg(sc, vw, ora.AGG_SCENE).astype(np.float32)
    s_ray = ora.sensitivity(sc, vw)["s"].astype(np.float32)
    errs = []
    for seed in range(4):
        for s in (s_scene, s_ray):
            w = ora.sample(s, 200, seed)["weights"]
            pv = ora.objective(sc, vw, w)["view_sums"]
            errs.append(abs(pv[:, 1].sum() - pv[:, 0].sum()) / pv[:, 0].sum())
    assert max(errs[0::2]) < 1e-7, errs
    assert min(errs[1::2]) > 5e-4, errs


def test_theorem2_sample_size_failure_rate(ora):
    """At m >= 3S/eps^2 log(2|Q'|/delta), the fixed objective is an eps-coreset
    on every ray in (far) more than a 1 - delta fraction of seeds."""
    sc, vw, _, _ = synth.make_config("tiny")
    vw1 = vw.subset([2])
    r = ora.sensitivity(sc, vw1)
    S = r["s"].sum()
    Qn = int((r["A"] > 0).sum())
    eps, delta = 0.5, 0.2
    m = int(math.ceil(3 * S / eps ** 2 * math.log(2 * Qn / delta)))
    fails = 0
    runs = 5
    on = r["A"] > 0
    for k in range(runs):
        w = ora.sample(r["s"].astype(np.float32), m, 77 + k)["weights"]
        ob = ora.objective(sc, vw1, w)
        err = np.abs(ob["A_fixed"][on] - r["A"][on]) / r["A"][on]
        fails += err.max() > eps
    assert fails <= math.floor(delta * runs)


# --------------------------------------------------------------------------
# Objectives (Section 3; Definition 2, Assumption 1, transfer lemma).
def test_unit_weights_reproduce_the_full_render(ora):
    sc, vw, _, _ = synth.make_config("tiny")
    ob = ora.objective(sc, vw, np.ones(sc.n))
    r = ora.sensitivity(sc, vw)
    assert np.allclose(ob["A"], r["A"], rtol=1e-15, atol=0)
    assert np.allclose(ob["A_fixed"], ob["A"], rtol=1e-15, atol=0)
    assert np.allclose(ob["A_true"], ob["A"], rtol=1e-15, atol=0)
    assert ob["gamma"] == 0.0 and ob["n_invalid"] == 0


def test_true_render_closed_form_two_gaussians(ora):
    al = np.array([0.4, 0.5], np.float32).astype(np.float64)
    sc, vw = _axis_stack(al, [[0.2, 0.2, 0.2]] * 2, [2.0, 3.0])
    mask = _central_ray_mask(vw)
    w = np.array([1.5, 0.8])
    ob = ora.objective(sc, vw, w, ora.default_params(query_mode=1), mask)
    ray = mask_index(vw)
    assert ob["A_true"][ray] == pytest.approx(w[0] * al[0] + w[1] * al[1] * (1 - w[0] * al[0]), rel=1e-13)
    assert ob["A_fixed"][ray] == pytest.approx(w[0] * al[0] + w[1] * al[1] * (1 - al[0]), rel=1e-13)
    gap = abs(math.log(1 - al[0]) - math.log(1 - w[0] * al[0]))
    assert ob["gamma"] == pytest.approx(gap, rel=1e-12)
    # an invalid weight (w rho >= 1) is counted
    ob2 = ora.objective(sc, vw, np.array([3.0, 1.0]), ora.default_params(query_mode=1), mask)
    assert ob2["n_invalid"] == 1


def test_transfer_sandwich(ora):
    """e^-gamma A^th_w <= A_w <= e^gamma A^th_w on valid rays (transfer lemma)."""
    sc, vw, m, seed = synth.make_config("tiny")
    r = ora.sensitivity(sc, vw)
    w = ora.sample(r["s"].astype(np.float32), 1500, seed)["weights"]
    ob = ora.objective(sc, vw, w)
    g = ob["gamma"]
    on = ob["A"] > 0
    lo = np.exp(-g) * ob["A_fixed"][on] * (1 - 1e-12)
    hi = np.exp(g) * ob["A_fixed"][on] * (1 + 1e-12)
    At = ob["A_true"][on]
    if ob["n_invalid"] == 0:
        assert np.all(At >= lo - 1e-300) and np.all(At <= hi + 1e-300)
    assert g > 0


def test_eps_rendered_closed_forms(ora):
    """Theorem 3's eps_r: gamma = 0 gives eps_c back; eps_c = 0 gives
    e^gamma - 1 (the upper branch wins for gamma > 0); it grows with both."""
    e = np.linspace(0, 0.9, 10)
    assert np.allclose(ora.eps_rendered(0.0, e), e, atol=1e-15)
    g = np.linspace(0, 3, 13)
    assert np.allclose(ora.eps_rendered(g, 0.0), np.expm1(g), rtol=1e-14, atol=1e-15)
    assert abs(ora.eps_rendered(np.log(2.0), 0.5) - max(1 - 0.5 * 0.5, 2 * 1.5 - 1)) < 1e-15
    G, E = np.meshgrid(np.linspace(0, 2, 9), np.linspace(0, 0.9, 9))
    r = ora.eps_rendered(G, E)
    assert np.all(np.diff(r, axis=0) > 0) and np.all(np.diff(r, axis=1) >= 0)
    assert np.all(r >= E - 1e-15)


def test_rendered_bound_holds_for_valid_weights(ora):
    """Theorem 3's deterministic step: for any valid w (every w rho < 1) with
    measured gamma and eps_c = max_q |A^th_w - A| / A, every ray satisfies
    |A_w - A| <= eps_r A.  Weights of 0.6-1.4 on a scene with alpha <= 0.6
    keep w rho < 1."""
    sc, vw, _, _ = synth.make_config("tiny")
    sc.opacity = np.ascontiguousarray(np.minimum(sc.opacity, 0.6).astype(np.float32))
    rng = np.random.default_rng(9)
    w = rng.uniform(0.6, 1.4, sc.n)
    ob = ora.objective(sc, vw, w)
    assert ob["n_invalid"] == 0
    on = ob["A"] > 0
    A, Af, At = ob["A"][on], ob["A_fixed"][on], ob["A_true"][on]
    eps_c = float(np.max(np.abs(Af - A) / A))
    g = ob["gamma"]
    assert g > 0 and 0 < eps_c < 1
    eps_r = float(ora.eps_rendered(g, eps_c))
    err = np.abs(At - A) / A
    assert np.all(err <= eps_r * (1 + 1e-9)), (err.max(), eps_r)
    # the reduced render really differs from the fixed relaxation here
    assert np.max(np.abs(At - Af) / Af) > 1e-2


# --------------------------------------------------------------------------
# Targeted pins for boundaries that random inputs rarely reach.
def test_cutoff_boundary_over_many_footprints(ora):
    """Across footprint sizes, exactly the pixels with d^2 <= r^2 are lit."""
    lit_band = 0
    for sig_px in (1.1, 1.37, 1.66, 2.0, 2.41, 2.93, 3.3):
        sc, vw = _single_gaussian_nocolor(ora, sig_px, 0.6, 33)
        W = int(vw.size[0, 0])
        prm = ora.default_params(query_mode=1)
        A = ora.sensitivity(sc, vw, prm)["A"].reshape(W, W)
        var = ora.project(sc, vw, prm)["cov"][0, 0, 0]
        ys, xs = np.mgrid[0:W, 0:W]
        d2 = ((xs + 0.5 - W / 2) ** 2 + (ys + 0.5 - W / 2) ** 2) / var
        clear = np.abs(d2 - 9.0) > 1e-9
        assert np.array_equal((A > 0)[clear], (d2 <= 9.0)[clear])
        lit_band += int(((d2 > 9.0) & (d2 < 9.2)).sum())
    assert lit_band > 0     # some pixels sit just outside the cutoff


def test_equal_keys_ordered_by_index(ora):
    """Two Gaussians at the same depth: the lower index is in front."""
    al = np.array([0.3, 0.7], np.float32).astype(np.float64)
    sc, vw = _axis_stack(al, [[0.5, 0.5, 0.5]] * 2, [2.5, 2.5])
    r = ora.sensitivity(sc, vw, ora.default_params(query_mode=1), _central_ray_mask(vw))
    A = 1 - (1 - al[0]) * (1 - al[1])
    assert np.allclose(r["s"], [al[0] / A, al[1] * (1 - al[0]) / A], rtol=1e-12)


def test_draw_target_exact_on_crafted_values(ora):
    rng = np.random.default_rng(9)
    cases = [(2 ** 128 - 1, 3), (2 ** 128 - 1, 2 ** 64 - 1), (2 ** 64 - 1, 2 ** 64 - 1),
             ((2 ** 64 - 1) << 64, 7), (0, 12345), (1 << 127, 5), ((1 << 64) - 2, 3)]
    for _ in range(2000):
        u = int(rng.integers(0, 2 ** 63)) << 65 | int(rng.integers(0, 2 ** 63)) << 2 | int(rng.integers(0, 4))
        Q = int(rng.integers(1, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        cases.append((u & (2 ** 128 - 1), Q))
    # values whose low-part carry decides the result
    for Q in (3, 5, 7, 2 ** 40 + 1):
        for k in range(1, 50):
            u_hi = ((k << 64) // Q) & (2 ** 64 - 1)
            for u_lo in (2 ** 64 - 1, 2 ** 64 - 2 ** 20, 2 ** 63):
                cases.append(((u_hi << 64) | u_lo, Q))
    for u, Q in cases:
        words = [(u >> (32 * j)) & 0xFFFFFFFF for j in range(4)]
        assert ora.draw_target(words, Q) == (u * Q) >> 128


def test_sampler_small_integer_cdf_boundaries(ora):
    """Sensitivities k 2^-40 give q_i = k exactly; with Q small every target
    hits prefix-sum boundaries, so the search must be 'first C_i > target'."""
    k = np.array([1, 2, 0, 3, 1, 4], np.float64)
    s = (k * 2.0 ** -40).astype(np.float32)
    assert np.array_equal(np.ceil(s.astype(np.float64) * 2.0 ** 40), k)
    C = np.cumsum(k).astype(np.int64)
    Q = int(C[-1])
    m, seed = 4000, 5
    counts = np.zeros(k.size, np.int64)
    for t in range(m):
        x = ora.philox4x32_10([t, 0, 0, 0], [seed, 0])
        u = int(x[0]) | (int(x[1]) << 32) | (int(x[2]) << 64) | (int(x[3]) << 96)
        counts[int(np.searchsorted(C, (u * Q) >> 128, side="right"))] += 1
    r = ora.sample(s, m, seed)
    assert np.array_equal(r["counts"].astype(np.int64), counts)
    assert r["counts"][2] == 0


def test_view_dependent_colour_uses_camera_centre(ora):
    """Degree-1 colour: c = 1/2 + sum_k f_k Y_k(d) with d the unit direction
    from the camera centre (placed by the test) to the mean."""
    eye = np.array([0.7, -3.1, 1.3])
    mean = np.array([0.2, 0.1, -0.3])
    sh = np.zeros((1, 4, 3))
    sh[0, 1:, :] = [[0.3, -0.2, 0.1], [0.5, 0.4, -0.6], [-0.7, 0.2, 0.3]]
    sc = make_explicit_scene([mean], [-3.0] * 3, ID_Q, 0.5, sh=sh, sh_degree=1)
    vw = make_camera_set([eye], [(0.0, 0.0, 0.0)], 32, 32, 60.0)
    pr = ora.project(sc, vw)
    d = (mean.astype(np.float32).astype(np.float64) - eye)
    d /= np.linalg.norm(d)
    c1 = math.sqrt(3 / (4 * math.pi))
    Y = np.array([c1 * d[1], c1 * d[2], c1 * d[0]])
    f = sh[0, 1:, :].astype(np.float32).astype(np.float64)
    expect = np.maximum(0.5 + Y @ f, 0)
    assert np.allclose(pr["rgb"][0, 0], expect, rtol=1e-9)
