"""Pins of the oracle's rounding scale of the true reduced render
(objective_true_scale), which sets the FP32 tolerance of A_w in the GPU
parity test.

E bounds the first-order change of A_w when every rho carries a relative
error of at most d: |dA_w| <= d E.  The pins check it against the oracle's
own objective (a separate routine) under an exact perturbation of the
opacities (rho is proportional to alpha), and against the one-pair case,
where the bound is attained.
"""
import math

import numpy as np
import pytest

from synth import make_camera_set, make_cluster_scene, make_explicit_scene, make_orbit_views, pack_bits

ID_Q = (1.0, 0.0, 0.0, 0.0)


def _axis_stack(alphas, colours, depths, W=31):
    means = [(d - 4.0, 0.0, 0.0) for d in depths]
    sc = make_explicit_scene(means, [math.log(0.01)] * 3, ID_Q, alphas, colours)
    return sc, make_camera_set([(-4.0, 0.0, 0.0)], [(0.0, 0.0, 0.0)], W, W, 60.0)


def _scaled(sc, factor):
    """The scene with every opacity times `factor` (float32), and the actual
    relative change of each opacity."""
    op = (sc.opacity.astype(np.float64) * factor).astype(np.float32)
    d = 1.0 - op.astype(np.float64) / sc.opacity.astype(np.float64)
    out = type(sc)(sc.mean, sc.log_scale, sc.quat, op, sc.sh, sc.sh_degree)
    return out, d


def _delta_true(ora, sc, vw, w, factor, mask=None, prm=None):
    base = ora.objective(sc, vw, w, prm, ray_mask=mask)["A_true"]
    sc2, d = _scaled(sc, factor)
    pert = ora.objective(sc2, vw, w, prm, ray_mask=mask)["A_true"]
    return np.abs(pert - base), float(np.max(np.abs(d))), base


def test_one_pair_per_ray_scale_is_the_value(ora):
    """With one Gaussian every ray holds one pair: no earlier factor, so E is
    |A_w| itself (and the first-order change is exactly d |A_w|)."""
    sc, vw = _axis_stack([0.7], [[0.3, 0.6, 0.2]], [4.0])
    w = np.array([3.0])
    E = ora.objective_true_scale(sc, vw, w)
    At = ora.objective(sc, vw, w)["A_true"]
    assert np.count_nonzero(At) >= 5
    assert np.allclose(E, np.abs(At), rtol=1e-13, atol=0.0)
    dA, d, _ = _delta_true(ora, sc, vw, w, 1.0 - 1e-4)
    on = E > 0
    assert np.allclose(dA[on], d * E[on], rtol=1e-3)


def test_two_pairs_near_an_invalid_factor(ora):
    """Central ray of two Gaussians on the axis (rho = alpha there), the
    first nearly black and with w rho = 0.9: the second pair's T_w = 1 - 0.9
    moves by nine times the relative error of rho, so A_w moves by about
    8 d A_w against the bound's 20 d A_w.  The bound holds and is within a
    factor three of the actual change."""
    sc, vw = _axis_stack([0.6, 0.5], [[0.001, 0.001, 0.001], [0.7, 0.2, 0.1]], [2.0, 3.0])
    W = int(vw.size[0, 0])
    centre = (W // 2) * W + W // 2
    w = np.array([0.9 / float(np.float32(0.6)), 1.5])
    keep = np.zeros(vw.n_rays, bool)
    keep[centre] = True
    mask = pack_bits(keep)
    E = ora.objective_true_scale(sc, vw, w, ray_mask=mask)
    dA, d, base = _delta_true(ora, sc, vw, w, 1.0 - 1e-5, mask)
    assert base[centre] > 0
    assert dA[centre] <= d * E[centre] * (1 + 1e-3)
    assert dA[centre] >= 0.33 * d * E[centre]
    assert E[centre] > 5 * abs(base[centre])      # the factor near 0 dominates


@pytest.mark.parametrize("mode", [0, 2])
def test_scale_bounds_the_change_on_a_sampled_coreset(ora, mode):
    """A cluster scene with coreset weights near n/m = 10 (many pairs with
    w rho >= 1): on every scored ray the change of A_w under a uniform
    relative perturbation of the opacities stays within d E (RGB-sum and L2
    objectives)."""
    sc = make_cluster_scene(600, 31, 2)
    vw = make_orbit_views(2, 32, 40, 32)
    prm = ora.default_params(query_mode=mode)
    s = ora.sensitivity(sc, vw, prm)["s"]
    w = ora.sample(s, 60, 5)["weights"]
    E = ora.objective_true_scale(sc, vw, w, prm)
    ob = ora.objective(sc, vw, w, prm)
    assert ob["n_invalid"] > 0
    dA, d, base = _delta_true(ora, sc, vw, w, 1.0 - 1e-6, prm=prm)
    on = E > 0
    assert on.sum() > 500
    fin = on & np.isfinite(E)
    assert np.all(dA[fin] <= d * E[fin] * (1 + 1e-2) + 1e-300)
    assert np.all(E[on] >= np.abs(base[on]) * (1 - 1e-12))
    ratio = dA[fin] / (d * E[fin])
    assert ratio.max() > 0.5                        # attained on some rays
