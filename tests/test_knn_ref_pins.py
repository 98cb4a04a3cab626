"""Pins of the oracle's neighbourhood features for the learned proposal
(brute-force k nearest means, float32 squared distances, ties by index, and
the 64 features built from them), each against something other than the
oracle itself: closed forms on a cubic lattice, scipy's k-d tree, and
identities of the attribute columns."""
import math

import numpy as np
import pytest

import synth

H = 0.125   # lattice spacing: squared distances h^2, 2 h^2, 3 h^2 are exact in float32


def _lattice(side=7):
    g = np.arange(side, dtype=np.float64) * H
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()]).astype(np.float32)
    return pts


def _lattice_scene(side=7, seed=0):
    pts = _lattice(side)
    n = pts.shape[1]
    rng = np.random.default_rng(seed)
    op = rng.uniform(0.05, 0.95, n).astype(np.float32)
    sc = synth.make_explicit_scene(pts.T, np.full((n, 3), -3.0), np.tile([1.0, 0, 0, 0], (n, 1)), op,
                                   colours=np.full((n, 3), 0.5))
    return sc, op


def test_lattice_neighbours_closed_form(ora):
    """On the cubic lattice an interior point's 16 nearest others are its 6
    face neighbours (distance h) and the 10 of its 12 edge neighbours
    (distance h sqrt 2) with the smallest indices: ties go by index."""
    side = 7
    sc, op = _lattice_scene(side)
    f, idx, d2 = ora.features(sc)
    lin = lambda i, j, k: (i * side + j) * side + k      # meshgrid 'ij' order
    for c in [(3, 3, 3), (2, 3, 4), (4, 2, 2)]:
        i = lin(*c)
        face = sorted(lin(c[0] + a, c[1] + b, c[2] + e) for a, b, e in
                      [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])
        edge = sorted(lin(c[0] + a, c[1] + b, c[2] + e)
                      for a in (-1, 0, 1) for b in (-1, 0, 1) for e in (-1, 0, 1)
                      if abs(a) + abs(b) + abs(e) == 2)
        want = face + edge[:10]
        assert idx[i].tolist() == want
        assert np.all(d2[i, :6] == np.float32(H * H)) and np.all(d2[i, 6:] == np.float32(2 * H * H))
        nb = op[want].astype(np.float64)
        d16 = math.sqrt(2.0) * H
        assert abs(f[i, 59] - math.log((6 * H + 10 * d16) / 16)) < 1e-12
        assert abs(f[i, 60] - math.log(d16)) < 1e-12
        assert abs(f[i, 61] - nb.mean()) < 1e-12
        assert f[i, 62] == nb.max()
        assert abs(f[i, 63] - math.log(nb.sum() / (4.0 / 3.0 * math.pi * d16 ** 3))) < 1e-12


def test_knn_matches_kdtree(ora):
    """Clustered means: neighbour distances equal scipy's k-d tree (float64)
    to float32 rounding; neighbour sets agree except where the float32
    distance of a swapped point ties the k-th distance within rounding."""
    from scipy.spatial import cKDTree
    sc = synth.make_cluster_scene(6000, 31, 0)
    mean = np.asarray(sc.mean, np.float32).reshape(3, -1)
    idx, d2 = ora.knn(mean)
    P = mean.T.astype(np.float64)
    dist, nb = cKDTree(P).query(P, k=17)
    dist, nb = dist[:, 1:], nb[:, 1:]
    got = np.sqrt(d2.astype(np.float64))
    assert np.all(np.abs(got - dist) <= 2e-6 * dist + 1e-9)
    differ = 0
    for i in range(P.shape[0]):
        a, b = set(idx[i].tolist()), set(nb[i].tolist())
        if a != b:
            differ += 1
            kth = dist[i, -1]
            for j in a ^ b:
                dj = np.linalg.norm(P[j] - P[i])
                assert abs(dj - kth) <= 2e-6 * kth, (i, j)
    assert differ <= 6


def test_small_scenes_and_missing_neighbours(ora):
    """Fewer than 17 points: missing neighbours are marked, features use the
    ones there are; one point alone gets the documented defaults."""
    rng = np.random.default_rng(5)
    for n in (1, 2, 5, 17):
        sc = synth.make_explicit_scene(rng.uniform(-1, 1, (n, 3)), np.full((n, 3), -3.0),
                                       np.tile([1.0, 0, 0, 0], (n, 1)), rng.uniform(0.1, 0.9, n),
                                       colours=np.full((n, 3), 0.5))
        f, idx, d2 = ora.features(sc)
        have = min(n - 1, 16)
        assert np.all(idx[:, :have] != np.uint32(0xFFFFFFFF))
        assert np.all(idx[:, have:] == np.uint32(0xFFFFFFFF)) and np.all(np.isinf(d2[:, have:]))
        assert not np.any(idx[:, :have] == np.arange(n)[:, None])       # never itself
        if n == 1:
            assert f[0, 59] == 0.0 and f[0, 60] == 0.0 and f[0, 61] == 0.0 and f[0, 62] == 0.0
            assert abs(f[0, 63] - math.log(1e-12 / (4.0 / 3.0 * math.pi))) < 1e-12
        else:
            P = np.asarray(sc.mean, np.float64).reshape(3, n).T
            D = np.linalg.norm(P[:, None] - P[None], axis=2)
            np.fill_diagonal(D, np.inf)
            assert np.allclose(np.sort(D, axis=1)[:, :have], np.sqrt(d2[:, :have].astype(np.float64)),
                               rtol=2e-6)


def test_attribute_columns(ora):
    """Columns 0-58 restate the attributes: mean and log-scale as given, a
    unit quaternion with w >= 0 that is +-the input direction, logit of the
    clamped opacity, and the SH planes with zeros past the degree."""
    sc = synth.make_cluster_scene(3000, 8, 1)
    n = sc.n
    q = np.asarray(sc.quat, np.float32).reshape(4, n).T.astype(np.float64)
    q[::5] *= -3.0          # sign and scale of the quaternion are irrelevant
    sc.quat = np.ascontiguousarray(q.T.astype(np.float32))
    f, _, _ = ora.features(sc)
    assert np.array_equal(f[:, 0:3], np.asarray(sc.mean, np.float32).reshape(3, n).T.astype(np.float64))
    assert np.array_equal(f[:, 3:6], np.asarray(sc.log_scale, np.float32).reshape(3, n).T.astype(np.float64))
    qq = f[:, 6:10]
    assert np.allclose(np.linalg.norm(qq, axis=1), 1.0, atol=1e-15) and np.all(qq[:, 0] >= 0)
    qin = np.asarray(sc.quat, np.float32).reshape(4, n).T.astype(np.float64)
    cosang = np.abs(np.sum(qq * qin, axis=1)) / np.linalg.norm(qin, axis=1)
    assert np.allclose(cosang, 1.0, atol=1e-12)
    a = np.clip(np.asarray(sc.opacity, np.float32), np.float32(1e-6), np.float32(1) - np.float32(1e-6))
    assert np.allclose(1.0 / (1.0 + np.exp(-f[:, 10])), a.astype(np.float64), rtol=1e-12, atol=0)
    sh = np.asarray(sc.sh, np.float32).reshape(-1, n)
    assert sh.shape[0] == 12
    assert np.array_equal(f[:, 11:23], sh.T.astype(np.float64))
    assert not f[:, 23:59].any()
