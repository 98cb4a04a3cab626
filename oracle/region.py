"""FP64 reference of the compact-region extension (Section 3.4: Assumption 2,
the rho-net definition and Theorem 4; appendix, compact-region extension
from representatives).

TEST INFRASTRUCTURE ONLY: used by the tests and never by the product
package; it shares no code with the HIP library.

A query is (camera pose, pixel).  On a region of poses around a
representative camera the distance between two queries of the same pixel is
the pose distance  d = |c - c'| + lam * angle(R R'^T)  (camera centres c,
world-to-camera rotations R, lam in length units per radian).  Given sampled
poses of the region:
  - a rho-net (Definition: every query within rho of a representative) is
    chosen greedily: the first pose, then repeatedly the pose farthest from
    the chosen ones, until every pose is within rho of one;
  - the Lipschitz constants of the full and reduced renders are estimated
    as the largest |A(q) - A(q')| / d(q, q') over pairs of sampled poses,
    per pixel, maximised over the pixels kept (Assumption 2, items ii-iii);
  - A_min is the smallest A over the kept pixels and sampled poses (item iv);
  - eps_0 is the largest |A - A_w| / A over the representatives;
  - Theorem 4:  eps_reg = eps_0 + ((1 + eps_0) L_full + L_w) rho / A_min.
"""
from __future__ import annotations

import numpy as np


def camera_centre(w2c):
    """c = -R^T t of a [12] row-major [R | t]."""
    M = np.asarray(w2c, np.float64).reshape(3, 4)
    return -M[:, :3].T @ M[:, 3]


def rotation_angle(Ra, Rb):
    """Angle of Ra Rb^T in [0, pi], from the sine of its skew part and the
    cosine of its trace (accurate for small and large angles alike)."""
    M = np.asarray(Ra, np.float64) @ np.asarray(Rb, np.float64).T
    s = 0.5 * np.linalg.norm([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    c = 0.5 * (np.trace(M) - 1.0)
    return float(np.arctan2(s, c))


def pose_distance(w2c_a, w2c_b, lam):
    Ra = np.asarray(w2c_a, np.float64).reshape(3, 4)[:, :3]
    Rb = np.asarray(w2c_b, np.float64).reshape(3, 4)[:, :3]
    return float(np.linalg.norm(camera_centre(w2c_a) - camera_centre(w2c_b)) + lam * rotation_angle(Ra, Rb))


def distance_matrix(w2c, lam):
    K = len(w2c)
    D = np.zeros((K, K))
    for i in range(K):
        for j in range(i + 1, K):
            D[i, j] = D[j, i] = pose_distance(w2c[i], w2c[j], lam)
    return D


def rho_net(D, rho):
    """Greedy representatives: returns (indices in the order chosen, the
    covering radius reached = max over poses of the distance to the nearest
    representative, which is <= rho)."""
    K = D.shape[0]
    net = [0]
    near = D[0].copy()
    while near.max() > rho:
        j = int(np.argmax(near))          # the first farthest pose
        net.append(j)
        near = np.minimum(near, D[j])
    return net, float(near.max())


def region_bound(A, Aw, D, net, keep):
    """A, Aw: [K][pixels] full and reduced renders at the sampled poses;
    D: [K][K] pose distances; net: representative indices; keep: [pixels]
    bools (pixels with A > 0 at every pose).  Returns a dict with L_full,
    L_w, A_min, eps_0, rho (covering radius of the net over the poses),
    eps_reg and the largest |A - A_w| / A over every sampled pose."""
    A = np.asarray(A, np.float64)[:, keep]
    Aw = np.asarray(Aw, np.float64)[:, keep]
    K = A.shape[0]
    L_full = L_w = 0.0
    for i in range(K):
        for j in range(i + 1, K):
            if D[i, j] > 0:
                L_full = max(L_full, float(np.max(np.abs(A[i] - A[j]))) / D[i, j])
                L_w = max(L_w, float(np.max(np.abs(Aw[i] - Aw[j]))) / D[i, j])
    A_min = float(A.min())
    err = np.abs(A - Aw) / A
    eps_0 = float(err[net].max())
    rho = float(np.min(D[:, net], axis=1).max())
    eps_reg = eps_0 + ((1.0 + eps_0) * L_full + L_w) * rho / A_min
    return {"L_full": L_full, "L_w": L_w, "A_min": A_min, "eps_0": eps_0, "rho": rho, "eps_reg": eps_reg,
            "max_err": float(err.max()), "err_per_pose": err.max(axis=1)}


def rho_for_target(eps_target, eps_0, L_full, L_w, A_min):
    """The corollary's cover radius: rho <= (eps_target - eps_0) A_min / ((1 + eps_0) L_full + L_w)."""
    return (eps_target - eps_0) * A_min / ((1.0 + eps_0) * L_full + L_w)
