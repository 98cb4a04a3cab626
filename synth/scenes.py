"""Seeded synthetic 3DGS scenes and pinhole camera sets.

The paper evaluates on real captured scenes (Mip-NeRF 360, Tanks & Temples,
Deep Blending; Section 4) that are not available here.  These generators stand
in for them with the shapes of the workloads the build is measured on:

* tiny scene: 2 000 Gaussians, uniform means in [-1,1]^3, log-scales
  N(-3.5, 0.5^2), uniform rotations, opacity sigmoid(N(0,1)), SH degree 0
  colours uniform in [0,1]; 4 views at 64x64 on a radius-3 sphere;
* cluster scene: 64 anisotropic clusters plus 10% uniform background,
  log-scales N(-4.5, 0.7^2), opacity sigmoid(N(0.5, 1.5^2)), SH degree 3;
  views on a jittered orbit at 1280x720 (or other resolutions).

Layout (structure of arrays, float32, C-contiguous), n Gaussians:
  mean      [3][n]            x, y, z
  log_scale [3][n]            per-axis log standard deviation
  quat      [4][n]            w, x, y, z (not necessarily unit length)
  opacity   [n]               alpha in (0, 1)
  sh        [(deg+1)^2][3][n] real SH coefficients, coefficient-major,
                              then channel (R, G, B)

Views are float64: world_to_cam [V][12] row-major [R | t] (p_cam = R p + t,
OpenCV axes: x right, y down, z forward), intrinsics [V][4] = fx, fy, cx, cy
in pixels, size [V][2] = width, height (int32).

Every array is drawn from numpy.random.Generator(PCG64(seed)) in a fixed order,
so a (recipe, seed) pair always yields the same bytes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Degree-0 real spherical harmonic, 1/(2 sqrt(pi)).  Used only to place the DC
# coefficient so that the degree-0 colour equals the drawn colour.
SH_C0 = 0.28209479177387814


@dataclasses.dataclass
class Scene:
    mean: np.ndarray        # [3, n] f32
    log_scale: np.ndarray   # [3, n] f32
    quat: np.ndarray        # [4, n] f32
    opacity: np.ndarray     # [n] f32
    sh: np.ndarray          # [K, 3, n] f32, K = (deg+1)^2
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.mean[:, idx]),
                     np.ascontiguousarray(self.log_scale[:, idx]),
                     np.ascontiguousarray(self.quat[:, idx]),
                     np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]), self.sh_degree)

    def attribute_bytes(self) -> int:
        return int(self.mean.nbytes + self.log_scale.nbytes + self.quat.nbytes
                   + self.opacity.nbytes + self.sh.nbytes)


@dataclasses.dataclass
class Views:
    world_to_cam: np.ndarray  # [V, 12] f64
    intrinsics: np.ndarray    # [V, 4] f64
    size: np.ndarray          # [V, 2] i32 (width, height)

    @property
    def n_views(self) -> int:
        return int(self.size.shape[0])

    @property
    def n_rays(self) -> int:
        return int(np.sum(self.size[:, 0].astype(np.int64) * self.size[:, 1]))

    def subset(self, idx) -> "Views":
        idx = np.asarray(idx)
        return Views(np.ascontiguousarray(self.world_to_cam[idx]),
                     np.ascontiguousarray(self.intrinsics[idx]),
                     np.ascontiguousarray(self.size[idx]))

    def ray_offsets(self) -> np.ndarray:
        """Start of each view's rays in the global (view-major, row-major) ray index."""
        per = self.size[:, 0].astype(np.int64) * self.size[:, 1]
        return np.concatenate([[0], np.cumsum(per)]).astype(np.int64)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _colours_to_sh(rng, n, degree, colours, hi_std):
    k = (degree + 1) ** 2
    sh = np.zeros((k, 3, n), dtype=np.float64)
    sh[0] = (colours.T - 0.5) / SH_C0
    if k > 1:
        sh[1:] = rng.normal(0.0, hi_std, size=(k - 1, 3, n))
    return sh


def make_tiny_scene(n: int = 2000, seed: int = 0) -> Scene:
    """Uniform tiny scene (2 000 Gaussians by default), SH degree 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mean = rng.uniform(-1.0, 1.0, size=(3, n))
    log_scale = rng.normal(-3.5, 0.5, size=(3, n))
    quat = _random_quats(rng, n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    colours = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = _colours_to_sh(rng, n, 0, colours, 0.0)
    return Scene(mean.astype(np.float32), log_scale.astype(np.float32),
                 quat.astype(np.float32), opacity.astype(np.float32),
                 sh.astype(np.float32), 0)


def make_cluster_scene(n: int, seed: int, sh_degree: int = 3,
                       n_clusters: int = 64, background: float = 0.10) -> Scene:
    """Clustered scene: 64 anisotropic clusters + uniform background."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(-0.7, 0.7, size=(n_clusters, 3))
    weights = rng.dirichlet(np.ones(n_clusters))
    sig = rng.uniform(0.02, 0.2, size=(n_clusters, 3))
    rots = np.stack([_quat_to_rot(q) for q in _random_quats(rng, n_clusters).T])
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    which = rng.choice(n_clusters, size=n_cl, p=weights)
    z = rng.standard_normal((n_cl, 3)) * sig[which]
    pts_cl = centres[which] + np.einsum("nij,nj->ni", rots[which], z)
    pts_bg = rng.uniform(-1.0, 1.0, size=(n_bg, 3))
    pts = np.concatenate([pts_cl, pts_bg], axis=0)
    perm = rng.permutation(n)
    pts = pts[perm]
    log_scale = rng.normal(-4.5, 0.7, size=(3, n))
    quat = _random_quats(rng, n)
    opacity = _sigmoid(rng.normal(0.5, 1.5, size=n))
    colours = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = _colours_to_sh(rng, n, sh_degree, colours, 0.1)
    return Scene(np.ascontiguousarray(pts.T).astype(np.float32),
                 log_scale.astype(np.float32), quat.astype(np.float32),
                 opacity.astype(np.float32), sh.astype(np.float32), sh_degree)


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """World-to-camera [R | t] (OpenCV axes) for a camera at `eye` facing `target`."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    return np.concatenate([R, t[:, None]], axis=1).reshape(12)


def _intrinsics(width, height, fov_deg):
    fx = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return np.array([fx, fx, width / 2.0, height / 2.0])


def make_tiny_views(width: int = 64, height: int = 64, fov_deg: float = 60.0) -> Views:
    """Four cameras at the vertices of a regular tetrahedron of radius 3."""
    s = math.sqrt(3.0)
    eyes = [(s, s, s), (s, -s, -s), (-s, s, -s), (-s, -s, s)]
    w2c = np.stack([look_at(e, (0.0, 0.0, 0.0)) for e in eyes])
    intr = np.stack([_intrinsics(width, height, fov_deg)] * 4)
    size = np.array([[width, height]] * 4, dtype=np.int32)
    return Views(w2c, intr, size)


def make_orbit_views(n_views: int, seed: int, width: int = 1280, height: int = 720,
                     fov_deg: float = 60.0, resolutions=None) -> Views:
    """Jittered orbit: azimuth 2pi(k+U(-1/2,1/2))/V, elevation 15deg+U(-10,10)deg,
    radius 3(1+U(-0.05,0.05)), target N(0, 0.02^2 I).  With `resolutions`, each
    view's (width, height) is drawn uniformly from that list."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w2c, intr, size = [], [], []
    for k in range(n_views):
        az = 2.0 * math.pi * (k + rng.uniform(-0.5, 0.5)) / n_views
        el = math.radians(15.0 + rng.uniform(-10.0, 10.0))
        rad = 3.0 * (1.0 + rng.uniform(-0.05, 0.05))
        tgt = rng.normal(0.0, 0.02, size=3)
        if resolutions is not None:
            width, height = resolutions[int(rng.integers(len(resolutions)))]
        eye = tgt + rad * np.array([math.cos(el) * math.cos(az),
                                    math.cos(el) * math.sin(az), math.sin(el)])
        w2c.append(look_at(eye, tgt))
        intr.append(_intrinsics(width, height, fov_deg))
        size.append((width, height))
    return Views(np.stack(w2c), np.stack(intr), np.array(size, dtype=np.int32))


def splitmix64(x):
    """SplitMix64 finaliser (Steele, Lea & Flood 2014), vectorised over uint64."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    return x


def ray_subsample_mask(views: Views, seed: int, modulus: int = 100) -> np.ndarray:
    """Bitset (uint32 words) over all rays, view-major then row-major: ray r is
    kept when splitmix64(seed xor r) mod `modulus` == 0."""
    n = views.n_rays
    r = np.arange(n, dtype=np.uint64)
    keep = (splitmix64(r ^ np.uint64(seed)) % np.uint64(modulus)) == 0
    return pack_bits(keep)


def block_subsample_mask(views: Views, seed: int, modulus: int = 100, block: int = 8) -> np.ndarray:
    """Bitset over all rays keeping whole block x block pixel squares (aligned
    to multiples of `block` in each view): square b (numbered view by view,
    row-major) is kept when splitmix64(seed xor b) mod `modulus` == 0."""
    keep_all = []
    b0 = 0
    for v in range(views.n_views):
        W, H = int(views.size[v, 0]), int(views.size[v, 1])
        bx, by = (W + block - 1) // block, (H + block - 1) // block
        ids = np.arange(bx * by, dtype=np.uint64) + np.uint64(b0)
        kb = ((splitmix64(ids ^ np.uint64(seed)) % np.uint64(modulus)) == 0).reshape(by, bx)
        b0 += bx * by
        ys, xs = np.mgrid[0:H, 0:W]
        keep_all.append(kb[ys // block, xs // block].reshape(-1))
    return pack_bits(np.concatenate(keep_all))


def pack_bits(keep: np.ndarray) -> np.ndarray:
    """Pack a boolean ray array into little-endian uint32 words (bit r%32 of word r//32)."""
    keep = np.asarray(keep, dtype=bool)
    n = keep.shape[0]
    words = (n + 31) // 32
    pad = np.zeros(words * 32, dtype=bool)
    pad[:n] = keep
    b = pad.reshape(words, 32).astype(np.uint64)
    w = (b << np.arange(32, dtype=np.uint64)).sum(axis=1)
    return w.astype(np.uint32)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    w = np.asarray(words, dtype=np.uint32).astype(np.uint64)
    bits = (w[:, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(-1)[:n].astype(bool)


def make_config(name: str):
    """Named workloads: returns (scene, views, m, seed) for 'tiny' and 'scene1m';
    'scene1m_views(k)' style subsets are built by the callers."""
    if name == "tiny":
        return make_tiny_scene(2000, 0), make_tiny_views(), 200, 0
    if name == "scene1m":
        return (make_cluster_scene(1_000_000, 1, 3), make_orbit_views(100, 101),
                100_000, 0)
    if name == "precision3m":
        return (make_cluster_scene(3_000_000, 3, 3),
                make_orbit_views(200, 103, 1920, 1080), 300_000, 0)
    raise KeyError(name)


def make_batch_specs(n_scenes: int = 16, seed: int = 2, n_lo: int = 50_000, n_hi: int = 2_000_000,
                     v_lo: int = 24, v_hi: int = 200,
                     resolutions=((640, 360), (1280, 720), (1920, 1080))):
    """Sizes of a batch of uneven scenes: Gaussian counts log-uniform in
    [n_lo, n_hi], view counts uniform in [v_lo, v_hi]; each view's resolution
    is drawn from `resolutions`.  Returns [(n, n_views, scene_seed, view_seed)]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_scenes):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        nv = int(rng.integers(v_lo, v_hi + 1))
        out.append((n, nv, 10_000 + 2 * k + seed * 1000, 10_001 + 2 * k + seed * 1000))
    return out


def make_batch(specs, resolutions=((640, 360), (1280, 720), (1920, 1080))):
    """(scene, views) pairs for make_batch_specs output (cluster scenes, SH
    degree 3, jittered orbits at mixed resolutions)."""
    return [(make_cluster_scene(n, ss, 3), make_orbit_views(nv, vs, resolutions=resolutions))
            for n, nv, ss, vs in specs]


def make_explicit_scene(means, log_scales, quats, opacity, colours=None, sh=None,
                        sh_degree: int = 0) -> Scene:
    """Scene from explicit per-Gaussian rows: means [n,3], log_scales [n,3],
    quats [n,4] (w,x,y,z), opacity [n], and either colours [n,3] (degree 0)
    or full SH coefficients sh [n, K, 3]."""
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = means.shape[0]
    ls = np.broadcast_to(np.asarray(log_scales, np.float64), (n, 3))
    q = np.broadcast_to(np.asarray(quats, np.float64), (n, 4))
    op = np.broadcast_to(np.asarray(opacity, np.float64), (n,))
    if sh is None:
        col = np.broadcast_to(np.asarray(colours if colours is not None else 0.5, np.float64), (n, 3))
        coeff = np.zeros((1, 3, n))
        coeff[0] = (col.T - 0.5) / SH_C0
        sh_degree = 0
    else:
        coeff = np.transpose(np.asarray(sh, np.float64), (1, 2, 0))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means.T), f(ls.T), f(q.T), f(op), f(coeff), sh_degree)


def make_camera_set(eyes, targets, width, height, fov_deg=60.0, up=(0.0, 0.0, 1.0)) -> Views:
    """Cameras at `eyes` facing `targets` (one each), all width x height."""
    w2c = np.stack([look_at(e, t, up) for e, t in zip(eyes, targets)])
    intr = np.stack([_intrinsics(width, height, fov_deg)] * len(w2c))
    size = np.array([[width, height]] * len(w2c), dtype=np.int32)
    return Views(w2c, intr, size)


def _ball(rng, radius):
    """A point uniform in the 3D ball of the given radius."""
    v = rng.normal(size=3)
    return v / np.linalg.norm(v) * radius * rng.uniform() ** (1.0 / 3.0)


def make_pose_region(w2c0, n_poses: int, pos_radius: float, ang_radius: float, seed: int = 0):
    """Camera poses around the world-to-camera pose `w2c0` ([12], [R | t]):
    the first is w2c0 itself; each other has its centre moved uniformly within
    `pos_radius` and its orientation turned by a rotation vector drawn
    uniformly within `ang_radius` radians (world frame).  Returns a list of
    [12] arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M0 = np.asarray(w2c0, np.float64).reshape(3, 4)
    R0, t0 = M0[:, :3], M0[:, 3]
    c0 = -R0.T @ t0
    out = [M0.ravel().copy()]
    for _ in range(n_poses - 1):
        w = _ball(rng, ang_radius)
        th = np.linalg.norm(w)
        K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]) / max(th, 1e-300)
        Rw = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * (K @ K)
        R = R0 @ Rw.T          # camera turned by Rw in the world frame
        c = c0 + _ball(rng, pos_radius)
        out.append(np.concatenate([R, (-R @ c)[:, None]], 1).ravel())
    return out
