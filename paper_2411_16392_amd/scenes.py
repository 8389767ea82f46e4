"""Seeded synthetic scenes and cameras for the quadric rasterizer.

This module only draws inputs: primitive parameters and camera poses.  It holds
none of the rendering arithmetic, so both the HIP path and the FP64 oracle can be
fed from it.  The datasets the paper evaluates on (DTU, Tanks and Temples,
Mip-NeRF 360; Sec. 4) are not available, so these scenes stand in for them with
the shapes of the five workloads below.

Primitive parameters follow the paper's statement of a quadric Gaussian
(Sec. 3.2, "Quadratic Gaussian Model"): centre c, orientation R (stored as a
unit quaternion w,x,y,z), two tangent-plane scales sigma_1, sigma_2 (standard
deviations), two curvature coefficients lambda_1, lambda_2 of the explicit
height z = lambda_1 x^2 + lambda_2 y^2 (the paper's lambda_i = sign(s_i) s_3/s_i^2,
Sec. 3.2 curvature paragraph), opacity and an RGB colour.

Cameras are world-to-camera (R, t) in the OpenCV convention (x right, y down,
z forward) with pinhole intrinsics fx, fy, cx, cy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32 = np.float32


@dataclass
class Scene:
    center: np.ndarray   # [P,3] float32
    quat: np.ndarray     # [P,4] float32, (w,x,y,z)
    scale: np.ndarray    # [P,2] float32, sigma_1, sigma_2 > 0
    curv: np.ndarray     # [P,2] float32, lambda_1, lambda_2
    opacity: np.ndarray  # [P]   float32
    rgb: np.ndarray      # [P,3] float32
    sh: np.ndarray | None = None  # [P,K,3] float32 spherical-harmonics coefficients (K = 1, 4, 9, 16), or None

    @property
    def n(self) -> int:
        return int(self.center.shape[0])

    @property
    def sh_degree(self) -> int:
        return -1 if self.sh is None else int(round(np.sqrt(self.sh.shape[1]))) - 1

    def arrays(self):
        return (self.center, self.quat, self.scale, self.curv, self.opacity, self.rgb)

    def subset(self, idx) -> "Scene":
        sub = Scene(*(np.ascontiguousarray(a[idx]) for a in self.arrays()))
        if self.sh is not None:
            sub.sh = np.ascontiguousarray(self.sh[idx])
        return sub


def with_sh(scene: Scene, degree: int, seed: int, scale: float = 0.3) -> Scene:
    """The scene with spherical-harmonics colour coefficients of `degree`
    ((degree + 1)^2 per channel): the constant terms uniform in [-1.5, 1.5],
    the band-l terms N(0, (scale / (l + 1))^2)."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    K = (degree + 1) ** 2
    sh = np.zeros((scene.n, K, 3), F32)
    sh[:, 0, :] = rng.uniform(-1.5, 1.5, (scene.n, 3))
    for k in range(1, K):
        l = int(np.floor(np.sqrt(k)))
        sh[:, k, :] = rng.normal(0.0, scale / (l + 1), (scene.n, 3))
    return Scene(scene.center, scene.quat, scene.scale, scene.curv, scene.opacity, scene.rgb, sh)


@dataclass
class Camera:
    R: np.ndarray        # [3,3] float32 world->camera rotation (rows = camera axes)
    t: np.ndarray        # [3]   float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16


@dataclass
class Config:
    index: int
    name: str
    scene: Scene
    cameras: list = field(default_factory=list)
    notes: str = ""


# ---------------------------------------------------------------------------
# small helpers (input generation only)
# ---------------------------------------------------------------------------

def look_at(eye, target=(0.0, 0.0, 0.0), width=128, height=128, f=None) -> Camera:
    """Pinhole camera at `eye` looking at `target`: z = normalize(target-eye),
    x = normalize(up x z) with up = (0,1,0) (or (0,0,1) when z is parallel to
    it), y = z x x; R = [x; y; z], t = -R eye.  f defaults to the image width,
    principal point at the image centre."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    up = np.array([0.0, 1.0, 0.0])
    if abs(np.dot(up, z)) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    x = np.cross(up, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z]).astype(F32)
    t = (-R.astype(np.float64) @ eye).astype(F32)
    f = float(width if f is None else f)
    return Camera(R=R, t=t, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                  width=int(width), height=int(height))


def look_dir(eye, direction, width, height, f=None) -> Camera:
    eye = np.asarray(eye, np.float64)
    return look_at(eye, eye + np.asarray(direction, np.float64), width, height, f)


def random_quats(rng, n) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def mat_to_quat(M: np.ndarray) -> np.ndarray:
    """Rotation matrices [n,3,3] (columns = local axes in world) -> unit
    quaternions (w,x,y,z), branch on the largest diagonal term for stability."""
    n = M.shape[0]
    q = np.empty((n, 4))
    tr = M[:, 0, 0] + M[:, 1, 1] + M[:, 2, 2]
    cases = np.stack([tr, M[:, 0, 0], M[:, 1, 1], M[:, 2, 2]], 1).argmax(1)
    for c in range(4):
        m = cases == c
        if not m.any():
            continue
        A = M[m]
        if c == 0:
            s = np.sqrt(1.0 + A[:, 0, 0] + A[:, 1, 1] + A[:, 2, 2]) * 2
            q[m] = np.stack([0.25 * s, (A[:, 2, 1] - A[:, 1, 2]) / s,
                             (A[:, 0, 2] - A[:, 2, 0]) / s, (A[:, 1, 0] - A[:, 0, 1]) / s], 1)
        elif c == 1:
            s = np.sqrt(1.0 + A[:, 0, 0] - A[:, 1, 1] - A[:, 2, 2]) * 2
            q[m] = np.stack([(A[:, 2, 1] - A[:, 1, 2]) / s, 0.25 * s,
                             (A[:, 0, 1] + A[:, 1, 0]) / s, (A[:, 0, 2] + A[:, 2, 0]) / s], 1)
        elif c == 2:
            s = np.sqrt(1.0 + A[:, 1, 1] - A[:, 0, 0] - A[:, 2, 2]) * 2
            q[m] = np.stack([(A[:, 0, 2] - A[:, 2, 0]) / s, (A[:, 0, 1] + A[:, 1, 0]) / s,
                             0.25 * s, (A[:, 1, 2] + A[:, 2, 1]) / s], 1)
        else:
            s = np.sqrt(1.0 + A[:, 2, 2] - A[:, 0, 0] - A[:, 1, 1]) * 2
            q[m] = np.stack([(A[:, 1, 0] - A[:, 0, 1]) / s, (A[:, 0, 2] + A[:, 2, 0]) / s,
                             (A[:, 1, 2] + A[:, 2, 1]) / s, 0.25 * s], 1)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def tangent_quats(rng, normals) -> np.ndarray:
    """Orientation whose local z axis is the given surface normal, with a
    uniform random twist about it."""
    n = normals / np.linalg.norm(normals, axis=1, keepdims=True)
    ref = np.where(np.abs(n[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    e1 = np.cross(ref, n)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(n, e1)
    psi = rng.uniform(0, 2 * np.pi, size=(n.shape[0], 1))
    c, s = np.cos(psi), np.sin(psi)
    a1 = c * e1 + s * e2
    a2 = -s * e1 + c * e2
    M = np.stack([a1, a2, n], axis=2)  # columns
    return mat_to_quat(M)


def log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


def curvatures(rng, n, lim, planar_frac=0.1):
    lam = rng.uniform(-lim, lim, size=(n, 2))
    planar = rng.random(n) < planar_frac
    lam[planar] = 0.0
    return lam


def _finish(center, quat, scale, curv, rng) -> Scene:
    n = center.shape[0]
    return Scene(center=np.ascontiguousarray(center, F32),
                 quat=np.ascontiguousarray(quat, F32),
                 scale=np.ascontiguousarray(scale, F32),
                 curv=np.ascontiguousarray(curv, F32),
                 opacity=np.ascontiguousarray(rng.uniform(0.1, 0.99, size=n), F32),
                 rgb=np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(n, 3)), F32))


def unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def scene_uniform_cube(n, seed, scale_range=(0.01, 0.1), curv_lim=2.0) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    center = rng.uniform(-1, 1, size=(n, 3))
    quat = random_quats(rng, n)
    scale = log_uniform(rng, *scale_range, size=(n, 2))
    curv = curvatures(rng, n, curv_lim)
    return _finish(center, quat, scale, curv, rng)


def scene_sphere(n, seed, jitter=0.02, scale_range=(0.01, 0.1), curv_lim=2.0) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    d = unit_vectors(rng, n)
    center = d + rng.normal(0, jitter, size=(n, 3))
    quat = tangent_quats(rng, d)
    scale = log_uniform(rng, *scale_range, size=(n, 2))
    curv = curvatures(rng, n, curv_lim)
    return _finish(center, quat, scale, curv, rng)


def scene_ellipsoids(n, seed, n_ell=8, jitter=0.01, scale_range=(0.002, 0.03), curv_lim=5.0) -> Scene:
    """Noisy closed surface: the outer surface of a union of random ellipsoids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C = rng.uniform(-0.5, 0.5, size=(n_ell, 3))
    rad = rng.uniform(0.3, 1.0, size=(n_ell, 3))
    Rs = np.stack([_quat_to_mat(q) for q in random_quats(rng, n_ell)])
    # approximate areas (Knud Thomsen) to share the points
    p = 1.6075
    a, b, c = rad[:, 0], rad[:, 1], rad[:, 2]
    area = 4 * np.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)
    pts, nrm = [], []
    have = 0
    while have < n:
        m = int((n - have) * 1.6) + 1024
        k = rng.choice(n_ell, size=m, p=area / area.sum())
        u = unit_vectors(rng, m)
        local = u * rad[k]
        x = C[k] + np.einsum("mij,mj->mi", Rs[k], local)
        # surface normal of the ellipsoid: R D^-2 R^T (x - C) = R (u / r)
        g = np.einsum("mij,mj->mi", Rs[k], u / rad[k])
        inside = np.zeros(m, bool)
        for j in range(n_ell):
            y = np.einsum("ji,mj->mi", Rs[j], x - C[j]) / rad[j]
            inside |= (np.sum(y * y, 1) < 1.0 - 1e-9) & (k != j)
        keep = ~inside
        pts.append(x[keep])
        nrm.append(g[keep])
        have += int(keep.sum())
    pts = np.concatenate(pts)[:n]
    nrm = np.concatenate(nrm)[:n]
    center = pts + rng.normal(0, jitter, size=(n, 3))
    quat = tangent_quats(rng, nrm)
    scale = log_uniform(rng, *scale_range, size=(n, 2))
    curv = curvatures(rng, n, curv_lim)
    return _finish(center, quat, scale, curv, rng)


def scene_unbounded(n, seed, shell_frac=0.7, bg_radius=50.0) -> Scene:
    """Nested noisy shells of radius 1..5 plus a uniform background ball."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_sh = int(round(n * shell_frac))
    n_bg = n - n_sh
    radii = np.arange(1, 6, dtype=np.float64)
    w = radii ** 2 / np.sum(radii ** 2)
    r = rng.choice(radii, size=n_sh, p=w)
    d = unit_vectors(rng, n_sh)
    c_sh = d * r[:, None] + rng.normal(0, 1, size=(n_sh, 3)) * (0.01 * r[:, None])
    q_sh = tangent_quats(rng, d)
    s_sh = log_uniform(rng, 0.002, 0.03, size=(n_sh, 2))
    rb = bg_radius * rng.random(n_bg) ** (1.0 / 3.0)
    c_bg = unit_vectors(rng, n_bg) * rb[:, None]
    q_bg = random_quats(rng, n_bg)
    s_bg = log_uniform(rng, 0.05, 1.0, size=(n_bg, 2))
    center = np.concatenate([c_sh, c_bg])
    quat = np.concatenate([q_sh, q_bg])
    scale = np.concatenate([s_sh, s_bg])
    perm = rng.permutation(n)
    curv = curvatures(rng, n, 5.0)
    return _finish(center[perm], quat[perm], scale[perm], curv, rng)


def _quat_to_mat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


RESOLUTIONS_SERVE = [(256, 256), (512, 384), (1280, 720), (1920, 1080)]


def make_config(i: int, seed: int | None = None, n_override: int | None = None,
                n_views: int | None = None) -> Config:
    """Workload i (0..4) with the seed defaulting to i."""
    seed = i if seed is None else seed
    if i == 0:
        n = n_override or 2000
        sc = scene_uniform_cube(n, seed)
        cams = [look_at((0, 0, -3), width=128, height=128, f=128)]
        return Config(0, "2K quadrics, uniform cube, 128x128", sc, cams)
    if i == 1:
        n = n_override or 100_000
        sc = scene_sphere(n, seed)
        cams = [look_at((0, 0, -3), width=800, height=600, f=800)]
        return Config(1, "100K quadrics on a unit sphere, 800x600", sc, cams)
    if i == 2:
        n = n_override or 500_000
        sc = scene_ellipsoids(n, seed)
        nv = 64 if n_views is None else n_views
        cams = []
        for k in range(nv):
            phi = 2 * np.pi * k / 64
            cams.append(look_at((3 * np.sin(phi), 0.0, -3 * np.cos(phi)), width=1600, height=1200, f=1600))
        return Config(2, "500K quadrics on 8 ellipsoids, 1600x1200 ring views", sc, cams)
    if i == 3:
        n = n_override or 3_000_000
        sc = scene_unbounded(n, seed)
        rng = np.random.Generator(np.random.PCG64(1000 + seed))
        nv = 4 if n_views is None else n_views
        cams = []
        for k in range(nv):
            eye = unit_vectors(rng, 1)[0] * 2.0 * rng.random() ** (1 / 3)
            d = unit_vectors(rng, 1)[0]
            if k % 2 == 0:
                cams.append(look_dir(eye, d, 1237, 822, 1237))
            else:
                cams.append(look_dir(eye, d, 1600, 1064, 1600))
        return Config(3, "3M quadrics, shells + background ball", sc, cams)
    if i == 4:
        n = n_override or 1_000_000
        sc = scene_unbounded(n, seed)
        return Config(4, "1M resident quadrics for serving", sc, [])
    raise ValueError(f"no workload {i}")


def serve_trace(n_requests: int, rate_hz: float = 500.0, seed: int = 4, radius: float = 3.0, sizes=None):
    """Poisson arrival trace: list of (arrival_s, Camera), resolutions drawn
    uniformly from `sizes` (default RESOLUTIONS_SERVE), eyes uniform on a
    sphere looking at the origin."""
    sizes = RESOLUTIONS_SERVE if sizes is None else list(sizes)
    rng = np.random.Generator(np.random.PCG64(2000 + seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arr = np.cumsum(gaps)
    out = []
    for k in range(n_requests):
        w, h = sizes[int(rng.integers(0, len(sizes)))]
        eye = unit_vectors(rng, 1)[0] * radius
        out.append((float(arr[k]), look_at(eye, width=w, height=h, f=w)))
    return out


def upstream_grads(rng_seed: int, height: int, width: int, crop=None):
    """dL/d(colour[3,H,W], depth[H,W], normal[3,H,W]) drawn i.i.d. N(0,1);
    with `crop` = (x0, y0, w, h) everything outside the crop is zero."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    g = rng.standard_normal((7, height, width)).astype(F32)
    if crop is not None:
        x0, y0, w, h = crop
        m = np.zeros((height, width), bool)
        m[y0:y0 + h, x0:x0 + w] = True
        g[:, ~m] = 0.0
    return g[0:3].copy(), g[3].copy(), g[4:7].copy()


def upstream_geometry_grads(rng_seed: int, height: int, width: int, crop=None):
    """dL/d(curvature[H,W], median depth[H,W], distortion[H,W]) drawn i.i.d.
    N(0,1) from their own stream; zero outside `crop` as above."""
    rng = np.random.Generator(np.random.PCG64([rng_seed, 3]))
    g = rng.standard_normal((3, height, width)).astype(F32)
    if crop is not None:
        x0, y0, w, h = crop
        m = np.zeros((height, width), bool)
        m[y0:y0 + h, x0:x0 + w] = True
        g[:, ~m] = 0.0
    return g[0].copy(), g[1].copy(), g[2].copy()
