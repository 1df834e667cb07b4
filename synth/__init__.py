"""Seeded synthetic scenes and cameras for the RaDe-GS rasterizer.

This module only draws random inputs.  It holds none of the rasterizer's
arithmetic, so both the CPU oracle (``oracle/``) and the HIP path use it as
their common source of inputs.  Every array it returns is the canonical FP32
input of a workload; both sides read the same arrays.

Conventions
-----------
* Cameras use OpenCV axes (x right, y down, z forward).  A view holds a
  world-to-camera rotation ``R`` (3x3, row-major) and translation ``t``, the
  intrinsics ``fx, fy, cx, cy`` in pixels and the image size.
* Gaussians carry already-activated parameters: ``scales`` are positive
  standard deviations (exp of the drawn log-scale), ``opacities`` lie in
  (0, 1) (sigmoid of the drawn logit), quaternions are (w, x, y, z) and unit
  length, ``sh`` is N x K x 3 with K = (degree + 1)^2, coefficient-major and
  RGB-minor.
* ``N(m, s)`` below means a normal draw with mean m and standard deviation s.
  Draws use ``numpy.random.default_rng(seed)`` in FP64 in the order written in
  each function and are cast to FP32 at the end.

Workloads (the sizes of the benchmark configurations):

==========================  ============================================
name                        recipe
==========================  ============================================
``plain_64x64_1k``          1 view 64x64 (fx=fy=64, cx=cy=32), 1,000
                            Gaussians, means U[-1,1]^3 + (0,0,3),
                            log-scales N(-3,0.5), opacity sigmoid(N(0,1)),
                            SH degree 0 whose colour is U[0,1]
``plain_800x800_200k``      1 view 800x800, 200k Gaussians uniform in the
                            radius-2 ball at distance 4, log-scales
                            N(-4,0.7), opacity sigmoid(N(0,1)), SH degree 3
                            with coefficients N(0,0.2)
``plain_1600x1064_1m``      1 view 1600x1064, 1M Gaussians in 64 anisotropic
                            clusters at distance 2..20, log-scales
                            N(-4.5,0.8), opacity sigmoid(N(1,1.5)), SH
                            degree 3 with coefficients N(0,0.2)
``batched_16views_1m``      the 1M-Gaussian cluster scene seen by 16 orbit
                            views of uneven size in 400x300..1600x1200
``recompute_32views_3m``    the cluster recipe with 3M Gaussians seen by 32
                            orbit views of 1600x1064
==========================  ============================================
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

__all__ = [
    "View", "Scene", "WORKLOADS", "make_workload", "make_scene_uniform_cube",
    "make_scene_ball", "make_scene_clusters", "make_views_orbit",
    "identity_view", "random_targets", "sh_coeffs_per_channel",
]

# Scale that maps U[-0.5, 0.5] draws onto degree-0 SH coefficients whose
# evaluated colour (coefficient * Y00 + 0.5) is U[0, 1]: Y00 = 1/(2*sqrt(pi)).
_DC_SCALE = 2.0 * math.sqrt(math.pi)


def sh_coeffs_per_channel(degree: int) -> int:
    return (degree + 1) * (degree + 1)


@dataclasses.dataclass
class View:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3,3) float32, world -> camera
    t: np.ndarray  # (3,)  float32

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    means: np.ndarray      # (N,3) float32
    scales: np.ndarray     # (N,3) float32, > 0
    quats: np.ndarray      # (N,4) float32, (w,x,y,z)
    opacities: np.ndarray  # (N,)  float32, in (0,1)
    sh: np.ndarray         # (N,K,3) float32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.scales[idx].copy(),
                     self.quats[idx].copy(), self.opacities[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree)


def identity_view(width: int, height: int, fx: float | None = None,
                  fy: float | None = None) -> View:
    """Camera at the origin looking down +z, f = W unless given, c = centre."""
    fx = float(width) if fx is None else float(fx)
    fy = float(width) if fy is None else float(fy)
    return View(int(width), int(height), fx, fy, width / 2.0, height / 2.0,
                np.eye(3, dtype=np.float32), np.zeros(3, dtype=np.float32))


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.normal(0.0, 1.0, size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from the QR factorisation of a normal matrix."""
    a = rng.normal(size=(3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _finish(means, log_scales, quats, logit_o, sh, degree) -> Scene:
    return Scene(
        means=np.ascontiguousarray(means, dtype=np.float32),
        scales=np.ascontiguousarray(np.exp(log_scales), dtype=np.float32),
        quats=np.ascontiguousarray(quats, dtype=np.float32),
        opacities=np.ascontiguousarray(_sigmoid(logit_o), dtype=np.float32),
        sh=np.ascontiguousarray(sh, dtype=np.float32),
        sh_degree=int(degree),
    )


def make_scene_uniform_cube(n: int = 1000, seed: int = 0, centre_z: float = 3.0,
                            log_scale_mu: float = -3.0, log_scale_sd: float = 0.5,
                            sh_degree: int = 0, half: float = 1.0) -> Scene:
    """Means U[-half,half]^3 + (0,0,centre_z).  Draw order: means, log-scales,
    quaternions, opacity logits, colour/SH."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-half, half, size=(n, 3)) + np.array([0.0, 0.0, centre_z])
    log_s = rng.normal(log_scale_mu, log_scale_sd, size=(n, 3))
    quats = _unit_quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n)
    k = sh_coeffs_per_channel(sh_degree)
    sh = np.zeros((n, k, 3))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    sh[:, 0, :] = (rgb - 0.5) * _DC_SCALE
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.2, size=(n, k - 1, 3))
    return _finish(means, log_s, quats, logit, sh, sh_degree)


def make_scene_ball(n: int = 200_000, seed: int = 1, centre=(0.0, 0.0, 4.0),
                    radius: float = 2.0, log_scale_mu: float = -4.0,
                    log_scale_sd: float = 0.7, sh_degree: int = 3) -> Scene:
    """Means uniform in a ball (direction = normalised normal draw, radius =
    R * U^(1/3)).  Draw order: directions, radii, log-scales, quaternions,
    opacity logits, SH coefficients (all N(0,0.2))."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, size=n) ** (1.0 / 3.0)
    means = np.asarray(centre)[None, :] + d * r[:, None]
    log_s = rng.normal(log_scale_mu, log_scale_sd, size=(n, 3))
    quats = _unit_quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n)
    k = sh_coeffs_per_channel(sh_degree)
    sh = rng.normal(0.0, 0.2, size=(n, k, 3))
    return _finish(means, log_s, quats, logit, sh, sh_degree)


def make_scene_clusters(n: int = 1_000_000, seed: int = 2, n_clusters: int = 64,
                        width: int = 1600, height: int = 1064,
                        dist_range=(2.0, 20.0), log_scale_mu: float = -4.5,
                        log_scale_sd: float = 0.8, logit_mu: float = 1.0,
                        logit_sd: float = 1.5, sh_degree: int = 3) -> Scene:
    """Mixture of anisotropic clusters in front of the identity camera.

    Per cluster k (drawn in this order): distance r_k ~ U[dist_range]; a pixel
    (u, v) ~ U[0,W] x U[0,H] whose viewing ray (f = W, c = image centre) gives
    the centre direction; per-axis extents r_k * 10^U(-2,-0.7); a uniform
    random rotation.  Then per Gaussian: unit normal offsets, log-scales,
    quaternions, opacity logits, SH coefficients N(0, 0.2).  Cluster sizes are
    n // n_clusters with the remainder spread over the first clusters.
    """
    rng = np.random.default_rng(seed)
    fx = float(width)
    cx, cy = width / 2.0, height / 2.0
    centres = np.zeros((n_clusters, 3))
    axes = np.zeros((n_clusters, 3, 3))
    for k in range(n_clusters):
        rk = rng.uniform(*dist_range)
        u = rng.uniform(0.0, width)
        v = rng.uniform(0.0, height)
        d = np.array([(u - cx) / fx, (v - cy) / fx, 1.0])
        d /= np.linalg.norm(d)
        centres[k] = rk * d
        sig = rk * 10.0 ** rng.uniform(-2.0, -0.7, size=3)
        rot = _random_rotation(rng)
        axes[k] = rot * sig[None, :]
    sizes = np.full(n_clusters, n // n_clusters)
    sizes[: n - sizes.sum()] += 1
    cid = np.repeat(np.arange(n_clusters), sizes)
    eps = rng.normal(size=(n, 3))
    means = centres[cid] + np.einsum("nij,nj->ni", axes[cid], eps)
    log_s = rng.normal(log_scale_mu, log_scale_sd, size=(n, 3))
    quats = _unit_quats(rng, n)
    logit = rng.normal(logit_mu, logit_sd, size=n)
    k = sh_coeffs_per_channel(sh_degree)
    sh = rng.normal(0.0, 0.2, size=(n, k, 3))
    return _finish(means, log_s, quats, logit, sh, sh_degree)


def _look_at(cam_pos: np.ndarray, target: np.ndarray) -> tuple:
    """World-to-camera (R, t) for OpenCV axes with world +y as 'down'."""
    f = target - cam_pos
    f = f / np.linalg.norm(f)
    down = np.array([0.0, 1.0, 0.0])
    x = np.cross(down, f)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f], axis=0)
    t = -R @ cam_pos
    return R, t


def make_views_orbit(scene_centroid: np.ndarray, radius: float, n_views: int,
                     seed: int, sizes: Sequence[tuple] | None = None,
                     size_range=((400, 1600), (300, 1200)),
                     elev_deg: float = 20.0) -> List[View]:
    """Orbit cameras looking at ``scene_centroid``.

    Draw order per view: width ~ U{lo..hi}, height ~ U{lo..hi} (skipped when
    ``sizes`` is given), azimuth ~ U[0, 2pi), elevation ~ U[-elev, elev] deg.
    Intrinsics f = W, c = image centre.
    """
    rng = np.random.default_rng(seed)
    views = []
    for i in range(n_views):
        if sizes is None:
            w = int(rng.integers(size_range[0][0], size_range[0][1] + 1))
            h = int(rng.integers(size_range[1][0], size_range[1][1] + 1))
        else:
            w, h = sizes[i]
        az = rng.uniform(0.0, 2.0 * math.pi)
        el = math.radians(rng.uniform(-elev_deg, elev_deg))
        off = radius * np.array([math.cos(el) * math.sin(az), -math.sin(el),
                                 math.cos(el) * math.cos(az)])
        R, t = _look_at(scene_centroid + off, scene_centroid)
        views.append(View(w, h, float(w), float(w), w / 2.0, h / 2.0,
                          R.astype(np.float32), t.astype(np.float32)))
    return views


def _cluster_orbit(scene: Scene, n_views: int, seed: int, sizes=None) -> List[View]:
    # Orbit around the centroid at 1.5x the largest centroid distance of the
    # cluster centres; the cluster centres are recovered as a coarse k-means
    # free proxy: the spread of the means themselves.
    m = scene.means.astype(np.float64)
    c = m.mean(axis=0)
    rad = 1.5 * float(np.quantile(np.linalg.norm(m - c, axis=1), 0.99))
    return make_views_orbit(c, rad, n_views, seed, sizes=sizes)


WORKLOADS = {
    "plain_64x64_1k": dict(views=1, n=1000),
    "plain_800x800_200k": dict(views=1, n=200_000),
    "plain_1600x1064_1m": dict(views=1, n=1_000_000),
    "batched_16views_1m": dict(views=16, n=1_000_000),
    "recompute_32views_3m": dict(views=32, n=3_000_000),
}


def make_workload(name: str, n: int | None = None) -> tuple:
    """(scene, views) of a named workload; ``n`` overrides the Gaussian count
    (for scaled-down parity runs of the same recipe)."""
    if name == "plain_64x64_1k":
        scene = make_scene_uniform_cube(n or 1000, seed=0)
        return scene, [identity_view(64, 64, 64.0, 64.0)]
    if name == "plain_800x800_200k":
        scene = make_scene_ball(n or 200_000, seed=1)
        return scene, [identity_view(800, 800)]
    if name == "plain_1600x1064_1m":
        scene = make_scene_clusters(n or 1_000_000, seed=2)
        return scene, [identity_view(1600, 1064)]
    if name == "batched_16views_1m":
        scene = make_scene_clusters(n or 1_000_000, seed=2)
        return scene, _cluster_orbit(scene, 16, seed=3)
    if name == "recompute_32views_3m":
        scene = make_scene_clusters(n or 3_000_000, seed=4)
        return scene, _cluster_orbit(scene, 32, seed=4,
                                     sizes=[(1600, 1064)] * 32)
    raise KeyError(name)


def random_targets(views: Sequence[View], seed: int) -> dict:
    """Random per-view targets for an L1 loss (colour U[0,1], both depths
    U[2,6], unit normals with n_z < 0, alpha U[0,1]); planar per view."""
    rng = np.random.default_rng(seed)
    out = {"color": [], "depth": [], "normal": [], "alpha": []}
    for v in views:
        p = v.pixels
        out["color"].append(rng.uniform(0, 1, size=(3, p)))
        out["depth"].append(rng.uniform(2, 6, size=(2, p)))
        n = rng.normal(size=(3, p))
        n /= np.linalg.norm(n, axis=0, keepdims=True)
        n[2] = -np.abs(n[2])
        out["normal"].append(n)
        out["alpha"].append(rng.uniform(0, 1, size=(1, p)))
    return {k: np.ascontiguousarray(np.concatenate([a.reshape(-1) for a in v]),
                                    dtype=np.float32) for k, v in out.items()}
