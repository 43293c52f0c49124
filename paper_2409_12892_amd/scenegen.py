"""Seeded synthetic inputs for the LM/PCG hot path (scenes, cameras, noise).

This module produces *inputs only*: Gaussian parameters, pinhole cameras,
parameter perturbations and pixel noise.  It holds none of the method's
arithmetic (no projection, blending, Jacobians or solves), so both the FP64
CPU oracle and the HIP path can consume exactly the same arrays.

Parameter layout (per Gaussian, structure-of-arrays ``x[P][N]`` float32, the
paper's per-attribute vector layout, supplement A.3):

    0..2    mean (world)
    3..5    log-scale
    6..9    quaternion (w, x, y, z), not normalised
    10      opacity logit
    11..    SH coefficients, index 11 + 3*k + ch (k = SH basis index, ch = RGB)

P = 11 + 3*(deg+1)**2, i.e. 14 at SH degree 0 and 59 at degree 3 (paper
section 3.1 and supplement A.3 count 59 parameters per Gaussian).

Cameras follow the OpenCV convention: camera x right, y down, z forward;
``R`` maps world to camera (row-major), ``t`` is the translation, pixel
coordinates are ``u = fx*x/z + cx``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "n_params", "Scene", "Cameras", "make_scene", "fibonacci_cameras",
    "perturb", "pixel_noise", "config_scene",
]


def n_params(sh_degree: int) -> int:
    """Parameters per Gaussian: 11 geometric/opacity + 3 per SH coefficient."""
    if sh_degree not in (0, 1, 2, 3):
        raise ValueError("sh_degree must be 0..3")
    return 11 + 3 * (sh_degree + 1) ** 2


@dataclasses.dataclass
class Scene:
    x: np.ndarray          # float32 [P][N]
    sh_degree: int
    seed: int

    @property
    def N(self) -> int:
        return int(self.x.shape[1])

    @property
    def P(self) -> int:
        return int(self.x.shape[0])


@dataclasses.dataclass
class Cameras:
    R: np.ndarray    # float32 [V,3,3] world->camera rotation (rows = camera axes)
    t: np.ndarray    # float32 [V,3]
    fx: np.ndarray   # float32 [V]
    fy: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    W: np.ndarray    # int32 [V]
    H: np.ndarray

    @property
    def V(self) -> int:
        return int(self.R.shape[0])

    def view(self, v: int) -> dict:
        return dict(R=self.R[v], t=self.t[v], fx=self.fx[v], fy=self.fy[v],
                    cx=self.cx[v], cy=self.cy[v], W=int(self.W[v]), H=int(self.H[v]))

    def subset(self, idx) -> "Cameras":
        idx = np.asarray(idx)
        return Cameras(self.R[idx], self.t[idx], self.fx[idx], self.fy[idx],
                       self.cx[idx], self.cy[idx], self.W[idx], self.H[idx])

    @staticmethod
    def concat(cams: list["Cameras"]) -> "Cameras":
        return Cameras(*[np.concatenate([getattr(c, f.name) for c in cams])
                         for f in dataclasses.fields(Cameras)])


def make_scene(N: int, sh_degree: int, seed: int, *,
               mean_lo: float = -1.0, mean_hi: float = 1.0,
               logscale_mu: float = -3.5, logscale_sigma: float = 0.3,
               sh_dc_sigma: float = 0.5, sh_rest_sigma: float = 0.05,
               rng: np.random.Generator | None = None) -> tuple[Scene, np.random.Generator]:
    """Draw a scene.  Draw order: means U[lo,hi]^3, log-scales N(mu,sigma),
    quaternions (normalised N(0,I4) draws), opacity logits N(0,1), SH
    (DC N(0,0.5), higher orders N(0,0.05)).  Returns the scene and the
    generator positioned after the scene draws, so perturbations and pixel
    noise come next from the same stream."""
    rng = np.random.default_rng(seed) if rng is None else rng
    P = n_params(sh_degree)
    K = (sh_degree + 1) ** 2
    mean = rng.uniform(mean_lo, mean_hi, size=(N, 3))
    logscale = rng.normal(logscale_mu, logscale_sigma, size=(N, 3))
    q = rng.normal(0.0, 1.0, size=(N, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = rng.normal(0.0, 1.0, size=(N,))
    sh_dc = rng.normal(0.0, sh_dc_sigma, size=(N, 1, 3))
    sh_rest = rng.normal(0.0, sh_rest_sigma, size=(N, K - 1, 3))
    sh = np.concatenate([sh_dc, sh_rest], axis=1)       # [N, K, 3]
    x = np.empty((P, N), dtype=np.float64)
    x[0:3] = mean.T
    x[3:6] = logscale.T
    x[6:10] = q.T
    x[10] = opac
    x[11:] = sh.reshape(N, 3 * K).T                     # index 11 + 3k + ch
    return Scene(np.ascontiguousarray(x.astype(np.float32)), sh_degree, seed), rng


def perturb(scene: Scene, rng: np.random.Generator, sigma: float = 0.02) -> np.ndarray:
    """Perturbed parameter copy x* = x + N(0, sigma) on every raw parameter."""
    d = rng.normal(0.0, sigma, size=scene.x.shape)
    return (scene.x.astype(np.float64) + d).astype(np.float32)


def pixel_noise(rng: np.random.Generator, cams: Cameras, sigma: float = 0.01) -> list[np.ndarray]:
    """Per-view pixel noise N(0, sigma), float32 [3][H][W] each."""
    return [rng.normal(0.0, sigma, size=(3, int(cams.H[v]), int(cams.W[v]))).astype(np.float32)
            for v in range(cams.V)]


def _look_at(cam_pos: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    fwd = -cam_pos / np.linalg.norm(cam_pos)
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(fwd @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])          # rows: camera x, y, z in world coords
    t = -R @ cam_pos
    return R, t


def fibonacci_cameras(V: int, W: int, H: int, *, radius: float = 4.0,
                      fov_x_deg: float = 60.0, phase: float = 0.0) -> Cameras:
    """V pinhole cameras on a Fibonacci lattice of a sphere, looking at the
    origin, up +z (+y near the poles), horizontal field of view fov_x,
    fx = fy = (W/2)/tan(fov_x/2), principal point at the image centre.
    ``phase`` rotates the lattice about z (disjoint lattices for subsets)."""
    golden = math.pi * (3.0 - math.sqrt(5.0))
    f = (W / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    Rs, ts = [], []
    for i in range(V):
        zc = 1.0 - 2.0 * (i + 0.5) / V
        rc = math.sqrt(max(0.0, 1.0 - zc * zc))
        phi = i * golden + phase
        pos = radius * np.array([rc * math.cos(phi), rc * math.sin(phi), zc])
        R, t = _look_at(pos)
        Rs.append(R)
        ts.append(t)
    f32 = np.float32
    return Cameras(np.asarray(Rs, dtype=f32), np.asarray(ts, dtype=f32),
                   np.full(V, f, f32), np.full(V, f, f32),
                   np.full(V, W / 2.0, f32), np.full(V, H / 2.0, f32),
                   np.full(V, W, np.int32), np.full(V, H, np.int32))


# Workload shapes used by the tests and the benchmark.  Each entry lists the
# scene size, SH degree, and the image subsets (views, width, height).
CONFIGS = {
    # tiny plain-method scene: 2,048 Gaussians, SH 0, 4 views 64x64, one subset
    "tiny": dict(N=2048, deg=0, seed=1, subsets=[(4, 64, 64)], n_iters=10, lam=1e-2),
    # paper-scale plain method: 1M Gaussians, SH 3, 32 views 1024x640, one subset
    "paper": dict(N=1_000_000, deg=3, seed=2, subsets=[(32, 1024, 640)], n_iters=8, lam=1e-2, lm_steps=5),
    # precision study: 20k Gaussians, SH 0, 4 views 128x128
    "precision": dict(N=20_000, deg=0, seed=3, subsets=[(4, 128, 128)], n_iters=10, lam=1e-2),
    # uneven batched subsets: 1.5M Gaussians, SH 3
    "batching": dict(N=1_500_000, deg=3, seed=4,
                     subsets=[(16, 512, 384), (24, 800, 600), (32, 1024, 640), (48, 1280, 720)],
                     n_iters=8, lam=1e-2),
    # learned-preconditioner deployment: 3M Gaussians, SH 3, 4 x 40 views 1280x720
    "learned": dict(N=3_000_000, deg=3, seed=5, subsets=[(40, 1280, 720)] * 4, n_iters=8, lam=1e-2),
}


def config_scene(name: str, *, N: int | None = None, subsets=None, seed: int | None = None,
                 deg: int | None = None):
    """Scene, per-subset cameras, perturbed parameters and per-subset pixel
    noise for a named workload (sizes may be overridden for smaller runs).
    Subsets get disjoint lattices (phase offset per subset)."""
    cfg = dict(CONFIGS[name])
    N = cfg["N"] if N is None else N
    subsets = cfg["subsets"] if subsets is None else subsets
    seed = cfg["seed"] if seed is None else seed
    deg = cfg["deg"] if deg is None else deg
    scene, rng = make_scene(N, deg, seed)
    cams = [fibonacci_cameras(v, w, h, phase=0.37 * i) for i, (v, w, h) in enumerate(subsets)]
    x_star = perturb(scene, rng)
    noise = [pixel_noise(rng, c) for c in cams]
    return dict(scene=scene, cams=cams, x_star=x_star, noise=noise, cfg=cfg)
