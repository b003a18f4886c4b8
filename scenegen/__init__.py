"""Seeded synthetic scenes and camera sets for object-aware Gaussian splatting.

This module only draws random inputs. It contains none of the scoring
arithmetic (projection, compositing, Jacobians, information gain): both the
FP64 oracle under ``oracle/`` and the HIP path read the arrays it returns.

Scene structure follows the paper's setting (Sec. III-A, Sec. IV-A):
Gaussians with mean, log-scale, raw quaternion, opacity logit, SH degree-0
colour and an object-logit vector of length K = n + 1 (ids 1..n are objects,
0 is background, Sec. III-A.1). Dense object clusters stand in for the
cluttered BlenderProc / GraspNet scenes; candidate cameras sit on a sphere
about the scene centre, half on an equal-latitude ring ("spiral" views) and
half at random (Sec. IV-A.1); the training set is 4 initial views biased to one
side (Sec. IV-A.3).

Every array is float32, structure-of-arrays: ``mean[3][n]``,
``log_scale[3][n]``, ``rot[4][n]`` (w, x, y, z), ``opacity_logit[n]``,
``rgb[3][n]``, ``obj_logit[k][n]``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

CAMERA_STREAM_OFFSET = 1_000_003
TARGET_POOL = 16  # object-centric targets are drawn among this many highest object clusters


@dataclasses.dataclass(frozen=True)
class SceneConfig:
    """Sizes and distributions of one synthetic workload."""
    name: str
    n: int                      # Gaussians
    clusters: int               # object clusters C
    k: int                      # object-vector length K
    n_views: int                # candidate views
    resolutions: tuple          # ((W, H, count), ...) in candidate order
    focal_at_640: float         # fx = fy = focal_at_640 * W / 640
    radius: tuple               # (lo, hi) camera distance in metres
    object_centric: bool = False
    n_train: int = 4


CONFIGS = {
    # 2k Gaussians, 8 clusters, K = 16, 8 views at 128x96 with f = 100.
    "tiny": SceneConfig("tiny", 2_000, 8, 16, 8, ((128, 96, 8),), 100.0 * 640 / 128, (0.6, 0.6)),
    # 200k Gaussians, 32 clusters, K = 32, 64 views at 640x480, f = 525.
    "mid": SceneConfig("mid", 200_000, 32, 32, 64, ((640, 480, 64),), 525.0, (0.6, 0.6)),
    # 1M Gaussians, 64 clusters, K = 64, 256 mixed-resolution views, radius U[0.4, 0.9],
    # object-centric on a seeded target.
    "batched": SceneConfig("batched", 1_000_000, 64, 64, 256,
                           ((320, 240, 86), (640, 480, 85), (1280, 720, 85)), 525.0, (0.4, 0.9),
                           object_centric=True),
    # 1M-Gaussian scene scored at 640x480 only (the 640x480 share of "batched").
    "batched640": SceneConfig("batched640", 1_000_000, 64, 64, 85, ((640, 480, 85),), 525.0,
                              (0.4, 0.9), object_centric=True),
    # 500k Gaussians, 32 clusters, 8 views at 640x480 (differentiation workload).
    "diff": SceneConfig("diff", 500_000, 32, 32, 8, ((640, 480, 8),), 525.0, (0.6, 0.6)),
    # 1M Gaussians, 2048 views at 80x60 (surrogate feature maps).
    "surrogate": SceneConfig("surrogate", 1_000_000, 64, 64, 2048, ((80, 60, 2048),), 525.0,
                             (0.6, 0.6)),
}


@dataclasses.dataclass
class Scene:
    n: int
    k: int
    mean: np.ndarray            # [3][n] f32
    log_scale: np.ndarray       # [3][n] f32
    rot: np.ndarray             # [4][n] f32, unit quaternion (w, x, y, z)
    opacity_logit: np.ndarray   # [n] f32
    rgb: np.ndarray             # [3][n] f32
    obj_logit: np.ndarray       # [k][n] f32
    cluster: np.ndarray         # [n] i32, object channel of each Gaussian
    confidence: np.ndarray      # [n] f32, the drawn per-Gaussian confidence U[0, 1)
    target: int = -1            # seeded target object id (object-centric), else -1


@dataclasses.dataclass
class Camera:
    R: np.ndarray               # [3][3] world -> camera, rows are camera axes (x right, y down, z fwd)
    t: np.ndarray               # [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def packed(self) -> np.ndarray:
        """Camera as 16 float32: R (9, row-major), t (3), fx, fy, cx, cy."""
        return np.concatenate([self.R.reshape(-1), self.t,
                               [self.fx, self.fy, self.cx, self.cy]]).astype(np.float32)


def make_scene(n: int, clusters: int, k: int, seed: int, object_centric: bool = False,
               cube: float = 0.2, spread: float = 0.05,
               scale_range: tuple = (0.002, 0.02)) -> Scene:
    """Draw one clustered scene.

    Draw order (fixed): cluster centres U[-cube, cube]^3; a permutation that
    assigns Gaussian g to cluster perm[g] mod C (equal sizes); means
    N(centre, spread^2) per axis; log-scales U[ln lo, ln hi] per axis;
    quaternions N(0, I4) normalised; opacity logits N(0, 1); colours U[0, 1)^3;
    confidences q ~ U[0, 1); the target id (object-centric workloads only).

    The object vector is one-hot by cluster and tempered by the confidence:
    logits o = log(q e_c + (1 - q)/K), so that softmax(o) equals that mixture
    exactly. Cluster c maps to channel c; channel 0 doubles as background.
    A target id, if asked for, is drawn last, uniformly from the TARGET_POOL object clusters
    (ids >= 1; channel 0 is the background) whose centres are highest: a target is specified
    from what the initial views observe, and a uniform draw over every object would often
    land on one buried at the bottom of the pile, which no elevated view sees.
    """
    if k < clusters:
        raise ValueError("object-vector length must cover every cluster")
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(-cube, cube, size=(clusters, 3))
    perm = rng.permutation(n)
    cluster = (perm % clusters).astype(np.int32)
    mean = centres[cluster] + rng.normal(0.0, spread, size=(n, 3))
    log_scale = rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]), size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity_logit = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    conf = rng.uniform(0.0, 1.0, size=n)
    mix = np.broadcast_to(((1.0 - conf) / k)[:, None], (n, k)).copy()
    mix[np.arange(n), cluster] += conf
    obj_logit = np.log(mix)
    target = -1
    if object_centric:
        pool = 1 + np.argsort(-centres[1:, 2], kind="stable")[:min(TARGET_POOL, clusters - 1)]
        target = int(pool[rng.integers(0, len(pool))])
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(n=n, k=k, mean=f32(mean.T), log_scale=f32(log_scale.T), rot=f32(q.T),
                 opacity_logit=f32(opacity_logit), rgb=f32(rgb.T), obj_logit=f32(obj_logit.T),
                 cluster=cluster, confidence=f32(conf), target=target)


def look_at(eye: np.ndarray, width: int, height: int, focal: float,
            target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> Camera:
    """Pinhole camera at ``eye`` looking at ``target``; OpenCV axes, zero roll."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    t = (-R.astype(np.float64) @ eye).astype(np.float32)
    return Camera(R=R, t=t, fx=float(np.float32(focal)), fy=float(np.float32(focal)),
                  cx=width / 2.0, cy=height / 2.0, width=width, height=height)


def _sphere_point(radius: float, elev: float, azim: float) -> np.ndarray:
    return radius * np.array([math.cos(elev) * math.cos(azim),
                              math.cos(elev) * math.sin(azim), math.sin(elev)])


def make_cameras(cfg: SceneConfig, seed: int):
    """Candidate and training cameras for ``cfg`` from their own seeded stream.

    Candidates: the first half on a ring at elevation 30 degrees with even
    azimuths and a seeded offset, the second half with elevation U[10, 80]
    degrees and azimuth U[0, 2 pi). Resolutions are assigned in the order of
    ``cfg.resolutions``. Training views: ``cfg.n_train`` views at elevation 45
    degrees inside one 90-degree azimuth sector. Radii are U[lo, hi].
    Returns (candidates, training) lists of Camera.
    """
    rng = np.random.Generator(np.random.PCG64(seed + CAMERA_STREAM_OFFSET))
    v = cfg.n_views
    n_ring = v // 2
    offset = rng.uniform(0.0, 2 * math.pi)
    lo, hi = cfg.radius
    res = []
    for (w, h, cnt) in cfg.resolutions:
        res += [(w, h)] * cnt
    assert len(res) == v
    cands: List[Camera] = []
    radii = rng.uniform(lo, hi, size=v)
    rand_el = rng.uniform(math.radians(10), math.radians(80), size=v - n_ring)
    rand_az = rng.uniform(0.0, 2 * math.pi, size=v - n_ring)
    for i in range(v):
        if i < n_ring:
            el, az = math.radians(30), offset + 2 * math.pi * i / max(n_ring, 1)
        else:
            el, az = rand_el[i - n_ring], rand_az[i - n_ring]
        w, h = res[i]
        cands.append(look_at(_sphere_point(radii[i], el, az), w, h, cfg.focal_at_640 * w / 640.0))
    sector = rng.uniform(0.0, 2 * math.pi)
    t_az = sector + rng.uniform(0.0, math.pi / 2, size=cfg.n_train)
    t_r = rng.uniform(lo, hi, size=cfg.n_train)
    w0, h0 = cfg.resolutions[len(cfg.resolutions) // 2][:2]
    train = [look_at(_sphere_point(t_r[i], math.radians(45), t_az[i]), w0, h0,
                     cfg.focal_at_640 * w0 / 640.0) for i in range(cfg.n_train)]
    return cands, train


def make_workload(name: str, seed: int = 0, n_views: Optional[int] = None):
    """(cfg, scene, candidates, training) for a named workload."""
    cfg = CONFIGS[name]
    scene = make_scene(cfg.n, cfg.clusters, cfg.k, seed, object_centric=cfg.object_centric)
    cands, train = make_cameras(cfg, seed)
    if n_views is not None:
        cands = cands[:n_views]
    return cfg, scene, cands, train


def tiny_scene(means, log_scales, quats, opacity_logits, rgbs, obj_logits) -> Scene:
    """Hand-built scene from per-Gaussian rows (used by closed-form tests)."""
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64).T, dtype=np.float32)
    ol = np.asarray(obj_logits, dtype=np.float64)
    n, k = ol.shape
    return Scene(n=n, k=k, mean=f32(means), log_scale=f32(log_scales), rot=f32(quats),
                 opacity_logit=np.asarray(opacity_logits, dtype=np.float32),
                 rgb=f32(rgbs), obj_logit=f32(ol), cluster=np.argmax(ol, axis=1).astype(np.int32),
                 confidence=np.ones(n, dtype=np.float32))
