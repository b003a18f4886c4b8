"""FP64 CPU oracle for object-aware next-best-view scoring (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package. The product library never does, and the oracle imports nothing from the
product: the two share only the seeded input generator ``scenegen``.

The arithmetic lives in ``ngs_oracle.cpp`` (plain C++17, FP64, no FMA
contraction); this module builds it with g++ and marshals numpy arrays through
ctypes. Every float32 input (scene, camera, constants) is widened exactly to
FP64, so the oracle sees the same numbers the GPU path sees.

Parity status: every function is pinned by the ``-m "not gpu"`` tests against
closed forms, brute force, finite differences or LAPACK; none is
"parity unpinned" except absolute gains on the paper's own scenes, which the
paper does not print.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ngs_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "_build", "libngs_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no FMA contraction) into oracle/_build/."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int32), ("k", C.c_int32), ("mean", C.c_void_p), ("log_scale", C.c_void_p),
                ("rot", C.c_void_p), ("opacity_logit", C.c_void_p), ("rgb", C.c_void_p),
                ("obj_logit", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Raster(C.Structure):
    _fields_ = [("tile", C.c_int32), ("z_near", C.c_double), ("eps2d", C.c_double),
                ("cutoff_q", C.c_double), ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("t_min", C.c_double), ("amb_rel", C.c_double)]


class _IG(C.Structure):
    _fields_ = [("lambda_prior", C.c_double), ("alpha_obj", C.c_double), ("alpha_opa", C.c_double),
                ("beta_d", C.c_double), ("beta_o", C.c_double), ("target_id", C.c_int32),
                ("outputs", C.c_int32), ("conf_on_train", C.c_int32), ("obj_eq2", C.c_int32),
                ("level", C.c_int32), ("criterion", C.c_int32)]


def _f32(x) -> float:
    return float(np.float32(x))


@dataclass
class RasterParams:
    """Rasterizer constants (3DGS pipeline readings); widened from float32."""
    tile: int = 16
    z_near: float = 0.05
    eps2d: float = 0.3
    cutoff_q: float = 9.0
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    amb_rel: float = 1e-5

    def c(self) -> _Raster:
        return _Raster(self.tile, _f32(self.z_near), _f32(self.eps2d), _f32(self.cutoff_q),
                       _f32(self.alpha_min), _f32(self.alpha_max), _f32(self.t_min), self.amb_rel)


@dataclass
class IGParams:
    """Information-gain constants: alpha_obj = alpha_opa = 0.3, beta_d = 10, beta_o = 1
    (Sec. IV-A.2); lambda_prior is the prior of the Hessian (a reading)."""
    lambda_prior: float = 0.1
    alpha_obj: float = 0.3
    alpha_opa: float = 0.3
    beta_d: float = 10.0
    beta_o: float = 1.0
    target_id: int = -1
    outputs: int = 7
    conf_on_train: int = 1
    obj_eq2: int = 1
    level: int = 2
    criterion: int = 0  # 0: log det (Eq. 6); 1: trace(H^-1)^-1 (the alternative f of Sec. III-B)

    def c(self) -> _IG:
        return _IG(_f32(self.lambda_prior), _f32(self.alpha_obj), _f32(self.alpha_opa), _f32(self.beta_d),
                   _f32(self.beta_o), self.target_id, self.outputs, self.conf_on_train, self.obj_eq2,
                   self.level, self.criterion)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB_PATH)
            P = C.c_void_p
            L.or_gaussian_terms.argtypes = [P, P, P, P, P, P, P]
            L.or_project.argtypes = [P, P, P] + [P] * 8
            L.or_lists.argtypes = [P, P, P, C.c_int64, P, P, P]
            L.or_lists.restype = C.c_int64
            L.or_render.argtypes = [P, P, P, P, C.c_int, C.c_int] + [P] * 9
            L.or_view_blocks.argtypes = [P, P, P, P, C.c_int]
            L.or_view_blocks.restype = C.c_void_p
            L.or_blocks_count.argtypes = [P]
            L.or_blocks_count.restype = C.c_int64
            L.or_blocks_pairs.argtypes = [P]
            L.or_blocks_pairs.restype = C.c_int64
            L.or_blocks_get.argtypes = [P, C.c_int64, P, P, P, P]
            L.or_blocks_free.argtypes = [P]
            L.or_logdet.argtypes = [C.c_int, P]
            L.or_logdet.restype = C.c_double
            L.or_trace_inv.argtypes = [C.c_int, P]
            L.or_trace_inv.restype = C.c_double
            L.or_pixel_rows.argtypes = [P, P, P, P, C.c_int, C.c_int, C.c_int, P, P, P, P]
            L.or_pixel_eval_frozen.argtypes = [P, P, P, P, C.c_int, C.c_int, C.c_int, P, P]
            L.or_score.argtypes = [P, C.c_int, P, C.c_int, P, P, P, C.c_int, P, P, P, P, P, P, P]
            L.or_last_score_seconds.argtypes = [P, C.c_int]
            L.or_last_score_seconds.restype = C.c_int
            L.or_set_setup_threads.argtypes = [C.c_int]
            L.or_train_blocks.argtypes = [P, C.c_int, P, P, P, C.c_int, C.c_int, P, P, P, P, P]
            L.or_render_grad.argtypes = [P, P, P, P, C.c_int, P, P, P, P]
            _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _SceneBuf:
    """Holds FP64 copies of a scenegen.Scene and its C view."""

    def __init__(self, scene):
        d = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.n, self.k = int(scene.n), int(scene.k)
        self.arrs = [d(scene.mean), d(scene.log_scale), d(scene.rot), d(scene.opacity_logit),
                     d(scene.rgb), d(scene.obj_logit)]
        self.c = _Scene(self.n, self.k, *[a.ctypes.data for a in self.arrs])


def _cam(cam) -> _Camera:
    R = np.asarray(cam.R, dtype=np.float32).reshape(-1).astype(np.float64)
    t = np.asarray(cam.t, dtype=np.float32).astype(np.float64)
    return _Camera((C.c_double * 9)(*R), (C.c_double * 3)(*t), _f32(cam.fx), _f32(cam.fy), _f32(cam.cx),
                   _f32(cam.cy), int(cam.width), int(cam.height))


def _cams(cams) -> C.Array:
    arr = (_Camera * max(1, len(cams)))()
    for i, c in enumerate(cams):
        arr[i] = _cam(c)
    return arr


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ------------------------------------------------------------------------------------------
# Public functions
# ------------------------------------------------------------------------------------------

def gaussian_terms(scene, ig: IGParams = IGParams()):
    """p = softmax(o) [n][k], kappa, sigma, c_g (Eq. 7 / Eq. 12), argmax k."""
    sb = _SceneBuf(scene)
    n, k = sb.n, sb.k
    p = np.zeros((n, k)); kap = np.zeros(n); sig = np.zeros(n); conf = np.zeros(n)
    am = np.zeros(n, dtype=np.int32)
    igc = ig.c()
    lib().or_gaussian_terms(C.byref(sb.c), C.byref(igc), _ptr(p), _ptr(kap), _ptr(sig), _ptr(conf), _ptr(am))
    return dict(p=p, kappa=kap, sigma=sig, conf=conf, argmax=am)


def project(scene, cam, rp: RasterParams = RasterParams()):
    """FP64 projection of every Gaussian for one camera."""
    sb = _SceneBuf(scene)
    n = sb.n
    out = dict(z=np.zeros(n), zkey=np.zeros(n, np.uint32), m=np.zeros((2, n)), cov=np.zeros((3, n)),
               conic=np.zeros((3, n)), radius=np.zeros(n, np.int32), rect=np.zeros((4, n), np.int32),
               valid=np.zeros(n, np.uint8))
    cc, rc = _cam(cam), rp.c()
    lib().or_project(C.byref(sb.c), C.byref(cc), C.byref(rc), _ptr(out["z"]), _ptr(out["zkey"]), _ptr(out["m"]),
                     _ptr(out["cov"]), _ptr(out["conic"]), _ptr(out["radius"]), _ptr(out["rect"]),
                     _ptr(out["valid"]))
    return out


def tile_lists(scene, cam, rp: RasterParams = RasterParams()):
    """Sorted (tile, depth, gid) lists: keys u64 [M], gids u32 [M], ranges u32 [2][tiles]."""
    sb = _SceneBuf(scene)
    cc, rc = _cam(cam), rp.c()
    nt = ((cam.width + rp.tile - 1) // rp.tile) * ((cam.height + rp.tile - 1) // rp.tile)
    m = lib().or_lists(C.byref(sb.c), C.byref(cc), C.byref(rc), 0, None, None, None)
    keys = np.zeros(max(m, 1), np.uint64); gids = np.zeros(max(m, 1), np.uint32)
    ranges = np.zeros((2, nt), np.uint32)
    lib().or_lists(C.byref(sb.c), C.byref(cc), C.byref(rc), m, _ptr(keys), _ptr(gids), _ptr(ranges))
    return dict(keys=keys[:m], gids=gids[:m], ranges=ranges, m=int(m))


def render(scene, cam, rp: RasterParams = RasterParams(), ig: IGParams = IGParams(), brute: bool = False,
           threads: Optional[int] = None):
    """FP64 images: rgb [3][H][W], depth, obj (O, Eq. 2) [k][H][W], objp (O', Eq. 1),
    t_final, id (argmax of O), kbar (mean kappa), ncontrib, ambiguous (u8)."""
    sb = _SceneBuf(scene)
    H, W, k = cam.height, cam.width, sb.k
    out = dict(rgb=np.zeros((3, H, W)), depth=np.zeros((H, W)), obj=np.zeros((k, H, W)),
               objp=np.zeros((k, H, W)), t_final=np.zeros((H, W)), id=np.zeros((H, W), np.int32),
               kbar=np.zeros((H, W)), ncontrib=np.zeros((H, W), np.int32),
               ambiguous=np.zeros((H, W), np.uint8))
    cc, rc, igc = _cam(cam), rp.c(), ig.c()
    lib().or_render(C.byref(sb.c), C.byref(cc), C.byref(rc), C.byref(igc), int(brute),
                    threads or default_threads(), *[_ptr(out[x]) for x in
                    ("rgb", "depth", "obj", "objp", "t_final", "id", "kbar", "ncontrib", "ambiguous")])
    return out


def render_grad(scene, cam, g_rgb=None, g_depth=None, g_obj=None, rp: RasterParams = RasterParams(),
                ig: IGParams = IGParams(), threads: Optional[int] = None) -> np.ndarray:
    """FP64 gradient [n][14 + k] (mu 3, log-scale 3, raw quaternion 4, opacity logit 1, rgb 3,
    object logits k) of a loss whose gradients w.r.t. the rendered rgb [3][H][W], depth [H][W]
    and object vector [k][H][W] (O of Eq. 2, or O' when ig.obj_eq2 = 0) are given."""
    sb = _SceneBuf(scene)
    d = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    gr, gd, go = d(g_rgb), d(g_depth), d(g_obj)
    out = np.zeros((sb.n, 14 + sb.k))
    cc, rc, igc = _cam(cam), rp.c(), ig.c()
    lib().or_render_grad(C.byref(sb.c), C.byref(cc), C.byref(rc), C.byref(igc), threads or default_threads(),
                         _ptr(gr) if gr is not None else None, _ptr(gd) if gd is not None else None,
                         _ptr(go) if go is not None else None, _ptr(out))
    return out


@dataclass
class ViewBlocks:
    gids: np.ndarray
    rgb: np.ndarray   # [U][14][14]
    d: np.ndarray     # [U][11][11]
    o: np.ndarray     # [U][11+k][11+k]
    pairs: int


def view_blocks(scene, cam, rp: RasterParams = RasterParams(), ig: IGParams = IGParams(),
                threads: Optional[int] = None) -> ViewBlocks:
    """Unweighted per-Gaussian information blocks A^f_g of one view (Eq. 6)."""
    sb = _SceneBuf(scene)
    cc, rc, igc = _cam(cam), rp.c(), ig.c()
    L = lib()
    h = L.or_view_blocks(C.byref(sb.c), C.byref(cc), C.byref(rc), C.byref(igc), threads or default_threads())
    try:
        u = L.or_blocks_count(h)
        lo = 11 + sb.k
        gids = np.zeros(u, np.int32)
        a_rgb = np.zeros((u, 14, 14)); a_d = np.zeros((u, 11, 11)); a_o = np.zeros((u, lo, lo))
        g = C.c_int32()
        for i in range(u):
            L.or_blocks_get(h, i, C.byref(g), _ptr(a_rgb[i]), _ptr(a_d[i]), _ptr(a_o[i]))
            gids[i] = g.value
        pairs = L.or_blocks_pairs(h)
    finally:
        L.or_blocks_free(h)
    return ViewBlocks(gids, a_rgb, a_d, a_o, int(pairs))


def logdet(A: np.ndarray) -> float:
    A = np.ascontiguousarray(A, dtype=np.float64)
    return float(lib().or_logdet(A.shape[0], _ptr(A)))


def trace_inv(A: np.ndarray) -> float:
    """trace(A^-1) of an SPD matrix by the oracle's Cholesky."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    return float(lib().or_trace_inv(A.shape[0], _ptr(A)))


def pixel_rows(scene, cam, px: int, py: int, rp: RasterParams = RasterParams(), ig: IGParams = IGParams(),
               cap: int = 512):
    """Jacobian rows of every channel at one pixel, for each contributor front to back."""
    sb = _SceneBuf(scene)
    k = sb.k
    cc, rc, igc = _cam(cam), rp.c(), ig.c()
    contrib = np.zeros(cap, np.int32)
    rr = np.zeros((cap, 3, 14)); rd = np.zeros((cap, 11)); ro = np.zeros((cap, k, 11 + k))
    nc = lib().or_pixel_rows(C.byref(sb.c), C.byref(cc), C.byref(rc), C.byref(igc), px, py, cap,
                             _ptr(contrib), _ptr(rr), _ptr(rd), _ptr(ro))
    if nc > cap:
        return pixel_rows(scene, cam, px, py, rp, ig, cap=nc)
    return dict(gids=contrib[:nc], rgb=rr[:nc], d=rd[:nc], o=ro[:nc])


def pixel_eval_frozen(scene, cam, px: int, py: int, seq: Sequence[int], rp: RasterParams = RasterParams(),
                      ig: IGParams = IGParams()) -> np.ndarray:
    """Outputs [rgb 3, depth, object k] at one pixel for a fixed front-to-back sequence."""
    sb = _SceneBuf(scene)
    cc, rc, igc = _cam(cam), rp.c(), ig.c()
    seq = np.ascontiguousarray(seq, dtype=np.int32)
    out = np.zeros(4 + sb.k)
    lib().or_pixel_eval_frozen(C.byref(sb.c), C.byref(cc), C.byref(rc), C.byref(igc), px, py, len(seq),
                               _ptr(seq), _ptr(out))
    return out


@dataclass
class ScoreResult:
    status: int
    ig_train: np.ndarray   # [T][3] raw gains of the training views
    ig_cand: np.ndarray    # [V][3] raw gains of the candidates
    norm: np.ndarray       # [3] Eq. 10 normalisers
    scores: np.ndarray     # [V][4] normalised rgb, depth, object, combined (Eq. 11)
    best: int
    stats: np.ndarray      # [V][2] touched Gaussians U, contributing pairs P
    trace_total: np.ndarray = None  # [3] S_T of the trace criterion (0 for log det)
    seconds: tuple = (0.0, 0.0)     # wall clock: training information + normalisers, candidates
    cand_seconds: np.ndarray = None  # [V] wall clock of each candidate


def score(scene, train_cams, cand_cams, rp: RasterParams = RasterParams(), ig: IGParams = IGParams(),
          threads: Optional[int] = None, setup_threads: int = 0) -> ScoreResult:
    """Full next-best-view scoring of the candidates given the training views. setup_threads
    > 0 runs the training views on that many threads (timing of the candidates alone)."""
    lib().or_set_setup_threads(int(setup_threads))
    sb = _SceneBuf(scene)
    nt, nc = len(train_cams), len(cand_cams)
    tc, cc = _cams(train_cams), _cams(cand_cams)
    rc, igc = rp.c(), ig.c()
    igt = np.zeros((max(nt, 1), 3)); igcand = np.zeros((max(nc, 1), 3)); norm = np.zeros(3)
    sc = np.zeros((max(nc, 1), 4)); best = C.c_int32(-1); stats = np.zeros((max(nc, 1), 2), np.int64)
    tt = np.zeros(3)
    st = lib().or_score(C.byref(sb.c), nt, tc, nc, cc, C.byref(rc), C.byref(igc), threads or default_threads(),
                        _ptr(igt), _ptr(igcand), _ptr(norm), _ptr(sc), C.byref(best), _ptr(stats), _ptr(tt))
    secs = np.zeros(2 + nc)
    lib().or_last_score_seconds(_ptr(secs), 2 + nc)
    lib().or_set_setup_threads(0)
    return ScoreResult(int(st), igt[:nt], igcand[:nc], norm, sc[:nc], int(best.value), stats[:nc], tt,
                       (float(secs[0]), float(secs[1])), secs[2:])


def train_blocks(scene, train_cams, query: Sequence[int], rp: RasterParams = RasterParams(),
                 ig: IGParams = IGParams(), threads: Optional[int] = None):
    """H_T blocks (prior + weighted training information) for the queried Gaussians."""
    sb = _SceneBuf(scene)
    k = sb.k
    lo = 11 + k
    q = np.ascontiguousarray(query, dtype=np.int32)
    nq = len(q)
    hr = np.zeros((nq, 14, 14)); hd = np.zeros((nq, 11, 11)); ho = np.zeros((nq, lo, lo))
    touched = np.zeros(nq, np.uint8)
    tc = _cams(train_cams)
    rc, igc = rp.c(), ig.c()
    lib().or_train_blocks(C.byref(sb.c), len(train_cams), tc, C.byref(rc), C.byref(igc),
                          threads or default_threads(), nq, _ptr(q), _ptr(hr), _ptr(hd), _ptr(ho), _ptr(touched))
    return dict(rgb=hr, d=hd, o=ho, touched=touched.astype(bool))
