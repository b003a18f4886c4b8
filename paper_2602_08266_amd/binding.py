"""ctypes binding of libngs (include/ngs.h): argument marshalling only.

Every step of the scoring path runs in the HIP kernels of libngs.so; this module only
allocates device buffers with torch, fills the C structs and calls the entry points with
the same names. It raises when the library has not been built: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NGS_LIB") or os.path.join(HERE, "_build", "libngs.so")

NGS_OK, NGS_INVALID_ARG, NGS_CAPACITY, NGS_WORKSPACE_TOO_SMALL = 0, -1, -2, -3
NGS_HIP_ERROR, NGS_DEGENERATE, NGS_UNSUPPORTED = -4, -5, -6
MODE_SCORE, MODE_ACCUMULATE = 0, 1
OUT_RGB, OUT_DEPTH, OUT_OBJ = 1, 2, 4
STATS_LEN = 14
EXPORTS = ["ngs_create", "ngs_destroy", "ngs_status_string", "ngs_version", "ngs_last_hip_error",
           "ngs_workspace_size", "ngs_prepare_scene", "ngs_project", "ngs_count_pairs", "ngs_bin_sort", "ngs_render",
           "ngs_info_gain", "ngs_info_gain_static", "ngs_hessian_reset", "ngs_hessian_finalize", "ngs_training_setup", "ngs_score_batch",
           "ngs_score_graph_create", "ngs_score_graph_launch", "ngs_score_graph_destroy", "ngs_set_tuning",
           "ngs_get_tuning",
           "ngs_render_backward", "ngs_profile_enable", "ngs_profile_enable_class", "ngs_profile_kernels", "ngs_profile_kernel_name",
           "ngs_profile_read", "ngs_sur_workspace_size", "ngs_sur_sync_bf16", "ngs_sur_forward", "ngs_sur_backward",
           "ngs_sur_mse", "ngs_sur_adam", "ngs_sur_features", "ngs_sur_novelty", "ngs_sur_render_features", "ngs_sur_pick", "ngs_gemm_bf16"]


class NgsError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed: {msg} ({status})")
        self.status = status


P = C.c_void_p


class ngs_scene(C.Structure):
    _fields_ = [("n", C.c_int32), ("k", C.c_int32), ("mean", P), ("log_scale", P), ("rot", P),
                ("opacity_logit", P), ("rgb", P), ("obj_logit", P), ("prob", P), ("opacity", P),
                ("kappa", P), ("conf", P), ("label", P), ("cov3", P)]


class ngs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class ngs_raster_params(C.Structure):
    _fields_ = [("tile", C.c_int32), ("z_near", C.c_float), ("eps2d", C.c_float), ("cutoff_q", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float)]


class ngs_ig_params(C.Structure):
    _fields_ = [("lambda_prior", C.c_float), ("alpha_obj", C.c_float), ("alpha_opa", C.c_float),
                ("beta_d", C.c_float), ("beta_o", C.c_float), ("target_id", C.c_int32), ("outputs", C.c_uint32),
                ("conf_on_train", C.c_int32), ("obj_eq2", C.c_int32), ("mode", C.c_int32),
                ("criterion", C.c_int32), ("trace_total", C.c_double * 3)]


class ngs_projected(C.Structure):
    _fields_ = [("mean2d", P), ("conic", P), ("depth", P), ("zkey", P), ("rect", P), ("count", P), ("splat", P)]


class ngs_tile_lists(C.Structure):
    _fields_ = [("keys", P), ("gids", P), ("capacity", C.c_int64), ("n_pairs", P), ("ranges", P)]


class ngs_image(C.Structure):
    _fields_ = [("rgb", P), ("depth", P), ("obj", P), ("t_final", P), ("mean_conf", P), ("argmax_id", P),
                ("n_contrib", P)]


class ngs_hessian(C.Structure):
    _fields_ = [("k", C.c_int32), ("capacity", C.c_int32), ("slot_of", P), ("n_slots", P), ("gid_of", P),
                ("h_rgb", P), ("h_d", P), ("h_o", P), ("logdet", P), ("trinv", P)]


class ngs_image_grad(C.Structure):
    _fields_ = [("rgb", P), ("depth", P), ("obj", P)]


class ngs_scene_grad(C.Structure):
    _fields_ = [("mean", P), ("log_scale", P), ("rot", P), ("opacity_logit", P), ("rgb", P), ("obj_logit", P)]


SUR_LAYERS, SUR_WIDTH, SUR_IN = 6, 128, (4, 60, 80)
# (in, out, kernel taps) of the surrogate's layers: four 3x3 convolutions, two fully connected
SUR_SHAPES = [(4, 32, 9), (32, 64, 9), (64, 128, 9), (128, 128, 9), (128, 128, 1), (128, 1, 1)]


class ngs_sur_params(C.Structure):
    _fields_ = [("w", P * SUR_LAYERS), ("b", P * SUR_LAYERS), ("w_bf16", P * SUR_LAYERS)]


class ngs_dims(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int64), ("width", C.c_int64), ("height", C.c_int64),
                ("max_pairs", C.c_int64), ("max_slots", C.c_int64), ("views_in_flight", C.c_int64)]


_lib = None


def lib():
    """Loads libngs.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        i32 = C.c_int32
        L.ngs_create.argtypes = [C.c_int, C.POINTER(P)]
        L.ngs_destroy.argtypes = [P]
        L.ngs_status_string.argtypes = [i32]
        L.ngs_status_string.restype = C.c_char_p
        L.ngs_version.restype = i32
        L.ngs_last_hip_error.argtypes = [P]
        L.ngs_last_hip_error.restype = i32
        L.ngs_workspace_size.argtypes = [i32, P, C.POINTER(C.c_size_t)]
        L.ngs_prepare_scene.argtypes = [P, P, P, P]
        L.ngs_project.argtypes = [P, P, P, P, P, P]
        L.ngs_bin_sort.argtypes = [P, P, P, P, P, P, P, C.c_size_t, P]
        L.ngs_count_pairs.argtypes = [P, P, P, i32, P, P, P, C.c_size_t, P]
        L.ngs_render.argtypes = [P, P, P, P, P, P, P, P]
        L.ngs_info_gain.argtypes = [P, P, P, P, P, P, P, P, P, P, P, C.c_size_t, P]
        L.ngs_info_gain_static.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
        L.ngs_hessian_reset.argtypes = [P, P, i32, P]
        L.ngs_hessian_finalize.argtypes = [P, P, P]
        L.ngs_score_batch.argtypes = [P, P, P, P, P, i32, P, P, P, P, P, P, P, P, C.c_size_t, P]
        L.ngs_training_setup.argtypes = [P, P, P, P, i32, P, P, P, P, P, P, P, C.c_size_t, P]
        L.ngs_score_graph_create.argtypes = [P, P, P, P, P, i32, P, P, P, P, P, P, P, P, P, C.c_size_t,
                                             C.POINTER(P)]
        L.ngs_score_graph_launch.argtypes = [P, P]
        L.ngs_set_tuning.argtypes = [P, P]
        L.ngs_get_tuning.argtypes = [P, P]
        L.ngs_score_graph_destroy.argtypes = [P]
        L.ngs_render_backward.argtypes = [P, P, P, P, P, P, i32, P, P, P, C.c_size_t, P]
        L.ngs_sur_workspace_size.argtypes = [i32, C.POINTER(C.c_size_t)]
        L.ngs_sur_sync_bf16.argtypes = [P, P, P]
        L.ngs_sur_forward.argtypes = [P, P, P, i32, P, P, C.c_size_t, P]
        L.ngs_sur_backward.argtypes = [P, P, P, i32, P, P, P, C.c_size_t, P]
        L.ngs_sur_mse.argtypes = [P, P, P, i32, P, P, P]
        L.ngs_sur_adam.argtypes = [P, P, P, P, P, C.c_float, C.c_float, C.c_float, C.c_float, i32, P]
        L.ngs_sur_features.argtypes = [P, P, i32, i32, i32, C.c_float, P, i32, i32, P]
        L.ngs_sur_novelty.argtypes = [P, P, P, C.c_float, P, P]
        L.ngs_sur_render_features.argtypes = [P, P, P, i32, P, P, C.c_float, P, P, P, C.c_size_t, P]
        L.ngs_gemm_bf16.argtypes = [P, i32, i32, i32, i32, i32, P, i32, P, i32, P, i32, C.c_float, P]
        L.ngs_sur_pick.argtypes = [P, P, P, P, P, i32, P, i32, P, P, P, P, P, P, P, P, P, C.c_size_t, P]
        L.ngs_profile_enable.argtypes = [P, i32]
        L.ngs_profile_enable_class.argtypes = [P, i32]
        L.ngs_profile_kernels.restype = i32
        L.ngs_profile_kernel_name.argtypes = [i32]
        L.ngs_profile_kernel_name.restype = C.c_char_p
        L.ngs_profile_read.argtypes = [P, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        for name in EXPORTS:
            if name not in ("ngs_status_string", "ngs_version", "ngs_last_hip_error", "ngs_profile_kernels",
                            "ngs_profile_kernel_name"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(fn: str, status: int, ctx=None):
    if status != NGS_OK:
        msg = lib().ngs_status_string(status).decode()
        if ctx is not None and status == NGS_HIP_ERROR:
            msg += f" (hipError {lib().ngs_last_hip_error(ctx.handle)})"
        raise NgsError(fn, status, msg)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stats(t: Optional[torch.Tensor]):
    """Pointer of a statistics tensor: int64, contiguous, on the GPU, NGS_STATS_LEN long."""
    if t is None:
        return None
    if t.dtype != torch.int64 or not t.is_contiguous() or not t.is_cuda or t.numel() < STATS_LEN:
        raise ValueError(f"stats must be a contiguous int64 GPU tensor of {STATS_LEN} entries")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ref(x):
    return C.byref(x)


# ------------------------------------------------------------------------------------------
# Parameter structs
# ------------------------------------------------------------------------------------------

def raster_params(tile=16, z_near=0.05, eps2d=0.3, cutoff_q=9.0, alpha_min=1.0 / 255.0, alpha_max=0.99,
                  t_min=1e-4) -> ngs_raster_params:
    return ngs_raster_params(tile, z_near, eps2d, cutoff_q, alpha_min, alpha_max, t_min)


def ig_params(lambda_prior=0.1, alpha_obj=0.3, alpha_opa=0.3, beta_d=10.0, beta_o=1.0, target_id=-1,
              outputs=7, conf_on_train=1, obj_eq2=1, mode=MODE_SCORE, criterion=0) -> ngs_ig_params:
    """criterion: 0 = log det (Eq. 6), 1 = trace(H^-1)^-1 (trace_total is filled by NbvScorer.setup)."""
    return ngs_ig_params(lambda_prior, alpha_obj, alpha_opa, beta_d, beta_o, target_id, outputs, conf_on_train,
                         obj_eq2, mode, criterion, (C.c_double * 3)(0.0, 0.0, 0.0))


def camera(cam) -> ngs_camera:
    """ngs_camera from an object with R (3x3), t (3), fx, fy, cx, cy, width, height."""
    import numpy as np
    R = np.asarray(cam.R, dtype=np.float32).reshape(-1)
    t = np.asarray(cam.t, dtype=np.float32).reshape(-1)
    return ngs_camera((C.c_float * 9)(*R.tolist()), (C.c_float * 3)(*t.tolist()), cam.fx, cam.fy, cam.cx, cam.cy,
                      int(cam.width), int(cam.height))


# ------------------------------------------------------------------------------------------
# Context and device-resident objects
# ------------------------------------------------------------------------------------------

class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check("ngs_create", lib().ngs_create(device, C.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().ngs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceScene:
    """Scene arrays resident on the GPU (float32 SoA) plus the derived arrays."""

    def __init__(self, scene, device: str = "cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        self.n, self.k = int(scene.n), int(scene.k)
        self.mean, self.log_scale, self.rot = f(scene.mean), f(scene.log_scale), f(scene.rot)
        self.opacity_logit, self.rgb, self.obj_logit = f(scene.opacity_logit), f(scene.rgb), f(scene.obj_logit)
        n, k = self.n, self.k
        self.prob = torch.empty((max(n, 1), k), dtype=torch.float32, device=device)
        self.opacity = torch.empty(max(n, 1), dtype=torch.float32, device=device)
        self.kappa = torch.empty_like(self.opacity)
        self.conf = torch.empty_like(self.opacity)
        self.label = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.cov3 = None  # allocated by ngs_prepare_scene, which fills it
        self.device = device

    def c(self) -> ngs_scene:
        return ngs_scene(self.n, self.k, _p(self.mean), _p(self.log_scale), _p(self.rot), _p(self.opacity_logit),
                         _p(self.rgb), _p(self.obj_logit), _p(self.prob), _p(self.opacity), _p(self.kappa),
                         _p(self.conf), _p(self.label), _p(getattr(self, "cov3", None)))


@dataclass
class Projected:
    mean2d: torch.Tensor
    conic: torch.Tensor
    depth: torch.Tensor
    zkey: torch.Tensor
    rect: torch.Tensor
    count: torch.Tensor
    splat: Optional[torch.Tensor] = None

    def c(self) -> ngs_projected:
        return ngs_projected(_p(self.mean2d), _p(self.conic), _p(self.depth), _p(self.zkey), _p(self.rect),
                             _p(self.count), _p(self.splat))


@dataclass
class TileLists:
    keys: Optional[torch.Tensor]
    gids: torch.Tensor
    n_pairs: torch.Tensor
    ranges: torch.Tensor
    capacity: int

    def c(self) -> ngs_tile_lists:
        return ngs_tile_lists(_p(self.keys), _p(self.gids), self.capacity, _p(self.n_pairs), _p(self.ranges))


class Hessian:
    """Training information store H_T (packed FP64 blocks of the touched Gaussians)."""

    def __init__(self, n: int, k: int, capacity: int, device: str = "cuda"):
        lo = 11 + k
        cap = max(int(capacity), 1)
        self.k, self.capacity = k, int(capacity)
        self.slot_of = torch.full((max(n, 1),), -1, dtype=torch.int32, device=device)
        self.n_slots = torch.zeros(1, dtype=torch.int32, device=device)
        self.gid_of = torch.full((cap,), -1, dtype=torch.int32, device=device)
        self.h_rgb = torch.zeros((cap, 105), dtype=torch.float64, device=device)
        self.h_d = torch.zeros((cap, 66), dtype=torch.float64, device=device)
        self.h_o = torch.zeros((cap, 68 + 12 * k), dtype=torch.float64, device=device)
        self.logdet = torch.zeros((3, cap), dtype=torch.float64, device=device)
        self.trinv = torch.zeros((3, cap), dtype=torch.float64, device=device)

    def c(self) -> ngs_hessian:
        return ngs_hessian(self.k, self.capacity, _p(self.slot_of), _p(self.n_slots), _p(self.gid_of),
                           _p(self.h_rgb), _p(self.h_d), _p(self.h_o), _p(self.logdet), _p(self.trinv))


def workspace_size(op: int, n: int, k: int, width: int = 0, height: int = 0, max_pairs: int = 0,
                   max_slots: int = 0, views_in_flight: int = 0) -> int:
    d = ngs_dims(n, k, width, height, max_pairs, max_slots, views_in_flight)
    b = C.c_size_t()
    _check("ngs_workspace_size", lib().ngs_workspace_size(op, _ref(d), C.byref(b)))
    return int(b.value)


def _bytes(nbytes: int, device: str = "cuda") -> torch.Tensor:
    try:
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    except torch.OutOfMemoryError:
        # blocks cached by torch's allocator from earlier (freed) workspaces of other sizes
        # can leave no contiguous range free: hand them back to the device and try once more
        torch.cuda.empty_cache()
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ------------------------------------------------------------------------------------------

def ngs_prepare_scene(ctx: Context, scene: DeviceScene, ig: ngs_ig_params):
    if getattr(scene, "cov3", None) is None:
        scene.cov3 = torch.empty((9, max(scene.n, 1)), dtype=torch.float64, device=scene.device)
    sc = scene.c()
    _check("ngs_prepare_scene", lib().ngs_prepare_scene(ctx.handle, _ref(sc), _ref(ig), _stream()), ctx)


def ngs_project(ctx: Context, scene: DeviceScene, cam: ngs_camera, rp: ngs_raster_params) -> Projected:
    n, dev = max(scene.n, 1), scene.device
    out = Projected(torch.empty((2, n), dtype=torch.float32, device=dev),
                    torch.empty((3, n), dtype=torch.float32, device=dev),
                    torch.empty(n, dtype=torch.float32, device=dev),
                    torch.empty(n, dtype=torch.int32, device=dev),
                    torch.empty((n, 4), dtype=torch.int16, device=dev),
                    torch.empty(n, dtype=torch.int32, device=dev),
                    torch.empty((n, 8), dtype=torch.float32, device=dev))
    sc, pc = scene.c(), out.c()
    _check("ngs_project", lib().ngs_project(ctx.handle, _ref(sc), _ref(cam), _ref(rp), _ref(pc), _stream()), ctx)
    return out


def ngs_bin_sort(ctx: Context, scene: DeviceScene, proj: Projected, cam: ngs_camera, rp: ngs_raster_params,
                 capacity: int = 1 << 20, want_keys: bool = False) -> TileLists:
    """Sorted tile lists; grows the capacity and retries when the library reports CAPACITY."""
    dev = scene.device
    tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    while True:
        cap = max(int(capacity), 1)
        lists = TileLists(torch.empty(cap, dtype=torch.int64, device=dev) if want_keys else None,
                          torch.empty(cap, dtype=torch.int32, device=dev),
                          torch.zeros(1, dtype=torch.int64, device=dev),
                          torch.empty((2, max(tiles, 1)), dtype=torch.int32, device=dev), cap)
        ws = _bytes(workspace_size(0, scene.n, scene.k, max_pairs=cap), dev)
        sc, pc, lc = scene.c(), proj.c(), lists.c()
        st = lib().ngs_bin_sort(ctx.handle, _ref(sc), _ref(pc), _ref(cam), _ref(rp), _ref(lc), _p(ws),
                                ws.numel(), _stream())
        if st == NGS_CAPACITY:
            capacity = int(lists.n_pairs.item())
            continue
        _check("ngs_bin_sort", st, ctx)
        return lists


def ngs_count_pairs(ctx: Context, scene: DeviceScene, cams: Sequence[ngs_camera], rp: ngs_raster_params,
                    ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Pair count M of every candidate (device int64 [V]): the capacity pre-pass of a batch."""
    nv = len(cams)
    pairs = torch.zeros(max(nv, 1), dtype=torch.int64, device=scene.device)
    if ws is None:
        ws = _bytes(workspace_size(5, scene.n, scene.k), scene.device)
    arr = (ngs_camera * max(nv, 1))(*cams)
    sc = scene.c()
    _check("ngs_count_pairs", lib().ngs_count_pairs(ctx.handle, _ref(sc), arr, nv, _ref(rp), _p(pairs), _p(ws),
                                                    ws.numel(), _stream()), ctx)
    return pairs[:nv]


def ngs_render(ctx: Context, scene: DeviceScene, proj: Projected, lists: TileLists, cam: ngs_camera,
               rp: ngs_raster_params, want_obj: bool = True) -> Dict[str, torch.Tensor]:
    H, W, dev = cam.height, cam.width, scene.device
    f = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
    out = dict(rgb=f(3, H, W), depth=f(H, W), obj=f(scene.k, H, W) if want_obj else None, t_final=f(H, W),
               mean_conf=f(H, W), argmax_id=torch.empty((H, W), dtype=torch.int32, device=dev),
               n_contrib=torch.empty((H, W), dtype=torch.int32, device=dev))
    img = ngs_image(*[_p(out[x]) for x in ("rgb", "depth", "obj", "t_final", "mean_conf", "argmax_id",
                                           "n_contrib")])
    sc, pc, lc = scene.c(), proj.c(), lists.c()
    _check("ngs_render", lib().ngs_render(ctx.handle, _ref(sc), _ref(pc), _ref(lc), _ref(cam), _ref(rp), _ref(img),
                                          _stream()), ctx)
    return out


def ngs_render_backward(ctx: Context, scene: DeviceScene, proj: Projected, lists: TileLists, cam: ngs_camera,
                        rp: ngs_raster_params, g_rgb: Optional[torch.Tensor] = None,
                        g_depth: Optional[torch.Tensor] = None, g_obj: Optional[torch.Tensor] = None,
                        obj_eq2: bool = True, ws: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
    """dL/d(scene parameters) from dL/d(rendered rgb [3][H][W], depth [H][W], obj [k][H][W])."""
    n, k, dev = max(scene.n, 1), scene.k, scene.device
    f = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
    out = dict(mean=f(3, n), log_scale=f(3, n), rot=f(4, n), opacity_logit=f(n), rgb=f(3, n), obj_logit=f(k, n))
    gi = [None if x is None else x.detach().to(torch.float32).contiguous() for x in (g_rgb, g_depth, g_obj)]
    if ws is None:
        ws = _bytes(workspace_size(3, scene.n, scene.k), dev)
    img = ngs_image_grad(*[_p(x) for x in gi])
    sgr = ngs_scene_grad(*[_p(out[x]) for x in ("mean", "log_scale", "rot", "opacity_logit", "rgb", "obj_logit")])
    sc, pc, lc = scene.c(), proj.c(), lists.c()
    _check("ngs_render_backward", lib().ngs_render_backward(ctx.handle, _ref(sc), _ref(pc), _ref(lc), _ref(cam),
                                                            _ref(rp), int(bool(obj_eq2)), _ref(img), _ref(sgr),
                                                            _p(ws), ws.numel(), _stream()), ctx)
    return out


class RenderFunction(torch.autograd.Function):
    """Differentiable tile rasterizer of one view: scene parameter tensors (float32 SoA on the
    GPU: mean [3][n], log_scale [3][n], rot [4][n], opacity_logit [n], rgb [3][n], obj_logit
    [k][n]) -> rgb [3][H][W], depth [H][W], obj [k][H][W] (O of Eq. 2). Forward and backward
    run in libngs; the lists are rebuilt from the current parameters on every forward."""

    @staticmethod
    def forward(fctx, mean, log_scale, rot, opacity_logit, rgb, obj_logit, ctx, cam, rp, capacity):
        ds = DeviceScene.__new__(DeviceScene)
        ds.n, ds.k, ds.device = int(mean.shape[1]), int(obj_logit.shape[0]), str(mean.device)
        c = lambda t: t.detach().to(torch.float32).contiguous()
        ds.mean, ds.log_scale, ds.rot = c(mean), c(log_scale), c(rot)
        ds.opacity_logit, ds.rgb, ds.obj_logit = c(opacity_logit), c(rgb), c(obj_logit)
        n = max(ds.n, 1)
        ds.prob = torch.empty((n, ds.k), dtype=torch.float32, device=ds.device)
        ds.opacity = torch.empty(n, dtype=torch.float32, device=ds.device)
        ds.kappa, ds.conf = torch.empty_like(ds.opacity), torch.empty_like(ds.opacity)
        ds.label = torch.empty(n, dtype=torch.int32, device=ds.device)
        ngs_prepare_scene(ctx, ds, ig_params())
        proj = ngs_project(ctx, ds, cam, rp)
        lists = ngs_bin_sort(ctx, ds, proj, cam, rp, capacity=capacity)
        img = ngs_render(ctx, ds, proj, lists, cam, rp, want_obj=True)
        fctx.state = (ctx, ds, proj, lists, cam, rp)
        return img["rgb"], img["depth"], img["obj"]

    @staticmethod
    def backward(fctx, g_rgb, g_depth, g_obj):
        ctx, ds, proj, lists, cam, rp = fctx.state
        g = ngs_render_backward(ctx, ds, proj, lists, cam, rp, g_rgb, g_depth, g_obj, obj_eq2=True)
        return g["mean"], g["log_scale"], g["rot"], g["opacity_logit"], g["rgb"], g["obj_logit"], None, None, None, None


def render(mean, log_scale, rot, opacity_logit, rgb, obj_logit, ctx: Context, cam: ngs_camera,
           rp: Optional[ngs_raster_params] = None, capacity: int = 1 << 24):
    """Autograd entry of the rasterizer (see RenderFunction)."""
    return RenderFunction.apply(mean, log_scale, rot, opacity_logit, rgb, obj_logit, ctx, cam,
                                rp if rp is not None else raster_params(), capacity)


def ngs_gemm_bf16(ctx: Context, a: torch.Tensor, b: torch.Tensor, trans_a: bool = False, trans_b: bool = False,
                  c: Optional[torch.Tensor] = None, beta: float = 0.0) -> torch.Tensor:
    """c = op(a) op(b) (+ beta c) with BF16 operands (torch.bfloat16) and FP32 output."""
    assert a.dtype == torch.bfloat16 and b.dtype == torch.bfloat16
    a, b = a.contiguous(), b.contiguous()
    m, k = (a.shape[1], a.shape[0]) if trans_a else (a.shape[0], a.shape[1])
    kb, n = (b.shape[1], b.shape[0]) if trans_b else (b.shape[0], b.shape[1])
    assert k == kb
    if c is None:
        c = torch.zeros((m, n), dtype=torch.float32, device=a.device)
    _check("ngs_gemm_bf16", lib().ngs_gemm_bf16(ctx.handle, int(trans_a), int(trans_b), m, n, k, _p(a), a.shape[1],
                                                _p(b), b.shape[1], _p(c), c.shape[1], float(beta), _stream()), ctx)
    return c


class Surrogate:
    """The learned view scorer's parameters, gradients and Adam moments (torch tensors on the
    GPU; every pass runs in libngs)."""

    def __init__(self, ctx: Context, device: str = "cuda", seed: int = 0, max_batch: int = 256):
        self.ctx, self.device, self.max_batch = ctx, device, max_batch
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.w, self.b = [], []
        for (ci, co, taps) in SUR_SHAPES:
            fan_in = ci * taps
            self.w.append((torch.randn((co, ci * taps), generator=g) * (2.0 / fan_in) ** 0.5).to(device))
            self.b.append(torch.zeros(co, device=device))
        self.wb = [torch.empty(w.shape, dtype=torch.bfloat16, device=device) for w in self.w]
        self.gw = [torch.zeros_like(w) for w in self.w]
        self.gb = [torch.zeros_like(x) for x in self.b]
        self.mw = [torch.zeros_like(w) for w in self.w]
        self.mb = [torch.zeros_like(x) for x in self.b]
        self.vw = [torch.zeros_like(w) for w in self.w]
        self.vb = [torch.zeros_like(x) for x in self.b]
        self.step = 0
        self.ws = _bytes(self.workspace_size(max_batch), device)
        self.sync()

    @staticmethod
    def workspace_size(batch: int) -> int:
        v = C.c_size_t()
        _check("ngs_sur_workspace_size", lib().ngs_sur_workspace_size(batch, C.byref(v)))
        return int(v.value)

    def _c(self, w, b, wb=None) -> ngs_sur_params:
        s = ngs_sur_params()
        for l in range(SUR_LAYERS):
            s.w[l], s.b[l] = _p(w[l]), _p(b[l])
            s.w_bf16[l] = _p(wb[l]) if wb is not None else None
        return s

    def params(self) -> ngs_sur_params:
        return self._c(self.w, self.b, self.wb)

    def sync(self):
        p = self.params()
        _check("ngs_sur_sync_bf16", lib().ngs_sur_sync_bf16(self.ctx.handle, _ref(p), _stream()), self.ctx)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x [4][B][60][80] FP32 -> predictions [B]."""
        B = int(x.shape[1])
        assert B <= self.max_batch and tuple(x.shape[2:]) == SUR_IN[1:] and x.shape[0] == 4
        x = x.contiguous()
        pred = torch.empty(B, dtype=torch.float32, device=self.device)
        p = self.params()
        _check("ngs_sur_forward", lib().ngs_sur_forward(self.ctx.handle, _ref(p), _p(x), B, _p(pred), _p(self.ws),
                                                        self.ws.numel(), _stream()), self.ctx)
        return pred

    def backward(self, x: torch.Tensor, dpred: torch.Tensor):
        """Gradients (into self.gw, self.gb) of the last forward on x."""
        B = int(x.shape[1])
        p, g = self.params(), self._c(self.gw, self.gb)
        _check("ngs_sur_backward", lib().ngs_sur_backward(self.ctx.handle, _ref(p), _p(x), B, _p(dpred.contiguous()),
                                                          _ref(g), _p(self.ws), self.ws.numel(), _stream()), self.ctx)

    def mse(self, pred: torch.Tensor, target: torch.Tensor):
        B = int(pred.shape[0])
        dpred = torch.empty_like(pred)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check("ngs_sur_mse", lib().ngs_sur_mse(self.ctx.handle, _p(pred), _p(target.contiguous()), B, _p(dpred),
                                                _p(loss), _stream()), self.ctx)
        return loss, dpred

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        p, g = self.params(), self._c(self.gw, self.gb)
        m, v = self._c(self.mw, self.mb), self._c(self.vw, self.vb)
        _check("ngs_sur_adam", lib().ngs_sur_adam(self.ctx.handle, _ref(p), _ref(g), _ref(m), _ref(v), lr, beta1, beta2,
                                                  eps, self.step, _stream()), self.ctx)

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float = 1e-3) -> torch.Tensor:
        pred = self.forward(x)
        loss, dpred = self.mse(pred, target)
        self.backward(x, dpred)
        self.adam(lr)
        return loss


def ngs_sur_features(ctx: Context, img: Dict[str, torch.Tensor], k: int, depth_scale: float, x: torch.Tensor,
                     index: int):
    """Writes view `index`'s four input channels from an ngs_render output into x [4][B][60][80]."""
    H, W = img["depth"].shape
    im = ngs_image(_p(img["rgb"]), _p(img["depth"]), None, _p(img["t_final"]), _p(img["mean_conf"]),
                   _p(img["argmax_id"]), None)
    _check("ngs_sur_features", lib().ngs_sur_features(ctx.handle, _ref(im), W, H, k, float(depth_scale), _p(x),
                                                      int(x.shape[1]), index, _stream()), ctx)


class FeatureRenderer:
    """Batched 80x60 feature maps of many candidates (ngs_sur_render_features)."""

    def __init__(self, ctx: Context, scene: DeviceScene, max_pairs: int = 1 << 23, views_in_flight: int = 0):
        self.ctx, self.scene = ctx, scene
        self.dims = ngs_dims(scene.n, scene.k, SUR_IN[2], SUR_IN[1], max_pairs, 0, views_in_flight)
        self.buf = _bytes(workspace_size(4, scene.n, scene.k, max_pairs=max_pairs, views_in_flight=views_in_flight),
                          scene.device)

    def __call__(self, cams: Sequence[ngs_camera], rp: ngs_raster_params, depth_scale: float,
                 x: Optional[torch.Tensor] = None, weight: Optional[torch.Tensor] = None) -> torch.Tensor:
        nv = len(cams)
        if x is None:
            x = torch.empty((4, nv, SUR_IN[1], SUR_IN[2]), dtype=torch.float32, device=self.scene.device)
        arr = (ngs_camera * nv)(*cams)
        sc = self.scene.c()
        _check("ngs_sur_render_features", lib().ngs_sur_render_features(
            self.ctx.handle, _ref(sc), arr, nv, _ref(rp), _p(weight), float(depth_scale), _p(x), _ref(self.dims),
            _p(self.buf),
            self.buf.numel(), _stream()), self.ctx)
        return x


def ngs_sur_novelty(ctx: Context, scene: DeviceScene, h: Optional[Hessian], lambda_prior: float) -> torch.Tensor:
    """Per-Gaussian confidence x novelty against the training store h (see ngs_surrogate.h)."""
    out = torch.empty(max(scene.n, 1), dtype=torch.float32, device=scene.device)
    sc = scene.c()
    hc = h.c() if h is not None else None
    _check("ngs_sur_novelty", lib().ngs_sur_novelty(ctx.handle, _ref(sc), _ref(hc) if hc is not None else None,
                                                    float(lambda_prior), _p(out), _stream()), ctx)
    return out


def ngs_sur_pick(ctx: Context, scene: DeviceScene, h: Optional[Hessian], normalisers: Sequence[float],
                 cams: Sequence[ngs_camera], pred: torch.Tensor, rescore: int, rp: ngs_raster_params,
                 ig: ngs_ig_params, ws: "ScoreWorkspace", stats: Optional[torch.Tensor] = None):
    """Exact re-score of the network's best `rescore` candidates and the exact argmax among
    them (one library call). Returns (best index into cams, chosen indices, scores [R][4],
    raw gains [R][3])."""
    nv = len(cams)
    r = max(1, min(int(rescore), nv))
    dev = scene.device
    chosen = (C.c_int32 * r)()
    scores = torch.empty((r, 4), dtype=torch.float32, device=dev)
    ig_raw = torch.empty((r, 3), dtype=torch.float64, device=dev)
    best = C.c_int32(-1)
    arr = (ngs_camera * nv)(*cams)
    norm = (C.c_double * 3)(*[float(x) for x in normalisers])
    sc = scene.c()
    hc = h.c() if h is not None else None
    pred = pred.contiguous()
    _check("ngs_sur_pick", lib().ngs_sur_pick(ctx.handle, _ref(sc), _ref(hc) if hc is not None else None, norm, arr,
                                              nv, _p(pred), r, _ref(rp), _ref(ig), chosen, _p(scores), _p(ig_raw),
                                              C.byref(best), _stats(stats), _ref(ws.dims), _p(ws.buf), ws.buf.numel(),
                                              _stream()), ctx)
    return int(best.value), list(chosen), scores, ig_raw


class IgWorkspace:
    def __init__(self, scene: DeviceScene, max_slots: int = 1 << 16):
        self.buf = _bytes(workspace_size(1, scene.n, scene.k, max_slots=max_slots), scene.device)


def ngs_info_gain(ctx: Context, scene: DeviceScene, proj: Projected, lists: TileLists, cam: ngs_camera,
                  rp: ngs_raster_params, ig: ngs_ig_params, h: Optional[Hessian], ws: IgWorkspace,
                  stats: Optional[torch.Tensor] = None) -> torch.Tensor:
    out = torch.zeros(3, dtype=torch.float64, device=scene.device)
    sc, pc, lc = scene.c(), proj.c(), lists.c()
    hc = h.c() if h is not None else None
    _check("ngs_info_gain", lib().ngs_info_gain(ctx.handle, _ref(sc), _ref(pc), _ref(lc), _ref(cam), _ref(rp),
                                                _ref(ig), _ref(hc) if hc is not None else None, _p(out),
                                                _stats(stats), _p(ws.buf), ws.buf.numel(), _stream()), ctx)
    return out


def ngs_info_gain_static(ctx: Context, scene: DeviceScene, proj: Projected, lists: TileLists, cam: ngs_camera,
                         rp: ngs_raster_params, ig: ngs_ig_params, h: Optional[Hessian], out: torch.Tensor,
                         stats: Optional[torch.Tensor] = None) -> torch.Tensor:
    """ngs_info_gain on the library's fixed device scratch array (no allocation in the call);
    `out` is a caller-owned FP64 [3] device tensor."""
    sc, pc, lc = scene.c(), proj.c(), lists.c()
    hc = h.c() if h is not None else None
    _check("ngs_info_gain_static", lib().ngs_info_gain_static(ctx.handle, _ref(sc), _ref(pc), _ref(lc), _ref(cam),
                                                              _ref(rp), _ref(ig), _ref(hc) if hc is not None else None,
                                                              _p(out), _stats(stats), _stream()), ctx)
    return out


def ngs_hessian_reset(ctx: Context, h: Hessian, n: int):
    hc = h.c()
    _check("ngs_hessian_reset", lib().ngs_hessian_reset(ctx.handle, _ref(hc), n, _stream()), ctx)


def ngs_hessian_finalize(ctx: Context, h: Hessian):
    hc = h.c()
    _check("ngs_hessian_finalize", lib().ngs_hessian_finalize(ctx.handle, _ref(hc), _stream()), ctx)


class ScoreWorkspace:
    """Scratch of ngs_score_batch and the dims it was sized (and is carved) with."""

    def __init__(self, scene: DeviceScene, max_pairs: int, max_slots: int = 1 << 16, views_in_flight: int = 0):
        self.dims = ngs_dims(scene.n, scene.k, 0, 0, max_pairs, max_slots, views_in_flight)
        self.buf = _bytes(workspace_size(2, scene.n, scene.k, max_pairs=max_pairs, max_slots=max_slots,
                                         views_in_flight=views_in_flight), scene.device)


def ngs_score_batch(ctx: Context, scene: DeviceScene, h: Optional[Hessian], normalisers: Sequence[float],
                    cams: Sequence[ngs_camera], rp: ngs_raster_params, ig: ngs_ig_params, ws: ScoreWorkspace,
                    stats: Optional[torch.Tensor] = None):
    nv = len(cams)
    dev = scene.device
    scores = torch.empty((max(nv, 1), 4), dtype=torch.float32, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)
    ig_raw = torch.empty((max(nv, 1), 3), dtype=torch.float64, device=dev)
    arr = (ngs_camera * max(nv, 1))(*cams)
    norm = (C.c_double * 3)(*[float(x) for x in normalisers])
    sc = scene.c()
    hc = h.c() if h is not None else None
    _check("ngs_score_batch", lib().ngs_score_batch(ctx.handle, _ref(sc), _ref(hc) if hc is not None else None,
                                                    norm, arr, nv, _ref(rp), _ref(ig), _p(scores), _p(best),
                                                    _p(ig_raw), _stats(stats), _ref(ws.dims), _p(ws.buf), ws.buf.numel(),
                                                    _stream()), ctx)
    return scores[:nv], best, ig_raw[:nv]


def ngs_training_setup(ctx: Context, scene: DeviceScene, h: Hessian, train: Sequence[ngs_camera],
                       rp: ngs_raster_params, ig: ngs_ig_params, ws: ScoreWorkspace):
    """H_T and the Eq. 10 normalisers of the training views (one library call). Returns device
    tensors (normalisers [3], trace_total [3], ig_train [T][3])."""
    nt = len(train)
    dev = scene.device
    norm = torch.zeros(3, dtype=torch.float64, device=dev)
    trace_total = torch.zeros(3, dtype=torch.float64, device=dev)
    ig_train = torch.zeros((max(nt, 1), 3), dtype=torch.float64, device=dev)
    arr = (ngs_camera * max(nt, 1))(*train)
    sc, hc = scene.c(), h.c()
    _check("ngs_training_setup", lib().ngs_training_setup(ctx.handle, _ref(sc), _ref(hc), arr, nt, _ref(rp), _ref(ig),
                                                          _p(norm), _p(trace_total), _p(ig_train), _ref(ws.dims),
                                                          _p(ws.buf), ws.buf.numel(), _stream()), ctx)
    return norm, trace_total, ig_train[:nt]


class ngs_tuning(C.Structure):
    _fields_ = [("ig_lanes_per_pixel", C.c_int32), ("ig_waves_per_simd", C.c_int32), ("bin_chunk", C.c_int32),
                ("groups_in_flight", C.c_int32)]


def ngs_set_tuning(ctx: Context, ig_lanes_per_pixel: int = 0, ig_waves_per_simd: int = 0, bin_chunk: int = 0,
                   groups_in_flight: int = 0):
    t = ngs_tuning(int(ig_lanes_per_pixel), int(ig_waves_per_simd), int(bin_chunk), int(groups_in_flight))
    _check("ngs_set_tuning", lib().ngs_set_tuning(ctx.handle, _ref(t)), ctx)


def ngs_get_tuning(ctx: Context) -> Dict[str, int]:
    t = ngs_tuning()
    _check("ngs_get_tuning", lib().ngs_get_tuning(ctx.handle, _ref(t)), ctx)
    return {"ig_lanes_per_pixel": int(t.ig_lanes_per_pixel), "ig_waves_per_simd": int(t.ig_waves_per_simd),
            "bin_chunk": int(t.bin_chunk), "groups_in_flight": int(t.groups_in_flight)}


class ScoreGraph:
    """A scoring batch captured into a HIP graph (ngs_score_graph_create) and replayed with
    one launch. It binds the cameras and parameters by value and the scene, the store h, the
    workspace and its own output tensors by address: after the scene or h change in place, or
    `normalisers` (a device tensor) is updated, replay() scores against the new contents."""

    def __init__(self, ctx: Context, scene: DeviceScene, h: Optional[Hessian], cams: Sequence[ngs_camera],
                 rp: ngs_raster_params, ig: ngs_ig_params, ws: ScoreWorkspace, normalisers=(1.0, 1.0, 1.0),
                 stats: Optional[torch.Tensor] = None):
        nv = len(cams)
        dev = scene.device
        self.ctx, self.scene, self.h, self.ws, self.stats = ctx, scene, h, ws, stats
        self.norm = torch.tensor([float(x) for x in normalisers], dtype=torch.float64, device=dev)
        self.scores = torch.empty((nv, 4), dtype=torch.float32, device=dev)
        self.best = torch.empty(1, dtype=torch.int32, device=dev)
        self.ig_raw = torch.empty((nv, 3), dtype=torch.float64, device=dev)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        arr = (ngs_camera * max(nv, 1))(*cams)
        sc = scene.c()
        hc = h.c() if h is not None else None
        self._rp, self._ig = rp, ig
        handle = C.c_void_p()
        torch.cuda.synchronize()
        _check("ngs_score_graph_create", lib().ngs_score_graph_create(
            ctx.handle, _ref(sc), _ref(hc) if hc is not None else None, _p(self.norm), arr, nv, _ref(rp), _ref(ig),
            _p(self.scores), _p(self.best), _p(self.ig_raw), _stats(stats), _p(self.overflow), _ref(ws.dims), _p(ws.buf),
            ws.buf.numel(), C.byref(handle)), ctx)
        self.handle = handle

    def replay(self, normalisers=None):
        """One launch of the whole batch on the current stream; returns (scores, best, ig_raw)."""
        if normalisers is not None:
            self.norm.copy_(torch.tensor([float(x) for x in normalisers], dtype=torch.float64))
        _check("ngs_score_graph_launch", lib().ngs_score_graph_launch(self.handle, _stream()), self.ctx)
        return self.scores, self.best, self.ig_raw

    def close(self):
        if getattr(self, "handle", None):
            lib().ngs_score_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def score_workspace(scene: DeviceScene, max_pairs: int, max_slots: int = 1 << 16,
                    views_in_flight: int = 0) -> ScoreWorkspace:
    return ScoreWorkspace(scene, max_pairs, max_slots, views_in_flight)


def ngs_profile_enable(ctx: Context, on: bool, only: Optional[str] = None):
    """Event timing of every kernel class, or with `only` (a class name) of that class alone."""
    L = lib()
    if on and only is not None:
        names = [L.ngs_profile_kernel_name(i).decode() for i in range(L.ngs_profile_kernels())]
        _check("ngs_profile_enable_class", L.ngs_profile_enable_class(ctx.handle, names.index(only)), ctx)
    else:
        _check("ngs_profile_enable", L.ngs_profile_enable(ctx.handle, 1 if on else 0), ctx)


def ngs_profile_read(ctx: Context) -> Dict[str, tuple]:
    """{kernel class: (total ms, launches)} of the event profile."""
    L = lib()
    out = {}
    for i in range(L.ngs_profile_kernels()):
        ms, cnt = C.c_double(), C.c_int64()
        _check("ngs_profile_read", L.ngs_profile_read(ctx.handle, i, C.byref(ms), C.byref(cnt)), ctx)
        out[L.ngs_profile_kernel_name(i).decode()] = (ms.value, cnt.value)
    return out


# ------------------------------------------------------------------------------------------
# The next-best-view scoring pipeline
# ------------------------------------------------------------------------------------------

class NbvScorer:
    """Training setup (H_T and Eq. 10 normalisers) and candidate scoring on one GPU."""

    def __init__(self, ctx: Context, scene: DeviceScene, rp: ngs_raster_params, ig: ngs_ig_params,
                 max_pairs: int = 1 << 24, max_slots: int = 1 << 16, store_capacity: int = 1 << 17,
                 views_in_flight: int = 0):
        self.ctx, self.scene, self.rp, self.ig = ctx, scene, rp, ig
        self.max_pairs, self.max_slots, self.views_in_flight = max_pairs, max_slots, views_in_flight
        ngs_prepare_scene(ctx, scene, ig)
        self.h = Hessian(scene.n, scene.k, store_capacity, scene.device)
        self.norm = None
        self.ig_train = None
        self.ws = None

    def workspace(self) -> "ScoreWorkspace":
        """The batch workspace for the current views_in_flight (allocated on first use)."""
        if self.ws is None:
            self.ws = score_workspace(self.scene, self.max_pairs, self.max_slots, self.views_in_flight)
        return self.ws

    def _view(self, cam: ngs_camera):
        proj = ngs_project(self.ctx, self.scene, cam, self.rp)
        lists = ngs_bin_sort(self.ctx, self.scene, proj, cam, self.rp, capacity=self.max_pairs)
        return proj, lists

    def setup(self, train_cams: Sequence[ngs_camera]):
        """H_T and the Eq. 10 normalisers of the training views (ngs_training_setup); the
        values come back to the host for ngs_score_batch, which takes them by value."""
        norm, trace_total, ig_train = ngs_training_setup(self.ctx, self.scene, self.h, list(train_cams), self.rp,
                                                         self.ig, self.workspace())
        self.ig_train = ig_train.cpu().numpy()
        if self.ig.criterion == 1:
            st = trace_total.cpu().numpy()
            self.ig.trace_total = (C.c_double * 3)(*[float(x) for x in st])
            self.trace_total = st
        self.norm = norm.cpu().numpy()
        return self.norm

    def score(self, cams: Sequence[ngs_camera], stats: Optional[torch.Tensor] = None, scaled: bool = True):
        """Scores the candidates. scaled=False drops the Eq. 10 normalisation (normalisers 1)."""
        norm = self.norm if scaled else [1.0, 1.0, 1.0]
        return ngs_score_batch(self.ctx, self.scene, self.h, norm, cams, self.rp, self.ig, self.workspace(), stats)

    def greedy(self, train_cams: Sequence[ngs_camera], cand_cams: Sequence[ngs_camera], steps: int,
               follow: Optional[Sequence[int]] = None, scaled: bool = True):
        """Greedy next-best-view sequence without retraining: each step scores the remaining
        candidates against the training set, then moves the chosen one (the argmax, or
        follow[step] when given) into the training set, so its information joins H_T and the
        Eq. 10 normalisers of the next step. Returns one dict per step."""
        chosen: list = []
        remaining = list(range(len(cand_cams)))
        out = []
        for s in range(min(steps, len(cand_cams))):
            self.setup(list(train_cams) + [cand_cams[i] for i in chosen])
            scores, best, raw = self.score([cand_cams[i] for i in remaining], scaled=scaled)
            b = remaining[int(best.item())]
            pick = b if follow is None else int(follow[s])
            out.append({"remaining": list(remaining), "scores": scores.cpu().numpy(), "raw": raw.cpu().numpy(),
                        "best": b, "norm": self.norm.copy()})
            chosen.append(pick)
            remaining.remove(pick)
        return out
