"""FP64 reference of the learned view scorer (test infrastructure only: the tests and the
benchmark's CPU baseline use it; nothing in the product imports it).

The network is an addition of this project, not of arXiv 2602.08266: four 3x3 convolutions
(stride 2, padding 1, ReLU; 4 -> 32 -> 64 -> 128 -> 128 channels on 60x80 inputs), a global
average pool and two fully connected layers (128 -> 128 with ReLU -> 1). Layouts follow the
library: activations [C][B][H][W], convolution weights [out][in * 9] with index
in * 9 + kh * 3 + kw, fully connected weights [out][in].

Written plainly: im2col by slicing, one matrix product per layer, explicit backward. With
`bf16=True` the operands of every product are rounded to bfloat16 (round to nearest even) at
the points where the GPU kernels hold them in BF16 - weights, the im2col of activations, the
pooled and hidden activations, and the pre-activation gradients - and everything else stays
FP64, so the GPU (FP32 accumulation) can be compared tightly. With `bf16=False` it is the
plain FP64 network, pinned by finite differences.
"""
from __future__ import annotations

import numpy as np

CONV = [(4, 32), (32, 64), (64, 128), (128, 128)]
WIDTH = 128
IN_H, IN_W = 60, 80


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (via float32, round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def out_size(n: int) -> int:
    return (n + 2 - 3) // 2 + 1


def im2col(x: np.ndarray) -> np.ndarray:
    """x [C][B][H][W] -> col [C * 9][B * Ho * Wo] for a 3x3 kernel, stride 2, padding 1."""
    C, B, H, W = x.shape
    Ho, Wo = out_size(H), out_size(W)
    xp = np.zeros((C, B, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    col = np.zeros((C, 9, B, Ho, Wo))
    for kh in range(3):
        for kw in range(3):
            col[:, kh * 3 + kw] = xp[:, :, kh:kh + 2 * Ho:2, kw:kw + 2 * Wo:2]
    return col.reshape(C * 9, B * Ho * Wo)


def col2im(dcol: np.ndarray, C: int, B: int, H: int, W: int) -> np.ndarray:
    """Adjoint of im2col: scatter-add dcol [C * 9][B * Ho * Wo] back to [C][B][H][W]."""
    Ho, Wo = out_size(H), out_size(W)
    d = dcol.reshape(C, 9, B, Ho, Wo)
    dxp = np.zeros((C, B, H + 2, W + 2))
    for kh in range(3):
        for kw in range(3):
            dxp[:, :, kh:kh + 2 * Ho:2, kw:kw + 2 * Wo:2] += d[:, kh * 3 + kw]
    return dxp[:, :, 1:H + 1, 1:W + 1]


def forward(w, b, x, bf=True):
    """Returns (pred [B], cache). w, b: lists of 6 arrays (shapes as in the module doc)."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    B = x.shape[1]
    a = np.asarray(x, dtype=np.float64)
    cache = {"col": [], "act": [], "shape": []}
    for l, (ci, co) in enumerate(CONV):
        _, _, H, W = a.shape
        col = r(im2col(a))
        z = r(w[l]) @ col + np.asarray(b[l], np.float64)[:, None]
        act = np.maximum(z, 0.0)
        cache["col"].append(col)
        cache["act"].append(act)
        cache["shape"].append((ci, H, W))
        a = act.reshape(co, B, out_size(H), out_size(W))
    pool = r(a.reshape(WIDTH, B, -1).mean(axis=2))
    hid = np.maximum(r(w[4]) @ pool + np.asarray(b[4], np.float64)[:, None], 0.0)
    hidr = r(hid)
    pred = (r(w[5]) @ hidr + np.asarray(b[5], np.float64)[:, None])[0]
    cache.update(pool=pool, hid=hid, hidr=hidr, S=a.shape[2] * a.shape[3], B=B)
    return pred, cache


def backward(w, cache, dpred, bf=True):
    """Gradients (gw, gb) of a loss with dL/dpred = dpred, from the forward cache."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    B, S = cache["B"], cache["S"]
    gw, gb = [None] * 6, [None] * 6
    dz = np.asarray(dpred, np.float64)[None, :]
    gb[5] = dz.sum(axis=1)
    gw[5] = r(dz) @ cache["hidr"].T
    dh = r(w[5]).T @ r(dz)
    dz = dh * (cache["hid"] > 0)
    gb[4] = dz.sum(axis=1)
    gw[4] = r(dz) @ cache["pool"].T
    dpool = r(w[4]).T @ r(dz)
    da = np.repeat(dpool[:, :, None] / S, S, axis=2).reshape(WIDTH, -1)
    for l in range(3, -1, -1):
        ci, H, W = cache["shape"][l]
        dz = da * (cache["act"][l] > 0)
        gb[l] = dz.sum(axis=1)
        gw[l] = r(dz) @ cache["col"][l].T
        if l == 0:
            break
        dcol = r(w[l]).T @ r(dz)
        da = col2im(dcol, ci, B, H, W).reshape(ci, -1)
    return gw, gb


def mse(pred, target):
    d = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(d * d)), 2.0 * d / len(d)
