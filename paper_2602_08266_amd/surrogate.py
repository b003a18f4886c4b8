"""Learned view scorer: data from the exact scorer, training and evaluation (the network and
all its passes run in libngs; see include/ngs_surrogate.h).

A sample is one candidate view of a seeded scene: its four 80x60 feature maps (depth, final
transmittance, argmax object id, mean confidence, from ngs_render) and, as the label, the
view's exact next-best-view score (Eq. 11 of the paper on Eq. 10-normalised gains, whole-scene
confidence Eq. 7, four training views per scene) from ngs_score_batch. The surrogate ranks
candidates; the exact scorer re-scores its best ones and stays the judge.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import binding as B

DEPTH_SCALE = 0.6  # m: candidate radius of the surrogate workload


@dataclass
class SceneSamples:
    x: torch.Tensor       # [4][V][60][80] FP32 features
    y: torch.Tensor       # [V] exact combined score (Eq. 11)
    raw: torch.Tensor     # [V][3] exact gains IG_rgb, IG_d, IG_o
    seconds_features: float
    seconds_exact: float


def scene_samples(ctx: B.Context, scene, cands: Sequence, train: Sequence, views_in_flight: int = 4,
                  max_pairs: int = 1 << 23) -> SceneSamples:
    """Feature maps and exact scores of every candidate of one scene."""
    ds = B.DeviceScene(scene, "cuda")
    rp = B.raster_params()
    ig = B.ig_params(target_id=-1)
    B.ngs_prepare_scene(ctx, ds, ig)
    cams = [B.camera(c) for c in cands]
    fr = B.FeatureRenderer(ctx, ds, max_pairs=max_pairs, views_in_flight=views_in_flight)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = fr(cams, rp, DEPTH_SCALE)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    scorer = B.NbvScorer(ctx, ds, rp, ig, max_pairs=max_pairs, max_slots=max(scene.n, 1 << 16),
                         store_capacity=max(scene.n, 1 << 16), views_in_flight=views_in_flight)
    scorer.setup([B.camera(c) for c in train])
    scores, best, raw = scorer.score(cams)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return SceneSamples(x, scores[:, 3].clone(), raw.clone(), t1 - t0, t2 - t1)


def train(net: B.Surrogate, x: torch.Tensor, y: torch.Tensor, epochs: int = 12, batch: int = 256,
          lr: float = 1e-3, seed: int = 0, log=None) -> List[float]:
    """Adam on the mean squared error of standardised labels; returns per-epoch mean loss."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = int(x.shape[1])
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(x.device)
        rate = lr if ep < (2 * epochs) // 3 else lr * 0.3
        tot, cnt = torch.zeros((), device=x.device), 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            tot += net.train_step(x[:, idx].contiguous(), y[idx].contiguous(), lr=rate)[0]
            cnt += 1
        hist.append(float(tot) / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def predict(net: B.Surrogate, x: torch.Tensor, batch: int = 256) -> torch.Tensor:
    out = []
    for s in range(0, int(x.shape[1]), batch):
        out.append(net.forward(x[:, s:s + batch].contiguous()))
    return torch.cat(out)


@dataclass
class Agreement:
    top5_in_steps: float      # fraction of 32-candidate steps whose exact best is in the surrogate's top 5
    top1_in_steps: float
    fallback_best: float      # fraction of steps where re-scoring the surrogate's top 5 finds the exact best
    full_top32_hit: float     # per scene: exact best among the surrogate's 32 best of all candidates
    spearman: float
    regret: float             # mean relative score loss of the fallback pick vs the exact best


def agreement(pred: np.ndarray, exact: np.ndarray, scene_of: np.ndarray, step: int = 32, seed: int = 0) -> Agreement:
    rng = np.random.default_rng(seed)
    t5 = t1 = fb = 0
    regret = []
    steps = 0
    hits, nsc = 0, 0
    for s in np.unique(scene_of):
        idx = np.where(scene_of == s)[0]
        p, e = pred[idx], exact[idx]
        nsc += 1
        hits += int(np.argmax(e) in np.argsort(-p)[:32])
        perm = rng.permutation(len(idx))
        for q in range(0, len(perm) - step + 1, step):
            c = perm[q:q + step]
            best = c[np.argmax(e[c])]
            order = c[np.argsort(-p[c])]
            t5 += int(best in order[:5])
            t1 += int(best == order[0])
            pick = order[:5][np.argmax(e[order[:5]])]
            fb += int(pick == best)
            regret.append((e[best] - e[pick]) / max(abs(e[best]), 1e-12))
            steps += 1
    from scipy.stats import spearmanr
    rho = float(np.mean([spearmanr(pred[scene_of == s], exact[scene_of == s])[0] for s in np.unique(scene_of)]))
    return Agreement(t5 / steps, t1 / steps, fb / steps, hits / nsc, rho, float(np.mean(regret)))
