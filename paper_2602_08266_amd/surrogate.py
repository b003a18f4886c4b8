"""Learned view scorer: data from the exact scorer, training and evaluation (the network and
all its passes run in libngs; see include/ngs_surrogate.h).

A sample is one candidate view of a seeded scene: its four 80x60 feature maps (depth, final
transmittance, argmax object id, and the ray average of confidence x novelty against the
training information, from the library's feature render) and, as the label, the view's exact
next-best-view score (Eq. 11 of the paper on Eq. 10-normalised gains, whole-scene confidence
Eq. 7, four training views per scene) from ngs_score_batch. The surrogate ranks candidates;
the exact scorer re-scores its best ones and makes the final choice. Without the novelty channel the
maps say nothing about what the training views already observed, which the gain depends on.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import autotune as AT
from . import binding as B

DEPTH_SCALE = 0.6  # m: candidate radius of the surrogate workload

# launch shapes of the exact scorer, tuned once per process and scene size / resolution
_TUNED = {}


@dataclass
class SceneSamples:
    x: torch.Tensor       # [4][V][60][80] FP32 features
    y: torch.Tensor       # [V] exact combined score (Eq. 11)
    raw: torch.Tensor     # [V][3] exact gains IG_rgb, IG_d, IG_o
    seconds_features: float
    seconds_exact: float
    seconds_rescore: float  # exact scoring of `rescore` of the candidates in one batch


def scene_samples(ctx: B.Context, scene, cands: Sequence, train: Sequence, views_in_flight: int = 8,
                  max_pairs: int = 1 << 23, rescore: int = 32, feature_in_flight: int = 32) -> SceneSamples:
    """Feature maps and exact scores of every candidate of one scene."""
    ds = B.DeviceScene(scene, "cuda")
    rp = B.raster_params()
    ig = B.ig_params(target_id=-1)
    B.ngs_prepare_scene(ctx, ds, ig)
    cams = [B.camera(c) for c in cands]
    scorer = B.NbvScorer(ctx, ds, rp, ig, max_pairs=max_pairs, max_slots=max(scene.n, 1 << 16),
                         store_capacity=max(scene.n, 1 << 16), views_in_flight=views_in_flight)
    scorer.setup([B.camera(c) for c in train])
    key = (scene.n, scene.k, cams[0].width, cams[0].height)
    if key not in _TUNED:
        _TUNED[key] = AT.tune_score(ctx, scorer, cams, sample=64, vif=(8, 16, 32))
    else:
        AT.apply(ctx, scorer, _TUNED[key])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scores, best, raw = scorer.score(cams)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fr = B.FeatureRenderer(ctx, ds, max_pairs=max_pairs, views_in_flight=feature_in_flight)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nov = B.ngs_sur_novelty(ctx, ds, scorer.h, ig.lambda_prior)
    x = fr(cams, rp, DEPTH_SCALE, weight=nov)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    scorer.score(cams[:rescore])
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    return SceneSamples(x, scores[:, 3].clone(), raw.clone(), t3 - t2, t1 - t0, t4 - t3)


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


class Pipeline:
    """What the surrogate-guided choice needs for one scene: the device scene (whole-scene
    confidence, Eq. 7), the exact scorer set up on the training views (H_T, Eq. 10
    normalisers), the per-Gaussian novelty weights and the batched feature renderer."""

    def __init__(self, ctx: B.Context, scene, train: Sequence, views_in_flight: int = 32,
                 max_pairs: int = 1 << 23, feature_in_flight: int = 32):
        self.ctx = ctx
        self.rp = B.raster_params()
        self.ds = B.DeviceScene(scene, "cuda")
        ig = B.ig_params(target_id=-1)
        self.scorer = B.NbvScorer(ctx, self.ds, self.rp, ig, max_pairs=max_pairs, max_slots=max(scene.n, 1 << 16),
                                  store_capacity=max(scene.n, 1 << 16), views_in_flight=views_in_flight)
        self.scorer.setup([B.camera(c) for c in train])
        self.weight = B.ngs_sur_novelty(ctx, self.ds, self.scorer.h, ig.lambda_prior)
        self.fr = B.FeatureRenderer(ctx, self.ds, max_pairs=max_pairs, views_in_flight=feature_in_flight)


@dataclass
class Pick:
    best: int                 # index (into the candidates) of the exact argmax among the re-scored
    pred: torch.Tensor        # [V] network predictions
    chosen: List[int]         # the re-scored candidates, by descending prediction
    scores: torch.Tensor      # [R][4] their exact scores (Eq. 10-11)
    seconds: float            # wall clock of the whole choice (features, network, re-score)


def pick(ctx: B.Context, scorer: B.NbvScorer, net: B.Surrogate, fr: B.FeatureRenderer, cams: Sequence,
         rp, weight: Optional[torch.Tensor], rescore: int = 256, batch: int = 256) -> Pick:
    """The surrogate-guided next-best-view choice: the candidates' feature maps and the
    network's predictions, then the exact scorer on the network's best `rescore` candidates and
    the exact argmax among them (ngs_sur_pick). The scorer must be set up (H_T, normalisers)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = fr(cams, rp, DEPTH_SCALE, weight=weight)
    pred = predict(net, x, batch)
    best, chosen, scores, _ = B.ngs_sur_pick(ctx, scorer.scene, scorer.h, scorer.norm, cams, pred, rescore, rp,
                                             scorer.ig, scorer.workspace())
    torch.cuda.synchronize()
    return Pick(best, pred, chosen, scores, time.perf_counter() - t0)


@dataclass
class Agreement:
    """Ranking agreement of the surrogate with the exact scores on held-out scenes. The
    pipeline ranks a candidate set with the surrogate, re-scores its `rescore` best exactly and
    takes the exact argmax among them."""
    top5_full: float          # per scene (all candidates): the pipeline's pick is in the exact top 5
    best_full: float          # ... and is the exact best
    top5_subsets: float       # the same over disjoint random subsets of `subset` candidates
    best_subsets: float
    top5_in_steps: float      # 32-candidate subsets: the exact best is in the surrogate's own top 5
    spearman: float           # mean per-scene rank correlation of predicted and exact scores
    regret: float             # mean relative score lost by the pipeline's pick (subsets)
    sets_full: int
    sets_subsets: int


def pipeline_pick(pred: np.ndarray, exact: np.ndarray, rescore: int) -> int:
    top = np.argsort(-pred, kind="stable")[:rescore]
    return int(top[np.argmax(exact[top])])


def agreement(pred: np.ndarray, exact: np.ndarray, scene_of: np.ndarray, rescore: int = 32, subset: int = 256,
              seed: int = 0) -> Agreement:
    from scipy.stats import spearmanr
    rng = np.random.default_rng(seed)
    full5 = fullb = sub5 = subb = st5 = 0
    nfull = nsub = nst = 0
    regret, rho = [], []
    for s in np.unique(scene_of):
        idx = np.where(scene_of == s)[0]
        p, e = pred[idx], exact[idx]
        rank = np.argsort(-e, kind="stable")
        pick = pipeline_pick(p, e, rescore)
        full5 += int(pick in rank[:5])
        fullb += int(pick == rank[0])
        nfull += 1
        rho.append(spearmanr(p, e)[0])
        perm = rng.permutation(len(idx))
        for q in range(0, len(perm) - subset + 1, subset):
            c = perm[q:q + subset]
            pk = c[pipeline_pick(p[c], e[c], rescore)]
            r = c[np.argsort(-e[c], kind="stable")]
            sub5 += int(pk in r[:5])
            subb += int(pk == r[0])
            regret.append((e[r[0]] - e[pk]) / max(abs(e[r[0]]), 1e-12))
            nsub += 1
        for q in range(0, len(perm) - 32 + 1, 32):
            c = perm[q:q + 32]
            st5 += int(c[np.argmax(e[c])] in c[np.argsort(-p[c], kind="stable")[:5]])
            nst += 1
    return Agreement(full5 / nfull, fullb / nfull, sub5 / max(nsub, 1), subb / max(nsub, 1), st5 / max(nst, 1),
                     float(np.mean(rho)), float(np.mean(regret)) if regret else 0.0, nfull, nsub)
