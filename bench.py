"""Throughput of exact next-best-view scoring on one MI355X.

Workload: 1M Gaussians in 64 object clusters (object vector k = 64), object-centric scoring
of a seeded target (Eq. 12), candidate views at 640x480 (fx = fy = 525) on a sphere of
radius U[0.4, 0.9] m -- the 640x480 share of the mixed-resolution batch. One step scores
every candidate view: projection, binning and sorting, the fused compositing +
information-gain walk, the FP64 finalize, Eq. 10-11 and the argmax. The training set
(4 views: H_T and the Eq. 10 normalisers) is built once before timing and reported apart.

Prints one JSON line. With --gpus N > 1 it exits: the scorer runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate views scored/sec at 1M Gaussians 640x480 (exact vs surrogate); % HBM peak"
HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2602_08266_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# Algorithmic HBM bytes per kernel class, from per-step counts: n Gaussians, k, views V,
# pairs M, walked (tile, list entry) pairs W and touched weighted Gaussians U (all summed
# over the step's views).
def algorithmic_bytes(name, n, k, V, M, W, U, W2=0):
    if name == "project":
        return V * n * (40 + 40)                 # mean, log-scale, quaternion in; 2D mean, conic, depth, key, rect, count out
    if name == "depth_sort_scatter":
        return V * 4 * n * 16                    # 4 passes, key + value in and out
    if name == "depth_sort_hist":
        return V * 4 * n * 4
    if name == "count_scan":
        return V * n * 16
    if name == "tile_part_hist":
        return V * n * 12                        # rank order and the rect of every Gaussian
    if name == "tile_part_scatter":
        return 4 * M + V * n * 12                # final gid per pair + the same per-Gaussian reads
    if name == "ig_front":
        # front-to-back walk: list entry, 2D mean, conic and opacity of every walked entry
        return W * 28
    if name == "ig_back":
        # back-to-front walk over the W2 entries from a tile's last contributor to its nearest
        # weighted one: list entry, geometry, weight flag, depth, colour and the k-long
        # probability row (the object suffixes of the weighted Gaussians in front sum the rows
        # of every contributing Gaussian behind them); the statistics (94 + 6k floats) of every
        # touched weighted Gaussian written
        return W2 * (48 + 4 * k) + U * 4 * (94 + 6 * k)
    return None


def path_bytes(n, k, V, M, U):
    """Compulsory HBM bytes of one scoring step (all views): geometry and c_g read, the
    projection written and read back, every pair emitted once and reordered once, the
    touched Gaussians' object rows, statistics written and read, and their stored training
    blocks read (factored object block)."""
    return V * n * 48 + V * n * 72 + M * 36 + U * (4 * k + 40) + U * 8 * (94 + 6 * k) + U * 8 * (105 + 66 + 68 + 12 * k)


KERNEL_FILES = {
    "project": ["project.hip", "common.hpp"], "depth_sort_scatter": ["sort.hip", "common.hpp"],
    "depth_sort_hist": ["sort.hip", "common.hpp"], "count_scan": ["bin.hip", "common.hpp"],
    "tile_part_hist": ["bin.hip", "common.hpp"], "tile_part_scatter": ["bin.hip", "common.hpp"],
    "ig_front": ["info_gain.hip", "common.hpp"], "ig_back": ["info_gain.hip", "common.hpp"],
    "ig_finalize": ["finalize.hip", "common.hpp"],
}


def read_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it still matches
    the kernel's source; else None."""
    path = os.path.join(PROFILE_DIR, f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash(KERNEL_FILES.get(kernel, [])):
        return None
    return d.get("hbm_bytes_per_launch")


def ig_flops(name, k, P1, P2, R):
    """FP32 operations of the information-gain walk kernels, from their own counts.
    ig_front: P1 contributing (pixel, Gaussian) pairs of the front-to-back pass (offset,
    quadratic form, opacity and transmittance: 15 each). ig_back: P2 contributing pairs of the
    back-to-front pass (the same 15, T recovery 4, suffix updates of colour, depth and the k
    object channels 2 (4 + k)) and R per-pixel records of weighted Gaussians (y and the channel
    weights 24 + 5k, record products 36, and the 94 + 6k products summed into the statistics:
    2 (94 + 6k))."""
    if name == "ig_front":
        return 15 * P1
    if name == "ig_back":
        return (19 + 2 * (4 + k)) * P2 + (60 + 5 * k + 2 * (94 + 6 * k)) * R
    return None


def cpu_baseline(workload_name, seed, views=3, threads=None):
    """The FP64 oracle timed on the host on a bounded sample: the first `views` candidate
    views of the workload scored against the training set's H_T and Eq. 10 normalisers (built
    by the oracle from the 4 training views first and timed apart); the oracle splits each
    view's work across its threads."""
    import oracle
    import scenegen
    cfg, scene, cands, train = scenegen.make_workload(workload_name, seed)
    ig = oracle.IGParams(target_id=scene.target)
    th = threads or oracle.default_threads()
    r = oracle.score(scene, train, cands[:views], ig=ig, threads=th)
    setup_s, cand_s = r.seconds
    mode = "object-centric" if scene.target >= 0 else "whole scene"
    return {"value": views / cand_s, "unit": "views/s", "cores": th, "kind": "oracle",
            "sample": f"{views} candidate views ({cands[0].width}x{cands[0].height}, {scene.n} Gaussians, k={scene.k}, "
                      f"{mode}) scored against H_T of the {len(train)} training views, FP64: {cand_s:.1f} s "
                      f"for the candidates (H_T and normalisers {setup_s:.1f} s, not counted)"}


def cpu_plan(args):
    """The oracle timed as planned for the reported CPU baseline: a seeded 16-candidate subset
    scored against the training H_T, on all host cores (one call) and single-threaded (two
    views, the training set built on all cores first), seconds per candidate view (median)."""
    import statistics

    import numpy as np

    import oracle
    import scenegen
    cfg, scene, cands, train = scenegen.make_workload(args.workload, args.seed)
    ig = oracle.IGParams(target_id=scene.target)
    rng = np.random.default_rng(args.seed + 7)
    subset = sorted(rng.choice(len(cands), size=min(16, len(cands)), replace=False).tolist())
    allc = oracle.default_threads()
    out = {"workload": args.workload, "subset": subset, "oracle_threads": allc, "host_cpu_count": os.cpu_count()}
    log = lambda m: (sys.stderr.write(m + "\n"), sys.stderr.flush())
    r = oracle.score(scene, train, [cands[v] for v in subset], ig=ig, threads=allc)
    per = [float(x) for x in r.cand_seconds]
    log(f"all cores ({allc} threads): setup {r.seconds[0]:.1f} s, candidates {per}")
    out["all_cores"] = {"threads": allc, "views": len(subset), "median_s_per_view": statistics.median(per),
                        "views_per_s": 1.0 / statistics.median(per), "setup_s": r.seconds[0], "per_view_s": per}
    per1 = []
    for v in subset[:2]:
        r = oracle.score(scene, train, [cands[v]], ig=ig, threads=1, setup_threads=allc)
        per1.append(float(r.cand_seconds[0]))
        log(f"single thread: view {v} {per1[-1]:.1f} s (setup on {allc} threads {r.seconds[0]:.1f} s)")
    out["single_thread"] = {"threads": 1, "views": len(per1), "median_s_per_view": statistics.median(per1),
                            "views_per_s": 1.0 / statistics.median(per1), "per_view_s": per1}
    print(json.dumps(out), flush=True)


def run_backward(args):
    """Refinement step: for every view, render the scene (projection, binning, compositing),
    an L1 colour + L1 depth + cross-entropy object loss against targets rendered from a
    perturbed copy of the scene, and the backward rasterizer."""
    import numpy as np
    import torch

    import scenegen
    from paper_2602_08266_amd import binding as B

    torch.cuda.set_device(0)
    cfg, scene, cands, train = scenegen.make_workload("diff", args.seed, n_views=args.views)
    V = len(cands)
    ctx = B.Context(0)
    rp = B.raster_params()
    cams = [B.camera(c) for c in cands]
    rng = np.random.default_rng(args.seed + 17)
    t = lambda a, grad=False: torch.as_tensor(np.asarray(a, np.float32), device="cuda").contiguous().requires_grad_(grad)
    tgt = [t(scene.mean + rng.normal(0, 0.005, scene.mean.shape)), t(scene.log_scale), t(scene.rot),
           t(scene.opacity_logit + rng.normal(0, 0.3, scene.opacity_logit.shape)), t(scene.rgb), t(scene.obj_logit)]
    targets = []
    with torch.no_grad():
        for c in cams:
            rgb, depth, obj = B.render(*tgt, ctx, c, rp, 48 << 20)
            targets.append((rgb.clone(), depth.clone(), obj.argmax(0)))
    params = [t(scene.mean, True), t(scene.log_scale, True), t(scene.rot, True), t(scene.opacity_logit, True),
              t(scene.rgb, True), t(scene.obj_logit, True)]

    def step():
        for p in params:
            p.grad = None
        total = 0.0
        for c, (trgb, tdep, tlab) in zip(cams, targets):
            rgb, depth, obj = B.render(*params, ctx, c, rp, 48 << 20)
            loss = (rgb - trgb).abs().mean() + (depth - tdep).abs().mean() + torch.nn.functional.nll_loss(
                torch.log(obj.clamp_min(1e-6)).unsqueeze(0), tlab.unsqueeze(0))
            loss.backward()
            total += float(loss.detach())
        return total

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-kernel breakdown from one profiled step outside the timed region; inside it only the
    # dominant kernel class carries timing events
    B.ngs_profile_enable(ctx, True)
    step()
    torch.cuda.synchronize()
    breakdown = {k: v for k, v in B.ngs_profile_read(ctx).items() if v[1] > 0}
    dom = max(breakdown, key=lambda k: breakdown[k][0])
    B.ngs_profile_enable(ctx, True, only=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = B.ngs_profile_read(ctx)
    B.ngs_profile_enable(ctx, False)
    K = args.steps
    ms_tot, launches = prof[dom]
    n, k, HW = scene.n, scene.k, cands[0].width * cands[0].height
    # compulsory bytes of one backward launch: the image gradients, the per-Gaussian screen
    # gradient rows (zeroed, written, read) and the parameter gradients written
    alg = {"bwd_tiles": HW * (4 + k) * 4 + n * (16 + k) * 4, "bwd_params": n * (16 + k) * 4 + n * (14 + k) * 4}.get(dom)
    avg_s = ms_tot / launches / 1e3
    roof = ({"bound": "hbm", "achieved": round(alg / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(alg / avg_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
             "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": int(alg)} if alg else
            {"bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None, "traffic": None, "kernel": dom,
             "avg_launch_us": round(avg_s * 1e6, 2)})
    print(json.dumps({
        "metric": "views/s of the differentiable rasterizer (forward + loss + backward), 500k Gaussians 640x480",
        "value": round(V * K / dt, 2), "unit": "views/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / K, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"diff: {n} Gaussians, k={k}, {V} views at {cands[0].width}x{cands[0].height}, "
                               "targets from a perturbed copy (mu + N(0, 5 mm), opacity logit + N(0, 0.3))",
                   "loss": "L1 rgb + L1 depth + object cross-entropy"},
        "roofline": roof, "loss": round(loss, 6),
        "kernels_ms_per_step": {kk: round(v[0], 3) for kk, v in sorted(breakdown.items(), key=lambda x: -x[1][0])}}),
          flush=True)


def run_surrogate(args):
    """Learned view scorer on the surrogate workload (1M Gaussians, k = 64, 2048 candidates at
    80x60 per scene, whole-scene confidence): exact labels from ngs_score_batch on seeded
    training scenes, training with the library's BF16 kernels, then on held-out scenes the
    ranking agreement with the exact scores and the throughput of both scorers."""
    import numpy as np
    import torch

    import scenegen
    from paper_2602_08266_amd import binding as B
    from paper_2602_08266_amd import surrogate as SG

    torch.cuda.set_device(0)
    ctx = B.Context(0)
    log = lambda m: (sys.stderr.write(m + "\n"), sys.stderr.flush())
    nv = args.views or 2048
    xs, ys, scene_of, raws = [], [], [], []
    t_feat = t_exact = 0.0
    seeds = list(range(args.sur_scenes)) + [1000 + i for i in range(args.sur_test_scenes)]
    for i, seed in enumerate(seeds):
        cfg, scene, cands, train = scenegen.make_workload("surrogate", seed, n_views=nv)
        s = SG.scene_samples(ctx, scene, cands, train, views_in_flight=8, rescore=args.sur_rescore)
        xs.append(s.x)
        ys.append(s.y)
        raws.append(s.raw)
        scene_of.append(np.full(nv, seed))
        if i >= args.sur_scenes:
            t_feat += s.seconds_features
            t_exact += s.seconds_exact
        log(f"scene {seed}: features {s.seconds_features:.2f} s, exact {s.seconds_exact:.2f} s")
        del scene
    ntr = args.sur_scenes * nv
    x = torch.cat(xs, dim=1)
    y = torch.cat(ys)
    del xs
    # labels standardised per scene: the network ranks the candidates of one scene, so the
    # scene-to-scene offset and spread of the exact scores are not part of its target
    yn = torch.cat([(t - t.mean()) / t.std() for t in ys])
    mu, sd = float(y[:ntr].mean()), float(y[:ntr].std())
    net = B.Surrogate(ctx, seed=args.seed, max_batch=256)
    B.ngs_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = SG.train(net, x[:, :ntr].contiguous(), yn[:ntr].contiguous(), epochs=args.sur_epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    prof = B.ngs_profile_read(ctx)
    B.ngs_profile_enable(ctx, False)
    xt = x[:, ntr:].contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = SG.predict(net, xt)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    ag = SG.agreement(pred.cpu().numpy(), y[ntr:].cpu().numpy(), np.concatenate(scene_of)[ntr:],
                      rescore=args.sur_rescore)
    ag_budget = {r: SG.agreement(pred.cpu().numpy(), y[ntr:].cpu().numpy(), np.concatenate(scene_of)[ntr:],
                                 rescore=r).__dict__ for r in (32, 64, 128, 256, 512)}
    if args.sur_dump:
        np.savez(args.sur_dump, pred=pred.cpu().numpy(), exact=y[ntr:].cpu().numpy(),
                 scene=np.concatenate(scene_of)[ntr:], raw=torch.cat(raws)[ntr:].cpu().numpy())
    # the product path on every held-out scene: SG.pick (feature maps, network, exact re-score of
    # the network's best candidates, exact argmax in the library) timed end to end, and its
    # choice ranked among the exact scores of all candidates
    t_pick, pipe_top5, pipe_best = 0.0, 0, 0
    for j, seed in enumerate(seeds[args.sur_scenes:]):
        cfg, scene, cands, train = scenegen.make_workload("surrogate", seed, n_views=nv)
        env = SG.Pipeline(ctx, scene, train)
        tuned = SG._TUNED.get((scene.n, scene.k, cands[0].width, cands[0].height))
        if tuned is not None:  # the exact scorer's launch shape tuned while labelling
            from paper_2602_08266_amd import autotune as AT
            AT.apply(ctx, env.scorer, tuned)
        cams = [B.camera(c) for c in cands]
        SG.pick(ctx, env.scorer, net, env.fr, cams, env.rp, env.weight, rescore=args.sur_rescore)
        pk = SG.pick(ctx, env.scorer, net, env.fr, cams, env.rp, env.weight, rescore=args.sur_rescore)
        e = ys[args.sur_scenes + j].cpu().numpy()
        rank = np.argsort(-e, kind="stable")
        pipe_top5 += int(pk.best in rank[:5])
        pipe_best += int(pk.best == rank[0])
        t_pick += pk.seconds
        log(f"held-out scene {seed}: pick {pk.best} (exact rank {int(np.where(rank == pk.best)[0][0])}), "
            f"{pk.seconds:.3f} s")
        del env, scene
    ptr = SG.predict(net, x[:, :min(ntr, 4 * nv)].contiguous())
    ag_train = SG.agreement(ptr.cpu().numpy(), y[:min(ntr, 4 * nv)].cpu().numpy(),
                            np.concatenate(scene_of)[:min(ntr, 4 * nv)])
    # matrix-core work of training: 2 flops per multiply-add of every GEMM of forward and backward
    per_view_fwd = sum(2 * co * ci * 9 * ho * wo for (ci, co, _), (ho, wo) in
                       zip(B.SUR_SHAPES[:4], [(30, 40), (15, 20), (8, 10), (4, 5)])) + 2 * (128 * 128 + 128)
    steps = args.sur_epochs * (ntr // 256)
    gemm_ms, gemm_n = prof.get("sur_gemm", (0.0, 0))
    gemm_tflops = 3 * per_view_fwd * 256 * steps / (gemm_ms / 1e3) / 1e12 if gemm_ms > 0 else None
    nt = args.sur_test_scenes * nv
    # the surrogate pipeline as the product runs it (SG.pick) against exact scoring of every
    # candidate (ngs_score_batch)
    sur_views_s = nt / t_pick
    exact_views_s = nt / t_exact
    print(json.dumps({
        "metric": "candidate views scored/sec, learned surrogate (80x60 feature maps + BF16 network) vs exact IG",
        "value": round(sur_views_s, 2), "unit": "views/s", "n_gpus": 1, "higher_is_better": True,
        "vs_baseline": None, "dtype": "bf16 network / f32 features", "data": "synthetic",
        "config": {"workload": f"surrogate: 1M Gaussians, k=64, {nv} candidates at 80x60 per scene, whole-scene "
                               f"confidence; {args.sur_scenes} training scenes ({ntr} pairs), "
                               f"{args.sur_test_scenes} held-out scenes",
                   "network": "4 conv 3x3 s2 (4-32-64-128-128) + avg pool + FC 128-128-1, BF16 MFMA, FP32 accumulate"},
        "exact_views_s": round(exact_views_s, 2), "speedup": round(sur_views_s / exact_views_s, 3),
        "pipeline": {"seconds": round(t_pick, 3), "scenes": args.sur_test_scenes, "rescore": args.sur_rescore,
                     "pick_in_exact_top5": pipe_top5, "pick_is_exact_best": pipe_best},
        "surrogate_feature_s": round(t_feat, 3), "surrogate_network_s": round(t_net, 4),
        "exact_s": round(t_exact, 3),
        "rescore": args.sur_rescore, "agreement_heldout": ag.__dict__,
        "agreement_heldout_by_rescore": ag_budget, "agreement_train": ag_train.__dict__,
        "train": {"pairs": ntr, "epochs": args.sur_epochs, "seconds": round(t_train, 2),
                  "loss_per_epoch": [round(h, 4) for h in hist], "label_mean": mu, "label_std": sd},
        "roofline": {"bound": "mfma", "kernel": "sur_gemm",
                     "achieved": round(gemm_tflops, 2) if gemm_tflops else None, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(gemm_tflops / 2500.0, 5) if gemm_tflops else None, "traffic": None,
                     "avg_launch_us": round(gemm_ms / gemm_n * 1e3, 2) if gemm_n else None}}), flush=True)


ALU_PEAK_TFLOPS = 157.3  # FP32 vector: 256 CUs x 128 lanes x 2 (FMA) x 2.4 GHz, the published MI355X figure


def _round_up(x, m):
    return (int(x) + m - 1) // m * m


def make_scorer(B, ctx, ds, scene, rp, ig, cams, train, in_flight, log):
    """Scorer whose pair capacity comes from the pre-pass (ngs_count_pairs) over the
    candidates and the training views, rounded up to 1M pairs; whole-scene scoring takes a
    statistics slot for every Gaussian that can contribute, one target a few per cent of n."""
    pairs = B.ngs_count_pairs(ctx, ds, list(cams) + list(train), rp).cpu()
    max_pairs = _round_up(int(pairs.max()), 1 << 20)
    slots = 1 << 16 if scene.target >= 0 else _round_up(scene.n, 1 << 16)
    log(f"capacity pre-pass: max pairs {int(pairs.max())} -> capacity {max_pairs}, slots {slots}")
    scorer = B.NbvScorer(ctx, ds, rp, ig, max_pairs=max_pairs, max_slots=slots, store_capacity=1 << 17,
                         views_in_flight=in_flight)
    return scorer, pairs[:len(cams)]


def serialized_roofline(B, ctx, scorer, cams, scene, K_views, log):
    """One view in flight (launches never overlap): every kernel class bracketed by events for
    the per-kernel breakdown, then only the dominant class, whose average launch duration and
    kernel-counted work give the roofline. Also returns the per-view counts of the kernels."""
    import torch
    saved = scorer.views_in_flight
    scorer.views_in_flight = 1
    scorer.ws = None
    scorer.score(cams)
    torch.cuda.synchronize()
    B.ngs_profile_enable(ctx, True)
    scorer.score(cams)
    torch.cuda.synchronize()
    breakdown = {k: v for k, v in B.ngs_profile_read(ctx).items() if v[1] > 0}
    dom = max(breakdown, key=lambda k: breakdown[k][0])
    stats = torch.zeros(B.STATS_LEN, dtype=torch.int64, device="cuda:0")
    B.ngs_profile_enable(ctx, True, only=dom)
    torch.cuda.synchronize()
    scorer.score(cams, stats)
    torch.cuda.synchronize()
    ms_tot, launches = B.ngs_profile_read(ctx)[dom]
    B.ngs_profile_enable(ctx, False)
    scorer.views_in_flight = saved
    scorer.ws = None
    st = stats.cpu().numpy().astype(np.float64)
    V = len(cams)
    counts = {"pairs_M": st[1] / V, "touched_weighted_U": st[2] / V, "contrib_pairs_P": st[3] / V,
              "walked_entries_W": st[4] / V, "back_to_front_entries": st[6] / V,
              "back_to_front_contrib_pairs": st[7] / V, "weighted_records": st[8] / V,
              "contrib_tile_pairs_F": st[9] / V}
    avg_s = ms_tot / launches / 1e3
    per_launch = launches / V  # launches of the class per view
    n, k = scene.n, scene.k
    alg = algorithmic_bytes(dom, n, k, 1, st[1] / V, st[4] / V, st[2] / V, st[6] / V)
    roof = {"kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2), "launches_timed": int(launches),
            "views_in_flight": 1, "traffic": read_traffic(dom, scorer_workload_name(scene))}
    hbm = None
    if alg is not None:
        b = alg / per_launch
        hbm = {"achieved": round(b / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(b / avg_s / 1e9 / HBM_PEAK_GBS, 5), "algorithmic_bytes_per_launch": int(b)}
    if dom in ("ig_front", "ig_back"):
        fl = ig_flops(dom, k, st[3] / V, st[7] / V, st[8] / V) / per_launch
        tf = fl / avg_s / 1e12
        roof.update({"bound": "alu", "achieved": round(tf, 3), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / ALU_PEAK_TFLOPS, 5), "flops_per_launch": int(fl), "hbm": hbm})
    elif hbm is not None:
        roof.update({"bound": "hbm", "achieved": hbm["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": hbm["frac"], "algorithmic_bytes_per_launch": hbm["algorithmic_bytes_per_launch"]})
    else:
        roof.update({"bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None})
    # where the back-to-front walk's wavefronts spend their time (shader-clock cycles summed
    # over them): the workgroup barrier before each batch, staging the batch, walking it, and
    # the records of weighted contributors (a part of the walking)
    cyc = st[10] + st[11] + st[12]
    if cyc > 0:
        roof["back_walk_wave_cycles"] = {
            "per_view": round(cyc / V), "barrier": round(st[10] / cyc, 4), "staging": round(st[11] / cyc, 4),
            "walking": round(st[12] / cyc, 4), "records_within_walking": round(st[13] / cyc, 4)}
    bd = {kk: round(v[0] / V * 1e3, 2) for kk, v in sorted(breakdown.items(), key=lambda x: -x[1][0])}
    log(f"serialized pass: dominant {dom} {avg_s * 1e6:.1f} us per launch; per-view us {bd}")
    return roof, counts, bd


_WORKLOAD_OF_SCENE = {}


def scorer_workload_name(scene):
    return _WORKLOAD_OF_SCENE.get(id(scene), "")


def run_exact(args, log):
    import numpy as np  # noqa: F401
    import torch

    import scenegen
    from paper_2602_08266_amd import binding as B

    torch.cuda.set_device(0)
    cfg, scene, cands, train = scenegen.make_workload(args.workload, args.seed, n_views=args.views)
    _WORKLOAD_OF_SCENE[id(scene)] = args.workload
    V = len(cands)
    ctx = B.Context(0)
    ds = B.DeviceScene(scene, "cuda:0")
    rp = B.raster_params()
    ig = B.ig_params(target_id=scene.target)
    cam_c = [B.camera(c) for c in cands]
    cam_t = [B.camera(c) for c in train]
    scorer, pairs = make_scorer(B, ctx, ds, scene, rp, ig, cam_c, cam_t, args.in_flight, log)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norm = scorer.setup(cam_t)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    tune = None
    if not args.no_autotune:
        # launch shapes from the package's tuning cache for this device and workload, else
        # (or with --retune) timed now on 64 of the candidates
        from paper_2602_08266_amd import autotune
        if args.retune and os.path.exists(args.retune):
            os.remove(args.retune)
        tune = autotune.tune_score(ctx, scorer, cam_c, sample=64, cache=args.retune or autotune.CACHE,
                                   write_cache=bool(args.retune), log=log)
    elif args.ig_lpp:
        B.ngs_set_tuning(ctx, args.ig_lpp)
    if args.serialized_only:
        roofline, counts, breakdown = serialized_roofline(B, ctx, scorer, cam_c, scene, V, log)
        lpp = B.ngs_get_tuning(ctx)["ig_lanes_per_pixel"]
        ctx.close()
        return {"serialized_only": True, "roofline": roofline, "counts_per_view": counts,
                "kernels_us_per_view_serialized": breakdown, "views": V, "ig_lanes_per_pixel": lpp}
    for _ in range(args.warmup):
        scorer.score(cam_c)
    torch.cuda.synchronize()
    # headline: K scoring steps of every candidate, nothing but the scorer's own kernels
    times = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        scores, best, raw = scorer.score(cam_c)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    dt = sum(times)
    K = args.steps
    graph = None
    if not args.no_graph:
        # the same batch captured once into a HIP graph, replayed with one launch per step
        g = B.ScoreGraph(ctx, ds, scorer.h, cam_c, rp, ig, scorer.workspace(), normalisers=norm)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            g.replay()
        torch.cuda.synchronize()
        gdt = time.perf_counter() - t0
        graph = {"views_per_s": round(V * K / gdt, 2), "ms_per_step": round(gdt * 1e3 / K, 3),
                 "overflow": int(g.overflow.item()), "best_view": int(g.best.item()),
                 "max_rel_diff_vs_eager": float(((g.ig_raw - raw).abs() / raw.abs().clamp_min(1e-300)).max())}
        g.close()
    roofline, counts, breakdown = (None, {}, {})
    if not args.no_profile:
        roofline, counts, breakdown = serialized_roofline(B, ctx, scorer, cam_c, scene, V, log)
    value = V * K / dt
    ms_per_step = dt * 1e3 / K
    path = None
    if counts:
        # M of the 3DGS binning (the capacity pre-pass counts it; the scoring path's own lists
        # keep only the pairs a walk can take, counts["pairs_M"])
        pb = path_bytes(scene.n, scene.k, 1, float(pairs[:V].double().mean()), counts["touched_weighted_U"])
        path = {"algorithmic_bytes_per_view": int(pb), "achieved_GBs": round(pb * value / 1e9, 1),
                "frac_of_hbm_peak": round(pb * value / 1e9 / HBM_PEAK_GBS, 4)}
    mode = f"object-centric target {scene.target}" if scene.target >= 0 else "whole-scene confidence (Eq. 7)"
    res = sorted({(c.width, c.height) for c in cands})
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "views/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {scene.n} Gaussians, {cfg.clusters} clusters, k={scene.k}, "
                               f"{V} candidate views at {', '.join(f'{w}x{h}' for w, h in res)}, {mode}, "
                               f"radius U{list(cfg.radius)} m, {len(train)} training views",
                   "views_per_step": V, "gaussians": scene.n, "k": scene.k, "scorer": "exact",
                   "views_in_flight": scorer.views_in_flight,
                   "ig_lanes_per_pixel": B.ngs_get_tuning(ctx)["ig_lanes_per_pixel"],
                   "ig_waves_per_simd": B.ngs_get_tuning(ctx)["ig_waves_per_simd"],
                   "bin_chunk": B.ngs_get_tuning(ctx)["bin_chunk"],
                   "groups_in_flight": B.ngs_get_tuning(ctx)["groups_in_flight"],
                   "pair_capacity": scorer.max_pairs},
        "roofline": roofline, "path": path, "setup_ms": round(setup_ms, 1),
        "ms_per_step_median": round(float(np.median(times)) * 1e3, 3),
        "counts_per_view": counts, "pairs_per_view_prepass": {"max": int(pairs.max()), "mean": float(pairs.double().mean())},
        "best_view": int(best.item()), "normalisers": [float(x) for x in norm],
        "kernels_us_per_view_serialized": breakdown, "graph": graph,
        "autotune": None if tune is None else {"cached": tune.cached, "views_in_flight": tune.views_in_flight,
                                               "ig_lanes_per_pixel": tune.ig_lanes_per_pixel,
                                               "ig_waves_per_simd": tune.ig_waves_per_simd,
                                               "bin_chunk": tune.bin_chunk,
                                               "groups_in_flight": tune.groups_in_flight,
                                               "sample_ms_per_view": round(tune.ms_per_view, 4), "table": tune.table},
    }
    if args.workload == "batched640" and not args.no_mixed and args.views is None:
        del scorer
        torch.cuda.empty_cache()
        out["mixed_batch"] = run_mixed(args, B, ctx, log)
    ctx.close()
    return out


def run_mixed(args, B, ctx, log):
    """The mixed-resolution batch on the same 1M-Gaussian scene: 256 candidates (86 at 320x240,
    85 at 640x480, 85 at 1280x720) scored in one call per step, capacity from the pre-pass."""
    import numpy as np  # noqa: F401
    import torch

    import scenegen
    cfg, scene, cands, train = scenegen.make_workload("batched", args.seed)
    ds = B.DeviceScene(scene, "cuda:0")
    rp = B.raster_params()
    ig = B.ig_params(target_id=scene.target)
    cam_c = [B.camera(c) for c in cands]
    scorer, pairs = make_scorer(B, ctx, ds, scene, rp, ig, cam_c, [B.camera(c) for c in train],
                                args.in_flight, log)
    scorer.setup([B.camera(c) for c in train])
    tuned = B.ngs_get_tuning(ctx)
    scorer.views_in_flight = args.mixed_in_flight
    scorer.ws = None
    scorer.score(cam_c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        scores, best, raw = scorer.score(cam_c)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    V = len(cands)
    # the same 256-view batch captured once into a HIP graph: one launch per step
    g = B.ScoreGraph(ctx, ds, scorer.h, cam_c, rp, ig, scorer.workspace(), normalisers=scorer.norm)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    gdt = time.perf_counter() - t0
    graph = {"views_per_s": round(V * args.steps / gdt, 2), "ms_per_step": round(gdt * 1e3 / args.steps, 3),
             "overflow": int(g.overflow.item()), "best_view": int(g.best.item()),
             "max_rel_diff_vs_eager": float(((g.ig_raw - raw).abs() / raw.abs().clamp_min(1e-300)).max())}
    g.close()
    by_res = {}
    for (w, h) in sorted({(c.width, c.height) for c in cands}):
        idx = [i for i, c in enumerate(cands) if (c.width, c.height) == (w, h)]
        by_res[f"{w}x{h}"] = {"views": len(idx), "mean_pairs": float(pairs[idx].double().mean()),
                              "max_pairs": int(pairs[idx].max())}
    res = {"workload": f"batched: {scene.n} Gaussians, k={scene.k}, {V} candidates (86 at 320x240, 85 at 640x480, "
                       f"85 at 1280x720), object-centric target {scene.target}, radius U{list(cfg.radius)} m",
           "views_per_s": round(V * args.steps / dt, 2), "ms_per_step": round(dt * 1e3 / args.steps, 3),
           "views_in_flight": scorer.views_in_flight, "ig_lanes_per_pixel": tuned["ig_lanes_per_pixel"],
           "pair_capacity": scorer.max_pairs, "by_resolution": by_res, "best_view": int(best.item()), "graph": graph}
    log(f"mixed batch: {res['views_per_s']} views/s")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched640")
    ap.add_argument("--views", type=int, default=None, help="limit candidate views per step")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--in-flight", type=int, default=8, help="candidate views scored concurrently")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the serialized pass (one view in flight, kernels bracketed by events) that gives "
                         "the roofline and the per-kernel breakdown")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-resolution batch (256 views of 320x240, 640x480, 1280x720)")
    ap.add_argument("--mixed-in-flight", type=int, default=32, help="views in flight of the mixed batch")
    ap.add_argument("--serialized-only", action="store_true",
                    help="only the setup and the serialized pass (one view in flight): the run whose rocprofv3 "
                         "kernel trace gives the dominant kernel's launch duration")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="only time the CPU oracle on a 16-view subset (all cores, and single-threaded)")
    ap.add_argument("--backward", action="store_true",
                    help="time the differentiable rasterizer (forward + loss + backward) on the 500k-Gaussian workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --in-flight and --ig-lpp instead of the autotuned launch shapes")
    ap.add_argument("--retune", default="", metavar="CACHE",
                    help="time every launch shape on 64 candidates (ignoring the package's tuning cache) and "
                         "write the result to CACHE")
    ap.add_argument("--ig-lpp", type=int, default=0, help="with --no-autotune: lanes per pixel of the IG kernel")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the second timed region, which replays the batch captured in a HIP graph")
    ap.add_argument("--surrogate", action="store_true",
                    help="train the learned view scorer on exact scores of seeded scenes and compare it with exact scoring")
    ap.add_argument("--sur-scenes", type=int, default=24, help="training scenes (2048 views each)")
    ap.add_argument("--sur-test-scenes", type=int, default=8)
    ap.add_argument("--sur-epochs", type=int, default=20)
    ap.add_argument("--sur-rescore", type=int, default=256,
                    help="candidates (of each scene's 2048) the exact scorer re-scores")
    ap.add_argument("--sur-dump", default="", help="write held-out predictions and exact scores (.npz)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (for scaling rocprofv3 FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the scorer is not sharded across GPUs "
              "(views would be split across GPUs with one all-gather of the scores).", file=sys.stderr)
        sys.exit(2)
    if args.backward:
        run_backward(args)
        return
    if args.surrogate:
        run_surrogate(args)
        return

    if args.cpu_plan:
        cpu_plan(args)
        return
    log = lambda m: (sys.stderr.write(m + "\n"), sys.stderr.flush())
    out = run_exact(args, log)
    if not args.no_cpu_baseline and not args.serialized_only:
        log("timing the CPU oracle on a sample of the candidates...")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
