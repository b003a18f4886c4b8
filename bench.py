"""Throughput of exact next-best-view scoring on one MI355X.

Workload: 1M Gaussians in 64 object clusters (object vector k = 64), object-centric scoring
of a seeded target (Eq. 12), candidate views at 640x480 (fx = fy = 525) on a sphere of
radius U[0.4, 0.9] m -- the 640x480 share of the mixed-resolution batch. One step scores
every candidate view: projection, binning and sorting, the fused compositing +
information-gain walk, the FP64 finalize, Eq. 10-11 and the argmax. The training set
(4 views: H_T and the Eq. 10 normalisers) is built once before timing and reported apart.

Prints one JSON line. With --gpus N > 1 it exits: this build targets one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

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
    if name == "ig_tiles":
        # front-to-back walk: list entry, 2D mean, conic and opacity of every walked entry;
        # back-to-front walk over the W2 entries from a tile's last contributor to its nearest
        # weighted one: weight flag, depth, colour and the k-long probability row (the object
        # suffixes of the weighted Gaussians in front sum the rows of every contributing
        # Gaussian behind them); the statistics (94 + 6k floats) of every touched weighted
        # Gaussian written
        return W * 28 + W2 * (24 + 4 * k) + U * 4 * (94 + 6 * k)
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
    "ig_tiles": ["info_gain.hip", "common.hpp"], "ig_finalize": ["finalize.hip", "common.hpp"],
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


def cpu_baseline(workload_name, seed, views=3, threads=None):
    """The FP64 oracle timed on the host on a bounded sample: the first `views` candidate
    views of the workload scored against H_T = lambda I (training blocks would triple the
    time). Each view's work is split across the oracle's threads."""
    import oracle
    import scenegen
    cfg, scene, cands, train = scenegen.make_workload(workload_name, seed)
    ig = oracle.IGParams(target_id=scene.target)
    th = threads or oracle.default_threads()
    t0 = time.perf_counter()
    oracle.score(scene, [], cands[:views], ig=ig, threads=th)
    dt = time.perf_counter() - t0
    return {"value": views / dt, "unit": "views/s", "cores": th, "kind": "oracle",
            "sample": f"{views} candidate views ({cands[0].width}x{cands[0].height}, {scene.n} Gaussians, k={scene.k}, "
                      f"object-centric), H_T = lambda I, FP64, {dt:.1f} s"}


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
    t_feat = t_exact = t_rescore = 0.0
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
            t_rescore += s.seconds_rescore
        log(f"scene {seed}: features {s.seconds_features:.2f} s, exact {s.seconds_exact:.2f} s, "
            f"exact re-score of 32 {s.seconds_rescore:.3f} s")
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
    # the surrogate pipeline: feature maps and network for every candidate, then the exact
    # re-score of its 32 best per scene
    sur_views_s = nt / (t_feat + t_net + t_rescore)
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
        "surrogate_feature_s": round(t_feat, 3), "surrogate_network_s": round(t_net, 4),
        "surrogate_rescore_s": round(t_rescore, 3), "exact_s": round(t_exact, 3),
        "rescore": args.sur_rescore, "agreement_heldout": ag.__dict__,
        "agreement_heldout_by_rescore": ag_budget, "agreement_train": ag_train.__dict__,
        "train": {"pairs": ntr, "epochs": args.sur_epochs, "seconds": round(t_train, 2),
                  "loss_per_epoch": [round(h, 4) for h in hist], "label_mean": mu, "label_std": sd},
        "roofline": {"bound": "mfma", "kernel": "sur_gemm",
                     "achieved": round(gemm_tflops, 2) if gemm_tflops else None, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(gemm_tflops / 2500.0, 5) if gemm_tflops else None, "traffic": None,
                     "avg_launch_us": round(gemm_ms / gemm_n * 1e3, 2) if gemm_n else None}}), flush=True)


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
    ap.add_argument("--no-profile", action="store_true", help="do not bracket kernels with events")
    ap.add_argument("--backward", action="store_true",
                    help="time the differentiable rasterizer (forward + loss + backward) on the 500k-Gaussian workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --in-flight and --ig-lpp instead of the autotuned launch shapes")
    ap.add_argument("--retune", default="", metavar="CACHE",
                    help="time every launch shape on 32 candidates (ignoring the package's tuning cache) and "
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
        print("bench.py measures one GPU only: the scorer is not sharded across GPUs in this build "
              "(views would be split across GPUs with one all-gather of the scores).", file=sys.stderr)
        sys.exit(2)
    if args.backward:
        run_backward(args)
        return
    if args.surrogate:
        run_surrogate(args)
        return

    import numpy as np
    import torch

    import scenegen
    from paper_2602_08266_amd import binding as B

    torch.cuda.set_device(0)
    cfg, scene, cands, train = scenegen.make_workload(args.workload, args.seed, n_views=args.views)
    V = len(cands)
    ctx = B.Context(0)
    ds = B.DeviceScene(scene, "cuda:0")
    rp = B.raster_params()
    ig = B.ig_params(target_id=scene.target)
    scorer = B.NbvScorer(ctx, ds, rp, ig, max_pairs=48 << 20, max_slots=1 << 16, store_capacity=1 << 17,
                         views_in_flight=args.in_flight)
    cam_c = [B.camera(c) for c in cands]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norm = scorer.setup([B.camera(c) for c in train])
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    tune = None
    if not args.no_autotune:
        # launch shapes from the package's tuning cache for this device and workload, else
        # (or with --retune) timed now on 32 of the candidates
        from paper_2602_08266_amd import autotune
        if args.retune and os.path.exists(args.retune):
            os.remove(args.retune)
        tune = autotune.tune_score(ctx, scorer, cam_c, sample=32, cache=args.retune or autotune.CACHE,
                                   write_cache=bool(args.retune),
                                   log=lambda m: (sys.stderr.write(m + "\n"), sys.stderr.flush()))
    elif args.ig_lpp:
        B.ngs_set_tuning(ctx, args.ig_lpp)
    stats = torch.zeros(B.STATS_LEN, dtype=torch.int64, device="cuda:0")
    for _ in range(args.warmup):
        scorer.score(cam_c, stats)
    torch.cuda.synchronize()
    breakdown, dom = {}, None
    if not args.no_profile:
        # per-kernel breakdown from one more step with every kernel class bracketed by events,
        # outside the timed region; inside it only the dominant class carries events
        B.ngs_profile_enable(ctx, True)
        scorer.score(cam_c)
        torch.cuda.synchronize()
        breakdown = {k: v for k, v in B.ngs_profile_read(ctx).items() if v[1] > 0}
        dom = max(breakdown, key=lambda k: breakdown[k][0])
        B.ngs_profile_enable(ctx, True, only=dom)
    stats.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        scores, best, raw = scorer.score(cam_c, stats)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = B.ngs_profile_read(ctx) if not args.no_profile else {}
    B.ngs_profile_enable(ctx, False)
    st = stats.cpu().numpy()
    graph = None
    if not args.no_graph:
        # the same batch captured once into a HIP graph, replayed with one launch per step
        g = B.ScoreGraph(ctx, ds, scorer.h, cam_c, rp, ig, scorer.ws, normalisers=norm)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        gdt = time.perf_counter() - t0
        gbest = int(g.best.item())
        graph = {"views_per_s": round(V * args.steps / gdt, 2), "ms_per_step": round(gdt * 1e3 / args.steps, 3),
                 "overflow": int(g.overflow.item()), "best_view": gbest,
                 "max_rel_diff_vs_eager": float(((g.ig_raw - raw).abs() / raw.abs().clamp_min(1e-300)).max())}
        g.close()
    K = args.steps
    ms_per_step = dt * 1e3 / K
    value = V * K / dt
    # per step counts (stats accumulate over the timed calls)
    M_step = int(st[1]) / K
    W_step = int(st[4]) / K
    U_step = int(st[2]) / K
    W2_step = int(st[6]) / K
    roofline = None
    if prof and prof.get(dom, (0.0, 0))[1] > 0:
        ms_tot, launches = prof[dom]
        alg = algorithmic_bytes(dom, scene.n, scene.k, V, M_step, W_step, U_step, W2_step)
        if alg is not None:
            per_launch = alg / (launches / K)
            avg_s = ms_tot / launches / 1e3
            achieved = per_launch / avg_s / 1e9
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(dom, args.workload),
                        "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2),
                        "algorithmic_bytes_per_launch": int(per_launch)}
        else:
            roofline = {"bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                        "traffic": None, "kernel": dom, "avg_launch_us": round(ms_tot / launches * 1e3, 2)}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "views/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {scene.n} Gaussians, {cfg.clusters} clusters, k={scene.k}, "
                               f"{V} candidate views at {cands[0].width}x{cands[0].height}, object-centric target "
                               f"{scene.target}, radius U{list(cfg.radius)} m, 4 training views",
                   "views_per_step": V, "gaussians": scene.n, "k": scene.k, "scorer": "exact",
                   "views_in_flight": scorer.views_in_flight, "ig_lanes_per_pixel": B.ngs_get_tuning(ctx)["ig_lanes_per_pixel"]},
        "roofline": roofline,
        "path": {"algorithmic_bytes_per_view": int(path_bytes(scene.n, scene.k, V, M_step, U_step) / V),
                 "achieved_GBs": round(path_bytes(scene.n, scene.k, V, M_step, U_step) / (ms_per_step / 1e3) / 1e9, 1),
                 "frac_of_hbm_peak": round(path_bytes(scene.n, scene.k, V, M_step, U_step) / (ms_per_step / 1e3) / 1e9
                                           / HBM_PEAK_GBS, 4)},
        "setup_ms": round(setup_ms, 1),
        "pairs_per_view": M_step / V, "walked_entries_per_view": W_step / V,
        "back_to_front_entries_per_view": W2_step / V,
        "contrib_pairs_per_view": int(st[3]) / K / V, "touched_weighted_per_view": int(st[2]) / K / V,
        "best_view": int(best.item()), "normalisers": [float(x) for x in norm],
        "kernels_ms_per_step": {k: round(v[0], 3) for k, v in sorted(breakdown.items(), key=lambda x: -x[1][0])},
        "graph": graph,
        "autotune": None if tune is None else {"cached": tune.cached, "views_in_flight": tune.views_in_flight,
                                               "ig_lanes_per_pixel": tune.ig_lanes_per_pixel,
                                               "sample_ms_per_view": round(tune.ms_per_view, 4), "table": tune.table},
    }
    if not args.no_cpu_baseline:
        sys.stderr.write("timing the CPU oracle on one view...\n")
        sys.stderr.flush()
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
